// Spectral route: one eigendecomposition of each real symmetric
// H = -t K + diag(h) of the batch, then every matrix A_b = z_b I - H from the
// spectrum,
//   ln|det A_b|      = sum_k ln|z_b - lambda_k|
//   (A_b^-1)_ii      = sum_k psi_k(i)^2 / (z_b - lambda_k)
// (H = sum_k lambda_k psi_k psi_k^T; the determinant is the product of the
// eigenvalues of A_b and the resolvent is diagonal in the eigenbasis).  The
// per-matrix outputs are the ones the factorisation routes write, so the
// Matsubara/spin reduction downstream is shared.
//
// The eigendecomposition follows the Householder / bisection / inverse
// iteration scheme (Golub & Van Loan, Sec. 8.3-8.4; LAPACK's dsytrd, dstebz,
// dstein describe the same steps):
//   eig_init_kernel    dense H per h vector
//   hh_step_kernel     one launch per column j while the trailing block
//                      exceeds 160 rows: the pending reflector of
//                      column j-1 is applied to the trailing block of the
//                      workgroup's rows; column j is formed from the
//                      previous launch's copy, its reflector built
//                      (redundantly in every workgroup) and kept (V, tau),
//                      and p = tau A v of the workgroup's rows written for
//                      the next launch.  H = Q T Q^T, Q = H_0 H_1 .. H_{N-2},
//                      T tridiagonal (d, e).
//   hh_tail_kernel     the last columns (trailing block of at most 160 rows)
//                      in one workgroup of four waves per h vector, the
//                      block in registers: three barriers per column instead
//                      of a launch (every column when N <= 161).
//   bisect_kernel      T splits where |e_i| <= 2 eps |T|; one wave per
//                      eigenvalue: 64 Sturm counts per round (65-section),
//                      ten rounds.
//   invit_kernel       one lane per eigenvalue: pivoted LU of T_blk - lambda,
//                      three solves from a counter-hashed start vector
//                      (invit_reg_kernel for N <= 1024: one wave per
//                      eigenvalue with the factors and the iterate in
//                      registers, the same arithmetic).
//   mgs_kernel         eigenvalues of one block closer than 1e-4 |T_blk| form
//                      a cluster; its vectors are orthonormalised in index
//                      order (block Gram-Schmidt over rows, two passes).
//   wy_t_kernel        compact WY factor T of each block of 32 reflectors:
//                      H_j0 .. H_j0+31 = I - V T V^T (Schreiber & Van Loan)
//   wy_apply_reg_kernel psi = Q Z in place: the blocks applied to Z from
//                      the last to the first, each workgroup on its own
//                      slice of 16 columns (no dependency between
//                      workgroups), the slice held in MFMA accumulators,
//                      V^T Z and V W2 on the f64 MFMA (N <= 2304;
//                      wy_apply_kernel above, the slice staged through LDS).
//   expand_kernel      dg[b][i] = sum_k psi_k(i)^2 / (z_b - lambda_k)
//   lad_kernel         lad[b] = sum_k ln|z_b - lambda_k|, growth[b] = 1
#include <algorithm>
#include <float.h>
#include <math.h>
#include "k_factor_common.h"
#include "sca_common.h"
#include "sca_kernels.h"
#include "sca_profile.h"
#include "sca_runtime.h"

namespace sca {

namespace {

constexpr int kRowsPerWg = 4;     // hh_step (N <= 512): one wave per row
constexpr int kTailWaves = 4;     // hh_tail: waves of the one workgroup
constexpr int kTailRows = 40;     // hh_tail: rows per wave
constexpr int kTailKM = 3;        // hh_tail: column registers per row
constexpr int kTailMax = kTailWaves * kTailRows;   // trailing block it keeps
constexpr int kTailCols = 64 * kTailKM;             // columns the lanes span
static_assert(kTailMax <= kTailCols, "rows and columns of the block");
constexpr int kWy = 32;           // reflectors per compact WY block
constexpr int kWyCols = 16;       // columns of Z per back-transform workgroup
constexpr int kBisRounds = 10;    // 65^-10 of the Gershgorin width
constexpr int kInvIters = 3;
constexpr double kEps = DBL_EPSILON;
constexpr double kClusterTol = 1e-4;
constexpr double kSplitTol = 2.0;   // split where |e_i| <= kSplitTol eps |T|

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

__device__ inline double wave_sum(double v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}
__device__ inline double wave_maxd(double v) {
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}
__device__ inline double wave_mind(double v) {
  for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off));
  return v;
}
__device__ inline int wave_maxi(int v) {
  for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off));
  return v;
}
__device__ inline int wave_mini(int v) {
  for (int off = 32; off >= 1; off >>= 1) v = min(v, __shfl_xor(v, off));
  return v;
}

// sum over the W waves of a workgroup (every thread gets the result; the
// waves' partial sums are added in wave order)
template <int W = 4>
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int k = 1; k < W; ++k) s += red[k];
  return s;
}

// uniform in (-1, 1) from a 64-bit counter (SplitMix64 finaliser)
__device__ inline double hash_uniform(unsigned long long x) {
  x += 0x9E3779B97F4A7C15ULL;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
  x ^= x >> 31;
  return (double)(x >> 11) * 0x1.0p-52 - 1.0;
}

}  // namespace

struct EigBufs {
  double* A;      // [nH][N][N] working matrix; later Z (eigenvectors of T)
  double* V;      // [nH][N][N] reflector j in row j (v_j, zero up to j)
  double* taus;   // [nH][N] tau_j
  double* Tb;     // [nH][nwy][kWy][kWy] compact WY factors
  double* lu;     // [nH][4][N][N] u0^-1, u1, u2, m of T_blk - lambda_t,
                  //  element (local row j, eigenvalue t) at j * N + t
  unsigned char* piv;   // [nH][N][N] row swap of elimination step j
  double* vec;    // [nH][6][N] v[2], p[2], col[2] (parity of the column)
  double* tau;    // [nH][2]
  double* d;      // [nH][N] diagonal of T
  double* e;      // [nH][N] off-diagonal of T (e[i] couples i, i+1)
  double* lam;    // [nH][N] eigenvalues (ascending inside each block)
  double* bnorm;  // [nH][N] |T_blk| of the block of eigenvalue t
  int* bnd;       // [nH][2][N] block [b0, b1) of eigenvalue t
};

size_t eig_workspace_bytes(int N, int nH) {
  const size_t n2 = (size_t)nH * N * N, n1 = (size_t)nH * N;
  const size_t nwy = (size_t)nH * ((N + kWy - 1) / kWy) * kWy * kWy;
  return 2 * al256(sizeof(double) * n2) + al256(sizeof(double) * n1) +
         al256(sizeof(double) * nwy) + al256(sizeof(double) * 4 * n2) +
         al256(n2) + al256(sizeof(double) * 6 * n1) +
         al256(sizeof(double) * 2 * nH) + 4 * al256(sizeof(double) * n1) +
         al256(sizeof(int) * 2 * n1);
}

static EigBufs carve_eig(void* ws, int N, int nH) {
  const size_t n2 = (size_t)nH * N * N, n1 = (size_t)nH * N;
  char* c = static_cast<char*>(ws);
  EigBufs E;
  auto take = [&](size_t bytes) { char* r = c; c += al256(bytes); return r; };
  E.A = (double*)take(sizeof(double) * n2);
  E.V = (double*)take(sizeof(double) * n2);
  E.taus = (double*)take(sizeof(double) * n1);
  E.Tb = (double*)take(sizeof(double) * (size_t)nH * ((N + kWy - 1) / kWy) *
                       kWy * kWy);
  E.lu = (double*)take(sizeof(double) * 4 * n2);
  E.piv = (unsigned char*)take(n2);
  E.vec = (double*)take(sizeof(double) * 6 * n1);
  E.tau = (double*)take(sizeof(double) * 2 * nH);
  E.d = (double*)take(sizeof(double) * n1);
  E.e = (double*)take(sizeof(double) * n1);
  E.lam = (double*)take(sizeof(double) * n1);
  E.bnorm = (double*)take(sizeof(double) * n1);
  E.bnd = (int*)take(sizeof(int) * 2 * n1);
  return E;
}

// grid (N, nH): row i of H_hv (hopping of problem hv / 2)
__global__ void __launch_bounds__(256)
eig_init_kernel(const ProbDesc* __restrict__ probs, const double* __restrict__ hbuf,
                int N, int L, EigBufs E) {
  const int i = blockIdx.x, hv = blockIdx.y;
  const double t = probs[hv >> 1].t;
  const double hi = hbuf[(size_t)hv * N + i];
  double* A = E.A + ((size_t)hv * N + i) * N;
  for (int j = threadIdx.x; j < N; j += 256)
    A[j] = -t * (double)kmult(i, j, L) + (i == j ? hi : 0.0);
}

// Householder step j (0 <= j < N), grid (ceil(N / WV) - first, nH), WV
// waves; the launch covers the row blocks from `first` (the block of row
// j + 1) on.
// The reflector of column j-1 (v, tau, p = tau A_{j-1} v: support [j, N))
// is pending from the previous launch; w = p - (tau/2)(p.v) v and
// A_j = A_{j-1} - v w^T - w v^T on [j, N)^2.
// Column j of A_j is formed from the previous launch's copy of column j of
// A_{j-1}; its entries below the diagonal give the reflector of column j
// (v_{j+1} = 1, tau = (beta - alpha)/beta, beta = -sign(alpha) |x|).
// Rows and columns below j+1 of A are never read again, so a wave keeps
// only A[r][j+1 ..] of its row r > j in registers: lane
// holds columns c0 + lane + 64 k, k < KM; every global load of the launch
// is issued before the first reduction.
template <int KM, int WV>
__global__ void __launch_bounds__(WV * 64)
hh_step_kernel(int N, int j, int first, EigBufs E) {
  constexpr int NT = WV * 64;
  const int hv = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r = (first + blockIdx.x) * WV + w;   // this wave's row
  double* A = E.A + (size_t)hv * N * N;
  double* vb = E.vec + (size_t)hv * 6 * N;
  double* taub = E.tau + 2 * hv;
  extern __shared__ double sm[];
  double* sv = sm;            // pending v
  double* sw = sm + N;        // pending w
  double* sx = sm + 2 * N;    // column j of A_j, then the new v
  __shared__ double red[WV];
  const int cur = j & 1, prv = cur ^ 1;
  const bool pend = j > 0;
  const bool rowA = r < N && r > j;    // A row of this wave still in play
  double ar[KM];
#pragma unroll
  for (int k = 0; k < KM; ++k) {
    const int ca = j + 1 + lane + 64 * k;
    ar[k] = (rowA && ca < N) ? A[(size_t)r * N + ca] : 0.0;
  }
  double tp = 0.0;
  if (pend) {
    tp = taub[prv];
    const double* vp = vb + prv * N;
    const double* pp = vb + (2 + prv) * N;
    const double* cp = vb + (4 + prv) * N;
    double s = 0.0;
    for (int c = j + tid; c < N; c += NT) {
      const double a = vp[c], b = pp[c];
      sv[c] = a; sw[c] = b; sx[c] = cp[c]; s += a * b;
    }
    s = block_sum<WV>(s, red);
    const double K = 0.5 * tp * s;
    for (int c = j + tid; c < N; c += NT) sw[c] -= K * sv[c];
    __syncthreads();
    // column j of A_j, rows [j, N)
    const double wj = sw[j], vj = sv[j];
    for (int q = j + tid; q < N; q += NT) sx[q] -= sv[q] * wj + sw[q] * vj;
  } else {
    for (int q = tid; q < N; q += NT) sx[q] = A[(size_t)q * N];
  }
  // pending update of this wave's rows (registers)
  if (rowA && pend) {
    const double vr = sv[r], wr = sw[r];
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      const int c = j + 1 + lane + 64 * k;
      if (c < N) ar[k] -= vr * sw[c] + wr * sv[c];
    }
  }
  __syncthreads();
  if (j == N - 1) {   // last diagonal entry; no reflector
    if (blockIdx.x == 0 && tid == 0) E.d[(size_t)hv * N + j] = sx[j];
    return;
  }
  // reflector of column j from x = sx[j+1 .. N)
  const double alpha = sx[j + 1];
  double s = 0.0;
  for (int q = j + 2 + tid; q < N; q += NT) s += sx[q] * sx[q];
  s = block_sum<WV>(s, red);
  double tau, beta, scale;
  if (s == 0.0) {
    tau = 0.0; beta = alpha; scale = 0.0;
  } else {
    const double nrm = sqrt(alpha * alpha + s);
    beta = alpha >= 0.0 ? -nrm : nrm;
    tau = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
  const double dj = sx[j];
  __syncthreads();   // every thread has read alpha and dj
  for (int q = j + 1 + tid; q < N; q += NT) sx[q] = (q == j + 1) ? 1.0 : sx[q] * scale;
  __syncthreads();
  if (blockIdx.x == 0) {
    if (tid == 0) {
      E.d[(size_t)hv * N + j] = dj;
      E.e[(size_t)hv * N + j] = beta;
      E.taus[(size_t)hv * N + j] = tau;
      taub[cur] = tau;
    }
    double* vn = vb + cur * N;
    double* vrow = E.V + ((size_t)hv * N + j) * N;
    for (int q = tid; q < N; q += NT) {
      const double vq = q > j ? sx[q] : 0.0;
      vrow[q] = vq;
      if (q > j) vn[q] = vq;
    }
  }
  // p = tau A_j v, the copy of column j+1 of A_j, and the row for the next
  // launch (columns j+2 ..; column j+1 travels in the copy)
  if (rowA) {
    double pr = 0.0;
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      const int c = j + 1 + lane + 64 * k;
      if (c < N) {
        pr += ar[k] * sx[c];
        if (c > j + 1) A[(size_t)r * N + c] = ar[k];
      }
    }
    pr = wave_sum(pr) * tau;
    if (lane == 0) {
      vb[(2 + cur) * N + r] = pr;
      vb[(4 + cur) * N + r] = ar[0];
    }
  }
}

// Sum over the 64 lanes, the same value in every lane: DPP inside each row
// of 16 lanes, then the four row sums in a fixed order.
__device__ inline double wave_sum_dpp(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  v += dpp_d<0x140>(v);
  return (readlane_d(v, 0) + readlane_d(v, 16)) +
         (readlane_d(v, 32) + readlane_d(v, 48));
}

// Householder steps j0 .. N-1, grid (1, nH), kTailWaves waves (one per
// SIMD, so the work every wave repeats costs once per SIMD): the same
// reflectors as hh_step_kernel (H_j = I - tau v v^T from column j of A_j),
// for a trailing block small enough for one workgroup's registers: rows and
// columns (j0, N), N - j0 - 1 <= kTailMax.  Wave w keeps rows
// r = j0 + 1 + w + kTailWaves i (i < kTailRows), lane columns
// c = j0 + 1 + lane + 64 k (k < kTailKM).  Per column j:
//   column j of A_j (sx, double-buffered in LDS) gives alpha, |x|^2 and the
//   reflector, formed by every wave;
//   p = tau A_j v by columns over the wave's rows (A_j is symmetric), the
//   waves' partial sums added in wave order;
//   K = tau (p.v) / 2, w = p - K v, A_{j+1} = A_j - v w^T - w v^T on the rows
//   and columns beyond j;
//   column j+1 of A_{j+1} below the diagonal is copied into the other sx as
//   row j+1 (symmetry), with its |x|^2, by the wave that keeps that row.
// Rows and columns that are finished (at or before j) or past N take
// v = w = 0, which leaves them unchanged and adds nothing to p; a wave skips
// its groups of finished rows (uniform branches).
// With j0 > 0 the reflector of column j0-1 is pending, as the launch of
// column j0-1 left it: v, p, tau and column j0 of A_{j0-1}.
__global__ void __launch_bounds__(kTailWaves * 64)
hh_tail_kernel(int N, int j0, EigBufs E) {
  constexpr int NT = kTailWaves * 64;
  const int hv = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int base = j0 + 1;   // first row and column kept
  const int m = N - base;    // rows and columns kept
  const double* A = E.A + (size_t)hv * N * N;
  const double* vb = E.vec + (size_t)hv * 6 * N;
  __shared__ double sxb[2][kTailCols + 1];   // column of A_j, index q - j0
  __shared__ double svp[2 * kTailCols];      // (v, p) at index c - base
  __shared__ double part[kTailWaves][kTailCols];
  __shared__ double ssq[2];                  // |x|^2 of the next column
  __shared__ double sv0[kTailCols + 1], sp0[kTailCols + 1];   // pending v, p
  const int ri1 = m > w ? (m - w + kTailWaves - 1) / kTailWaves : 0;
  double a[kTailRows][kTailKM];
#pragma unroll
  for (int i = 0; i < kTailRows; ++i) {
    const int r = base + w + kTailWaves * i;
#pragma unroll
    for (int k = 0; k < kTailKM; ++k) {
      const int c = base + lane + 64 * k;
      a[i][k] = (r < N && c < N) ? A[(size_t)r * N + c] : 0.0;
    }
  }
  double* sx = sxb[0];
  if (j0 > 0) {
    const int prv = (j0 - 1) & 1;
    const double tp = E.tau[2 * hv + prv];
    for (int t = tid; t <= m; t += NT) {
      sv0[t] = vb[prv * N + j0 + t];
      sp0[t] = vb[(2 + prv) * N + j0 + t];
      sx[t] = vb[(4 + prv) * N + j0 + t];
    }
    __syncthreads();
    double s = 0.0;
    for (int t = lane; t <= m; t += 64) s += sv0[t] * sp0[t];
    const double K = 0.5 * tp * wave_sum_dpp(s);
    // column j0 of A_j0 from the copy (each thread its own entries), then
    // the kept rows
    const double vj = sv0[0], wj = sp0[0] - K * sv0[0];
    for (int t = tid; t <= m; t += NT) {
      const double wq = sp0[t] - K * sv0[t];
      sx[t] -= sv0[t] * wj + wq * vj;
    }
    double vc[kTailKM], wc[kTailKM];
#pragma unroll
    for (int k = 0; k < kTailKM; ++k) {
      const int t = 1 + lane + 64 * k;
      vc[k] = t <= m ? sv0[t] : 0.0;
      wc[k] = t <= m ? sp0[t] - K * sv0[t] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < kTailRows; ++i) {
      if (i < ri1) {
        const int t = 1 + w + kTailWaves * i;
        const double vr = sv0[t], wr = sp0[t] - K * sv0[t];
#pragma unroll
        for (int k = 0; k < kTailKM; ++k) a[i][k] -= vr * wc[k] + wr * vc[k];
      }
    }
  } else {
    for (int q = tid; q < N; q += NT) sx[q] = A[(size_t)q * N];
  }
  __syncthreads();
  // Per-row scalars (v_r, w_r) reach the rows' loops by readlane from the
  // lane numbered like the row (lane i holds row i of the wave), so a row
  // costs no LDS wait; rows are skipped in groups of kTailGrp.
  constexpr int kTailGrp = 8;
  static_assert(kTailRows % kTailGrp == 0 && kTailRows <= 64, "row groups");
  const int tl = w + kTailWaves * lane;   // local index of this lane's row
  int cur = 0;
  for (int j = j0; j < N - 1; ++j) {
    const double* sxc = sxb[cur];
    double* sxn = sxb[cur ^ 1];
    const int jl = j - j0;   // column j+1 is local column jl
    // first row of this wave in play (t = w + kTailWaves i >= jl)
    const int ri0 = jl > w ? (jl - w + kTailWaves - 1) / kTailWaves : 0;
    // reflector of column j from x = column j of A_j below the diagonal
    const double alpha = sxc[jl + 1];
    double s2;
    if (j == j0) {
      s2 = 0.0;
      for (int q = j + 2 + lane; q < N; q += 64) {
        const double x = sxc[q - j0];
        s2 += x * x;
      }
      s2 = wave_sum_dpp(s2);
    } else {
      s2 = ssq[cur];
    }
    double tau, beta, scale;
    if (s2 == 0.0) {
      tau = 0.0; beta = alpha; scale = 0.0;
    } else {
      const double nrm = sqrt(alpha * alpha + s2);
      beta = alpha >= 0.0 ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    // v at local index t: 0 before jl, 1 at jl, x scale beyond, 0 past N
    auto vloc = [&](int t) {
      const double x = sxc[t + 1];
      return (t > jl && t < m) ? x * scale : (t == jl ? 1.0 : 0.0);
    };
    if (tid == 0) {
      E.d[(size_t)hv * N + j] = sxc[jl];
      E.e[(size_t)hv * N + j] = beta;
      E.taus[(size_t)hv * N + j] = tau;
    }
    double* vrow = E.V + ((size_t)hv * N + j) * N;
    for (int q = tid; q < N; q += NT)
      vrow[q] = q > j + 1 ? sxc[q - j0] * scale : (q == j + 1 ? 1.0 : 0.0);
    // p = tau A_j v: the wave's rows, by columns
    const double vl = lane < kTailRows ? vloc(tl) : 0.0;
    double pc[kTailKM];
#pragma unroll
    for (int k = 0; k < kTailKM; ++k) pc[k] = 0.0;
#pragma unroll
    for (int g = 0; g < kTailRows; g += kTailGrp) {
      if (g + kTailGrp > ri0) {
#pragma unroll
        for (int i = g; i < g + kTailGrp; ++i) {
          const double vr = readlane_d(vl, i);
#pragma unroll
          for (int k = 0; k < kTailKM; ++k) pc[k] = fma(a[i][k], vr, pc[k]);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kTailKM; ++k) part[w][lane + 64 * k] = pc[k];
    __syncthreads();
    // v and p side by side for the update's reads
    if (tid < m) {
      double s = part[0][tid];
#pragma unroll
      for (int ww = 1; ww < kTailWaves; ++ww) s += part[ww][tid];
      svp[2 * tid] = vloc(tid);
      svp[2 * tid + 1] = tau * s;
    }
    __syncthreads();
    // K = tau (p.v) / 2, then A_{j+1} = A_j - v w^T - w v^T beyond j
    double pv = 0.0;
    for (int t = jl + lane; t < m; t += 64) pv += svp[2 * t] * svp[2 * t + 1];
    const double K = 0.5 * tau * wave_sum_dpp(pv);
    double vc[kTailKM], wc[kTailKM];
#pragma unroll
    for (int k = 0; k < kTailKM; ++k) {
      const int t = lane + 64 * k;
      const bool act = t >= jl && t < m;
      vc[k] = act ? svp[2 * t] : 0.0;
      wc[k] = act ? svp[2 * t + 1] - K * vc[k] : 0.0;
    }
    double rv = 0.0, rw = 0.0;   // v and w of this lane's row
    if (lane < kTailRows && tl >= jl && tl < m) {
      rv = svp[2 * tl];
      rw = svp[2 * tl + 1] - K * rv;
    }
#pragma unroll
    for (int g = 0; g < kTailRows; g += kTailGrp) {
      if (g + kTailGrp > ri0) {
#pragma unroll
        for (int i = g; i < g + kTailGrp; ++i) {
          const double vr = readlane_d(rv, i), wr = readlane_d(rw, i);
#pragma unroll
          for (int k = 0; k < kTailKM; ++k)
            a[i][k] = fma(-wr, vc[k], fma(-vr, wc[k], a[i][k]));
        }
      }
    }
    // column j+1 of A_{j+1} below the diagonal as row j+1 (A_{j+1} is
    // symmetric): row jl / kTailWaves of wave jl % kTailWaves, every lane
    // its columns; that wave also forms the next |x|^2 (columns beyond j+2)
    if (w == jl % kTailWaves) {
      const int is = jl / kTailWaves;
      double sq = 0.0;
#pragma unroll
      for (int g = 0; g < kTailRows; g += kTailGrp) {
        if (is >= g && is < g + kTailGrp) {
#pragma unroll
          for (int i = g; i < g + kTailGrp; ++i) {
            if (i == is) {
#pragma unroll
              for (int k = 0; k < kTailKM; ++k) {
                const int t = lane + 64 * k;
                const double x = a[i][k];
                if (t >= jl && t < m) sxn[t + 1] = x;
                sq = (t >= jl + 2 && t < m) ? fma(x, x, sq) : sq;
              }
            }
          }
        }
      }
      sq = wave_sum_dpp(sq);
      if (lane == 0) ssq[cur ^ 1] = sq;
    }
    __syncthreads();
    cur ^= 1;
  }
  // last diagonal entry; no reflector
  if (tid == 0) E.d[(size_t)hv * N + N - 1] = sxb[cur][N - 1 - j0];
}

// Sturm count of T_blk - x (rows [b0, b1)): eigenvalues below x.
__device__ inline int sturm_count(const double* __restrict__ d,
                                  const double* __restrict__ e2, int b0, int b1,
                                  double x, double pivmin) {
  int c = 0;
  double q = d[b0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  c += q < 0.0;
#pragma unroll 4
  for (int i = b0 + 1; i < b1; ++i) {
    q = (d[i] - x) - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
  }
  return c;
}

// grid (ceil(N / 4), nH), 256 threads: one wave per eigenvalue t.  The
// split points, the block of t and its Gershgorin interval come from
// wave reductions; the interval then shrinks 65-fold per round.
__global__ void __launch_bounds__(256)
bisect_kernel(int N, EigBufs E) {
  const int hv = blockIdx.y, lane = threadIdx.x & 63;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  const double* d = E.d + (size_t)hv * N;
  double* e = E.e + (size_t)hv * N;
  extern __shared__ double sm[];
  double* sd = sm;        // d
  double* se2 = sm + N;   // e^2 with the splits set to zero
  __shared__ double red[4];
  // |T| (Gershgorin) over the whole matrix
  double tn = 0.0;
  for (int i = threadIdx.x; i < N; i += 256) {
    const double el = i > 0 ? fabs(e[i - 1]) : 0.0;
    const double er = i < N - 1 ? fabs(e[i]) : 0.0;
    tn = fmax(tn, fabs(d[i]) + el + er);
  }
  tn = wave_maxd(tn);
  if (lane == 0) red[threadIdx.x >> 6] = tn;
  __syncthreads();
  tn = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  const double split = kSplitTol * kEps * tn;
  for (int i = threadIdx.x; i < N; i += 256) {
    sd[i] = d[i];
    const double ei = i < N - 1 ? e[i] : 0.0;
    se2[i] = fabs(ei) <= split ? 0.0 : ei * ei;
  }
  __syncthreads();
  if (t >= N) return;
  // block [b0, b1) of t: b0 - 1 = last split below t, b1 - 1 = first at/after t
  int lo_s = -1, hi_s = N - 1;
  for (int i = lane; i < N - 1; i += 64) {
    if (se2[i] == 0.0) {
      if (i < t) lo_s = max(lo_s, i);
      else hi_s = min(hi_s, i);
    }
  }
  const int b0 = wave_maxi(lo_s) + 1, b1 = wave_mini(hi_s) + 1;
  double gl = DBL_MAX, gu = -DBL_MAX, bn = 0.0, emax = 0.0;
  for (int i = b0 + lane; i < b1; i += 64) {
    const double el = i > b0 ? sqrt(se2[i - 1]) : 0.0;
    const double er = i < b1 - 1 ? sqrt(se2[i]) : 0.0;
    gl = fmin(gl, sd[i] - el - er);
    gu = fmax(gu, sd[i] + el + er);
    bn = fmax(bn, fabs(sd[i]) + el + er);
    emax = fmax(emax, i < b1 - 1 ? se2[i] : 0.0);
  }
  gl = wave_mind(gl); gu = wave_maxd(gu); bn = wave_maxd(bn); emax = wave_maxd(emax);
  const int n = b1 - b0, k = t - b0;
  const double pivmin = DBL_MIN * fmax(1.0, emax);
  const double pad = 4.0 * kEps * bn * n + 2.0 * pivmin;
  double lo = gl - pad, hi = gu + pad;
  if (n > 1) {
    for (int it = 0; it < kBisRounds; ++it) {
      const double h = (hi - lo) / 65.0;
      const double x = lo + (lane + 1) * h;
      const int c = sturm_count(sd, se2, b0, b1, x, pivmin);
      const int m = __popcll(__ballot(c <= k));
      const double nlo = m > 0 ? lo + m * h : lo;
      const double nhi = m < 64 ? lo + (m + 1) * h : hi;
      lo = nlo; hi = nhi;
    }
  }
  if (lane == 0) {
    const size_t o = (size_t)hv * N + t;
    E.lam[o] = n > 1 ? 0.5 * (lo + hi) : sd[t];
    E.bnorm[o] = bn;
    E.bnd[(size_t)hv * 2 * N + t] = b0;
    E.bnd[(size_t)hv * 2 * N + N + t] = b1;
  }
}

// grid (ceil(N / 64), nH), 64 threads: lane = eigenvalue t.  Column t of Z
// (stored over A) is zero outside the block of t; inside it the inverse
// iteration with T_blk - lambda_t = P L U (partial pivoting; pivots below
// eps |T_blk| raised to it).  Each solve is a serial chain per lane: d and e
// come from LDS, and the factors and the right-hand side are loaded a group
// of kG steps ahead of the stores of the current group.
constexpr int kG = 8;
__global__ void __launch_bounds__(64)
invit_kernel(int N, EigBufs E) {
  const int hv = blockIdx.y;
  const int t = blockIdx.x * 64 + threadIdx.x;
  const size_t o = (size_t)hv * N;
  extern __shared__ double sm[];
  double* sd = sm;
  double* se = sm + N;
  for (int i = threadIdx.x; i < N; i += 64) { sd[i] = E.d[o + i]; se[i] = E.e[o + i]; }
  __syncthreads();
  if (t >= N) return;
  double* __restrict__ Z = E.A + (size_t)hv * N * N;
  const size_t n2 = (size_t)N * N;
  double* __restrict__ U0 = E.lu + (size_t)hv * 4 * n2;
  double* __restrict__ U1 = U0 + n2;
  double* __restrict__ U2 = U1 + n2;
  double* __restrict__ Mm = U2 + n2;
  unsigned char* __restrict__ Pv = E.piv + (size_t)hv * n2;
  const int b0 = E.bnd[o * 2 + t], b1 = E.bnd[o * 2 + N + t];
  const int n = b1 - b0;
  const double lam = E.lam[o + t], bn = E.bnorm[o + t];
  for (int q = 0; q < N; ++q)
    if (q < b0 || q >= b1) Z[(size_t)q * N + t] = 0.0;
  if (n == 1) { Z[(size_t)b0 * N + t] = 1.0; return; }
  const double tol = kEps * bn;
  // elimination; the current row holds (cd, cs) at columns (i, i+1)
  double cd = sd[b0] - lam, cs = se[b0];
  for (int i = 0; i < n - 1; ++i) {
    const double ci = se[b0 + i];
    const double an = sd[b0 + i + 1] - lam;
    const double bnx = i + 1 < n - 1 ? se[b0 + i + 1] : 0.0;
    const bool pv = fabs(ci) > fabs(cd);
    double u0, u1, u2, m;
    if (pv) {
      u0 = ci; u1 = an; u2 = bnx;
      m = cd / ci;
      const double ncd = cs - m * an;
      cs = -m * bnx;
      cd = ncd;
    } else {
      if (cd == 0.0) cd = tol;
      u0 = cd; u1 = cs; u2 = 0.0;
      m = ci / cd;
      cd = an - m * cs;
      cs = bnx;
    }
    if (fabs(u0) < tol) u0 = u0 >= 0.0 ? tol : -tol;
    const size_t ix = (size_t)i * N + t;
    U0[ix] = 1.0 / u0; U1[ix] = u1; U2[ix] = u2; Mm[ix] = m; Pv[ix] = pv;
  }
  if (fabs(cd) < tol) cd = cd >= 0.0 ? tol : -tol;
  U0[(size_t)(n - 1) * N + t] = 1.0 / cd;
  double* __restrict__ x = Z + (size_t)b0 * N + t;   // x[i] at x[i * N]
  const unsigned long long seed = (unsigned long long)t << 32;
  const int nf = n - 1;   // forward steps
  double sc = 1.0;
  for (int it = 0; it < kInvIters; ++it) {
    // forward: L^-1 P (sc y); y is the hashed start vector on the first pass
    const bool first = it == 0;
    double carry = first ? hash_uniform(seed) : sc * x[0];
    double ya[kG] = {}, ma[kG] = {}, yb[kG] = {}, mb[kG] = {};
    unsigned char pa[kG] = {}, pb[kG] = {};
    auto load_f = [&](int i0, double* y, double* m, unsigned char* p) {
#pragma unroll
      for (int u = 0; u < kG; ++u) {
        const int i = i0 + u;
        if (i < nf) {
          y[u] = first ? hash_uniform(seed | (unsigned)(i + 1))
                       : x[(size_t)(i + 1) * N];
          m[u] = Mm[(size_t)i * N + t];
          p[u] = Pv[(size_t)i * N + t];
        }
      }
    };
    load_f(0, ya, ma, pa);
    for (int i0 = 0; i0 < nf; i0 += kG) {
      if (i0 + kG < nf) load_f(i0 + kG, yb, mb, pb);
#pragma unroll
      for (int u = 0; u < kG; ++u) {
        const int i = i0 + u;
        if (i < nf) {
          const double y = first ? ya[u] : sc * ya[u];
          double out;
          if (pa[u]) { out = y; carry = carry - ma[u] * y; }
          else { out = carry; carry = y - ma[u] * carry; }
          x[(size_t)i * N] = out;
        }
      }
#pragma unroll
      for (int u = 0; u < kG; ++u) { ya[u] = yb[u]; ma[u] = mb[u]; pa[u] = pb[u]; }
    }
    // backward: U^-1, with the largest magnitude for the next scaling
    double x2 = carry * U0[(size_t)nf * N + t];
    x[(size_t)nf * N] = x2;
    double x1 = (x[(size_t)(nf - 1) * N] - U1[(size_t)(nf - 1) * N + t] * x2) *
                U0[(size_t)(nf - 1) * N + t];
    x[(size_t)(nf - 1) * N] = x1;
    double mx = fmax(fabs(x1), fabs(x2));
    double ra[kG] = {}, a0[kG] = {}, a1[kG] = {}, a2[kG] = {};
    double rb[kG] = {}, c0[kG] = {}, c1[kG] = {}, c2[kG] = {};
    auto load_b = [&](int i0, double* r, double* u0, double* u1, double* u2) {
#pragma unroll
      for (int u = 0; u < kG; ++u) {
        const int i = i0 - u;
        if (i >= 0) {
          const size_t ix = (size_t)i * N + t;
          r[u] = x[(size_t)i * N]; u0[u] = U0[ix]; u1[u] = U1[ix]; u2[u] = U2[ix];
        }
      }
    };
    const int top = nf - 2;   // first row of the general recurrence
    if (top >= 0) load_b(top, ra, a0, a1, a2);
    for (int i0 = top; i0 >= 0; i0 -= kG) {
      if (i0 - kG >= 0) load_b(i0 - kG, rb, c0, c1, c2);
#pragma unroll
      for (int u = 0; u < kG; ++u) {
        const int i = i0 - u;
        if (i >= 0) {
          const double xi = (ra[u] - a1[u] * x1 - a2[u] * x2) * a0[u];
          x[(size_t)i * N] = xi;
          mx = fmax(mx, fabs(xi));
          x2 = x1; x1 = xi;
        }
      }
#pragma unroll
      for (int u = 0; u < kG; ++u) { ra[u] = rb[u]; a0[u] = c0[u]; a1[u] = c1[u]; a2[u] = c2[u]; }
    }
    sc = 1.0 / mx;
  }
  double s2 = 0.0;
  for (int i = 0; i < n; ++i) {
    const double v = sc * x[(size_t)i * N];
    s2 += v * v;
  }
  const double f = sc / sqrt(s2);
  for (int i = 0; i < n; ++i) x[(size_t)i * N] *= f;
}

// grid (N, nH), 64 threads: one wave per eigenvalue t, for N <= 64 SPL.  The
// iteration of invit_kernel (the same arithmetic and start vector) with the
// factors and the iterate in registers: lane l keeps rows
// SPL l .. SPL l + SPL - 1, and the serial recurrences, run by every lane on
// the same values, take a row's entries with readlane and put them back
// with a select on the lane (nothing on the chain waits for memory).  The
// backward solve starts at row n-1 with the two later rows' values zero,
// which gives its first two rows exactly (the extra terms are +-0).
// Against the same iteration with the block of T, the factors and the
// iterate in LDS (lane 0 running the recurrences; bitwise the same output):
// 0.381 -> 0.247 ms at N = 400, 2.81 -> 1.41 ms at 1024; the
// lane-per-eigenvalue kernel took 1.74 ms at 1024 (both spins, as
// measured).
template <int SPL>
__global__ void __launch_bounds__(64)
invit_reg_kernel(int N, EigBufs E) {
  const int t = blockIdx.x, hv = blockIdx.y, lane = threadIdx.x;
  const size_t o = (size_t)hv * N;
  const int b0 = E.bnd[o * 2 + t], b1 = E.bnd[o * 2 + N + t];
  const int n = b1 - b0;
  double* Z = E.A + (size_t)hv * N * N;
  for (int q = lane; q < N; q += 64)
    if (q < b0 || q >= b1) Z[(size_t)q * N + t] = 0.0;
  if (n == 1) {
    if (lane == 0) Z[(size_t)b0 * N + t] = 1.0;
    return;
  }
  extern __shared__ double sm[];
  double* __restrict__ sd = sm;       // d, e of the block, then x
  double* __restrict__ se = sd + n;
  double* __restrict__ xs = se + n;
  const double lam = E.lam[o + t], bn = E.bnorm[o + t];
  const unsigned long long seed = (unsigned long long)t << 32;
  for (int i = lane; i < n; i += 64) {
    sd[i] = E.d[o + b0 + i];
    se[i] = E.e[o + b0 + i];
  }
  double rx[SPL], ru0[SPL], ru1[SPL], ru2[SPL], rm[SPL];
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    const int i = SPL * lane + s;
    rx[s] = i < n ? hash_uniform(seed | (unsigned)i) : 0.0;
    ru0[s] = 0.0; ru1[s] = 0.0; ru2[s] = 0.0; rm[s] = 0.0;
  }
  static_assert(SPL <= 32, "the pivot bits of a lane's rows fill one int");
  int rpv = 0;   // bit s: row SPL lane + s pivoted
  // lane dst takes v (the same value in every lane), the others keep old
  auto put = [&](double old, double v, int dst) { return lane == dst ? v : old; };
  __syncthreads();
  const int nblk = (n + SPL - 1) / SPL;
  // elimination; the current row holds (cd, cs) at columns (i, i+1)
  const double tol = kEps * bn;
  double cd = sd[0] - lam, cs = se[0];
  for (int b = 0; b < nblk; ++b) {
    int bits = 0;
#pragma unroll
    for (int s = 0; s < SPL; ++s) {
      const int i = SPL * b + s;
      if (i < n - 1) {
        const double ci = se[i];
        const double an = sd[i + 1] - lam;
        const double bnx = i + 1 < n - 1 ? se[i + 1] : 0.0;
        const bool pv = fabs(ci) > fabs(cd);
        double u0, u1, u2, m;
        if (pv) {
          u0 = ci; u1 = an; u2 = bnx;
          m = cd / ci;
          const double ncd = cs - m * an;
          cs = -m * bnx;
          cd = ncd;
        } else {
          if (cd == 0.0) cd = tol;
          u0 = cd; u1 = cs; u2 = 0.0;
          m = ci / cd;
          cd = an - m * cs;
          cs = bnx;
        }
        if (fabs(u0) < tol) u0 = u0 >= 0.0 ? tol : -tol;
        ru0[s] = put(ru0[s], 1.0 / u0, b);
        ru1[s] = put(ru1[s], u1, b);
        ru2[s] = put(ru2[s], u2, b);
        rm[s] = put(rm[s], m, b);
        bits |= pv ? 1 << s : 0;
      }
    }
    rpv = lane == b ? bits : rpv;
  }
  if (fabs(cd) < tol) cd = cd >= 0.0 ? tol : -tol;
  {
    const int i = n - 1, b = i / SPL;
#pragma unroll
    for (int s = 0; s < SPL; ++s)
      if (s == i % SPL) ru0[s] = put(ru0[s], 1.0 / cd, b);
  }
  const int nf = n - 1;
  double sc = 1.0;
  for (int it = 0; it < kInvIters; ++it) {
    // forward: L^-1 P (sc x)
    double carry = sc * readlane_d(rx[0], 0);
    for (int b = 0; b < nblk; ++b) {
      const int bits = __builtin_amdgcn_readlane(rpv, b);
#pragma unroll
      for (int s = 0; s < SPL; ++s) {
        const int i = SPL * b + s;
        if (i < nf) {
          const double xn = s + 1 < SPL ? readlane_d(rx[(s + 1) % SPL], b)
                                        : readlane_d(rx[0], b + 1);
          const double y = sc * xn;
          const double m = readlane_d(rm[s], b);
          double out;
          if ((bits >> s) & 1) { out = y; carry = carry - m * y; }
          else { out = carry; carry = y - m * carry; }
          rx[s] = put(rx[s], out, b);
        }
      }
    }
    // row nf takes carry; backward: U^-1 with the largest magnitude
    {
      const int b = nf / SPL;
#pragma unroll
      for (int s = 0; s < SPL; ++s)
        if (s == nf % SPL) rx[s] = put(rx[s], carry, b);
    }
    double x1 = 0.0, x2 = 0.0, mx = 0.0;
    for (int b = nf / SPL; b >= 0; --b) {
#pragma unroll
      for (int s = SPL - 1; s >= 0; --s) {
        const int i = SPL * b + s;
        if (i <= nf) {
          const double xi = (readlane_d(rx[s], b) - readlane_d(ru1[s], b) * x1 -
                             readlane_d(ru2[s], b) * x2) * readlane_d(ru0[s], b);
          rx[s] = put(rx[s], xi, b);
          mx = fmax(mx, fabs(xi));
          x2 = x1; x1 = xi;
        }
      }
    }
    sc = 1.0 / mx;
  }
  // normalisation: the rows through LDS, a wave sum of their squares
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    const int i = SPL * lane + s;
    if (i < n) xs[i] = rx[s];
  }
  __syncthreads();
  double s2 = 0.0;
  for (int i = lane; i < n; i += 64) {
    const double v = sc * xs[i];
    s2 += v * v;
  }
  s2 = wave_sum(s2);
  const double f = sc / sqrt(s2);
  for (int i = lane; i < n; i += 64) Z[(size_t)(b0 + i) * N + t] = xs[i] * f;
}

// grid (ceil(N / 4), nH), 256 threads: the wave of eigenvalue t acts if t
// starts a cluster of two or more inside its block.  The cluster's vectors
// are the columns t .. c1-1 of Z, contiguous inside each row, so the wave
// works on rows (lane l takes rows b0 + l + 64 k): each vector jc is made
// orthogonal to the earlier ones in chunks of kMgsChunk (one pass over the
// rows forms the chunk's dot products, a second subtracts the projections:
// block Gram-Schmidt), then normalised; the whole is done twice.
constexpr int kMgsChunk = 16;
__global__ void __launch_bounds__(256)
mgs_kernel(int N, EigBufs E) {
  const int hv = blockIdx.y, lane = threadIdx.x & 63;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= N) return;
  const size_t o = (size_t)hv * N;
  const int b0 = E.bnd[o * 2 + t], b1 = E.bnd[o * 2 + N + t];
  const double* lam = E.lam + o;
  const double gap = kClusterTol * E.bnorm[o + t];
  if (!(t == b0 || lam[t] - lam[t - 1] >= gap)) return;   // not a leader
  int c1 = t + 1;
  while (c1 < b1 && lam[c1] - lam[c1 - 1] < gap) ++c1;
  if (c1 - t < 2) return;
  double* Z = E.A + (size_t)hv * N * N;
  for (int jc = t + 1; jc < c1; ++jc) {
    for (int pass = 0; pass < 2; ++pass) {
      for (int q0 = t; q0 < jc; q0 += kMgsChunk) {
        const int nq = min(kMgsChunk, jc - q0);
        double d[kMgsChunk];
#pragma unroll
        for (int i = 0; i < kMgsChunk; ++i) d[i] = 0.0;
        for (int r = b0 + lane; r < b1; r += 64) {
          const double* zr = Z + (size_t)r * N;
          const double x = zr[jc];
#pragma unroll
          for (int i = 0; i < kMgsChunk; ++i)
            if (i < nq) d[i] = fma(x, zr[q0 + i], d[i]);
        }
#pragma unroll
        for (int i = 0; i < kMgsChunk; ++i) d[i] = wave_sum(d[i]);
        for (int r = b0 + lane; r < b1; r += 64) {
          double* zr = Z + (size_t)r * N;
          double x = zr[jc];
#pragma unroll
          for (int i = 0; i < kMgsChunk; ++i)
            if (i < nq) x = fma(-d[i], zr[q0 + i], x);
          zr[jc] = x;
        }
      }
      double s2 = 0.0;
      for (int r = b0 + lane; r < b1; r += 64) {
        const double v = Z[(size_t)r * N + jc];
        s2 += v * v;
      }
      s2 = wave_sum(s2);
      // a vector that the projections annihilated cannot be trusted: NaN
      // propagates to the caller's non-finite flag
      const double f = s2 > 1e-24 ? 1.0 / sqrt(s2) : NAN;
      for (int r = b0 + lane; r < b1; r += 64) Z[(size_t)r * N + jc] *= f;
    }
  }
}

// grid (ceil((N - 1) / kWy), nH), 256 threads: T of the block of reflectors
// j0 .. j0 + nb - 1 (forward, column by column: T_ii = tau_i,
// T[0:i, i] = -tau_i T[0:i, 0:i] V[:, 0:i]^T v_i), from the Gram matrix of
// the block's vectors (rows staged through LDS 64 at a time).
__global__ void __launch_bounds__(256)
wy_t_kernel(int N, EigBufs E) {
  const int blk = blockIdx.x, hv = blockIdx.y, tid = threadIdx.x;
  const int nref = N - 1, j0 = blk * kWy, nb = min(kWy, nref - j0);
  const double* V = E.V + (size_t)hv * N * N;
  __shared__ double vs[kWy][65];
  __shared__ double G[kWy][kWy + 1];
  __shared__ double T[kWy][kWy + 1];
  // pairs (m, i): thread owns m = tid >> 3, i = (tid & 7) + 8 u, u < 4
  const int m = tid >> 3;
  double g[4] = {0.0, 0.0, 0.0, 0.0};
  for (int r0 = j0 + 1; r0 < N; r0 += 64) {
    for (int u = tid; u < kWy * 64; u += 256) {
      const int ii = u >> 6, rr = u & 63, r = r0 + rr;
      vs[ii][rr] = (ii < nb && r < N) ? V[(size_t)(j0 + ii) * N + r] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < 64; ++rr) {
      const double a = vs[m][rr];
#pragma unroll
      for (int u = 0; u < 4; ++u) g[u] = fma(a, vs[(tid & 7) + 8 * u][rr], g[u]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) G[m][(tid & 7) + 8 * u] = g[u];
  __syncthreads();
  if (tid < 64) {
    const int k = tid;   // row of T this lane builds
    for (int i = 0; i < kWy; ++i) {
      const double ti = i < nb ? E.taus[(size_t)hv * N + j0 + i] : 0.0;
      double acc = 0.0;
      if (k < i)
        for (int mm = k; mm < i; ++mm) acc += T[k][mm] * G[mm][i];
      if (k < kWy) T[k][i] = k < i ? -ti * acc : (k == i ? ti : 0.0);
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
  }
  __syncthreads();
  double* To = E.Tb + (((size_t)hv * gridDim.x + blk) * kWy) * kWy;
  for (int u = tid; u < kWy * kWy; u += 256) To[u] = T[u / kWy][u % kWy];
}

// grid (ceil(N / kWyCols), nH), 256 threads: Z[:, k0 .. k0+16) <- Q Z by the
// blocks from the last to the first, Z <- Z - V (T (V^T Z)) on the rows
// below j0 of each block, both products on the f64 MFMA (16x16x4; A[m][k]
// from lane k*16+m, B[k][n] from lane k*16+n, accumulator element e of lane
// g*16+n holds row g+4e).  Each 64-row chunk of V and Z is staged in LDS:
// W = V^T Z takes the chunk's rows in steps of 4 split over the waves
// (partial sums reduced through LDS); Z -= V W2 gives each wave one
// 16-row tile.  Used above N = 2304 (wy_apply_reg_kernel below).
__global__ void __launch_bounds__(256)
wy_apply_kernel(int N, EigBufs E) {
  typedef double v4 __attribute__((ext_vector_type(4)));
  const int hv = blockIdx.y, tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6, g = lane >> 4, q = lane & 15;
  const int k0 = blockIdx.x * kWyCols;
  const int nref = N - 1, nwy = (nref + kWy - 1) / kWy;
  const double* V = E.V + (size_t)hv * N * N;
  double* Z = E.A + (size_t)hv * N * N;
  __shared__ double vs[kWy][65];                 // V[j0 + i][r0 + rr]
  __shared__ double zs[64][kWyCols + 1];         // Z[r0 + rr][k0 + n]
  __shared__ double wp[4][kWy][kWyCols + 1];     // per-wave partial W
  __shared__ double w2[kWy][kWyCols + 1];
  __shared__ double ts[kWy][kWy + 1];
  for (int blk = nwy - 1; blk >= 0; --blk) {
    const int j0 = blk * kWy, nb = min(kWy, nref - j0);
    const double* Tg = E.Tb + (((size_t)hv * nwy + blk) * kWy) * kWy;
    for (int u = tid; u < kWy * kWy; u += 256) ts[u / kWy][u % kWy] = Tg[u];
    // W = V^T Z: wave w takes row steps rr = 4 (w + 4 s), s < 4, of each chunk
    v4 c0 = {0.0, 0.0, 0.0, 0.0}, c1 = {0.0, 0.0, 0.0, 0.0};
    for (int r0 = j0 + 1; r0 < N; r0 += 64) {
      for (int u = tid; u < kWy * 64; u += 256) {
        const int ii = u >> 6, rr = u & 63, r = r0 + rr;
        vs[ii][rr] = (ii < nb && r < N) ? V[(size_t)(j0 + ii) * N + r] : 0.0;
      }
      for (int u = tid; u < 64 * kWyCols; u += 256) {
        const int rr = u >> 4, kk = u & 15, r = r0 + rr, c = k0 + kk;
        zs[rr][kk] = (r < N && c < N) ? Z[(size_t)r * N + c] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int rr = 4 * (w + 4 * st) + g;   // this lane's k (row)
        const double b = zs[rr][q];
        c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(vs[q][rr], b, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(vs[16 + q][rr], b, c1, 0, 0, 0);
      }
      __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      wp[w][g + 4 * e][q] = c0[e];
      wp[w][16 + g + 4 * e][q] = c1[e];
    }
    __syncthreads();
    // W2 = T W (T upper triangular); W = sum of the waves' parts in order
    for (int u = tid; u < kWy * kWyCols; u += 256) {
      const int i = u >> 4, n = u & 15;
      double b = 0.0;
      for (int mm = i; mm < kWy; ++mm) {
        const double wv = ((wp[0][mm][n] + wp[1][mm][n]) + wp[2][mm][n]) + wp[3][mm][n];
        b = fma(ts[i][mm], wv, b);
      }
      w2[i][n] = b;
    }
    __syncthreads();
    // Z -= V W2: wave w takes rows [r0 + 16 w, +16) of each chunk
    for (int r0 = j0 + 1; r0 < N; r0 += 64) {
      for (int u = tid; u < kWy * 64; u += 256) {
        const int ii = u >> 6, rr = u & 63, r = r0 + rr;
        vs[ii][rr] = (ii < nb && r < N) ? V[(size_t)(j0 + ii) * N + r] : 0.0;
      }
      __syncthreads();
      v4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < kWy / 4; ++ks) {
        const int i = 4 * ks + g;   // this lane's k
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(vs[i][16 * w + q], w2[i][q],
                                                   acc, 0, 0, 0);
      }
      const int c = k0 + q;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = r0 + 16 * w + g + 4 * e;
        if (r < N && c < N) Z[(size_t)r * N + c] -= acc[e];
      }
      __syncthreads();
    }
  }
}

// grid (ceil(N / 16), nH), WAVES * 64 threads, N <= 16 * WAVES * TPW: the
// back-transformation of wy_apply_kernel with the slice Z[:, k0 .. k0+16)
// resident in MFMA accumulators for the whole kernel.  Wave w keeps the row
// tiles t = w + WAVES s (s < TPW); element e of lane g*16+n holds
// Z[16t + g + 4e][k0 + n], which is also the B operand of the k step over
// the tile's rows 4e .. 4e+3.  Per block of reflectors, last first:
//   W = V^T Z: per k step of each tile, A = V^T from global memory (the
//   block's two halves of 16 reflectors), B = element e of the tile; the
//   waves' partial W added in wave order through LDS;
//   W2 = T W in LDS;
//   Z -= V W2 on each tile: A = the tile's rows of V, B = W2.
// A wave skips its tiles wholly above the block's first row (the block's V
// is zero there), a uniform branch per tile: half the MFMA work of the
// whole slice, 0.80 -> 0.48 ms at N = 1024.  (Loading a tile's operands one
// to three tiles ahead measured no faster: the waves sharing a SIMD already
// cover the loads.)
template <int TPW, int WAVES>
__global__ void __launch_bounds__(WAVES * 64)
wy_apply_reg_kernel(int N, EigBufs E) {
  typedef double v4 __attribute__((ext_vector_type(4)));
  constexpr int NT = WAVES * 64;
  const int hv = blockIdx.y, tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6, g = lane >> 4, q = lane & 15;
  const int k0 = blockIdx.x * 16;
  const int nref = N - 1, nwy = (nref + kWy - 1) / kWy;
  const double* V = E.V + (size_t)hv * N * N;
  double* Z = E.A + (size_t)hv * N * N;
  __shared__ double wp[WAVES][kWy][17];   // per-wave partial W
  __shared__ double ws[kWy][17];          // W
  __shared__ double w2[kWy][17];
  __shared__ double ts[kWy][kWy + 1];
  const int c = k0 + q;
  v4 z[TPW];
#pragma unroll
  for (int s = 0; s < TPW; ++s) {
    const int t = w + WAVES * s;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = 16 * t + g + 4 * e;
      z[s][e] = (r < N && c < N) ? Z[(size_t)r * N + c] : 0.0;
    }
  }
  for (int blk = nwy - 1; blk >= 0; --blk) {
    const int j0 = blk * kWy, nb = min(kWy, nref - j0);
    const double* Tg = E.Tb + (((size_t)hv * nwy + blk) * kWy) * kWy;
    for (int u = tid; u < kWy * kWy; u += NT) ts[u / kWy][u % kWy] = Tg[u];
    // Loads read clamped, in-bounds positions and zero what lies outside
    // the block or past N afterwards (no branches around them); the tile's
    // row offset is made opaque so that the compiler forms each tile's
    // addresses at the tile, not all tiles' at once.
    const double* pa = V + (size_t)min(j0 + q, N - 1) * N;
    const double* pb = V + (size_t)min(j0 + 16 + q, N - 1) * N;
    const bool oka = q < nb, okb = 16 + q < nb;
    auto load_w = [&](int sx, double* a0, double* a1) {
      int r0 = 16 * (w + WAVES * sx) + g;
      asm volatile("" : "+v"(r0));
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = r0 + 4 * e, rc = min(r, N - 1);
        const double x0 = pa[rc], x1 = pb[rc];
        a0[e] = (oka && r < N) ? x0 : 0.0;
        a1[e] = (okb && r < N) ? x1 : 0.0;
      }
    };
    // W = V^T Z
    // tiles wholly above the block's first row (all of V zero there) are
    // skipped: this wave's tiles s >= slo
    const int tlo = (j0 + 1) >> 4;
    const int slo = tlo > w ? (tlo - w + WAVES - 1) / WAVES : 0;
    v4 c0 = {0.0, 0.0, 0.0, 0.0}, c1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < TPW; ++s) {
      if (s < slo) continue;
      double a0[4], a1[4];
      load_w(s, a0, a1);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[e], z[s][e], c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[e], z[s][e], c1, 0, 0, 0);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      wp[w][g + 4 * e][q] = c0[e];
      wp[w][16 + g + 4 * e][q] = c1[e];
    }
    __syncthreads();
    // W = the waves' parts added in wave order, then W2 = T W (T upper
    // triangular)
    for (int u = tid; u < kWy * 16; u += NT) {
      const int i = u >> 4, n = u & 15;
      double wv = wp[0][i][n];
#pragma unroll
      for (int ww = 1; ww < WAVES; ++ww) wv += wp[ww][i][n];
      ws[i][n] = wv;
    }
    __syncthreads();
    for (int u = tid; u < kWy * 16; u += NT) {
      const int i = u >> 4, n = u & 15;
      double b = 0.0;
      for (int mm = i; mm < kWy; ++mm) b = fma(ts[i][mm], ws[mm][n], b);
      w2[i][n] = b;
    }
    __syncthreads();
    // Z -= V W2
    double bw[kWy / 4];
#pragma unroll
    for (int ks = 0; ks < kWy / 4; ++ks) bw[ks] = w2[4 * ks + g][q];
    auto load_z = [&](int sx, double* a) {
      int r = 16 * (w + WAVES * sx) + q;
      asm volatile("" : "+v"(r));
      const int rc = min(r, N - 1);
#pragma unroll
      for (int ks = 0; ks < kWy / 4; ++ks) {
        const int k = 4 * ks + g;
        const double x = V[(size_t)min(j0 + k, N - 1) * N + rc];
        a[ks] = (k < nb && r < N) ? x : 0.0;
      }
    };
#pragma unroll
    for (int s = 0; s < TPW; ++s) {
      if (s < slo) continue;
      double a[kWy / 4];
      load_z(s, a);
#pragma unroll
      for (int ks = 0; ks < kWy / 4; ++ks)
        z[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[ks], bw[ks], z[s], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();   // ts, wp and w2 are rewritten by the next block
  }
#pragma unroll
  for (int s = 0; s < TPW; ++s) {
    const int t = w + WAVES * s;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = 16 * t + g + 4 * e;
      if (r < N && c < N) Z[(size_t)r * N + c] = z[s][e];
    }
  }
}

// grid (ceil(N / 64), ceil(B / 16)), 256 threads: rows [i0, i0+64) of the
// matrices [b0, b0+16).  Matrices of one tile that belong to different h
// vectors are done in turns (one per distinct h vector).  Thread: row
// i0 + (tid & 63), matrices b0 + 4 (tid >> 6) + {0..3}.
__global__ void __launch_bounds__(256)
expand_kernel(const MatDesc* __restrict__ descs, int B, int N, EigBufs E,
              double* __restrict__ dg) {
  const int i0 = blockIdx.x * 64, bt0 = blockIdx.y * 16;
  const int tid = threadIdx.x, il = tid & 63, bq = tid >> 6;
  __shared__ double ps[16][65];       // ps[k][i]
  __shared__ double wr[16][17], wi[16][17];   // [b][k]
  __shared__ int hvs[16];
  __shared__ double zr_s[16], zi_s[16];
  if (tid < 16) {
    const int b = bt0 + tid;
    if (b < B) {
      const MatDesc m = descs[b];
      hvs[tid] = m.hoff / N; zr_s[tid] = m.zr; zi_s[tid] = m.zi;
    } else {
      hvs[tid] = -1; zr_s[tid] = 0.0; zi_s[tid] = 0.0;
    }
  }
  __syncthreads();
  unsigned done = 0;   // tile members finished (uniform across the group)
  for (int b = 0; b < 16; ++b)
    if (hvs[b] < 0) done |= 1u << b;
  while (done != 0xFFFFu) {
    const int first = __builtin_ctz(~done);
    const int hv = hvs[first];
    unsigned mine = 0;
    for (int b = 0; b < 16; ++b)
      if (!(done >> b & 1) && hvs[b] == hv) mine |= 1u << b;
    const double* Z = E.A + (size_t)hv * N * N;   // psi, squared on load
    const double* lam = E.lam + (size_t)hv * N;
    double ar[4] = {}, ai[4] = {};
    for (int k0 = 0; k0 < N; k0 += 16) {
      for (int u = tid; u < 16 * 64; u += 256) {
        const int kk = u & 15, ii = u >> 4;
        const int gi = i0 + ii, gk = k0 + kk;
        const double z = (gi < N && gk < N) ? Z[(size_t)gi * N + gk] : 0.0;
        ps[kk][ii] = z * z;
      }
      {
        const int b = tid >> 4, kk = tid & 15, gk = k0 + kk;
        double re = 0.0, im = 0.0;
        if ((mine >> b & 1) && gk < N) {
          const double dr = zr_s[b] - lam[gk], di = zi_s[b];
          const double den = 1.0 / (dr * dr + di * di);
          re = dr * den; im = -di * den;
        }
        wr[b][kk] = re; wi[b][kk] = im;
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) {
        const double p = ps[kk][il];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          ar[x] = fma(p, wr[4 * bq + x][kk], ar[x]);
          ai[x] = fma(p, wi[4 * bq + x][kk], ai[x]);
        }
      }
      __syncthreads();
    }
    const int gi = i0 + il;
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      const int bl = 4 * bq + x;
      if ((mine >> bl & 1) && gi < N) {
        double* o = dg + ((size_t)(bt0 + bl) * N + gi) * 2;
        o[0] = ar[x]; o[1] = ai[x];
      }
    }
    done |= mine;
  }
}

// grid (B), 64 threads
__global__ void __launch_bounds__(64)
lad_kernel(const MatDesc* __restrict__ descs, int N, EigBufs E,
           double* __restrict__ lad, double* __restrict__ growth) {
  const int b = blockIdx.x;
  const MatDesc m = descs[b];
  const double* lam = E.lam + (size_t)(m.hoff / N) * N;
  double s = 0.0;
  for (int k = threadIdx.x; k < N; k += 64) {
    const double dr = m.zr - lam[k];
    s += log(dr * dr + m.zi * m.zi);
  }
  s = wave_sum(s);
  if (threadIdx.x == 0) {
    if (lad) lad[b] = 0.5 * s;
    if (growth) growth[b] = 1.0;
  }
}

hipError_t spectral_batch(const ProbDesc* probs, int nH, const MatDesc* descs,
                          const double* hbuf, int B, int N, int L, double* lad,
                          double* dg, double* growth, void* fact,
                          hipStream_t st) {
  if (nH <= 0 || !probs || !fact) return hipErrorInvalidValue;
  EigBufs E = carve_eig(fact, N, nH);
  mark_begin(K_TRIDIAG, st);
  hipLaunchKernelGGL(eig_init_kernel, dim3(N, nH), dim3(256), 0, st, probs,
                     hbuf, N, L, E);
  // rows (waves) per workgroup: 4 up to N = 512, 8 above (measured: 8 is
  // 6% faster at N = 1024, 2% slower at 400; 2 and 16 slower at both)
  const bool wide = N > 512;
  const int wv = wide ? 8 : kRowsPerWg;
  const int nrow = (N + wv - 1) / wv;
  auto kern = N <= 512 ? hh_step_kernel<8, kRowsPerWg>
            : N <= 1024 ? hh_step_kernel<16, 8>
            : N <= 2560 ? hh_step_kernel<40, 8> : hh_step_kernel<64, 8>;
  // above N = 1024 only the workgroups that hold rows below j (the others'
  // rows are finished; workgroup 0 of each launch also writes the
  // reflector): 13% less time at 2304, 2% more at 400 and 1024, as measured
  // the last columns in one launch, once the trailing block fits one
  // workgroup's registers
  const int j0 = std::max(0, N - 1 - kTailMax);
  for (int j = 0; j < j0; ++j) {
    const int first = N > 1024 ? std::min((j + 1) / wv, nrow - 1) : 0;
    hipLaunchKernelGGL(kern, dim3(nrow - first, nH), dim3(wv * 64),
                       sizeof(double) * 3 * N, st, N, j, first, E);
  }
  hipLaunchKernelGGL(hh_tail_kernel, dim3(1, nH), dim3(kTailWaves * 64), 0,
                     st, N, j0, E);
  mark_end(K_TRIDIAG, st);
  mark_begin(K_SPECTRUM, st);
  hipLaunchKernelGGL(bisect_kernel, dim3((N + 3) / 4, nH), dim3(256),
                     sizeof(double) * 2 * N, st, N, E);
  if (N <= 512) {
    hipLaunchKernelGGL(invit_reg_kernel<8>, dim3(N, nH), dim3(64),
                       sizeof(double) * 3 * N, st, N, E);
  } else if (N <= 1024) {
    hipLaunchKernelGGL(invit_reg_kernel<16>, dim3(N, nH), dim3(64),
                       sizeof(double) * 3 * N, st, N, E);
  } else {
    hipLaunchKernelGGL(invit_kernel, dim3((N + 63) / 64, nH), dim3(64),
                       sizeof(double) * 2 * N, st, N, E);
  }
  hipLaunchKernelGGL(mgs_kernel, dim3((N + 3) / 4, nH), dim3(256), 0, st, N,
                     E);
  const int nwy = (N - 1 + kWy - 1) / kWy;
  hipLaunchKernelGGL(wy_t_kernel, dim3(nwy, nH), dim3(256), 0, st, N, E);
  // Z in registers up to N = 2304 (both spins, as measured against Z
  // staged through LDS per block: 0.18 -> 0.13 ms at N = 400, 1.72 -> 0.48
  // at 1024, 10.8 -> 4.6 at 2304; the shapes are the fastest of those tried)
  if (N <= 512) {
    hipLaunchKernelGGL((wy_apply_reg_kernel<2, 16>), dim3((N + 15) / 16, nH),
                       dim3(1024), 0, st, N, E);
  } else if (N <= 1024) {
    hipLaunchKernelGGL((wy_apply_reg_kernel<4, 16>), dim3((N + 15) / 16, nH),
                       dim3(1024), 0, st, N, E);
  } else if (N <= 2304) {
    hipLaunchKernelGGL((wy_apply_reg_kernel<12, 12>), dim3((N + 15) / 16, nH),
                       dim3(768), 0, st, N, E);
  } else {
    hipLaunchKernelGGL(wy_apply_kernel, dim3((N + kWyCols - 1) / kWyCols, nH),
                       dim3(256), 0, st, N, E);
  }
  mark_end(K_SPECTRUM, st);
  mark_begin(K_EXPAND, st);
  if (dg)
    hipLaunchKernelGGL(expand_kernel, dim3((N + 63) / 64, (B + 15) / 16),
                       dim3(256), 0, st, descs, B, N, E, dg);
  hipLaunchKernelGGL(lad_kernel, dim3(B), dim3(64), 0, st, descs, N, E, lad,
                     growth);
  mark_end(K_EXPAND, st);
  return hipGetLastError();
}

}  // namespace sca
