// FP32 factor route with FP64 refinement.
//
// After the complex64 LU (P A ~ L U) and the complex64 triangular inverses
// W ~ U^-1, V ~ L^-1 (stored in place in F, original-row order):
//
//   wv_gemm_kernel   X = fl32(W V) on the f32 MFMA; Z = X P ~ A^-1, i.e.
//                    Z[i][r] = X[i][pos(r)].
//   refine_kernel    in FP64, per block of 32 pivot positions q (i = perm[q]):
//     * one Newton step for the diagonal of the inverse,
//         Z' = Z (2I - A Z)  =>  Z'_ii = 2 Z_ii - sum_j Z_ij (A Z)_ji,
//       whose error is O(|A^-1| |I - A Z|^2): FP32 accuracy squared;
//     * the log-determinant from the identity, exact for any Y,
//         ln|det A| = ln|det(A Y)| - ln|det Y|,  Y = W V P,
//       with |det Y| = prod |w_kk| (V unit lower) and
//         ln|det(A Y)| = Re ln det(I - R) = -Re tr R + O(|R|^2),
//         R = I - A Y,  tr(A Y) = sum over the 5 N non-zeros of A of
//         A_ij Y_ji, each Y_ji = W[j, :] . V[:, pos(i)] summed in FP64 from
//         the stored FP32 values (their products are exact in FP64).
//   finalize_kernel  fixed-order sum of the per-block log-det parts.
//
// A = z I - H with H = -t K + diag(h) is applied as its 5-point stencil.
#include <math.h>
#include "sca_common.h"
#include "sca_blocked.h"
#include "sca_profile.h"

namespace sca {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ inline f4 mma32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int GT = 64;   // output tile of the W V product
constexpr int GK = 16;   // k chunk

}  // namespace

// X[i][c] = sum_{k >= max(i, c)} W[i][k] V[k][c], V[c][c] = 1.
// W[i][k] is stored at F[perm[i]][k] (k >= i), V[k][c] at F[perm[k]][c]
// (k > c).  256 threads: 4 waves, each a 32 x 32 quarter of the 64 x 64 tile
// (2 x 2 MFMA tiles, real and imaginary accumulators).  Np is a multiple of
// 16; the tiles past Np are masked.
__global__ void __launch_bounds__(256)
wv_gemm_kernel(int Np, const float* __restrict__ F, const int* __restrict__ perm_g,
               float* __restrict__ X) {
  const int b = blockIdx.z;
  const int i0 = blockIdx.y * GT, c0 = blockIdx.x * GT;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = lane >> 4, q = lane & 15;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  __shared__ float Wr[GT][GK + 1], Wi[GT][GK + 1];   // [i][k]
  __shared__ float Vr[GK][GT + 1], Vi[GK][GT + 1];   // [k][c]
  __shared__ int prow[GT], pk[GK];
  const size_t plane = (size_t)Np * Np;
  const float* Fr = F + (size_t)b * 2 * plane;
  const float* Fi = Fr + plane;
  const int* perm = perm_g + (size_t)b * Np;
  if (tid < GT) prow[tid] = i0 + tid < Np ? perm[i0 + tid] : 0;
  f4 ar[2][2], ai[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      ar[a][c] = (f4){0.f, 0.f, 0.f, 0.f};
      ai[a][c] = (f4){0.f, 0.f, 0.f, 0.f};
    }
  const int kstart = (i0 > c0 ? i0 : c0);   // multiple of GT, so of GK
  for (int k0 = kstart; k0 < Np; k0 += GK) {
    __syncthreads();
    if (tid < GK) pk[tid] = perm[k0 + tid];
    // W tile: rows i0.., columns k0..k0+GK (upper: k >= i)
    for (int e = tid; e < GT * GK; e += 256) {
      const int r = e / GK, k = e % GK;
      const int gi = i0 + r, gk = k0 + k;
      float xr = 0.f, xi = 0.f;
      if (gk >= gi && gi < Np) {
        const size_t o = (size_t)prow[r] * Np + gk;
        xr = Fr[o];
        xi = Fi[o];
      }
      Wr[r][k] = xr;
      Wi[r][k] = xi;
    }
    __syncthreads();
    // V tile: rows k0.., columns c0..c0+GT (unit lower: k > c, 1 at k == c)
    for (int e = tid; e < GK * GT; e += 256) {
      const int k = e / GT, c = e % GT;
      const int gk = k0 + k, gc = c0 + c;
      float vr = 0.f, vi = 0.f;
      if (gc >= Np) {
        // masked column
      } else if (gk > gc) {
        const size_t o = (size_t)pk[k] * Np + gc;
        vr = Fr[o];
        vi = Fi[o];
      } else if (gk == gc) {
        vr = 1.f;
      }
      Vr[k][c] = vr;
      Vi[k][c] = vi;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < GK / 4; ++ks) {
      const int k = 4 * ks + g;
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const float w_r = Wr[wr + 16 * a + q][k], w_i = Wi[wr + 16 * a + q][k];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const float v_r = Vr[k][wc + 16 * c + q], v_i = Vi[k][wc + 16 * c + q];
          ar[a][c] = mma32(w_r, v_r, ar[a][c]);
          ar[a][c] = mma32(-w_i, v_i, ar[a][c]);
          ai[a][c] = mma32(w_r, v_i, ai[a][c]);
          ai[a][c] = mma32(w_i, v_r, ai[a][c]);
        }
      }
    }
  }
  float* Xr = X + (size_t)b * 2 * plane;
  float* Xi = Xr + plane;
  // f32 accumulator: element j of lane (g, q) holds row 4g + j, column q
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int gi = i0 + wr + 16 * a + 4 * g + j, gc = c0 + wc + 16 * c + q;
        if (gi < Np && gc < Np) {
          const size_t o = (size_t)gi * Np + gc;
          Xr[o] = ar[a][c][j];
          Xi[o] = ai[a][c][j];
        }
      }
}

// --------------------------------------------------------------------------

namespace {
constexpr int RQ = 32;   // pivot positions per workgroup
constexpr int RS = 32;   // s chunk (Newton step)
constexpr int RK = 16;   // k chunk (log-det: rows of W staged in LDS)
}  // namespace

__global__ void __launch_bounds__(256)
refine_kernel(int N, int Np, int L, const MatDesc* __restrict__ descs,
              const double* __restrict__ hbuf, const float* __restrict__ F,
              const int* __restrict__ perm_g, const float* __restrict__ X,
              double* __restrict__ dg, double* __restrict__ ldpart) {
  const int b = blockIdx.y;
  const int q0 = blockIdx.x * RQ;
  const int tid = threadIdx.x;
  const MatDesc dsc = descs[b];
  const double* h = hbuf + dsc.hoff;
  const size_t plane = (size_t)Np * Np;
  const float* Fr = F + (size_t)b * 2 * plane;
  const float* Fi = Fr + plane;
  const float* Xr = X + (size_t)b * 2 * plane;
  const float* Xi = Xr + plane;
  const int* perm = perm_g + (size_t)b * Np;

  __shared__ int iq[RQ];                       // i = perm[q]
  __shared__ int nbr[RQ][5];                   // {i} and its 4 neighbours
  // Newton step: X[i][s-chunk] and (A Z)[perm s][i]; the log-det phase
  // reuses the same space for its chunk of the 5 RQ rows of W
  __shared__ double nw_s[2 * RQ * (RS + 1) + 2 * RS * (RQ + 1)];
  double (*zr_s)[RS + 1] = reinterpret_cast<double (*)[RS + 1]>(nw_s);
  double (*zi_s)[RS + 1] = zr_s + RQ;
  double (*ar_s)[RQ + 1] = reinterpret_cast<double (*)[RQ + 1]>(nw_s + 2 * RQ * (RS + 1));
  double (*ai_s)[RQ + 1] = ar_s + RS;
  float (*wr_s)[RK + 1] = reinterpret_cast<float (*)[RK + 1]>(nw_s);
  float (*wi_s)[RK + 1] = wr_s + 5 * RQ;
  __shared__ float vr_s[RK][RQ + 1], vi_s[RK][RQ + 1];      // V[k][q]
  __shared__ int wrow_s[5 * RQ], jrow_s[5 * RQ];
  __shared__ double part_r[8][RQ], part_i[8][RQ];
  __shared__ double tr_part[256], ld_part[RQ];

  if (tid < RQ) {
    const int q = q0 + tid;
    const int i = (q < Np) ? perm[q] : Np;
    iq[tid] = i;
    if (i < N) {
      const int x = i % L, y = i / L;
      nbr[tid][0] = i;
      nbr[tid][1] = (x + 1) % L + L * y;
      nbr[tid][2] = (x + L - 1) % L + L * y;
      nbr[tid][3] = x + L * ((y + 1) % L);
      nbr[tid][4] = x + L * ((y + L - 1) % L);
    } else {
      for (int k = 0; k < 5; ++k) nbr[tid][k] = -1;
    }
  }
  __syncthreads();

  // ---- Newton step for Z_ii, i = perm[q] -----------------------------------
  // acc[q] = sum_s X[i][s] (A Z)_{perm[s], i},
  // (A Z)_{r, i} = (z - h_r) X[r][q] + t sum_{l ~ r} X[l][q]
  const int ql = tid % RQ, part = tid / RQ;   // 8 parts of the s-chunk
  double acc_r = 0.0, acc_i = 0.0;
  for (int s0 = 0; s0 < Np; s0 += RS) {
    __syncthreads();
    for (int e = tid; e < RQ * RS; e += 256) {
      const int a = e / RS, sl = e % RS;
      const int i = iq[a], s = s0 + sl;
      double xr = 0.0, xi = 0.0;
      if (i < N && s < Np) {
        const size_t o = (size_t)i * Np + s;
        xr = Xr[o];
        xi = Xi[o];
      }
      zr_s[a][sl] = xr;
      zi_s[a][sl] = xi;
    }
    for (int e = tid; e < RS * RQ; e += 256) {
      const int sl = e / RQ, a = e % RQ;
      const int s = s0 + sl, q = q0 + a;
      double vr = 0.0, vi = 0.0;
      if (s < Np && q < Np) {
        const int r = perm[s];
        if (r < N) {
          const double cr = dsc.zr - h[r], ci = dsc.zi;
          const size_t o = (size_t)r * Np + q;
          const double xr = Xr[o], xi = Xi[o];
          vr = cr * xr - ci * xi;
          vi = cr * xi + ci * xr;
          const int x = r % L, y = r / L;
          const int ls[4] = {(x + 1) % L + L * y, (x + L - 1) % L + L * y,
                             x + L * ((y + 1) % L), x + L * ((y + L - 1) % L)};
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const size_t ol = (size_t)ls[k] * Np + q;
            vr += dsc.t * (double)Xr[ol];
            vi += dsc.t * (double)Xi[ol];
          }
        }
      }
      ar_s[sl][a] = vr;
      ai_s[sl][a] = vi;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < RS / 8; ++k) {
      const int sl = part * (RS / 8) + k;
      const double xr = zr_s[ql][sl], xi = zi_s[ql][sl];
      const double yr = ar_s[sl][ql], yi = ai_s[sl][ql];
      acc_r += xr * yr - xi * yi;
      acc_i += xr * yi + xi * yr;
    }
  }
  part_r[part][ql] = acc_r;
  part_i[part][ql] = acc_i;
  __syncthreads();
  if (tid < RQ) {
    const int i = iq[tid], q = q0 + tid;
    if (i < N) {
      double sr = 0.0, si = 0.0;
      for (int p = 0; p < 8; ++p) { sr += part_r[p][tid]; si += part_i[p][tid]; }
      const size_t o = (size_t)i * Np + q;
      dg[((size_t)b * N + i) * 2 + 0] = 2.0 * (double)Xr[o] - sr;
      dg[((size_t)b * N + i) * 2 + 1] = 2.0 * (double)Xi[o] - si;
    }
  }

  // ---- log-det: tr(A Y) over this block's columns, -sum ln|w_qq| ---------
  // thread (a, k5) with a = tid / 5 < RQ handles Y_{nbr[a][k5], i_a}; the
  // rows of W it needs are staged in LDS a chunk of RK columns at a time
  const int a5 = tid / 5, k5 = tid % 5;
  const bool act = (tid < 5 * RQ) && (a5 < RQ) && nbr[a5 < RQ ? a5 : 0][k5] >= 0;
  const int jrow = act ? nbr[a5][k5] : 0;
  double yr = 0.0, yi = 0.0;
  // W[j][k] lives at F[perm[j]][k] for k >= j
  if (tid < 5 * RQ) {
    wrow_s[tid] = act ? perm[jrow] : -1;
    jrow_s[tid] = jrow;
  }
  for (int k0 = 0; k0 < Np; k0 += RK) {
    __syncthreads();
    for (int e = tid; e < 5 * RQ * RK; e += 256) {
      const int p = e / RK, kl = e % RK, k = k0 + kl;
      const int wr = wrow_s[p];
      float xr = 0.f, xi = 0.f;
      if (wr >= 0 && k < Np && k >= jrow_s[p]) {
        const size_t o = (size_t)wr * Np + k;
        xr = Fr[o];
        xi = Fi[o];
      }
      wr_s[p][kl] = xr;
      wi_s[p][kl] = xi;
    }
    for (int e = tid; e < RK * RQ; e += 256) {
      const int kl = e / RQ, a = e % RQ;
      const int k = k0 + kl, q = q0 + a;
      float vr = 0.f, vi = 0.f;
      if (k < Np && q < Np) {
        if (k > q) {
          const size_t o = (size_t)perm[k] * Np + q;
          vr = Fr[o];
          vi = Fi[o];
        } else if (k == q) {
          vr = 1.f;
        }
      }
      vr_s[kl][a] = vr;
      vi_s[kl][a] = vi;
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int kl = 0; kl < RK; ++kl) {
        const double wr_ = wr_s[tid][kl], wi_ = wi_s[tid][kl];
        const double vr = vr_s[kl][a5], vi = vi_s[kl][a5];
        yr += wr_ * vr - wi_ * vi;
        yi += wr_ * vi + wi_ * vr;
      }
    }
  }
  double contrib = 0.0;
  if (act) {
    const int i = iq[a5];
    // A_{i j}: diagonal z - h_i, neighbours t (K_ij counts coinciding ones)
    double cr, ci;
    if (k5 == 0) { cr = dsc.zr - h[i]; ci = dsc.zi; }
    else { cr = dsc.t; ci = 0.0; }
    contrib = cr * yr - ci * yi;   // Re(A_ij Y_ji)
  }
  tr_part[tid] = contrib;
  __syncthreads();
  if (tid < RQ) {
    double s = 0.0;
    for (int k = 0; k < 5; ++k) s += tr_part[5 * tid + k];
    const int q = q0 + tid;
    double lw = 0.0;
    if (q < Np && iq[tid] < N) {
      // w_qq at F[perm[q]][q]; -ln|w_qq| - 1 + Re(row contribution)
      const size_t o = (size_t)perm[q] * Np + q;
      lw = -log(hypot((double)Fr[o], (double)Fi[o]));
      s -= 1.0;
    } else {
      s = 0.0;
    }
    ld_part[tid] = lw + s;
  }
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int k = 0; k < RQ; ++k) s += ld_part[k];
    ldpart[(size_t)b * gridDim.x + blockIdx.x] = s;
  }
}

// lad[b] = sum of the per-block parts, in block order.
__global__ void finalize_logdet_kernel(const double* __restrict__ ldpart,
                                       int nblocks, int B,
                                       double* __restrict__ lad) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double s = 0.0;
  for (int k = 0; k < nblocks; ++k) s += ldpart[(size_t)b * nblocks + k];
  lad[b] = s;
}

int refine_blocks(int Np) { return (Np + RQ - 1) / RQ; }

hipError_t launch_wv_gemm(int B, int Np, const float* F, const int* perm,
                          float* X, hipStream_t st) {
  if (Np % GK) return hipErrorInvalidValue;
  const int nt = (Np + GT - 1) / GT;
  mark_begin(K_WVGEMM, st);
  hipLaunchKernelGGL(wv_gemm_kernel, dim3(nt, nt, B), dim3(256), 0,
                     st, Np, F, perm, X);
  mark_end(K_WVGEMM, st);
  return hipGetLastError();
}

hipError_t launch_refine(int B, int N, int Np, int L, const MatDesc* descs,
                         const double* hbuf, const float* F, const int* perm,
                         const float* X, double* dg, double* ldpart,
                         double* lad, hipStream_t st) {
  const int nb = refine_blocks(Np);
  mark_begin(K_REFINE, st);
  hipLaunchKernelGGL(refine_kernel, dim3(nb, B), dim3(256), 0, st, N, Np, L,
                     descs, hbuf, F, perm, X, dg, ldpart);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    hipLaunchKernelGGL(finalize_logdet_kernel, dim3((B + 127) / 128),
                       dim3(128), 0, st, ldpart, nb, B, lad);
  mark_end(K_REFINE, st);
  return e != hipSuccess ? e : hipGetLastError();
}

}  // namespace sca
