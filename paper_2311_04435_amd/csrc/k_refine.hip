// FP32 factor route with FP64 refinement.
//
// After the complex64 LU (P A ~ L U) and the complex64 triangular inverses
// W ~ U^-1, V ~ L^-1 (stored in place in F, original-row order), with
// Y = W V P the approximate inverse whose determinant is known exactly,
// |det Y| = prod |w_kk| (V is unit lower):
//
//   wv_gemm_kernel   X = fl32(W V) on the f32 MFMA, stored transposed
//                    (XT[c][i] = X[i][c]); Z = X P ~ A^-1, so row q of XT
//                    is column perm[q] of Z in site order.  While the tiles
//                    of W and V pass through LDS it also sums, in FP64 from
//                    the stored FP32 values (their products are exact in
//                    FP64), the entries Y_ji = W[j, :] . V[:, pos(i)] at the
//                    5N non-zeros A_ij, and each tile's share of
//                    tr(A Y) = sum_ij A_ij Y_ji (real part).
//   refine_kernel    in FP64, per column i of Z (one row of XT):
//     * one Newton step for the diagonal of the inverse.  A is complex
//       symmetric; with Z = A^-1 + E and the residual R = I - A Z
//       (E = -A^-1 R),
//         Z^T A Z = A^-1 + E + E^T + E^T A E,   E^T A E = R^T A^-1 R,
//       so d_i = 2 Z_ii - c_i^T A c_i (c_i: column i of Z) misses
//       (A^-1)_ii by -(R^T A^-1 R)_ii: the FP32 residual squared, as for
//       the full Newton step Z (2I - A Z).  A acts through its 5-point
//       stencil on the column, so each row of XT is read once;
//     * its positions' part of -sum ln|w_qq| - N.
//   finalize_logdet_kernel   fixed-order sum of the parts:
//         ln|det A| = ln|det(A Y)| - ln|det Y|
//                   = Re ln det(I - R') - ln|det Y|     (R' = I - A Y)
//                   = Re tr(A Y) - N - sum ln|w_kk| + O(|R'|^2).
//
// A = z I - H with H = -t K + diag(h); its off-diagonal entries are t
// (K_ij counts directions; on these lattices, L >= 10, the 4 neighbours
// are distinct).
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

constexpr int GT = 64;          // output tile of the W V product
constexpr int GK = 16;          // k chunk
constexpr int kSlots = GT * 5;  // trace entries a tile may hold: 5 per column

// Site of stencil slot d of site s: itself, +x, -x, +y, -y.
__device__ inline int stencil_site(int s, int d, int L) {
  const int x = s % L, y = s / L;
  switch (d) {
    case 0: return s;
    case 1: return (x + 1) % L + L * y;
    case 2: return (x + L - 1) % L + L * y;
    case 3: return x + L * ((y + 1) % L);
    default: return x + L * ((y + L - 1) % L);
  }
}

__device__ inline double wave_sum_xor(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace

// XT[c][i] = X[i][c] = sum_{k >= max(i, c)} W[i][k] V[k][c], V[c][c] = 1.
// W[i][k] is stored at F[perm[i]][k] (k >= i), V[k][c] at F[perm[k]][c]
// (k > c).  256 threads: each wave owns a 32 x 32 quarter of the 64 x 64
// tile (2 x 2 MFMA tiles, real and imaginary accumulators); Np is a multiple
// of 16 and the tiles past Np are masked.  The next k chunk of W and V is
// loaded into registers while the current one is multiplied.
//
// The grid is one-dimensional and XCD-aware: workgroup g runs on XCD g % 8
// (round-robin dispatch), and the tiles of matrix b are the workgroups
// g = (b % 8) + 8 (T (b / 8) + tile), T tiles per matrix, so all of a
// matrix's tiles share one XCD's L2, which holds its factors (1.4 MB at
// N = 400) while they are read once per tile.
//
// Trace: column c of the tile (position c, site s = perm[c]) needs Y_jc for
// the 5 sites j of the stencil of s (A_sj != 0) that fall in the tile's
// rows.  They are listed in the order e = 5 cl + d (d: self, +x, -x, +y,
// -y); entry e is summed in FP64 by lane (e / 4) % 64 of wave e % 4 as the
// tiles pass, and the tile's sum of Re(A_sj Y_jc), in list order, goes to
// ldpart[b][tile].
constexpr int kGemmThreads = 256;

__global__ void __launch_bounds__(kGemmThreads)
__attribute__((amdgpu_waves_per_eu(4)))
wv_gemm_kernel(int N, int Np, int L, int B, int nt,
               const MatDesc* __restrict__ descs,
               const double* __restrict__ hbuf, const float* __restrict__ F,
               const int* __restrict__ perm_g, float* __restrict__ XT,
               double* __restrict__ ldpart, int nparts) {
  const int T = nt * nt;
  const int gid = blockIdx.x, slot = gid >> 3;
  const int b = (gid & 7) + 8 * (slot / T);
  if (b >= B) return;
  const int tile = slot % T;
  const int i0 = (tile / nt) * GT, c0 = (tile % nt) * GT;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = lane >> 4, q = lane & 15;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  __shared__ float Wr[GT][GK + 1], Wi[GT][GK + 1];   // [i][k]
  __shared__ float Vr[GK][GT + 1], Vi[GK][GT + 1];   // [k][c]
  __shared__ int ent_j[kSlots], ent_c[kSlots];
  __shared__ double ent_r[kSlots], ent_i[kSlots], slot_s[kSlots];
  __shared__ int ns_s;
  const size_t plane = (size_t)Np * Np;
  const float* Fr = F + (size_t)b * 2 * plane;
  const float* Fi = Fr + plane;
  const int* perm = perm_g + (size_t)b * Np;

  // the tile's trace entries, compacted in order by wave 0: lane l examines
  // column l (up to 5 entries) and places them after the lower lanes'
  if (w == 0) {
    const MatDesc dsc = descs[b];
    const int c = c0 + lane;
    const int s = c < Np ? perm[c] : N;
    int jj[5], cnt = 0;
#pragma unroll
    for (int d = 0; d < 5; ++d) {
      jj[d] = -1;
      if (s < N) {
        const int j = stencil_site(s, d, L);
        if (j >= i0 && j < i0 + GT && j < N) { jj[d] = j - i0; ++cnt; }
      }
    }
    int incl = cnt;   // inclusive prefix sum over the lanes
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int v = __shfl_up(incl, o, 64);
      if (lane >= o) incl += v;
    }
    if (lane == 63) ns_s = incl;
    int pos = incl - cnt;
    const double hs = s < N ? hbuf[dsc.hoff + s] : 0.0;
#pragma unroll
    for (int d = 0; d < 5; ++d)
      if (jj[d] >= 0) {
        ent_j[pos] = jj[d];
        ent_c[pos] = lane;
        ent_r[pos] = d == 0 ? dsc.zr - hs : dsc.t;
        ent_i[pos] = d == 0 ? dsc.zi : 0.0;
        ++pos;
      }
  }

  // loader assignment: W element (r, k) = (tid / 16 + 16 u, tid % 16),
  // V element (k, c) = (tid / 64 + 4 u, tid % 64), u < 4
  const int lk = tid & 15, lr = tid >> 4;
  const int vc = tid & 63, vk = tid >> 6;
  int prow[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = i0 + lr + 16 * u;
    prow[u] = r < Np ? perm[r] : 0;
  }
  float pwr[4], pwi[4], pvr[4], pvi[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int gi = i0 + lr + 16 * u, gk = k0 + lk;
      float xr = 0.f, xi = 0.f;
      if (gk >= gi && gi < Np) {
        const size_t o = (size_t)prow[u] * Np + gk;
        xr = Fr[o];
        xi = Fi[o];
      }
      pwr[u] = xr;
      pwi[u] = xi;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int gk = k0 + vk + 4 * u, gc = c0 + vc;
      float vr = 0.f, vi = 0.f;
      if (gc < Np) {
        if (gk > gc) {
          const size_t o = (size_t)perm[gk] * Np + gc;
          vr = Fr[o];
          vi = Fi[o];
        } else if (gk == gc) {
          vr = 1.f;
        }
      }
      pvr[u] = vr;
      pvi[u] = vi;
    }
  };

  f4 ar[2][2], ai[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      ar[a][c] = (f4){0.f, 0.f, 0.f, 0.f};
      ai[a][c] = (f4){0.f, 0.f, 0.f, 0.f};
    }
  const int kstart = (i0 > c0 ? i0 : c0);   // multiple of GT, so of GK
  load(kstart);
  __syncthreads();   // the entry list
  const int ns = ns_s;
  // this lane's entries: e0 = 4 lane + w, and e0 + 256
  const int e0 = 4 * lane + w, e1 = e0 + 256;
  const bool v0 = e0 < ns, v1 = e1 < ns;
  const int j0 = v0 ? ent_j[e0] : 0, cc0 = v0 ? ent_c[e0] : 0;
  const int j1 = v1 ? ent_j[e1] : 0, cc1 = v1 ? ent_c[e1] : 0;
  double y0r = 0.0, y0i = 0.0, y1r = 0.0, y1i = 0.0;

  for (int k0 = kstart; k0 < Np; k0 += GK) {
    __syncthreads();   // the previous chunk's tiles are no longer read
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      Wr[lr + 16 * u][lk] = pwr[u];
      Wi[lr + 16 * u][lk] = pwi[u];
      Vr[vk + 4 * u][vc] = pvr[u];
      Vi[vk + 4 * u][vc] = pvi[u];
    }
    __syncthreads();
    if (k0 + GK < Np) load(k0 + GK);   // in flight during the products
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
    // exact-product FP64 sums of this lane's trace entries
    if (v0) {
#pragma unroll
      for (int kk = 0; kk < GK; ++kk) {
        const double w_r = Wr[j0][kk], w_i = Wi[j0][kk];
        const double v_r = Vr[kk][cc0], v_i = Vi[kk][cc0];
        y0r += w_r * v_r - w_i * v_i;
        y0i += w_r * v_i + w_i * v_r;
      }
    }
    if (v1) {
#pragma unroll
      for (int kk = 0; kk < GK; ++kk) {
        const double w_r = Wr[j1][kk], w_i = Wi[j1][kk];
        const double v_r = Vr[kk][cc1], v_i = Vi[kk][cc1];
        y1r += w_r * v_r - w_i * v_i;
        y1i += w_r * v_i + w_i * v_r;
      }
    }
  }
  float* Tr = XT + (size_t)b * 2 * plane;
  float* Ti = Tr + plane;
  // f32 accumulator: element j of lane (g, q) holds row 4g + j, column q;
  // in XT the four rows are adjacent (Np is a multiple of 16)
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int gi = i0 + wr + 16 * a + 4 * g, gc = c0 + wc + 16 * c + q;
      if (gi < Np && gc < Np) {
        const size_t o = (size_t)gc * Np + gi;
        *reinterpret_cast<f4*>(Tr + o) = ar[a][c];
        *reinterpret_cast<f4*>(Ti + o) = ai[a][c];
      }
    }
  // the tile's share of Re tr(A Y), entries in list order: lane l of wave 0
  // sums entries 5l .. 5l+4, then a fixed butterfly over the lanes
  if (v0) slot_s[e0] = ent_r[e0] * y0r - ent_i[e0] * y0i;
  if (v1) slot_s[e1] = ent_r[e1] * y1r - ent_i[e1] * y1i;
  __syncthreads();
  if (w == 0) {
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const int e = 5 * lane + k;
      sum += e < ns ? slot_s[e] : 0.0;
    }
    sum = wave_sum_xor(sum);
    if (lane == 0) ldpart[(size_t)b * nparts + tile] = sum;
  }
}

// --------------------------------------------------------------------------

namespace {
constexpr int kRefineWaves = 4;
constexpr int kRefineThreads = 64 * kRefineWaves;
constexpr int kBatch = 8;   // column elements per lane loaded at a time
}  // namespace

size_t refine_lds_bytes(int N, int Np) {
  return sizeof(double) * (size_t)N                        // h
       + sizeof(float) * 2 * (size_t)kRefineWaves * N      // columns of Z
       + sizeof(int) * (size_t)Np                          // perm
       + sizeof(double) * kRefineThreads;                  // reduction
}

// grid (nsplit, B): workgroup s takes the positions q in
// [s * chunk, (s + 1) * chunk), chunk = ceil(Np / nsplit); wave w the
// positions w, w + 4, ... of its range.  Row q of XT (column i = perm[q] of
// Z, site order) is staged in the wave's LDS region, then lane l takes the
// sites l, l + 64, ...:
//   acc = sum_j Z_ji ((z - h_j) Z_ji + t sum_{l ~ j} Z_li)   (FP64)
//   dg[b][i] = 2 Z_ii - acc.
__global__ void __launch_bounds__(kRefineThreads)
refine_kernel(int N, int Np, int L, const MatDesc* __restrict__ descs,
              const double* __restrict__ hbuf, const float* __restrict__ F,
              const int* __restrict__ perm_g, const float* __restrict__ XT,
              double* __restrict__ dg, double* __restrict__ ldpart,
              int nparts, int part0) {
  extern __shared__ double lds_raw[];
  const int b = blockIdx.y, split = blockIdx.x, nsplit = gridDim.x;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double* h_s = lds_raw;
  double* red_s = h_s + N;
  float* z_s = reinterpret_cast<float*>(red_s + kRefineThreads);
  float* zr = z_s + (size_t)w * 2 * N;   // this wave's column: re, then im
  float* zi = zr + N;
  int* perm_s = reinterpret_cast<int*>(z_s + (size_t)kRefineWaves * 2 * N);

  const MatDesc dsc = descs[b];
  const size_t plane = (size_t)Np * Np;
  const float* Tr = XT + (size_t)b * 2 * plane;
  const float* Ti = Tr + plane;
  const int* perm = perm_g + (size_t)b * Np;
  for (int k = tid; k < N; k += kRefineThreads) h_s[k] = hbuf[dsc.hoff + k];
  for (int k = tid; k < Np; k += kRefineThreads) perm_s[k] = perm[k];
  __syncthreads();

  const int qc = (Np + nsplit - 1) / nsplit;
  const int qa = split * qc, qb = min(Np, qa + qc);
  // -ln|w_qq| - 1 over this workgroup's real positions (fixed order)
  {
    const float* Fr = F + (size_t)b * 2 * plane;
    double s = 0.0;
    for (int qq = qa + tid; qq < qb; qq += kRefineThreads) {
      if (perm_s[qq] < N) {
        const size_t o = (size_t)perm_s[qq] * Np + qq;   // w_qq at F[perm q][q]
        s += -log(hypot((double)Fr[o], (double)Fr[o + plane])) - 1.0;
      }
    }
    red_s[tid] = s;
    __syncthreads();
    for (int k = kRefineThreads / 2; k >= 1; k >>= 1) {
      if (tid < k) red_s[tid] += red_s[tid + k];
      __syncthreads();
    }
    if (tid == 0) ldpart[(size_t)b * nparts + part0 + split] = red_s[0];
  }

  const double zre = dsc.zr, zim = dsc.zi, t = dsc.t;
  // lattice coordinates of site lane + 64 k, advanced by 64 sites a step
  const int dx = 64 % L, dy = 64 / L;
  for (int qq = qa + w; qq < qb; qq += kRefineWaves) {
    const int i = perm_s[qq];
    if (i >= N) continue;   // padding position (uniform over the wave)
    const float* cr = Tr + (size_t)qq * Np;
    const float* ci = Ti + (size_t)qq * Np;
    // the column's loads go out kBatch per lane at a time
    for (int j0 = 0; j0 < N; j0 += 64 * kBatch) {
      float a[kBatch], c[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int j = j0 + 64 * u + lane;
        a[u] = j < N ? cr[j] : 0.f;
        c[u] = j < N ? ci[j] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int j = j0 + 64 * u + lane;
        if (j < N) { zr[j] = a[u]; zi[j] = c[u]; }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    double acc_r = 0.0, acc_i = 0.0;
    int x = lane % L, y = lane / L;
    for (int j = lane; j < N; j += 64) {
      const double ar = zr[j], ai = zi[j];
      const int xp = x + 1 == L ? 0 : x + 1, xm = x == 0 ? L - 1 : x - 1;
      const int yp = y + 1 == L ? 0 : y + 1, ym = y == 0 ? L - 1 : y - 1;
      const int ly = L * y;
      const double nr = (double)zr[xp + ly] + (double)zr[xm + ly] +
                        (double)zr[x + L * yp] + (double)zr[x + L * ym];
      const double ni = (double)zi[xp + ly] + (double)zi[xm + ly] +
                        (double)zi[x + L * yp] + (double)zi[x + L * ym];
      const double ur = zre - h_s[j];
      // (A c_i)_j = (z - h_j) Z_ji + t (sum of the neighbours)
      const double vr = ur * ar - zim * ai + t * nr;
      const double vi = ur * ai + zim * ar + t * ni;
      acc_r += ar * vr - ai * vi;
      acc_i += ar * vi + ai * vr;
      x += dx; y += dy;
      if (x >= L) { x -= L; ++y; }
    }
    acc_r = wave_sum_xor(acc_r);
    acc_i = wave_sum_xor(acc_i);
    if (lane == 0) {
      dg[((size_t)b * N + i) * 2 + 0] = 2.0 * (double)zr[i] - acc_r;
      dg[((size_t)b * N + i) * 2 + 1] = 2.0 * (double)zi[i] - acc_i;
    }
    // the next column overwrites this wave's region
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// lad[b] = sum of the per-matrix parts, in order.
__global__ void finalize_logdet_kernel(const double* __restrict__ ldpart,
                                       int nparts, int nused, int B,
                                       double* __restrict__ lad) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double s = 0.0;
  for (int k = 0; k < nused; ++k) s += ldpart[(size_t)b * nparts + k];
  lad[b] = s;
}

namespace {
int wv_tiles(int Np) { return (Np + GT - 1) / GT; }
}  // namespace

// Workgroups per matrix of the refinement: enough of them in all to fill
// the GPU several times over, at most one per 32 rows and at most
// kMaxSplits.
constexpr int kMaxSplits = 64;
int refine_splits(int N, int B) {
  int s = (4096 + B - 1) / B;
  const int smax = (N + 31) / 32;
  if (s > smax) s = smax;
  if (s > kMaxSplits) s = kMaxSplits;
  return s < 1 ? 1 : s;
}

// Parts per matrix of the log-determinant (tiles of W V, then the
// refinement's workgroups); the scratch holds this many for any B.
int refine_parts(int Np) {
  const int nt = wv_tiles(Np);
  return nt * nt + kMaxSplits;
}

hipError_t launch_wv_gemm(int B, int N, int Np, int L, const MatDesc* descs,
                          const double* hbuf, const float* F, const int* perm,
                          float* XT, double* ldpart, hipStream_t st) {
  if (Np % GK || L < 3) return hipErrorInvalidValue;
  const int nt = wv_tiles(Np);
  const int nparts = refine_parts(Np);
  const int grid = 8 * nt * nt * ((B + 7) / 8);
  mark_begin(K_WVGEMM, st);
  hipLaunchKernelGGL(wv_gemm_kernel, dim3(grid), dim3(kGemmThreads), 0, st, N,
                     Np, L, B, nt, descs, hbuf, F, perm, XT, ldpart, nparts);
  mark_end(K_WVGEMM, st);
  return hipGetLastError();
}

hipError_t launch_refine(int B, int N, int Np, int L, const MatDesc* descs,
                         const double* hbuf, const float* F, const int* perm,
                         const float* XT, double* dg, double* ldpart,
                         double* lad, hipStream_t st) {
  if (L < 3) return hipErrorInvalidValue;
  const int ns = refine_splits(N, B);
  const int nt = wv_tiles(Np);
  const int nparts = refine_parts(Np);
  const size_t lds = refine_lds_bytes(N, Np);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(refine_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  mark_begin(K_REFINE, st);
  hipLaunchKernelGGL(refine_kernel, dim3(ns, B), dim3(kRefineThreads), lds, st,
                     N, Np, L, descs, hbuf, F, perm, XT, dg, ldpart, nparts,
                     nt * nt);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    hipLaunchKernelGGL(finalize_logdet_kernel, dim3((B + 127) / 128),
                       dim3(128), 0, st, ldpart, nparts, nt * nt + ns, B, lad);
  mark_end(K_REFINE, st);
  return e != hipSuccess ? e : hipGetLastError();
}

}  // namespace sca
