// Symmetric route: A = L D L^T without pivoting, for the complex symmetric
// A_b = z_b I - H_b (H_b real symmetric).
//
// Why no pivoting is needed here: with z = w + i eta, eta > 0 (every
// Matsubara shift and every DOS shift), -iA has the positive definite
// Hermitian part eta I, every leading block of A keeps that property, so
// every leading block is non-singular and the elimination exists; Schur
// complements keep it too, which bounds the growth.  The kernel still
// measures the growth (max|U| / max|A| with U = D L^T, and max|L|) and marks
// the matrix for the pivoted LU when either exceeds kSymGrowthMax or a
// pivot is not finite.
//
// Work: (4/3) N^3 real flops for the factorisation (half the pivoted LU)
// and one triangular inverse instead of two; diag(A^-1) = diag(L^-T D^-1
// L^-1), i.e. (A^-1)_ii = sum_k (L^-1)_ki^2 / d_k.
//
// Layout.  The kernel keeps block ROW J (NB rows x columns >= c0) of the
// Schur complement in MFMA accumulators, so the triangular solve of the
// panel is a product from the left (the accumulator tile is directly the B
// operand).  It stores F = L^T row-major (row k holds column k of L, the
// diagonal holds d_k), so that the upper-triangle mode of trtri_kernel
// (identity permutation) turns F into V^T = L^-T in place, and writes
// 1/d_k to invd[b][k].  The inverted diagonal blocks go to tri like the
// LU's: L_JJ^-1 in the L slot, (L_JJ^-1)^T in the U slot (read by trtri).
//
//   ldlt_kernel     the factorisation, ln|det A| = sum ln|d_k|, growth,
//                   fallback flag
//   symdiag_kernel  (A^-1)_ii = sum_{k >= i} (V^T)_ik^2 / d_k
#include <math.h>
#include "sca_common.h"
#include "sca_blocked.h"
#include "k_factor_common.h"
#include "sca_profile.h"

namespace sca {

// Growth (max|U| / max|A|, or max|L|) above which the unpivoted factors of a
// matrix are replaced by the pivoted LU.
constexpr double kSymGrowthMax = 64.0;

// LDS: reductions, d and 1/d, then one region used first by the W~ double
// buffer of the update and then by the diagonal block, L_JJ^-1 and the
// inversion scratch.
template <typename T>
size_t ldlt_region_elems(int NB) {
  const size_t upd = 4 * (size_t)NB * (NB + 1);
  const size_t blk = 4 * (size_t)NB * (NB + 1) + (size_t)NB * NB;
  return upd > blk ? upd : blk;
}

template <typename T>
size_t ldlt_lds_bytes(int Np, int NB, int waves) {
  size_t b = 0;
  b += sizeof(double) * (64 * waves + 2 * waves);   // reductions
  b += sizeof(T) * 4 * Np;                          // d, 1/d (re, im)
  b += sizeof(T) * ldlt_region_elems<T>(NB);
  return b + 256;
}

template <typename T, int WAVES, int RT, int CT>
__global__ void __launch_bounds__(WAVES * 64)
ldlt_kernel(const MatDesc* __restrict__ descs, const double* __restrict__ hbuf,
            int N, int Np, int L, T* __restrict__ F, int* __restrict__ perm_out,
            T* __restrict__ tri, T* __restrict__ invd_out,
            double* __restrict__ lad, double* __restrict__ growth,
            int* __restrict__ fallback) {
  typedef Mma<T> M;
  typedef typename M::v4 V4;
  constexpr int NB = 16 * CT;
  constexpr int NT = WAVES * 64;
  constexpr int KPL = NB / 4;
  constexpr int LDB = NB + 1;
  extern __shared__ double lds_raw[];
  const int b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = lane >> 4, q = lane & 15;
  const int ntiles = Np >> 4;
  const int nblk = Np / NB;

  double* red = lds_raw;                 // [NT]
  double* wred = red + NT;               // [2][WAVES]
  T* dr_s = reinterpret_cast<T*>(wred + 2 * WAVES);
  T* di_s = dr_s + Np;
  T* er_s = di_s + Np;                   // 1/d
  T* ei_s = er_s + Np;
  T* region = ei_s + Np;
  T* wsr = region;                       // [2][NB][LDB]  W~[j][k] = L[c0+j][k] d_k
  T* wsi = wsr + 2 * NB * LDB;
  T* xsr = region;                       // diagonal block (LU form)
  T* xsi = xsr + NB * LDB;
  T* lsr = xsi + NB * LDB;               // L_JJ^-1
  T* lsi = lsr + NB * LDB;
  T* tr_ = lsi + NB * LDB;
  T* ti_ = tr_ + NB * NB / 2;

  const MatDesc dsc = descs[b];
  const double* h = hbuf + dsc.hoff;
  const size_t plane = (size_t)Np * Np;
  T* Fr = F + (size_t)b * 2 * plane;
  T* Fi = Fr + plane;
  T* Tb = tri + (size_t)b * nblk * 4 * NB * NB;

  V4 xr[RT][CT], xi[RT][CT];
  double umax = 0.0, lmax = 0.0, amax = 0.0;
  int bad = 0;

  for (int J = 0; J < nblk; ++J) {
    const int c0 = J * NB;
    // ---- 1. block row J of A: S[j][p] = A[c0 + j][p], p >= c0 ------------
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = c0 + 16 * ct + M::m(g, i);
        int n0 = -1, n1 = -1, n2 = -1, n3 = -1;
        double dre = 0.0;
        if (r < N) {
          const int x = r % L, y = r / L;
          n0 = (x + 1) % L + L * y;
          n1 = (x + L - 1) % L + L * y;
          n2 = x + L * ((y + 1) % L);
          n3 = x + L * ((y + L - 1) % L);
          dre = dsc.zr - h[r];
        }
#pragma unroll
        for (int s = 0; s < RT; ++s) {
          const int t = w + WAVES * s;
          const int p = 16 * t + q;
          double re = 0.0, im = 0.0;
          if (r < N && p < N) {
            re = dsc.t * (double)((p == n0) + (p == n1) + (p == n2) + (p == n3));
            if (p == r) { re += dre; im = dsc.zi; }
            if (t < ntiles && p >= c0) amax = fmax(amax, fabs(re) + fabs(im));
          } else if (r == p) {
            re = 1.0;
          }
          xr[s][ct][i] = T(re);
          xi[s][ct][i] = T(im);
        }
      }
    }

    // ---- 2. left-looking update: S -= W~_I L[p, I]^T over earlier blocks --
    for (int I = 0; I < J; ++I) {
      const int r0 = I * NB;
      T* wr = wsr + (I & 1) * NB * LDB;
      T* wi = wsi + (I & 1) * NB * LDB;
      // W~[j][k] = L[c0 + j][r0 + k] d_{r0 + k}, L[c0+j][r0+k] = F[r0+k][c0+j]
      for (int e = tid; e < NB * NB; e += NT) {
        const int j = e % NB, k = e / NB;
        const size_t o = (size_t)(r0 + k) * Np + c0 + j;
        const T lr = Fr[o], li = Fi[o];
        const T d_r = dr_s[r0 + k], d_i = di_s[r0 + k];
        wr[j * LDB + k] = lr * d_r - li * d_i;
        wi[j * LDB + k] = lr * d_i + li * d_r;
      }
      // one barrier per I: the buffer written here was last read two
      // iterations ago, before every wave passed the previous barrier
      __syncthreads();
#pragma unroll
      for (int s = 0; s < RT; ++s) {
        const int t = w + WAVES * s;
        if (t < ntiles && 16 * t >= c0) {
          // B operand: L^T[r0 + KPL g + ks][p] = F[r0 + KPL g + ks][p]
          const int p = 16 * t + q;
          T br[KPL], bi[KPL];
#pragma unroll
          for (int ks = 0; ks < KPL; ++ks) {
            const size_t o = (size_t)(r0 + KPL * g + ks) * Np + p;
            br[ks] = Fr[o];
            bi[ks] = Fi[o];
          }
#pragma unroll
          for (int ks = 0; ks < KPL; ++ks) {
            const int k = KPL * g + ks;
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
              const T ar = wr[(16 * ct + q) * LDB + k];
              const T ai = wi[(16 * ct + q) * LDB + k];
              xr[s][ct] = M::mma(-ar, br[ks], xr[s][ct]);
              xr[s][ct] = M::mma(ai, bi[ks], xr[s][ct]);
              xi[s][ct] = M::mma(-ar, bi[ks], xi[s][ct]);
              xi[s][ct] = M::mma(-ai, br[ks], xi[s][ct]);
            }
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }

    // ---- 3. diagonal block to LDS (the region the update used) -----------
    __syncthreads();
#pragma unroll
    for (int s = 0; s < RT; ++s) {
      const int t = w + WAVES * s;
      if (t >= (c0 >> 4) && t < ((c0 + NB) >> 4)) {
        const int col = 16 * t + q - c0;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            xsr[(16 * ct + M::m(g, i)) * LDB + col] = xr[s][ct][i];
            xsi[(16 * ct + M::m(g, i)) * LDB + col] = xi[s][ct][i];
          }
      }
    }
    __syncthreads();

    // ---- 4. unpivoted LU of the diagonal block (U = D L^T), all threads:
    //         per step k the multipliers of column k, a barrier, the
    //         rank-1 update of the trailing block, a barrier ---------------
    for (int k = 0; k < NB; ++k) {
      const double pr = xsr[k * LDB + k], pi = xsi[k * LDB + k];
      const double den = pr * pr + pi * pi;
      const double ir = pr / den, ii = -pi / den;
      if (tid > k && tid < NB) {
        const double ar = xsr[tid * LDB + k], ai = xsi[tid * LDB + k];
        const double lr = ar * ir - ai * ii, li = ar * ii + ai * ir;
        xsr[tid * LDB + k] = T(lr);
        xsi[tid * LDB + k] = T(li);
        lmax = fmax(lmax, fabs(lr) + fabs(li));
      }
      if (tid >= k && tid < NB)
        umax = fmax(umax, (double)fabs(xsr[k * LDB + tid]) +
                              (double)fabs(xsi[k * LDB + tid]));
      __syncthreads();
      const int m = NB - 1 - k;
      for (int e = tid; e < m * m; e += NT) {
        const int i = k + 1 + e / m, j = k + 1 + e % m;
        const T lr = xsr[i * LDB + k], li = xsi[i * LDB + k];
        const T ur = xsr[k * LDB + j], ui = xsi[k * LDB + j];
        xsr[i * LDB + j] -= lr * ur - li * ui;
        xsi[i * LDB + j] -= lr * ui + li * ur;
      }
      __syncthreads();
    }
    if (tid < NB) {
      const double pr = xsr[tid * LDB + tid], pi = xsi[tid * LDB + tid];
      const double den = pr * pr + pi * pi;
      bad |= !(den > 0.0) || !isfinite(den);
      dr_s[c0 + tid] = T(pr);
      di_s[c0 + tid] = T(pi);
      er_s[c0 + tid] = T(pr / den);
      ei_s[c0 + tid] = T(-pi / den);
    }
    __syncthreads();

    // ---- 5. L_JJ^-1 of the factored block ---------------------------------
    block_tri_inverses<T, NB, NT, false>(xsr, xsi, lsr, lsi, nullptr, nullptr,
                                         tr_, ti_, tid);

    // ---- 6. panel rows right of the block: U[j][p] = (L_JJ^-1 S)[j][p],
    //         L[p][c0 + j] = U[j][p] / d_j, stored at F[c0 + j][p] ---------
#pragma unroll
    for (int s = 0; s < RT; ++s) {
      const int t = w + WAVES * s;
      if (t < ntiles && 16 * t >= c0 + NB) {
        const int p = 16 * t + q;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          V4 ur = {T(0), T(0), T(0), T(0)}, ui = {T(0), T(0), T(0), T(0)};
#pragma unroll
          for (int c2 = 0; c2 < CT; ++c2)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              // k = 16 c2 + m(g, i): element i of the accumulator tile
              const int k = 16 * c2 + M::m(g, i);
              const T ar = lsr[(16 * ct + q) * LDB + k];
              const T ai = lsi[(16 * ct + q) * LDB + k];
              const T br = xr[s][c2][i], bi = xi[s][c2][i];
              ur = M::mma(ar, br, ur);
              ur = M::mma(-ai, bi, ur);
              ui = M::mma(ar, bi, ui);
              ui = M::mma(ai, br, ui);
            }
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int j = 16 * ct + M::m(g, i);
            const T vr = ur[i], vi = ui[i];
            umax = fmax(umax, (double)fabs(vr) + (double)fabs(vi));
            const T er = er_s[c0 + j], ei = ei_s[c0 + j];
            const T lr = vr * er - vi * ei, li = vr * ei + vi * er;
            lmax = fmax(lmax, (double)fabs(lr) + (double)fabs(li));
            Fr[(size_t)(c0 + j) * Np + p] = lr;
            Fi[(size_t)(c0 + j) * Np + p] = li;
          }
        }
      }
    }
    // ---- 7. the diagonal block of F (L^T part, d on the diagonal), 1/d,
    //         and the inverted diagonal blocks for trtri ------------------
    {
      T* Lr = Tb + (size_t)(J * 4 + 0) * NB * NB;
      T* Li = Lr + NB * NB;
      T* Ur = Li + NB * NB;
      T* Ui = Ur + NB * NB;
      for (int e = tid; e < NB * NB; e += NT) {
        const int rr = e / NB, cc = e % NB;
        T fr = T(0), fi = T(0);
        if (cc > rr) { fr = xsr[cc * LDB + rr]; fi = xsi[cc * LDB + rr]; }
        else if (cc == rr) { fr = dr_s[c0 + rr]; fi = di_s[c0 + rr]; }
        Fr[(size_t)(c0 + rr) * Np + c0 + cc] = fr;
        Fi[(size_t)(c0 + rr) * Np + c0 + cc] = fi;
        Lr[e] = lsr[rr * LDB + cc];
        Li[e] = lsi[rr * LDB + cc];
        Ur[e] = lsr[cc * LDB + rr];   // (L_JJ^-1)^T
        Ui[e] = lsi[cc * LDB + rr];
      }
      T* ir = invd_out + (size_t)b * 2 * Np;
      for (int k = tid; k < NB; k += NT) {
        ir[c0 + k] = er_s[c0 + k];
        ir[Np + c0 + k] = ei_s[c0 + k];
      }
    }
    __syncthreads();
  }

  for (int p = tid; p < Np; p += NT) perm_out[(size_t)b * Np + p] = p;
  // ln|det A| = sum_k ln|d_k|: strided partial sums, fixed-order total
  double lsum = 0.0;
  for (int k = tid; k < Np; k += NT)
    lsum += log(hypot((double)dr_s[k], (double)di_s[k]));
  for (int off = 32; off >= 1; off >>= 1) {
    umax = fmax(umax, __shfl_xor(umax, off));
    lmax = fmax(lmax, __shfl_xor(lmax, off));
    amax = fmax(amax, __shfl_xor(amax, off));
    bad |= __shfl_xor(bad, off);
  }
  __syncthreads();
  if (lane == 0) {
    wred[w] = fmax(umax, lmax * amax);
    wred[WAVES + w] = amax + (bad ? INFINITY : 0.0);
  }
  red[tid] = lsum;
  __syncthreads();
  if (tid == 0) {
    double u = 0.0, a = 0.0, l = 0.0;
    for (int ww = 0; ww < WAVES; ++ww) { u = fmax(u, wred[ww]); a = fmax(a, wred[WAVES + ww]); }
    for (int k = 0; k < NT; ++k) l += red[k];
    const double gr = u / a;
    const bool ok = isfinite(a) && isfinite(l) && gr <= kSymGrowthMax;
    growth[b] = isfinite(a) ? gr : INFINITY;
    lad[b] = l;
    fallback[b] = ok ? 0 : 1;
  }
}

// (A^-1)_ii = sum_{k >= i} (V^T)_ik^2 / d_k, V^T stored in place of L^T.
// One wave per row i (lanes over k, fixed-order combination).
template <typename T>
__global__ void __launch_bounds__(256)
symdiag_kernel(int N, int Np, const T* __restrict__ F,
               const T* __restrict__ invd, double* __restrict__ dg,
               const int* __restrict__ only, int want) {
  const int b = blockIdx.y;
  if (only && only[b] != want) return;   // matrix not selected
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + w;
  __shared__ double sr_s[4][64], si_s[4][64];
  const size_t plane = (size_t)Np * Np;
  const T* Fr = F + (size_t)b * 2 * plane;
  const T* Fi = Fr + plane;
  const T* er = invd + (size_t)b * 2 * Np;
  const T* ei = er + Np;
  double ar = 0.0, ai = 0.0;
  if (i < N) {
    for (int k = i + lane; k < Np; k += 64) {
      const double vr = Fr[(size_t)i * Np + k], vi = Fi[(size_t)i * Np + k];
      const double sqr = vr * vr - vi * vi, sqi = 2.0 * vr * vi;
      const double dr = er[k], di = ei[k];
      ar += sqr * dr - sqi * di;
      ai += sqr * di + sqi * dr;
    }
  }
  sr_s[w][lane] = ar;
  si_s[w][lane] = ai;
  __syncthreads();
  if (lane == 0 && i < N) {
    double tr = 0.0, ti = 0.0;
    for (int k = 0; k < 64; ++k) { tr += sr_s[w][k]; ti += si_s[w][k]; }
    dg[((size_t)b * N + i) * 2 + 0] = tr;
    dg[((size_t)b * N + i) * 2 + 1] = ti;
  }
}

namespace {

template <typename T, int WAVES, int RT, int CT>
hipError_t run_ldlt(const MatDesc* descs, const double* hbuf, int B, int N,
                    int Np, int L, T* F, int* perm, T* tri, T* invd,
                    double* lad, double* growth, int* fallback,
                    hipStream_t st) {
  const size_t lds = ldlt_lds_bytes<T>(Np, 16 * CT, WAVES);
  auto kern = ldlt_kernel<T, WAVES, RT, CT>;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  mark_begin(K_LDLT, st);
  hipLaunchKernelGGL(kern, dim3(B), dim3(WAVES * 64), lds, st, descs, hbuf, N,
                     Np, L, F, perm, tri, invd, lad, growth, fallback);
  mark_end(K_LDLT, st);
  return hipGetLastError();
}

}  // namespace

hipError_t blocked_ldlt_f64(const BlockedPlan& p, const MatDesc* descs,
                            const double* hbuf, int B, int N, int L, double* F,
                            int* perm, double* tri, double* invd, double* lad,
                            double* growth, int* fallback, hipStream_t st) {
  switch (p.cfg) {
    case 0: return run_ldlt<double, 4, 4, 2>(descs, hbuf, B, N, p.Np, L, F, perm, tri, invd, lad, growth, fallback, st);
    case 1: return run_ldlt<double, 8, 4, 2>(descs, hbuf, B, N, p.Np, L, F, perm, tri, invd, lad, growth, fallback, st);
    case 2: return run_ldlt<double, 16, 4, 1>(descs, hbuf, B, N, p.Np, L, F, perm, tri, invd, lad, growth, fallback, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_symdiag_f64(int B, int N, int Np, const double* F,
                              const double* invd, double* dg, hipStream_t st,
                              const int* only, int want) {
  mark_begin(K_SYMDIAG, st);
  hipLaunchKernelGGL(symdiag_kernel<double>, dim3((N + 3) / 4, B), dim3(256),
                     0, st, N, Np, F, invd, dg, only, want);
  mark_end(K_SYMDIAG, st);
  return hipGetLastError();
}

}  // namespace sca
