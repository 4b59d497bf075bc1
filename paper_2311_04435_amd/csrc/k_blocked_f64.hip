// Blocked FP64 path for lattices with N > 64 sites: one workgroup per
// matrix A_b = z_b I - H_b, complex arithmetic on the f64 MFMA
// (v_mfma_f64_16x16x4f64; four real products per complex tile product).
//
// Storage of the factors ("original-row order").  With P A = L U, row r of
// the factor array holds row pos(r) of L (left of the diagonal) and of U (on
// and right of it), where pos(r) is the position original row r was pivoted
// to: F[r][c] = (c < pos(r)) ? L[pos(r)][c] : U[pos(r)][c].  Later row swaps
// then never move anything already written, so the left-looking update of a
// block column reads L through the current permutation instead of swapping
// earlier columns.  F is planar (re plane, then im plane), row-major, with
// leading dimension Np (N rounded up to the block width; the padding is an
// identity block, which leaves ln|det| and the original diagonal unchanged).
//
// Kernels
//   lu_kernel      P A = L U, ln|det A| = sum ln|u_kk|, the inverses of the
//                  diagonal blocks L_JJ^-1 and U_JJ^-1, pivot growth.
//   trtri_kernel   W = U^-1 (block columns left to right) or V = L^-1 (right
//                  to left), in place; blockIdx.y picks which, both run in
//                  the same launch on disjoint triangles.
//   diagdot_kernel (A^-1)_ii = sum_s W[i][s] V[s][pos(i)]   (A^-1 = W V P)
#include <math.h>
#include "sca_common.h"
#include "sca_blocked.h"
#include "sca_profile.h"

namespace sca {

typedef double d4 __attribute__((ext_vector_type(4)));

namespace {

__device__ inline d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// f64 16x16x4 accumulator layout: lane l, element i holds row (l>>4) + 4 i,
// column l & 15.
__device__ inline int crow(int g, int i) { return g + 4 * i; }

__device__ inline void argmax_wave(double& mag, int& row) {
  for (int off = 32; off >= 1; off >>= 1) {
    double om = __shfl_xor(mag, off);
    int orow = __shfl_xor(row, off);
    if (om > mag || (om == mag && orow < row)) { mag = om; row = orow; }
  }
}

template <int NB>
struct LuLds {
  int* perm;          // [Np] position -> original row
  double* cmag;       // [2][WAVES]
  int* crowi;         // [2][WAVES]
  double *rAr, *rAi;  // [NB] row at the pivot position before the swap
  double *rBr, *rBi;  // [NB] pivot row
  double *mr, *mi;    // [Np] multipliers of the current column
  double *xsr, *xsi;  // [NB][NB+1] rows of a previous panel / diagonal block
  double *lsr, *lsi;  // [NB][NB+1] L_II^-1
  double *unr, *uni;  // [NB][NB+1] -U_IJ, or U_JJ^-1
};

constexpr int LD(int NB) { return NB + 1; }

}  // namespace

size_t lu_lds_bytes(int Np, int NB, int waves) {
  size_t b = 0;
  b += sizeof(int) * Np;
  b += sizeof(double) * 2 * waves + sizeof(int) * 2 * waves;
  b += sizeof(double) * 4 * NB;
  b += sizeof(double) * 2 * Np;
  b += sizeof(double) * 6 * NB * (NB + 1);
  return b + 64;
}

template <int WAVES, int RT, int CT>
__global__ void __launch_bounds__(WAVES * 64)
lu_kernel(const MatDesc* __restrict__ descs, const double* __restrict__ hbuf,
          int N, int Np, int L, double* __restrict__ F,
          int* __restrict__ perm_out, double* __restrict__ tri,
          double* __restrict__ lad, double* __restrict__ growth) {
  constexpr int NB = 16 * CT;
  constexpr int NT = WAVES * 64;
  constexpr int KPL = NB / 4;   // k values per lane group per panel
  extern __shared__ double lds_raw[];
  const int b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = lane >> 4, q = lane & 15;
  const int ntiles = Np >> 4;
  const int nblk = Np / NB;

  // carve LDS (doubles first for alignment)
  LuLds<NB> S;
  {
    double* d = lds_raw;
    S.mr = d; d += Np; S.mi = d; d += Np;
    S.rAr = d; d += NB; S.rAi = d; d += NB; S.rBr = d; d += NB; S.rBi = d; d += NB;
    S.xsr = d; d += NB * LD(NB); S.xsi = d; d += NB * LD(NB);
    S.lsr = d; d += NB * LD(NB); S.lsi = d; d += NB * LD(NB);
    S.unr = d; d += NB * LD(NB); S.uni = d; d += NB * LD(NB);
    S.cmag = d; d += 2 * WAVES;
    int* ip = reinterpret_cast<int*>(d);
    S.crowi = ip; ip += 2 * WAVES;
    S.perm = ip;
  }

  const MatDesc dsc = descs[b];
  const double* h = hbuf + dsc.hoff;
  const size_t plane = (size_t)Np * Np;
  double* Fr = F + (size_t)b * 2 * plane;
  double* Fi = Fr + plane;
  double* T = tri + (size_t)b * nblk * 4 * NB * NB;   // [nblk][2][2][NB][NB]

  for (int p = tid; p < Np; p += NT) S.perm[p] = p;
  __syncthreads();

  d4 xr[RT][CT], xi[RT][CT];
  double lsum = 0.0, umax = 0.0, amax = 0.0;

  for (int J = 0; J < nblk; ++J) {
    const int c0 = J * NB;
    // ---- 1. generate block column J: X[p][c] = A[perm[p]][c0 + c] ----------
#pragma unroll
    for (int s = 0; s < RT; ++s) {
      const int t = w + WAVES * s;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int p = 16 * t + crow(g, i);
        const int r = (t < ntiles) ? S.perm[p] : Np;
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
        for (int ct = 0; ct < CT; ++ct) {
          const int c = c0 + 16 * ct + q;
          double re = 0.0, im = 0.0;
          if (r < N && c < N) {
            re = dsc.t * (double)((c == n0) + (c == n1) + (c == n2) + (c == n3));
            if (c == r) { re += dre; im = dsc.zi; }
            amax = fmax(amax, fabs(re) + fabs(im));
          } else if (r == c) {
            re = 1.0;
          }
          xr[s][ct][i] = re;
          xi[s][ct][i] = im;
        }
      }
    }

    // ---- 2. left-looking updates from the previous panels ------------------
    for (int I = 0; I < J; ++I) {
      const int r0 = I * NB;
      // (a) panel-I rows of X -> xs; L_II^-1 -> ls
#pragma unroll
      for (int s = 0; s < RT; ++s) {
        const int t = w + WAVES * s;
        if (t >= (r0 >> 4) && t < ((r0 + NB) >> 4)) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int pr = 16 * t + crow(g, i) - r0;
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
              S.xsr[pr * LD(NB) + 16 * ct + q] = xr[s][ct][i];
              S.xsi[pr * LD(NB) + 16 * ct + q] = xi[s][ct][i];
            }
          }
        }
      }
      {
        const double* Lr = T + (size_t)(I * 4 + 0) * NB * NB;
        const double* Li = Lr + NB * NB;
        for (int e = tid; e < NB * NB; e += NT) {
          S.lsr[(e / NB) * LD(NB) + e % NB] = Lr[e];
          S.lsi[(e / NB) * LD(NB) + e % NB] = Li[e];
        }
      }
      __syncthreads();
      // (b) un = -(L_II^-1 xs) = -U_IJ ; one 16x16 real output tile per task
      for (int task = w; task < 2 * CT * CT; task += WAVES) {
        const int rt = task / (2 * CT), ct = (task >> 1) % CT, part = task & 1;
        d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < NB / 4; ++ks) {
          const int k = 4 * ks + g;
          const double ar = S.lsr[(16 * rt + q) * LD(NB) + k];
          const double ai = S.lsi[(16 * rt + q) * LD(NB) + k];
          const double br = S.xsr[k * LD(NB) + 16 * ct + q];
          const double bi = S.xsi[k * LD(NB) + 16 * ct + q];
          if (part == 0) { acc = mfma(ar, br, acc); acc = mfma(-ai, bi, acc); }
          else { acc = mfma(ar, bi, acc); acc = mfma(ai, br, acc); }
        }
        double* dst = part ? S.uni : S.unr;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          dst[(16 * rt + crow(g, i)) * LD(NB) + 16 * ct + q] = -acc[i];
      }
      __syncthreads();
      // (c) panel-I rows become U_IJ; rows below get X += L[:, I] (-U_IJ)
#pragma unroll
      for (int s = 0; s < RT; ++s) {
        const int t = w + WAVES * s;
        if (t >= (r0 >> 4) && t < ((r0 + NB) >> 4)) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int pr = 16 * t + crow(g, i) - r0;
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
              const double ur = -S.unr[pr * LD(NB) + 16 * ct + q];
              const double ui = -S.uni[pr * LD(NB) + 16 * ct + q];
              xr[s][ct][i] = ur;
              xi[s][ct][i] = ui;
              umax = fmax(umax, fabs(ur) + fabs(ui));
            }
          }
        } else if (t < ntiles && 16 * t >= r0 + NB) {
          // A operand: L[16t + q][r0 + KPL g + ks] read from original row
          const int ra = S.perm[16 * t + q];
          const double* pa_r = Fr + (size_t)ra * Np + r0 + KPL * g;
          const double* pa_i = Fi + (size_t)ra * Np + r0 + KPL * g;
          double ar[KPL], ai[KPL];
#pragma unroll
          for (int k = 0; k < KPL; ++k) { ar[k] = pa_r[k]; ai[k] = pa_i[k]; }
#pragma unroll
          for (int ks = 0; ks < KPL; ++ks) {
            const int k = KPL * g + ks;
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
              const double br = S.unr[k * LD(NB) + 16 * ct + q];
              const double bi = S.uni[k * LD(NB) + 16 * ct + q];
              xr[s][ct] = mfma(ar[ks], br, xr[s][ct]);
              xr[s][ct] = mfma(-ai[ks], bi, xr[s][ct]);
              xi[s][ct] = mfma(ar[ks], bi, xi[s][ct]);
              xi[s][ct] = mfma(ai[ks], br, xi[s][ct]);
            }
          }
        }
        // keep each row tile's operand loads next to its products (hoisting
        // all tiles' loads ahead would double the live registers)
        __builtin_amdgcn_sched_barrier(0);
      }
    }

    // ---- 3. panel factorisation of positions >= c0, column by column ------
#pragma unroll
    for (int cj = 0; cj < CT; ++cj) {
      for (int qj = 0; qj < 16; ++qj) {
        const int j = 16 * cj + qj;
        const int pj = c0 + j;
        const int par = j & 1;
        // A: pivot candidates (largest |Re|+|Im|, lowest position on ties)
        double best = -1.0;
        int brow = 0x7fffffff;
        if (q == qj) {
#pragma unroll
          for (int s = 0; s < RT; ++s) {
            const int t = w + WAVES * s;
            if (t < ntiles && 16 * t + 15 >= pj) {
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const int p = 16 * t + crow(g, i);
                const double m = fabs(xr[s][cj][i]) + fabs(xi[s][cj][i]);
                if (p >= pj && m > best) { best = m; brow = p; }
              }
            }
          }
        }
        argmax_wave(best, brow);
        if (lane == 0) { S.cmag[par * WAVES + w] = best; S.crowi[par * WAVES + w] = brow; }
        __syncthreads();
        // B: choose the pivot; owners publish the two rows to swap
        double bm = -1.0;
        int piv = 0x7fffffff;
#pragma unroll
        for (int ww = 0; ww < WAVES; ++ww) {
          const double m = S.cmag[par * WAVES + ww];
          const int rr = S.crowi[par * WAVES + ww];
          if (m > bm || (m == bm && rr < piv)) { bm = m; piv = rr; }
        }
        if (piv >= Np) piv = pj;   // no comparable entry (NaN column)
#pragma unroll
        for (int s = 0; s < RT; ++s) {
          const int t = w + WAVES * s;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int p = 16 * t + crow(g, i);
            if (t < ntiles && p == piv) {
#pragma unroll
              for (int ct = 0; ct < CT; ++ct) {
                S.rBr[16 * ct + q] = xr[s][ct][i];
                S.rBi[16 * ct + q] = xi[s][ct][i];
              }
            }
            if (t < ntiles && p == pj) {
#pragma unroll
              for (int ct = 0; ct < CT; ++ct) {
                S.rAr[16 * ct + q] = xr[s][ct][i];
                S.rAi[16 * ct + q] = xi[s][ct][i];
              }
            }
          }
        }
        if (tid == 0 && piv != pj) {
          const int tp = S.perm[pj];
          S.perm[pj] = S.perm[piv];
          S.perm[piv] = tp;
        }
        __syncthreads();
        // C: swap, scale the column below the pivot into multipliers
        const double pvr = S.rBr[j], pvi = S.rBi[j];
        const double den = pvr * pvr + pvi * pvi;
        const double ivr = pvr / den, ivi = -pvi / den;
#pragma unroll
        for (int s = 0; s < RT; ++s) {
          const int t = w + WAVES * s;
          if (t < ntiles) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int p = 16 * t + crow(g, i);
              if (piv != pj && p == pj) {
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) {
                  xr[s][ct][i] = S.rBr[16 * ct + q];
                  xi[s][ct][i] = S.rBi[16 * ct + q];
                }
              } else if (piv != pj && p == piv) {
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) {
                  xr[s][ct][i] = S.rAr[16 * ct + q];
                  xi[s][ct][i] = S.rAi[16 * ct + q];
                }
              }
              if (q == qj && p > pj) {
                const double ar = xr[s][cj][i], ai = xi[s][cj][i];
                const double lr = ar * ivr - ai * ivi;
                const double li = ar * ivi + ai * ivr;
                xr[s][cj][i] = lr;
                xi[s][cj][i] = li;
                S.mr[p] = lr;
                S.mi[p] = li;
              }
            }
          }
        }
        if (tid == 0) lsum += log(hypot(pvr, pvi));
        if (tid >= j && tid < NB) umax = fmax(umax, fabs(S.rBr[tid]) + fabs(S.rBi[tid]));
        __syncthreads();
        // D: rank-1 update of the columns right of j, rows below pj
#pragma unroll
        for (int s = 0; s < RT; ++s) {
          const int t = w + WAVES * s;
          if (t < ntiles && 16 * t + 15 > pj) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int p = 16 * t + crow(g, i);
              if (p > pj) {
                const double lr = S.mr[p], li = S.mi[p];
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) {
                  if (16 * ct + q > j) {
                    const double ur = S.rBr[16 * ct + q], ui = S.rBi[16 * ct + q];
                    xr[s][ct][i] -= lr * ur - li * ui;
                    xi[s][ct][i] -= lr * ui + li * ur;
                  }
                }
              }
            }
          }
        }
      }
    }

    // ---- 4. inverses of the diagonal blocks L_JJ (unit) and U_JJ ---------
#pragma unroll
    for (int s = 0; s < RT; ++s) {
      const int t = w + WAVES * s;
      if (t >= (c0 >> 4) && t < ((c0 + NB) >> 4)) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int pr = 16 * t + crow(g, i) - c0;
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            S.xsr[pr * LD(NB) + 16 * ct + q] = xr[s][ct][i];
            S.xsi[pr * LD(NB) + 16 * ct + q] = xi[s][ct][i];
          }
        }
      }
    }
    __syncthreads();
    if (tid < NB) {
      // column c of L_JJ^-1: Y[r][c] = -sum_{k=c}^{r-1} L[r][k] Y[k][c]
      const int c = tid;
      for (int r = 0; r < NB; ++r) {
        double yr, yi;
        if (r < c) { yr = 0.0; yi = 0.0; }
        else if (r == c) { yr = 1.0; yi = 0.0; }
        else {
          double sr = S.xsr[r * LD(NB) + c], si = S.xsi[r * LD(NB) + c];
          for (int k = c + 1; k < r; ++k) {
            const double lr = S.xsr[r * LD(NB) + k], li = S.xsi[r * LD(NB) + k];
            const double vr = S.lsr[k * LD(NB) + c], vi = S.lsi[k * LD(NB) + c];
            sr += lr * vr - li * vi;
            si += lr * vi + li * vr;
          }
          yr = -sr; yi = -si;
        }
        S.lsr[r * LD(NB) + c] = yr;
        S.lsi[r * LD(NB) + c] = yi;
      }
    } else if (tid < 2 * NB) {
      // column c of U_JJ^-1: Z[r][c] = -(sum_{k=r+1}^{c} U[r][k] Z[k][c]) / U[r][r]
      const int c = tid - NB;
      for (int r = NB - 1; r >= 0; --r) {
        double zr = 0.0, zi = 0.0;
        if (r <= c) {
          double sr = (r == c) ? 1.0 : 0.0, si = 0.0;
          for (int k = r + 1; k <= c; ++k) {
            const double ur = S.xsr[r * LD(NB) + k], ui = S.xsi[r * LD(NB) + k];
            const double vr = S.unr[k * LD(NB) + c], vi = S.uni[k * LD(NB) + c];
            sr -= ur * vr - ui * vi;
            si -= ur * vi + ui * vr;
          }
          const double pr = S.xsr[r * LD(NB) + r], pi = S.xsi[r * LD(NB) + r];
          const double dd = pr * pr + pi * pi;
          zr = (sr * pr + si * pi) / dd;
          zi = (si * pr - sr * pi) / dd;
        }
        S.unr[r * LD(NB) + c] = zr;
        S.uni[r * LD(NB) + c] = zi;
      }
    }
    __syncthreads();
    {
      double* Lr = T + (size_t)(J * 4 + 0) * NB * NB;
      double* Li = Lr + NB * NB;
      double* Ur = Li + NB * NB;
      double* Ui = Ur + NB * NB;
      for (int e = tid; e < NB * NB; e += NT) {
        const int rr = e / NB, cc = e % NB;
        Lr[e] = S.lsr[rr * LD(NB) + cc];
        Li[e] = S.lsi[rr * LD(NB) + cc];
        Ur[e] = S.unr[rr * LD(NB) + cc];
        Ui[e] = S.uni[rr * LD(NB) + cc];
      }
    }

    // ---- 5. store block column J at the original rows ---------------------
#pragma unroll
    for (int s = 0; s < RT; ++s) {
      const int t = w + WAVES * s;
      if (t < ntiles) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = S.perm[16 * t + crow(g, i)];
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            Fr[(size_t)r * Np + c0 + 16 * ct + q] = xr[s][ct][i];
            Fi[(size_t)r * Np + c0 + 16 * ct + q] = xi[s][ct][i];
          }
        }
      }
    }
    __syncthreads();
  }

  for (int p = tid; p < Np; p += NT) perm_out[(size_t)b * Np + p] = S.perm[p];
  // growth = max|u| / max|a| over the block
  for (int off = 32; off >= 1; off >>= 1) {
    umax = fmax(umax, __shfl_xor(umax, off));
    amax = fmax(amax, __shfl_xor(amax, off));
  }
  __syncthreads();
  if (lane == 0) { S.mr[w] = umax; S.mi[w] = amax; }
  __syncthreads();
  if (tid == 0) {
    double u = 0.0, a = 0.0;
    for (int ww = 0; ww < WAVES; ++ww) { u = fmax(u, S.mr[ww]); a = fmax(a, S.mi[ww]); }
    growth[b] = u / a;
    lad[b] = lsum;
  }
}

// --------------------------------------------------------------------------
// W = U^-1 (which == 0) or V = L^-1 (which == 1), in place in F.
//   W[:, J] = -(sum_{I<J} W[:, I] U[I, J]) U_JJ^-1  for rows above block J
//   V[:, J] = -(sum_{K>J} V[:, K] L[K, J]) L_JJ^-1  for rows below block J
// Each step forms Y = U[I,J] U_JJ^-1 (or L[K,J] L_JJ^-1) in LDS, then the
// waves accumulate their row tiles with the f64 MFMA.  W[a][k] lives where
// U[a][k] was (row perm[a]), V[r][k] where L[r][k] was.
size_t trtri_lds_bytes(int Np, int NB) {
  return sizeof(int) * Np + sizeof(double) * 6 * NB * (NB + 1) + 64;
}

template <int WAVES, int RT, int CT>
__global__ void __launch_bounds__(WAVES * 64)
trtri_kernel(int Np, double* __restrict__ F, const int* __restrict__ perm_g,
             const double* __restrict__ tri) {
  constexpr int NB = 16 * CT;
  constexpr int NT = WAVES * 64;
  constexpr int KPL = NB / 4;
  extern __shared__ double lds_raw[];
  const int b = blockIdx.x;
  const int upper = (blockIdx.y == 0);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = lane >> 4, q = lane & 15;
  const int ntiles = Np >> 4;
  const int nblk = Np / NB;
  double* xsr = lds_raw;                 // block of U or L
  double* xsi = xsr + NB * LD(NB);
  double* dir = xsi + NB * LD(NB);       // U_JJ^-1 or L_JJ^-1
  double* dii = dir + NB * LD(NB);
  double* yr_s = dii + NB * LD(NB);      // Y
  double* yi_s = yr_s + NB * LD(NB);
  int* perm = reinterpret_cast<int*>(yi_s + NB * LD(NB));
  const size_t plane = (size_t)Np * Np;
  double* Fr = F + (size_t)b * 2 * plane;
  double* Fi = Fr + plane;
  const double* T = tri + (size_t)b * nblk * 4 * NB * NB;
  for (int p = tid; p < Np; p += NT) perm[p] = perm_g[(size_t)b * Np + p];

  for (int jj = 0; jj < nblk; ++jj) {
    const int J = upper ? jj : nblk - 1 - jj;
    const int c0 = J * NB;
    __syncthreads();
    {
      const double* Dr = T + (size_t)(J * 4 + (upper ? 2 : 0)) * NB * NB;
      const double* Di = Dr + NB * NB;
      for (int e = tid; e < NB * NB; e += NT) {
        dir[(e / NB) * LD(NB) + e % NB] = Dr[e];
        dii[(e / NB) * LD(NB) + e % NB] = Di[e];
      }
    }
    d4 ar_[RT][CT], ai_[RT][CT];
#pragma unroll
    for (int s = 0; s < RT; ++s)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        ar_[s][ct] = (d4){0.0, 0.0, 0.0, 0.0};
        ai_[s][ct] = (d4){0.0, 0.0, 0.0, 0.0};
      }
    const int nsteps = upper ? J : nblk - 1 - J;
    for (int st = 0; st < nsteps; ++st) {
      const int I = upper ? st : J + 1 + st;   // block row of U[I,J] / L[I,J]
      const int r0 = I * NB;
      __syncthreads();
      for (int e = tid; e < NB * NB; e += NT) {
        const int rr = e / NB, cc = e % NB;
        const int orow = perm[r0 + rr];
        xsr[rr * LD(NB) + cc] = Fr[(size_t)orow * Np + c0 + cc];
        xsi[rr * LD(NB) + cc] = Fi[(size_t)orow * Np + c0 + cc];
      }
      __syncthreads();
      // Y = X_blk * D  (D = U_JJ^-1 or L_JJ^-1)
      for (int task = w; task < 2 * CT * CT; task += WAVES) {
        const int rt = task / (2 * CT), ct = (task >> 1) % CT, part = task & 1;
        d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < NB / 4; ++ks) {
          const int k = 4 * ks + g;
          const double a_r = xsr[(16 * rt + q) * LD(NB) + k];
          const double a_i = xsi[(16 * rt + q) * LD(NB) + k];
          const double b_r = dir[k * LD(NB) + 16 * ct + q];
          const double b_i = dii[k * LD(NB) + 16 * ct + q];
          if (part == 0) { acc = mfma(a_r, b_r, acc); acc = mfma(-a_i, b_i, acc); }
          else { acc = mfma(a_r, b_i, acc); acc = mfma(a_i, b_r, acc); }
        }
        double* dst = part ? yi_s : yr_s;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          dst[(16 * rt + crow(g, i)) * LD(NB) + 16 * ct + q] = acc[i];
      }
      __syncthreads();
      // acc[rows] += Tri[rows, I-cols] * Y, rows in the triangle's reach
#pragma unroll
      for (int s = 0; s < RT; ++s) {
        const int t = w + WAVES * s;
        const bool active = upper ? (t < (c0 >> 4) && 16 * t < r0 + NB)
                                  : (t < ntiles && t >= ((c0 + NB) >> 4) && 16 * t + 15 >= r0);
        if (active) {
          const int arow = 16 * t + q;     // A-operand row (position)
          const int orow = perm[arow];
          const double* pa_r = Fr + (size_t)orow * Np + r0 + KPL * g;
          const double* pa_i = Fi + (size_t)orow * Np + r0 + KPL * g;
          double a_r[KPL], a_i[KPL];
#pragma unroll
          for (int k = 0; k < KPL; ++k) {
            const int col = r0 + KPL * g + k;
            double vr = pa_r[k], vi = pa_i[k];
            if (upper) {
              if (col < arow) { vr = 0.0; vi = 0.0; }
            } else {
              if (col > arow) { vr = 0.0; vi = 0.0; }
              else if (col == arow) { vr = 1.0; vi = 0.0; }
            }
            a_r[k] = vr; a_i[k] = vi;
          }
#pragma unroll
          for (int ks = 0; ks < KPL; ++ks) {
            const int k = KPL * g + ks;
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
              const double b_r = yr_s[k * LD(NB) + 16 * ct + q];
              const double b_i = yi_s[k * LD(NB) + 16 * ct + q];
              ar_[s][ct] = mfma(a_r[ks], b_r, ar_[s][ct]);
              ar_[s][ct] = mfma(-a_i[ks], b_i, ar_[s][ct]);
              ai_[s][ct] = mfma(a_r[ks], b_i, ai_[s][ct]);
              ai_[s][ct] = mfma(a_i[ks], b_r, ai_[s][ct]);
            }
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    __syncthreads();
    // store -acc for the rows of the triangle, then the diagonal block
#pragma unroll
    for (int s = 0; s < RT; ++s) {
      const int t = w + WAVES * s;
      const bool active = upper ? (t < (c0 >> 4)) : (t < ntiles && t >= ((c0 + NB) >> 4));
      if (active) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int orow = perm[16 * t + crow(g, i)];
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            Fr[(size_t)orow * Np + c0 + 16 * ct + q] = -ar_[s][ct][i];
            Fi[(size_t)orow * Np + c0 + 16 * ct + q] = -ai_[s][ct][i];
          }
        }
      }
    }
    for (int e = tid; e < NB * NB; e += NT) {
      const int rr = e / NB, cc = e % NB;
      const bool mine = upper ? (cc >= rr) : (cc < rr);
      if (mine) {
        const int orow = perm[c0 + rr];
        Fr[(size_t)orow * Np + c0 + cc] = dir[rr * LD(NB) + cc];
        Fi[(size_t)orow * Np + c0 + cc] = dii[rr * LD(NB) + cc];
      }
    }
  }
}

// --------------------------------------------------------------------------
// (A^-1)_{perm[j]} = sum_{s >= max(perm[j], j)} W[perm[j]][s] V[s][j],
// V[j][j] = 1.  One workgroup per (64 positions j, matrix); W and V tiles
// are staged through LDS so both are read row-contiguously.
constexpr int kDD = 32;
constexpr int kDDParts = 8;   // 256 threads = 32 positions x 8 s-slices

__global__ void __launch_bounds__(256)
diagdot_kernel(int N, int Np, const double* __restrict__ F,
               const int* __restrict__ perm_g, double* __restrict__ dg) {
  const int j0 = blockIdx.x * kDD;
  const int b = blockIdx.y;
  const int tid = threadIdx.x;
  __shared__ double wr[kDD][kDD + 1], wi[kDD][kDD + 1];   // [j][s]
  __shared__ double vr[kDD][kDD + 1], vi[kDD][kDD + 1];   // [s][j]
  __shared__ int wrow[kDD], lo[kDD];
  __shared__ double pr_s[kDDParts][kDD], pi_s[kDDParts][kDD];
  const size_t plane = (size_t)Np * Np;
  const double* Fr = F + (size_t)b * 2 * plane;
  const double* Fi = Fr + plane;
  const int* perm = perm_g + (size_t)b * Np;
  if (tid < kDD) {
    const int j = j0 + tid;
    if (j < Np) {
      const int i = perm[j];
      wrow[tid] = perm[i];                 // storage row of W[i][.]
      lo[tid] = i > j ? i : j;             // first s of the sum
    } else {
      wrow[tid] = 0;
      lo[tid] = Np;
    }
  }
  const int jl = tid % kDD, part = tid / kDD;
  constexpr int SPP = kDD / kDDParts;      // s values per slice
  double accr = 0.0, acci = 0.0;
  for (int s0 = j0; s0 < Np; s0 += kDD) {
    __syncthreads();
    for (int e = tid; e < kDD * kDD; e += 256) {
      const int a = e / kDD, c = e % kDD;
      double x_r = 0.0, x_i = 0.0, y_r = 0.0, y_i = 0.0;
      // W tile: W[perm[j0 + a]][s0 + c]
      if (j0 + a < Np && s0 + c < Np) {
        x_r = Fr[(size_t)wrow[a] * Np + s0 + c];
        x_i = Fi[(size_t)wrow[a] * Np + s0 + c];
      }
      // V tile: V[s0 + a][j0 + c], stored at row perm[s0 + a]
      if (s0 + a < Np && j0 + c < Np) {
        const int vrow = perm[s0 + a];
        y_r = Fr[(size_t)vrow * Np + j0 + c];
        y_i = Fi[(size_t)vrow * Np + j0 + c];
      }
      wr[a][c] = x_r; wi[a][c] = x_i;
      vr[a][c] = y_r; vi[a][c] = y_i;
    }
    __syncthreads();
    const int j = j0 + jl;
    const int first = lo[jl];
#pragma unroll
    for (int k = 0; k < SPP; ++k) {
      const int sl = part * SPP + k;
      const int s = s0 + sl;
      if (s >= first && s < Np) {
        double yr = vr[sl][jl], yi = vi[sl][jl];
        if (s == j) { yr = 1.0; yi = 0.0; }
        const double xr_ = wr[jl][sl], xi_ = wi[jl][sl];
        accr += xr_ * yr - xi_ * yi;
        acci += xr_ * yi + xi_ * yr;
      }
    }
  }
  pr_s[part][jl] = accr;
  pi_s[part][jl] = acci;
  __syncthreads();
  if (tid < kDD) {
    const int j = j0 + tid;
    if (j < Np) {
      const int i = perm[j];
      if (i < N) {
        double sr = 0.0, si = 0.0;
        for (int pp = 0; pp < kDDParts; ++pp) { sr += pr_s[pp][tid]; si += pi_s[pp][tid]; }
        dg[((size_t)b * N + i) * 2 + 0] = sr;
        dg[((size_t)b * N + i) * 2 + 1] = si;
      }
    }
  }
}

// --------------------------------------------------------------------------

namespace {

template <int WAVES, int RT, int CT>
hipError_t run_lu(const MatDesc* descs, const double* hbuf, int B, int N,
                  int Np, int L, double* F, int* perm, double* tri,
                  double* lad, double* growth, hipStream_t st) {
  const size_t lds = lu_lds_bytes(Np, 16 * CT, WAVES);
  mark_begin(K_LU, st);
  hipLaunchKernelGGL((lu_kernel<WAVES, RT, CT>), dim3(B), dim3(WAVES * 64),
                     lds, st, descs, hbuf, N, Np, L, F, perm, tri, lad, growth);
  mark_end(K_LU, st);
  return hipGetLastError();
}

template <int WAVES, int RT, int CT>
hipError_t run_inv(int B, int N, int Np, double* F, const int* perm,
                   const double* tri, double* dg, hipStream_t st) {
  const size_t lds = trtri_lds_bytes(Np, 16 * CT);
  mark_begin(K_TRTRI, st);
  hipLaunchKernelGGL((trtri_kernel<WAVES, RT, CT>), dim3(B, 2), dim3(WAVES * 64),
                     lds, st, Np, F, perm, tri);
  mark_end(K_TRTRI, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  mark_begin(K_DIAGDOT, st);
  hipLaunchKernelGGL(diagdot_kernel, dim3((Np + kDD - 1) / kDD, B), dim3(256),
                     0, st, N, Np, F, perm, dg);
  mark_end(K_DIAGDOT, st);
  return hipGetLastError();
}

}  // namespace

BlockedPlan blocked_plan_f64(int N) {
  BlockedPlan p{};
  const int n16 = (N + 15) / 16 * 16;
  if (n16 <= 256) { p.cfg = 0; p.NB = 32; }
  else if (n16 <= 512) { p.cfg = 1; p.NB = 32; }
  else if (n16 <= 1024) { p.cfg = 2; p.NB = 16; }
  else { p.cfg = -1; p.NB = 0; return p; }
  p.Np = (N + p.NB - 1) / p.NB * p.NB;
  if ((p.cfg == 0 && p.Np > 256) || (p.cfg == 1 && p.Np > 512)) {
    // rounding up to the block width crossed into the next configuration
    p.cfg += 1;
    if (p.cfg == 2) { p.NB = 16; p.Np = n16; }
  }
  return p;
}

hipError_t blocked_lu_f64(const BlockedPlan& p, const MatDesc* descs,
                          const double* hbuf, int B, int N, int L, double* F,
                          int* perm, double* tri, double* lad, double* growth,
                          hipStream_t st) {
  switch (p.cfg) {
    case 0: return run_lu<4, 4, 2>(descs, hbuf, B, N, p.Np, L, F, perm, tri, lad, growth, st);
    case 1: return run_lu<8, 4, 2>(descs, hbuf, B, N, p.Np, L, F, perm, tri, lad, growth, st);
    case 2: return run_lu<8, 8, 1>(descs, hbuf, B, N, p.Np, L, F, perm, tri, lad, growth, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t blocked_inv_f64(const BlockedPlan& p, int B, int N, double* F,
                           const int* perm, const double* tri, double* dg,
                           hipStream_t st) {
  switch (p.cfg) {
    case 0: return run_inv<4, 4, 2>(B, N, p.Np, F, perm, tri, dg, st);
    case 1: return run_inv<8, 4, 2>(B, N, p.Np, F, perm, tri, dg, st);
    case 2: return run_inv<8, 8, 1>(B, N, p.Np, F, perm, tri, dg, st);
    default: return hipErrorInvalidValue;
  }
}

size_t blocked_factor_bytes_f64(const BlockedPlan& p, int B) {
  const size_t Np = p.Np, NB = p.NB;
  const size_t F = 2 * Np * Np * sizeof(double);
  const size_t perm = Np * sizeof(int);
  const size_t tri = (Np / NB) * 4 * NB * NB * sizeof(double);
  return (size_t)B * (F + perm + tri) + 3 * 256;
}

}  // namespace sca
