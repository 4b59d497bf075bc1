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
#include "k_factor_common.h"
#include "sca_profile.h"

namespace sca {

namespace {

template <typename T, int NB>
struct LuLds {
  int* perm;          // [Np] position -> original row
  double* cmag;       // [2][WAVES] best |Re|+|Im| of each wave (by column parity)
  int* crowi;         // [2][WAVES] its position
  T *rAr, *rAi;       // [2][NB] row at the pivot position before the swap
  T *slr, *sli;       // [2][WAVES][NB] each wave's candidate pivot row
  T *mr, *mi;         // [Np] multipliers of the current column
  T *xsr, *xsi;       // [NB][NB+1] rows of a previous panel / diagonal block
  T *lsr, *lsi;       // [NB][NB+1] L_II^-1
  T *unr, *uni;       // [NB][NB+1] -U_IJ, or U_JJ^-1
  T *tr_, *ti_;       // [NB*NB/2] scratch of the block inversion
  double* red;        // [NT] final reductions
  double* hs;         // [Np] row panel: the matrix's diagonal h
  int* nbr;           // [4][Np] row panel: the 4 lattice neighbours of a site
};

}  // namespace

// row panel: staging chunk width (columns) and staging size (elements of T)
// per wave
constexpr int rp_chunk(int waves) { return waves > 8 ? 4 : 8; }
constexpr int rp_stage_per_wave(int waves) { return 2 * 64 * (rp_chunk(waves) + 1); }

template <typename T>
size_t lu_lds_bytes(int Np, int NB, int waves, bool rp = false) {
  size_t b = 0;
  if (rp) {
    const long extra = (long)waves * rp_stage_per_wave(waves) - (6L * NB * (NB + 1) + (long)NB * NB);
    if (extra > 0) b += sizeof(T) * extra;
  }
  b += sizeof(int) * Np;
  if (rp) b += sizeof(double) * Np + sizeof(int) * 4 * Np;   // h, neighbours
  b += sizeof(double) * 2 * waves + sizeof(int) * 2 * waves;
  b += sizeof(double) * 64 * waves;        // final reductions
  b += sizeof(T) * 4 * NB;                 // rA [2][NB] re, im
  b += sizeof(T) * 4 * waves * NB;         // slots [2][W][NB] re, im
  b += sizeof(T) * 2 * Np;
  b += sizeof(T) * 6 * NB * (NB + 1);
  b += sizeof(T) * NB * NB;                // inversion scratch
  return b + 256;
}

// OCC: workgroups per CU the instance is sized for (its registers are
// capped at 512 / (OCC * WAVES / 4) per lane).
template <typename T, int WAVES, int RT, int CT, bool kRP = false, int OCC = 1>
__global__ void __launch_bounds__(WAVES * 64, OCC * WAVES / 4)
lu_kernel(const MatDesc* __restrict__ descs, const double* __restrict__ hbuf,
          int N, int Np, int L, T* __restrict__ F,
          int* __restrict__ perm_out, T* __restrict__ tri,
          double* __restrict__ lad, double* __restrict__ growth,
          const int* __restrict__ only, int want) {
  typedef Mma<T> M;
  typedef typename M::v4 V4;
  constexpr int NB = 16 * CT;
  constexpr int NT = WAVES * 64;
  constexpr int KPL = NB / 4;   // k values per lane group per panel
  extern __shared__ double lds_raw[];
  const int b = blockIdx.x;
  if (only && only[b] != want) return;   // matrix not selected
  const int tid0 = threadIdx.x;
  const int tid = tid0, lane = tid & 63, w = tid >> 6;
  const int ntiles = Np >> 4;
  const int nblk = Np / NB;

  // carve LDS (doubles first, then T arrays, then ints)
  LuLds<T, NB> S;
  {
    double* dd = lds_raw;
    S.cmag = dd; dd += 2 * WAVES;
    S.red = dd; dd += NT;
    if constexpr (kRP) { S.hs = dd; dd += Np; }
    T* d = reinterpret_cast<T*>(dd);
    S.mr = d; d += Np; S.mi = d; d += Np;
    S.rAr = d; d += 2 * NB; S.rAi = d; d += 2 * NB;
    S.slr = d; d += 2 * WAVES * NB; S.sli = d; d += 2 * WAVES * NB;
    S.xsr = d; d += NB * LD(NB); S.xsi = d; d += NB * LD(NB);
    S.lsr = d; d += NB * LD(NB); S.lsi = d; d += NB * LD(NB);
    S.unr = d; d += NB * LD(NB); S.uni = d; d += NB * LD(NB);
    S.tr_ = d; d += NB * NB / 2; S.ti_ = d; d += NB * NB / 2;
    if (kRP && d < S.xsr + WAVES * rp_stage_per_wave(WAVES)) d = S.xsr + WAVES * rp_stage_per_wave(WAVES);
    int* ip = reinterpret_cast<int*>(d);
    S.crowi = ip; ip += 2 * WAVES;
    S.perm = ip; ip += Np;
    S.nbr = ip;
  }

  const MatDesc dsc = descs[b];
  const double* h = hbuf + dsc.hoff;
  const size_t plane = (size_t)Np * Np;
  T* Fr = F + (size_t)b * 2 * plane;
  T* Fi = Fr + plane;
  T* Tb = tri + (size_t)b * nblk * 4 * NB * NB;   // [nblk][2][2][NB][NB]

  for (int p = tid; p < Np; p += NT) S.perm[p] = p;
  // row panel: h and each site's neighbours (+x, -x, +y, -y) once per
  // matrix, so that generating a block column divides by L nowhere and loads
  // nothing from global memory (the other instances keep their form: their
  // register allocation, hundreds of spilled VGPRs, is slower with it)
  if constexpr (kRP) {
    for (int p = tid; p < N; p += NT) S.hs[p] = h[p];
    for (int r = tid; r < N; r += NT) {
      const int x = r % L, y = r / L;
      S.nbr[r] = (x + 1) % L + L * y;
      S.nbr[Np + r] = (x + L - 1) % L + L * y;
      S.nbr[2 * Np + r] = x + L * ((y + 1) % L);
      S.nbr[3 * Np + r] = x + L * ((y + L - 1) % L);
    }
  }
  __syncthreads();

  V4 xr[RT][CT], xi[RT][CT];
  double lsum = 0.0, umax = 0.0, amax = 0.0;

  for (int J = 0; J < nblk; ++J) {
    const int c0 = J * NB;
    // row panel: per-block-column copies of the thread indices, so that
    // values derived from them are not hoisted out of this loop (they would
    // stay live through every phase and crowd the registers)
    int tid = tid0;
    if constexpr (kRP) asm volatile("" : "+v"(tid));
    const int lane = tid & 63;
    const int w = kRP ? __builtin_amdgcn_readfirstlane(tid >> 6) : tid >> 6;
    const int g = lane >> 4, q = lane & 15;
    // ---- 1. generate block column J: X[p][c] = A[perm[p]][c0 + c] ----------
#pragma unroll
    for (int s = 0; s < RT; ++s) {
      const int t = w + WAVES * s;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int p = 16 * t + M::m(g, i);
        const int r = (t < ntiles) ? S.perm[p] : Np;
        int n0 = -1, n1 = -1, n2 = -1, n3 = -1;
        double dre = 0.0;
        if (r < N) {
          if constexpr (kRP) {
            n0 = S.nbr[r];
            n1 = S.nbr[Np + r];
            n2 = S.nbr[2 * Np + r];
            n3 = S.nbr[3 * Np + r];
            dre = dsc.zr - S.hs[r];
          } else {
            const int x = r % L, y = r / L;
            n0 = (x + 1) % L + L * y;
            n1 = (x + L - 1) % L + L * y;
            n2 = x + L * ((y + 1) % L);
            n3 = x + L * ((y + L - 1) % L);
            dre = dsc.zr - h[r];
          }
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
          xr[s][ct][i] = T(re);
          xi[s][ct][i] = T(im);
        }
      }
      // one row tile at a time (hoisting every tile's index loads would
      // keep all their intermediate values live at once)
      if constexpr (kRP) __builtin_amdgcn_sched_barrier(0);
    }

    // ---- 2. left-looking updates from the previous panels ------------------
    if constexpr (kRP) {
    // The A operand of each step (L[rows below panel I][panel I], KPL values
    // per lane and row tile) and L_II^-1 are loaded one step ahead, so their
    // latency overlaps the previous step's products and barriers.
    // prefetch the A operand only while it fits beside the accumulators
    constexpr bool kPre = RT * KPL <= 16;
    constexpr int LSPT = (NB * NB + NT - 1) / NT;   // L_II^-1 elements per thread
    T ar_[RT][KPL], ai_[RT][KPL];
    T lsr_[LSPT], lsi_[LSPT];
    auto load_step = [&](int I) {
      const int r0 = I * NB;
      {
        const T* Lr = Tb + (size_t)(I * 4 + 0) * NB * NB;
#pragma unroll
        for (int u = 0; u < LSPT; ++u) {
          const int e = tid + u * NT;
          if (e < NB * NB) { lsr_[u] = Lr[e]; lsi_[u] = Lr[NB * NB + e]; }
        }
      }
      if constexpr (kPre) {
#pragma unroll
      for (int s = 0; s < RT; ++s) {
        const int t = w + WAVES * s;
        if (t < ntiles && 16 * t >= r0 + NB) {
          const int ra = S.perm[16 * t + q];
          const T* pa_r = Fr + (size_t)ra * Np + r0 + KPL * g;
          const T* pa_i = Fi + (size_t)ra * Np + r0 + KPL * g;
#pragma unroll
          for (int k = 0; k < KPL; ++k) { ar_[s][k] = pa_r[k]; ai_[s][k] = pa_i[k]; }
        }
      }
      }
    };
    // the generated block column is complete before the first operand loads
    // are issued (keeps the loads' registers out of the generation)
#pragma unroll
    for (int s = 0; s < RT; ++s)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
        asm volatile("" : "+v"(xr[s][ct]), "+v"(xi[s][ct]) :: "memory");
    if (J > 0) load_step(0);
    for (int I = 0; I < J; ++I) {
      const int r0 = I * NB;
      // (a) panel-I rows of X -> xs; L_II^-1 -> ls
#pragma unroll
      for (int s = 0; s < RT; ++s) {
        const int t = w + WAVES * s;
        if (t >= (r0 >> 4) && t < ((r0 + NB) >> 4)) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int pr = 16 * t + M::m(g, i) - r0;
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
              S.xsr[pr * LD(NB) + 16 * ct + q] = xr[s][ct][i];
              S.xsi[pr * LD(NB) + 16 * ct + q] = xi[s][ct][i];
            }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < LSPT; ++u) {
        const int e = tid + u * NT;
        if (e < NB * NB) {
          S.lsr[(e / NB) * LD(NB) + e % NB] = lsr_[u];
          S.lsi[(e / NB) * LD(NB) + e % NB] = lsi_[u];
        }
      }
      __syncthreads();
      // (b) un = -(L_II^-1 xs) = -U_IJ ; one 16x16 real output tile per task
      for (int task = w; task < 2 * CT * CT; task += WAVES) {
        const int rt = task / (2 * CT), ct = (task >> 1) % CT, part = task & 1;
        V4 acc = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int ks = 0; ks < NB / 4; ++ks) {
          const int k = 4 * ks + g;
          const T ar = S.lsr[(16 * rt + q) * LD(NB) + k];
          const T ai = S.lsi[(16 * rt + q) * LD(NB) + k];
          const T br = S.xsr[k * LD(NB) + 16 * ct + q];
          const T bi = S.xsi[k * LD(NB) + 16 * ct + q];
          if (part == 0) { acc = M::mma(ar, br, acc); acc = M::mma(-ai, bi, acc); }
          else { acc = M::mma(ar, bi, acc); acc = M::mma(ai, br, acc); }
        }
        T* dst = part ? S.uni : S.unr;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          dst[(16 * rt + M::m(g, i)) * LD(NB) + 16 * ct + q] = -acc[i];
      }
      __syncthreads();
      // (c) U_IJ to its rows of F; rows below panel I get X += L[:, I] (-U_IJ)
      for (int e = tid; e < NB * NB; e += NT) {
        const int rr = e / NB, cc = e % NB;
        const T ur = -S.unr[rr * LD(NB) + cc], ui = -S.uni[rr * LD(NB) + cc];
        const size_t o = (size_t)S.perm[r0 + rr] * Np + c0 + cc;
        Fr[o] = ur;
        Fi[o] = ui;
        umax = fmax(umax, (double)fabs(ur) + (double)fabs(ui));
      }
#pragma unroll
      for (int s = 0; s < RT; ++s) {
        const int t = w + WAVES * s;
        if (t < ntiles && 16 * t >= r0 + NB) {
          if constexpr (!kPre) {
            const int ra = S.perm[16 * t + q];
            const T* pa_r = Fr + (size_t)ra * Np + r0 + KPL * g;
            const T* pa_i = Fi + (size_t)ra * Np + r0 + KPL * g;
#pragma unroll
            for (int k = 0; k < KPL; ++k) { ar_[s][k] = pa_r[k]; ai_[s][k] = pa_i[k]; }
          }
#pragma unroll
          for (int ks = 0; ks < KPL; ++ks) {
            const int k = KPL * g + ks;
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
              const T br = S.unr[k * LD(NB) + 16 * ct + q];
              const T bi = S.uni[k * LD(NB) + 16 * ct + q];
              xr[s][ct] = M::mma(ar_[s][ks], br, xr[s][ct]);
              xr[s][ct] = M::mma(-ai_[s][ks], bi, xr[s][ct]);
              xi[s][ct] = M::mma(ar_[s][ks], bi, xi[s][ct]);
              xi[s][ct] = M::mma(ai_[s][ks], br, xi[s][ct]);
            }
          }
        }
        if constexpr (!kPre) __builtin_amdgcn_sched_barrier(0);
      }
      __builtin_amdgcn_sched_barrier(0);
      if (I + 1 < J) load_step(I + 1);
    }
    } else {
    for (int I = 0; I < J; ++I) {
      const int r0 = I * NB;
      // (a) panel-I rows of X -> xs; L_II^-1 -> ls
#pragma unroll
      for (int s = 0; s < RT; ++s) {
        const int t = w + WAVES * s;
        if (t >= (r0 >> 4) && t < ((r0 + NB) >> 4)) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int pr = 16 * t + M::m(g, i) - r0;
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
              S.xsr[pr * LD(NB) + 16 * ct + q] = xr[s][ct][i];
              S.xsi[pr * LD(NB) + 16 * ct + q] = xi[s][ct][i];
            }
          }
        }
      }
      {
        const T* Lr = Tb + (size_t)(I * 4 + 0) * NB * NB;
        const T* Li = Lr + NB * NB;
        for (int e = tid; e < NB * NB; e += NT) {
          S.lsr[(e / NB) * LD(NB) + e % NB] = Lr[e];
          S.lsi[(e / NB) * LD(NB) + e % NB] = Li[e];
        }
      }
      __syncthreads();
      // (b) un = -(L_II^-1 xs) = -U_IJ ; one 16x16 real output tile per task
      for (int task = w; task < 2 * CT * CT; task += WAVES) {
        const int rt = task / (2 * CT), ct = (task >> 1) % CT, part = task & 1;
        V4 acc = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int ks = 0; ks < NB / 4; ++ks) {
          const int k = 4 * ks + g;
          const T ar = S.lsr[(16 * rt + q) * LD(NB) + k];
          const T ai = S.lsi[(16 * rt + q) * LD(NB) + k];
          const T br = S.xsr[k * LD(NB) + 16 * ct + q];
          const T bi = S.xsi[k * LD(NB) + 16 * ct + q];
          if (part == 0) { acc = M::mma(ar, br, acc); acc = M::mma(-ai, bi, acc); }
          else { acc = M::mma(ar, bi, acc); acc = M::mma(ai, br, acc); }
        }
        T* dst = part ? S.uni : S.unr;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          dst[(16 * rt + M::m(g, i)) * LD(NB) + 16 * ct + q] = -acc[i];
      }
      __syncthreads();
      // (c) U_IJ is final: all threads copy it from LDS to its rows of F (the
      //     register copies of rows above the panel are not used again);
      //     rows below panel I get X += L[:, I] (-U_IJ)
      for (int e = tid; e < NB * NB; e += NT) {
        const int rr = e / NB, cc = e % NB;
        const T ur = -S.unr[rr * LD(NB) + cc], ui = -S.uni[rr * LD(NB) + cc];
        const size_t o = (size_t)S.perm[r0 + rr] * Np + c0 + cc;
        Fr[o] = ur;
        Fi[o] = ui;
        umax = fmax(umax, (double)fabs(ur) + (double)fabs(ui));
      }
#pragma unroll
      for (int s = 0; s < RT; ++s) {
        const int t = w + WAVES * s;
        if (t < ntiles && 16 * t >= r0 + NB) {
          // A operand: L[16t + q][r0 + KPL g + ks] read from original row
          const int ra = S.perm[16 * t + q];
          const T* pa_r = Fr + (size_t)ra * Np + r0 + KPL * g;
          const T* pa_i = Fi + (size_t)ra * Np + r0 + KPL * g;
          T ar[KPL], ai[KPL];
#pragma unroll
          for (int k = 0; k < KPL; ++k) { ar[k] = pa_r[k]; ai[k] = pa_i[k]; }
#pragma unroll
          for (int ks = 0; ks < KPL; ++ks) {
            const int k = KPL * g + ks;
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
              const T br = S.unr[k * LD(NB) + 16 * ct + q];
              const T bi = S.uni[k * LD(NB) + 16 * ct + q];
              xr[s][ct] = M::mma(ar[ks], br, xr[s][ct]);
              xr[s][ct] = M::mma(-ai[ks], bi, xr[s][ct]);
              xi[s][ct] = M::mma(ar[ks], bi, xi[s][ct]);
              xi[s][ct] = M::mma(ai[ks], br, xi[s][ct]);
            }
          }
        }
        // keep each row tile's operand loads next to its products (hoisting
        // all tiles' loads ahead would double the live registers)
        __builtin_amdgcn_sched_barrier(0);
      }
    }

    }

    if constexpr (kRP) {
    // ---- 3. one row per lane: lane L of wave w takes, for k < RPT, row
    //         L & 15 of its tile s = 4k + L/16 (position 16 (w + WAVES s) +
    //         L % 16), through a region of LDS private to the wave, CW
    //         columns at a time
    constexpr int RPT = (RT + 3) / 4;
    constexpr int CW = rp_chunk(WAVES);
    T yr[RPT][NB], yi[RPT][NB];
    int pos[RPT], org[RPT];
    T* stg = S.xsr + w * rp_stage_per_wave(WAVES);
    __syncthreads();   // the staging overlays LDS the update has read
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int s = 4 * k + (lane >> 4);
      const int p = 16 * (w + WAVES * s) + (lane & 15);
      const bool live = s < RT && p >= c0 && p < Np;
      pos[k] = live ? p : -1;
      org[k] = live ? S.perm[p] : 0;
#pragma unroll
      for (int cb = 0; cb < NB; cb += CW) {
        const int ct = cb >> 4, q0 = cb & 15;
#pragma unroll
        for (int sl = 0; sl < 4; ++sl) {
          const int ss = 4 * k + sl;
          if (ss < RT) {
            if (q >= q0 && q < q0 + CW) {
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const int r = 16 * sl + M::m(g, i);
                stg[2 * (r * (CW + 1) + q - q0)] = xr[ss][ct][i];
                stg[2 * (r * (CW + 1) + q - q0) + 1] = xi[ss][ct][i];
              }
            }
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int c = 0; c < CW; ++c) {
          yr[k][cb + c] = stg[2 * (lane * (CW + 1) + c)];
          yi[k][cb + c] = stg[2 * (lane * (CW + 1) + c) + 1];
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
    }
    // ---- 4. panel, one barrier per column.  Rows do not move: a row's
    //         position changes when it is swapped (pos), its data stays.
    auto column = [&](auto jc) {
      constexpr int j = decltype(jc)::value;
      const int pj = c0 + j;
      const int par = j & 1;
      // A: best row of this thread, then of the wave (largest |Re|+|Im|,
      //    lowest position on ties; NaN magnitudes count as 0)
      double m = -1.0;
      int mp = 0x7fffffff, mk = 0;
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        double a = (double)fabs(yr[k][j]) + (double)fabs(yi[k][j]);
        a = (a >= 0.0) ? a : 0.0;
        const bool better = pos[k] >= pj && (a > m || (a == m && pos[k] < mp));
        m = better ? a : m;
        mp = better ? pos[k] : mp;
        mk = better ? k : mk;
      }
      const double wm = wave_max_d(m);
      // lowest position among the lanes holding the maximum
      const int wp = wave_min_i((m == wm) ? mp : 0x7fffffff);
      const int wl = __ffsll((long long)__ballot(m == wm && mp == wp)) - 1;
      const int wk = __builtin_amdgcn_readlane(mk, wl);
      T* slot = S.slr + (par * WAVES + w) * 2 * NB;
      if (lane == 0) { S.cmag[par * WAVES + w] = wm; S.crowi[par * WAVES + w] = wp; }
      if (wm >= 0.0 && lane == wl) {
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
          if (k == wk) {
#pragma unroll
            for (int c = j; c < NB; ++c) { slot[2 * c] = yr[k][c]; slot[2 * c + 1] = yi[k][c]; }
          }
        }
      }
      __syncthreads();
      // B: the winner over the waves.  Lane v of every group of WAVES lanes
      //    reads wave v's candidate (magnitude, position and pivot value, in
      //    one round of independent loads); DPP steps inside the group then
      //    leave the winner (largest magnitude, lowest position on ties; the
      //    eligible positions are distinct, so it is unique) in every lane.
      static_assert(WAVES == 4 || WAVES == 8 || WAVES == 16, "group of waves");
      int cw = lane & (WAVES - 1);
      double bm = S.cmag[par * WAVES + cw];
      int piv = S.crowi[par * WAVES + cw];
      double pvr = S.slr[(par * WAVES + cw) * 2 * NB + 2 * j];
      double pvi = S.slr[(par * WAVES + cw) * 2 * NB + 2 * j + 1];
      auto merge = [&](auto ctl) {
        constexpr int C = decltype(ctl)::value;
        const double om = dpp_d<C>(bm), orr = dpp_d<C>(pvr), oi = dpp_d<C>(pvi);
        const int op = dpp_i<C>(piv), ow = dpp_i<C>(cw);
        const bool better = (om > bm) | ((om == bm) & (op < piv));
        bm = better ? om : bm;
        piv = better ? op : piv;
        cw = better ? ow : cw;
        pvr = better ? orr : pvr;
        pvi = better ? oi : pvi;
      };
      merge(std::integral_constant<int, 0xB1>{});   // lane pairs
      merge(std::integral_constant<int, 0x4E>{});   // quads
      if constexpr (WAVES >= 8) merge(std::integral_constant<int, 0x141>{});
      if constexpr (WAVES >= 16) merge(std::integral_constant<int, 0x140>{});
      piv = __builtin_amdgcn_readfirstlane(piv);
      const int ww = __builtin_amdgcn_readfirstlane(cw);
      const T* prow = S.slr + (par * WAVES + ww) * 2 * NB;
      const double rden = 1.0 / (pvr * pvr + pvi * pvi);
      const T ivr = T(pvr * rden), ivi = T(-pvi * rden);
      {
        const int cu = tid < j ? j : (tid < NB ? tid : NB - 1);
        const double au = (double)fabs(prow[2 * cu]) + (double)fabs(prow[2 * cu + 1]);
        umax = (tid >= j && tid < NB) ? fmax(umax, au) : umax;
      }
      // C: the pivot row moves to position pj, the row at pj to piv
#pragma unroll
      for (int k = 0; k < RPT; ++k)
        pos[k] = (pos[k] == piv) ? pj : (pos[k] == pj ? piv : pos[k]);
      // D: multipliers of the rows below the pivot (zero elsewhere, which
      //    leaves those rows unchanged), then the rank-1 update with the
      //    pivot row read from LDS four columns at a time
      T lr[RPT], li[RPT];
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const bool below = pos[k] > pj;
        const T ar = yr[k][j], ai = yi[k][j];
        lr[k] = below ? ar * ivr - ai * ivi : T(0);
        li[k] = below ? ar * ivi + ai * ivr : T(0);
        yr[k][j] = below ? lr[k] : ar;
        yi[k][j] = below ? li[k] : ai;
      }
#pragma unroll
      for (int cg = j + 1; cg < NB; cg += 4) {
        // compiler barrier: this group's pivot-row loads are not hoisted
        // above the previous group's products (they would all be live at once)
        asm volatile("" ::: "memory");
        T ur[4], ui[4];
#pragma unroll
        for (int c = 0; c < 4; ++c)
          if (cg + c < NB) { ur[c] = prow[2 * (cg + c)]; ui[c] = prow[2 * (cg + c) + 1]; }
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            if (cg + c < NB) {
              yr[k][cg + c] = fma(-lr[k], ur[c], fma(li[k], ui[c], yr[k][cg + c]));
              yi[k][cg + c] = fma(-lr[k], ui[c], fma(-li[k], ur[c], yi[k][cg + c]));
              // keep the products here (not sunk to their next use, which
              // would keep the loaded pivot row live)
              asm volatile("" : "+v"(yr[k][cg + c]), "+v"(yi[k][cg + c]));
            }
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    };
    StaticFor<0, NB>::run(column);
    // ---- 5. rows to F at their original rows, through the wave's LDS
    //         region CW columns at a time: a store then covers 16 rows x
    //         2 adjacent columns (one 64-byte run per row) instead of one
    //         element of 64 different rows
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
#pragma unroll
      for (int cb = 0; cb < NB; cb += CW) {
#pragma unroll
        for (int c = 0; c < CW; ++c) {
          stg[2 * (lane * (CW + 1) + c)] = yr[k][cb + c];
          stg[2 * (lane * (CW + 1) + c) + 1] = yi[k][cb + c];
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        constexpr int LPR = CW / 2;           // lanes per row
        constexpr int RPI = 64 / LPR;         // rows per store
#pragma unroll
        for (int it = 0; it < 64 / RPI; ++it) {
          const int src = RPI * it + lane / LPR, cp = 2 * (lane % LPR);
          const int spos = __shfl(pos[k], src), sorg = __shfl(org[k], src);
          const T* e = stg + 2 * (src * (CW + 1) + cp);
          if (spos >= 0) {
            // even element offsets: two elements form one aligned store
            typedef T T2 __attribute__((ext_vector_type(2)));
            T* dst = Fr + (size_t)sorg * Np + c0 + cb + cp;
            *reinterpret_cast<T2*>(dst) = T2{e[0], e[2]};
            *reinterpret_cast<T2*>(dst + plane) = T2{e[1], e[3]};
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
    }
    // the diagonal block goes to LDS that overlays the staging regions
    __syncthreads();
    // the diagonal block to LDS, positions to perm
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      if (pos[k] >= 0) {
        if (pos[k] < c0 + NB) {
          const int pr = pos[k] - c0;
#pragma unroll
          for (int c = 0; c < NB; ++c) {
            S.xsr[pr * LD(NB) + c] = yr[k][c];
            S.xsi[pr * LD(NB) + c] = yi[k][c];
          }
        }
        S.perm[pos[k]] = org[k];
      }
    }
    } else {
    // ---- 3. panel factorisation of positions >= c0, one barrier per column
    // Each wave finds its best candidate row for column j and publishes it
    // (|Re|+|Im|, position and the row's values) together with the row now
    // at the pivot position; after the barrier every lane picks the winner
    // (largest magnitude, lowest position on ties) and reads the pivot row
    // from LDS.  Multipliers go from the lane owning column j to the other
    // lanes of its row group through LDS inside the wave (no barrier).
#pragma unroll
    for (int cj = 0; cj < CT; ++cj) {
      for (int qj = 0; qj < 16; ++qj) {
        const int j = 16 * cj + qj;
        const int pj = c0 + j;
        const int par = j & 1;
        T* slr = S.slr + par * WAVES * NB;
        T* sli = S.sli + par * WAVES * NB;
        T* rar = S.rAr + par * NB;
        T* rai = S.rAi + par * NB;
        // A: wave candidate
        double best = -1.0;
        int brow = 0x7fffffff;
        if (q == qj) {
#pragma unroll
          for (int s = 0; s < RT; ++s) {
            const int t = w + WAVES * s;
            if (t < ntiles && 16 * t + 15 >= pj) {
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const int p = 16 * t + M::m(g, i);
                const double m = (double)fabs(xr[s][cj][i]) + (double)fabs(xi[s][cj][i]);
                if (p >= pj && m > best) { best = m; brow = p; }
              }
            }
          }
        }
        double wbest = readlane_d(best, qj);
        int wrow = __builtin_amdgcn_readlane(brow, qj);
#pragma unroll
        for (int gg = 1; gg < 4; ++gg) {
          const double m = readlane_d(best, qj + 16 * gg);
          const int rr = __builtin_amdgcn_readlane(brow, qj + 16 * gg);
          if (m > wbest || (m == wbest && rr < wrow)) { wbest = m; wrow = rr; }
        }
        if (lane == 0) { S.cmag[par * WAVES + w] = wbest; S.crowi[par * WAVES + w] = wrow; }
#pragma unroll
        for (int s = 0; s < RT; ++s) {
          const int t = w + WAVES * s;
          if (t < ntiles && 16 * t + 15 >= pj) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int p = 16 * t + M::m(g, i);
              if (p == wrow) {
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) {
                  slr[w * NB + 16 * ct + q] = xr[s][ct][i];
                  sli[w * NB + 16 * ct + q] = xi[s][ct][i];
                }
              }
              if (p == pj) {
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) {
                  rar[16 * ct + q] = xr[s][ct][i];
                  rai[16 * ct + q] = xi[s][ct][i];
                }
              }
            }
          }
        }
        __syncthreads();
        // B: the winner and its row
        double bm = -1.0;
        int piv = 0x7fffffff, wwin = 0;
#pragma unroll
        for (int ww = 0; ww < WAVES; ++ww) {
          const double m = S.cmag[par * WAVES + ww];
          const int rr = S.crowi[par * WAVES + ww];
          if (m > bm || (m == bm && rr < piv)) { bm = m; piv = rr; wwin = ww; }
        }
        const T* pvr_s = slr + wwin * NB;
        const T* pvi_s = sli + wwin * NB;
        if (piv >= Np) {   // no comparable entry (NaN column): keep row pj
          piv = pj;
          pvr_s = rar;
          pvi_s = rai;
        }
        T prr[CT], pri[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) { prr[ct] = pvr_s[16 * ct + q]; pri[ct] = pvi_s[16 * ct + q]; }
        const double pvr = pvr_s[j], pvi = pvi_s[j];
        const double rden = 1.0 / (pvr * pvr + pvi * pvi);
        const T ivr = T(pvr * rden), ivi = T(-pvi * rden);
        // C: swap; multipliers below the pivot (owner lanes of column j)
#pragma unroll
        for (int s = 0; s < RT; ++s) {
          const int t = w + WAVES * s;
          if (t < ntiles && 16 * t + 15 >= pj) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int p = 16 * t + M::m(g, i);
              if (piv != pj && p == pj) {
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) { xr[s][ct][i] = prr[ct]; xi[s][ct][i] = pri[ct]; }
              } else if (piv != pj && p == piv) {
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) {
                  xr[s][ct][i] = rar[16 * ct + q];
                  xi[s][ct][i] = rai[16 * ct + q];
                }
              }
              if (q == qj && p > pj) {
                const T ar = xr[s][cj][i], ai = xi[s][cj][i];
                const T lr = ar * ivr - ai * ivi;
                const T li = ar * ivi + ai * ivr;
                xr[s][cj][i] = lr;
                xi[s][cj][i] = li;
                S.mr[p] = lr;
                S.mi[p] = li;
              }
            }
          }
        }
        if (tid == 0) {
          if (piv != pj) {
            const int tp = S.perm[pj];
            S.perm[pj] = S.perm[piv];
            S.perm[piv] = tp;
          }
        }
        if (tid >= j && tid < NB) umax = fmax(umax, (double)fabs(pvr_s[tid]) + (double)fabs(pvi_s[tid]));
        // the multipliers of this wave's rows were written by this wave
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // D: rank-1 update of the columns right of j, rows below pj
#pragma unroll
        for (int s = 0; s < RT; ++s) {
          const int t = w + WAVES * s;
          if (t < ntiles && 16 * t + 15 > pj) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int p = 16 * t + M::m(g, i);
              if (p > pj) {
                const T lr = S.mr[p], li = S.mi[p];
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) {
                  if (16 * ct + q > j) {
                    xr[s][ct][i] -= lr * prr[ct] - li * pri[ct];
                    xi[s][ct][i] -= lr * pri[ct] + li * prr[ct];
                  }
                }
              }
            }
          }
        }
      }
    }

    // ---- 4. diagonal block to LDS (inverted after the store, when the
    //         block column registers are free)
#pragma unroll
    for (int s = 0; s < RT; ++s) {
      const int t = w + WAVES * s;
      if (t >= (c0 >> 4) && t < ((c0 + NB) >> 4)) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int pr = 16 * t + M::m(g, i) - c0;
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            S.xsr[pr * LD(NB) + 16 * ct + q] = xr[s][ct][i];
            S.xsi[pr * LD(NB) + 16 * ct + q] = xi[s][ct][i];
          }
        }
      }
    }
    // ---- 5. store rows >= c0 of block column J at the original rows -------
#pragma unroll
    for (int s = 0; s < RT; ++s) {
      const int t = w + WAVES * s;
      if (t < ntiles && 16 * t >= c0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = S.perm[16 * t + M::m(g, i)];
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            Fr[(size_t)r * Np + c0 + 16 * ct + q] = xr[s][ct][i];
            Fi[(size_t)r * Np + c0 + 16 * ct + q] = xi[s][ct][i];
          }
        }
      }
    }
    }
    // ---- 6. inverses of the diagonal blocks L_JJ (unit) and U_JJ --------
    __syncthreads();
    block_tri_inverses<T, NB, NT>(S.xsr, S.xsi, S.lsr, S.lsi, S.unr, S.uni,
                               S.tr_, S.ti_, tid);
    {
      T* Lr = Tb + (size_t)(J * 4 + 0) * NB * NB;
      T* Li = Lr + NB * NB;
      T* Ur = Li + NB * NB;
      T* Ui = Ur + NB * NB;
      for (int e = tid; e < NB * NB; e += NT) {
        const int rr = e / NB, cc = e % NB;
        Lr[e] = S.lsr[rr * LD(NB) + cc];
        Li[e] = S.lsi[rr * LD(NB) + cc];
        Ur[e] = S.unr[rr * LD(NB) + cc];
        Ui[e] = S.uni[rr * LD(NB) + cc];
      }
    }

    __syncthreads();
  }

  for (int p = tid; p < Np; p += NT) perm_out[(size_t)b * Np + p] = S.perm[p];
  // ln|det A| = sum_p ln|u_pp|, u_pp stored at row perm[p]; per-thread
  // strided partial sums, then a fixed-order combination
  for (int p = tid; p < Np; p += NT) {
    const size_t e = (size_t)S.perm[p] * Np + p;
    lsum += log(hypot((double)Fr[e], (double)Fi[e]));
  }
  // growth = max|u| / max|a| over the block
  for (int off = 32; off >= 1; off >>= 1) {
    umax = fmax(umax, __shfl_xor(umax, off));
    amax = fmax(amax, __shfl_xor(amax, off));
  }
  __syncthreads();
  if (lane == 0) { S.cmag[w] = umax; S.cmag[WAVES + w] = amax; }
  S.red[tid] = lsum;
  __syncthreads();
  if (tid == 0) {
    double u = 0.0, a = 0.0, l = 0.0;
    for (int ww = 0; ww < WAVES; ++ww) { u = fmax(u, S.cmag[ww]); a = fmax(a, S.cmag[WAVES + ww]); }
    for (int k = 0; k < NT; ++k) l += S.red[k];
    growth[b] = u / a;
    lad[b] = l;
  }
}

// --------------------------------------------------------------------------
// W = U^-1 (which == 0) or V = L^-1 (which == 1), in place in F.
//   W[:, J] = -(sum_{I<J} W[:, I] U[I, J]) U_JJ^-1  for rows above block J
//   V[:, J] = -(sum_{K>J} V[:, K] L[K, J]) L_JJ^-1  for rows below block J
// Each step forms Y = U[I,J] U_JJ^-1 (or L[K,J] L_JJ^-1) in LDS, then the
// waves accumulate their row tiles with the f64 MFMA.  W[a][k] lives where
// U[a][k] was (row perm[a]), V[r][k] where L[r][k] was.
template <typename T>
size_t trtri_lds_bytes(int Np, int NB) {
  return sizeof(int) * Np + sizeof(T) * 6 * NB * (NB + 1) + 64;
}

template <typename T, int WAVES, int RT, int CT, int OCC = 1>
__global__ void __launch_bounds__(WAVES * 64, OCC * WAVES / 4)
trtri_kernel(int Np, T* __restrict__ F, const int* __restrict__ perm_g,
             const T* __restrict__ tri, const int* __restrict__ only,
             int want) {
  typedef Mma<T> M;
  typedef typename M::v4 V4;
  constexpr int NB = 16 * CT;
  constexpr int NT = WAVES * 64;
  constexpr int KPL = NB / 4;
  extern __shared__ double lds_raw[];
  const int b = blockIdx.x;
  if (only && only[b] != want) return;   // matrix not selected
  const int upper = (blockIdx.y == 0);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = lane >> 4, q = lane & 15;
  const int ntiles = Np >> 4;
  const int nblk = Np / NB;
  T* xsr = reinterpret_cast<T*>(lds_raw);   // block of U or L
  T* xsi = xsr + NB * LD(NB);
  T* dir = xsi + NB * LD(NB);       // U_JJ^-1 or L_JJ^-1
  T* dii = dir + NB * LD(NB);
  T* yr_s = dii + NB * LD(NB);      // Y
  T* yi_s = yr_s + NB * LD(NB);
  int* perm = reinterpret_cast<int*>(yi_s + NB * LD(NB));
  const size_t plane = (size_t)Np * Np;
  T* Fr = F + (size_t)b * 2 * plane;
  T* Fi = Fr + plane;
  const T* Tb = tri + (size_t)b * nblk * 4 * NB * NB;
  for (int p = tid; p < Np; p += NT) perm[p] = perm_g[(size_t)b * Np + p];

  for (int jj = 0; jj < nblk; ++jj) {
    const int J = upper ? jj : nblk - 1 - jj;
    const int c0 = J * NB;
    __syncthreads();
    {
      const T* Dr = Tb + (size_t)(J * 4 + (upper ? 2 : 0)) * NB * NB;
      const T* Di = Dr + NB * NB;
      for (int e = tid; e < NB * NB; e += NT) {
        dir[(e / NB) * LD(NB) + e % NB] = Dr[e];
        dii[(e / NB) * LD(NB) + e % NB] = Di[e];
      }
    }
    V4 ar_[RT][CT], ai_[RT][CT];
#pragma unroll
    for (int s = 0; s < RT; ++s)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        ar_[s][ct] = (V4){T(0), T(0), T(0), T(0)};
        ai_[s][ct] = (V4){T(0), T(0), T(0), T(0)};
      }
    const int nsteps = upper ? J : nblk - 1 - J;
    // Loads run ahead of their use: the block X of the next step is fetched
    // during this step's products, and the A operand of each row tile in two
    // halves (k < KPL/2, k >= KPL/2), each half fetched while the previous
    // half's products run.  The active row tiles of a step form a range of
    // s (the triangle's reach), so the next half is known.
    constexpr int XE = (NB * NB + NT - 1) / NT;   // block-X elements per thread
    constexpr int KH = KPL / 2;
    T xbr[XE], xbi[XE];
    T abr[2][KH], abi[2][KH];
    auto step_I = [&](int st) { return upper ? st : J + 1 + st; };
    auto load_x = [&](int I) {
      const int r0 = I * NB;
#pragma unroll
      for (int u = 0; u < XE; ++u) {
        const int e = tid + u * NT;
        if (e < NB * NB) {
          const int orow = perm[r0 + e / NB];
          xbr[u] = Fr[(size_t)orow * Np + c0 + e % NB];
          xbi[u] = Fi[(size_t)orow * Np + c0 + e % NB];
        }
      }
    };
    // tile range [slo, shi) of the rows a step reaches
    auto tile_range = [&](int I, int& slo, int& shi) {
      const int r0 = I * NB;
      int tlo, thi;   // active t in [tlo, thi)
      if (upper) { tlo = 0; thi = min(c0 >> 4, (r0 + NB + 15) >> 4); }
      else { tlo = max((c0 + NB) >> 4, r0 >> 4); thi = ntiles; }
      // s with tlo <= w + WAVES s < thi
      slo = tlo > w ? (tlo - w + WAVES - 1) / WAVES : 0;
      shi = thi > w ? (thi - w + WAVES - 1) / WAVES : 0;
      if (shi > RT) shi = RT;
    };
    auto load_a = [&](int I, int s, int h) {
      const int r0 = I * NB;
      const int t = w + WAVES * s;
      const int arow = 16 * t + q;
      const int orow = perm[arow];
      const T* pa_r = Fr + (size_t)orow * Np + r0 + KPL * g + KH * h;
      const T* pa_i = Fi + (size_t)orow * Np + r0 + KPL * g + KH * h;
#pragma unroll
      for (int k = 0; k < KH; ++k) {
        const int col = r0 + KPL * g + KH * h + k;
        T vr = pa_r[k], vi = pa_i[k];
        if (upper) {
          if (col < arow) { vr = T(0); vi = T(0); }
        } else {
          if (col > arow) { vr = T(0); vi = T(0); }
          else if (col == arow) { vr = T(1); vi = T(0); }
        }
        abr[h][k] = vr; abi[h][k] = vi;
      }
    };
    if (nsteps > 0) load_x(step_I(0));
    for (int st = 0; st < nsteps; ++st) {
      const int I = step_I(st);
      int slo, shi;
      tile_range(I, slo, shi);
      if (slo < shi) load_a(I, slo, 0);   // first half, ahead of the Y products
      // xs was last read by the previous step's Y products, which ended at
      // that step's second barrier: no barrier is needed before writing it
#pragma unroll
      for (int u = 0; u < XE; ++u) {
        const int e = tid + u * NT;
        if (e < NB * NB) {
          xsr[(e / NB) * LD(NB) + e % NB] = xbr[u];
          xsi[(e / NB) * LD(NB) + e % NB] = xbi[u];
        }
      }
      __syncthreads();
      // Y = X_blk * D  (D = U_JJ^-1 or L_JJ^-1)
      for (int task = w; task < 2 * CT * CT; task += WAVES) {
        const int rt = task / (2 * CT), ct = (task >> 1) % CT, part = task & 1;
        V4 acc = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int ks = 0; ks < NB / 4; ++ks) {
          const int k = 4 * ks + g;
          const T a_r = xsr[(16 * rt + q) * LD(NB) + k];
          const T a_i = xsi[(16 * rt + q) * LD(NB) + k];
          const T b_r = dir[k * LD(NB) + 16 * ct + q];
          const T b_i = dii[k * LD(NB) + 16 * ct + q];
          if (part == 0) { acc = M::mma(a_r, b_r, acc); acc = M::mma(-a_i, b_i, acc); }
          else { acc = M::mma(a_r, b_i, acc); acc = M::mma(a_i, b_r, acc); }
        }
        T* dst = part ? yi_s : yr_s;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          dst[(16 * rt + M::m(g, i)) * LD(NB) + 16 * ct + q] = acc[i];
      }
      __syncthreads();
      if (st + 1 < nsteps) load_x(step_I(st + 1));
      // acc[rows] += Tri[rows, I-cols] * Y, rows in the triangle's reach
#pragma unroll
      for (int s = 0; s < RT; ++s) {
        if (s >= slo && s < shi) {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            // fetch the next half while this one's products run
            if (h == 0) load_a(I, s, 1);
            else if (s + 1 < shi) load_a(I, s + 1, 0);
#pragma unroll
            for (int kk = 0; kk < KH; ++kk) {
              const int k = KPL * g + KH * h + kk;
#pragma unroll
              for (int ct = 0; ct < CT; ++ct) {
                const T b_r = yr_s[k * LD(NB) + 16 * ct + q];
                const T b_i = yi_s[k * LD(NB) + 16 * ct + q];
                ar_[s][ct] = M::mma(abr[h][kk], b_r, ar_[s][ct]);
                ar_[s][ct] = M::mma(-abi[h][kk], b_i, ar_[s][ct]);
                ai_[s][ct] = M::mma(abr[h][kk], b_i, ai_[s][ct]);
                ai_[s][ct] = M::mma(abi[h][kk], b_r, ai_[s][ct]);
              }
            }
            __builtin_amdgcn_sched_barrier(0);
          }
        }
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
          const int orow = perm[16 * t + M::m(g, i)];
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

template <typename T>
__global__ void __launch_bounds__(256)
diagdot_kernel(int N, int Np, const T* __restrict__ F,
               const int* __restrict__ perm_g, double* __restrict__ dg,
               const int* __restrict__ only, int want) {
  const int j0 = blockIdx.x * kDD;
  const int b = blockIdx.y;
  if (only && only[b] != want) return;   // matrix not selected
  const int tid = threadIdx.x;
  __shared__ double wr[kDD][kDD + 1], wi[kDD][kDD + 1];   // [j][s]
  __shared__ double vr[kDD][kDD + 1], vi[kDD][kDD + 1];   // [s][j]
  __shared__ int wrow[kDD], lo[kDD];
  __shared__ double pr_s[kDDParts][kDD], pi_s[kDDParts][kDD];
  const size_t plane = (size_t)Np * Np;
  const T* Fr = F + (size_t)b * 2 * plane;
  const T* Fi = Fr + plane;
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
  constexpr int EPT = kDD * kDD / 256;     // tile elements per thread
  double accr = 0.0, acci = 0.0;
  // the tiles of the next s0 are loaded into registers while the current
  // ones are multiplied from LDS
  double xr_[EPT], xi_[EPT], yr_[EPT], yi_[EPT];
  auto load = [&](int s0) {
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = tid + 256 * u;
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
      xr_[u] = x_r; xi_[u] = x_i; yr_[u] = y_r; yi_[u] = y_i;
    }
  };
  __syncthreads();                         // wrow, lo
  load(j0);
  for (int s0 = j0; s0 < Np; s0 += kDD) {
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = tid + 256 * u;
      const int a = e / kDD, c = e % kDD;
      wr[a][c] = xr_[u]; wi[a][c] = xi_[u];
      vr[a][c] = yr_[u]; vi[a][c] = yi_[u];
    }
    __syncthreads();
    if (s0 + kDD < Np) load(s0 + kDD);
    const int j = j0 + jl;
    const int first = lo[jl];
#pragma unroll
    for (int k = 0; k < SPP; ++k) {
      const int sl = part * SPP + k;
      const int s = s0 + sl;
      if (s >= first && s < Np) {
        double yr = vr[sl][jl], yi = vi[sl][jl];
        if (s == j) { yr = 1.0; yi = 0.0; }
        const double x_r = wr[jl][sl], x_i = wi[jl][sl];
        accr += x_r * yr - x_i * yi;
        acci += x_r * yi + x_i * yr;
      }
    }
    __syncthreads();                       // the tiles are rewritten next
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

template <typename T, int WAVES, int RT, int CT, bool kRP = false, int OCC = 1>
hipError_t run_lu(const MatDesc* descs, const double* hbuf, int B, int N,
                  int Np, int L, T* F, int* perm, T* tri, double* lad,
                  double* growth, hipStream_t st, const int* only = nullptr,
                  int want = 0) {
  const size_t lds = lu_lds_bytes<T>(Np, 16 * CT, WAVES, kRP);
  auto kern = lu_kernel<T, WAVES, RT, CT, kRP, OCC>;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  const int cls = only ? K_FALLBACK : K_LU;
  mark_begin(cls, st);
  hipLaunchKernelGGL(kern, dim3(B), dim3(WAVES * 64), lds, st, descs, hbuf, N,
                     Np, L, F, perm, tri, lad, growth, only, want);
  mark_end(cls, st);
  return hipGetLastError();
}

// both: W = U^-1 and V = L^-1 (grid y = 2); otherwise only W.
template <typename T, int WAVES, int RT, int CT, int OCC = 1>
hipError_t run_trtri(int B, int Np, T* F, const int* perm, const T* tri,
                     hipStream_t st, bool both = true,
                     const int* only = nullptr, int want = 0) {
  const size_t lds = trtri_lds_bytes<T>(Np, 16 * CT);
  const int cls = !both ? K_TRTRI_SYM : only ? K_FALLBACK : K_TRTRI;
  mark_begin(cls, st);
  hipLaunchKernelGGL((trtri_kernel<T, WAVES, RT, CT, OCC>), dim3(B, both ? 2 : 1),
                     dim3(WAVES * 64), lds, st, Np, F, perm, tri, only, want);
  mark_end(cls, st);
  return hipGetLastError();
}

template <typename T>
hipError_t run_diagdot(int B, int N, int Np, const T* F, const int* perm,
                       double* dg, hipStream_t st, const int* only = nullptr,
                       int want = 0) {
  const int cls = only ? K_FALLBACK : K_DIAGDOT;
  mark_begin(cls, st);
  hipLaunchKernelGGL(diagdot_kernel<T>, dim3((Np + kDD - 1) / kDD, B),
                     dim3(256), 0, st, N, Np, F, perm, dg, only, want);
  mark_end(cls, st);
  return hipGetLastError();
}

}  // namespace

BlockedPlan blocked_plan(int N, bool fp32) {
  // Row tiles of 16 per wave; the block column (Np rows x NB) lives in MFMA
  // accumulators.  FP64: 4 waves x 4 tiles (Np <= 256), 8 x 4 (Np <= 512)
  // with NB = 32, then NB = 16 up to Np = 1024.  FP32 (half the registers):
  // the same up to 512, NB = 32 on 8 x 8 tiles up to 1024, NB = 16 on
  // 8 x 18 tiles up to 2304; Np is a multiple of 32.  FP32 with
  // 256 < Np <= 448 (cfg 4) runs the 8 x 4 LU and inverts with 4 waves x 7
  // tiles, two workgroups per CU (4.70 against 5.06 ms at Np = 416, as
  // measured; the LU as 4 x 7 at two per CU was slower, 8.2 against 6.0).
  BlockedPlan p{};
  p.cfg = -1;
  if (!fp32) {
    const int n32 = (N + 31) / 32 * 32, n16 = (N + 15) / 16 * 16;
    if (n32 <= 256) { p.cfg = 0; p.NB = 32; p.Np = n32; }
    else if (n32 <= 512) { p.cfg = 1; p.NB = 32; p.Np = n32; }
    else if (n16 <= 1024) { p.cfg = 2; p.NB = 16; p.Np = n16; }
  } else {
    const int n32 = (N + 31) / 32 * 32;
    if (n32 <= 256) { p.cfg = 0; p.NB = 32; p.Np = n32; }
    else if (n32 <= 448) { p.cfg = 4; p.NB = 32; p.Np = n32; }
    else if (n32 <= 512) { p.cfg = 1; p.NB = 32; p.Np = n32; }
    else if (n32 <= 1024) { p.cfg = 2; p.NB = 32; p.Np = n32; }
    else if (n32 <= 2304) { p.cfg = 3; p.NB = 16; p.Np = n32; }
  }
  if (p.cfg < 0) { p.NB = 0; p.Np = 0; }
  return p;
}

BlockedPlan blocked_plan_f64(int N) { return blocked_plan(N, false); }

hipError_t blocked_lu_f64(const BlockedPlan& p, const MatDesc* descs,
                          const double* hbuf, int B, int N, int L, double* F,
                          int* perm, double* tri, double* lad, double* growth,
                          hipStream_t st, const int* only, int want) {
  switch (p.cfg) {
    case 0: return run_lu<double, 4, 4, 2>(descs, hbuf, B, N, p.Np, L, F, perm, tri, lad, growth, st, only, want);
    case 1: return run_lu<double, 8, 4, 2, true>(descs, hbuf, B, N, p.Np, L, F, perm, tri, lad, growth, st, only, want);
    case 2: return run_lu<double, 16, 4, 1>(descs, hbuf, B, N, p.Np, L, F, perm, tri, lad, growth, st, only, want);
    default: return hipErrorInvalidValue;
  }
}

hipError_t blocked_inv_f64(const BlockedPlan& p, int B, int N, double* F,
                           const int* perm, const double* tri, double* dg,
                           hipStream_t st, const int* only, int want) {
  hipError_t e;
  switch (p.cfg) {
    case 0: e = run_trtri<double, 4, 4, 2>(B, p.Np, F, perm, tri, st, true, only, want); break;
    case 1: e = run_trtri<double, 8, 4, 2>(B, p.Np, F, perm, tri, st, true, only, want); break;
    case 2: e = run_trtri<double, 8, 8, 1>(B, p.Np, F, perm, tri, st, true, only, want); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  return run_diagdot<double>(B, N, p.Np, F, perm, dg, st, only, want);
}

hipError_t blocked_trtri_upper_f64(const BlockedPlan& p, int B, double* F,
                                   const int* perm, const double* tri,
                                   hipStream_t st, const int* only, int want) {
  switch (p.cfg) {
    case 0: return run_trtri<double, 4, 4, 2>(B, p.Np, F, perm, tri, st, false, only, want);
    case 1: return run_trtri<double, 8, 4, 2>(B, p.Np, F, perm, tri, st, false, only, want);
    case 2: return run_trtri<double, 8, 8, 1>(B, p.Np, F, perm, tri, st, false, only, want);
    default: return hipErrorInvalidValue;
  }
}

hipError_t blocked_lu_f32(const BlockedPlan& p, const MatDesc* descs,
                          const double* hbuf, int B, int N, int L, float* F,
                          int* perm, float* tri, double* lad, double* growth,
                          hipStream_t st) {
  switch (p.cfg) {
    case 0: return run_lu<float, 4, 4, 2>(descs, hbuf, B, N, p.Np, L, F, perm, tri, lad, growth, st);
    case 1: return run_lu<float, 8, 4, 2, true>(descs, hbuf, B, N, p.Np, L, F, perm, tri, lad, growth, st);
    case 2: return run_lu<float, 8, 8, 2>(descs, hbuf, B, N, p.Np, L, F, perm, tri, lad, growth, st);
    case 3: return run_lu<float, 8, 18, 1>(descs, hbuf, B, N, p.Np, L, F, perm, tri, lad, growth, st);
    case 4: return run_lu<float, 8, 4, 2, true>(descs, hbuf, B, N, p.Np, L, F, perm, tri, lad, growth, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t blocked_trtri_f32(const BlockedPlan& p, int B, float* F,
                             const int* perm, const float* tri,
                             hipStream_t st) {
  switch (p.cfg) {
    case 0: return run_trtri<float, 4, 4, 2>(B, p.Np, F, perm, tri, st);
    case 1: return run_trtri<float, 8, 4, 2>(B, p.Np, F, perm, tri, st);
    case 2: return run_trtri<float, 8, 8, 2>(B, p.Np, F, perm, tri, st);
    case 3: return run_trtri<float, 8, 18, 1>(B, p.Np, F, perm, tri, st);
    case 4: return run_trtri<float, 4, 7, 2, 2>(B, p.Np, F, perm, tri, st);
    default: return hipErrorInvalidValue;
  }
}

size_t blocked_factor_bytes(const BlockedPlan& p, int B, size_t elem) {
  const size_t Np = p.Np, NB = p.NB;
  const size_t F = 2 * Np * Np * elem;
  const size_t perm = Np * sizeof(int);
  const size_t tri = (Np / NB) * 4 * NB * NB * elem;
  return (size_t)B * (F + perm + tri) + 3 * 256;
}

size_t blocked_factor_bytes_f64(const BlockedPlan& p, int B) {
  return blocked_factor_bytes(p, B, sizeof(double));
}

}  // namespace sca
