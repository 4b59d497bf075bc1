// Fused small-matrix path: one workgroup factors one A_b = z_b I - H_b held
// entirely in LDS (N <= 64), then forms ln|det A_b| and diag(A_b^-1).
//
//   P A = L U            unblocked, partial pivoting (max |Re|+|Im|, lowest
//                        row on ties)
//   ln|det A| = sum_k ln|u_kk|
//   A^-1 = W V P,  W = U^-1, V = L^-1   =>   (A^-1)_ii = sum_k W_ik V_k,pos(i)
//
// where pos(i) is the position row i of A was pivoted to.  W and V overwrite
// U and L in place, one row per barrier step (W from the bottom, V from the
// top, in the same sweep).  This path serves the 4x4 .. 8x8 lattices; its
// cost is latency (barriers), not flops.
#include "sca_common.h"
#include "sca_kernels.h"
#include "sca_profile.h"

namespace sca {

template <int NMAX>
__device__ inline int lidx(int r, int c) { return r * (NMAX + 1) + c; }

__device__ inline void argmax_wave(double& mag, int& row) {
  for (int off = 32; off >= 1; off >>= 1) {
    double om = __shfl_xor(mag, off);
    int orow = __shfl_xor(row, off);
    if (om > mag || (om == mag && orow < row)) { mag = om; row = orow; }
  }
}

template <int NMAX, int NT>
__global__ void __launch_bounds__(NT)
small_factor_kernel(const MatDesc* __restrict__ descs,
                    const double* __restrict__ hbuf, int N, int L,
                    double* __restrict__ lad, double* __restrict__ dg,
                    double* __restrict__ growth) {
  __shared__ double ar[NMAX * (NMAX + 1)];
  __shared__ double ai[NMAX * (NMAX + 1)];
  __shared__ int perm[NMAX];
  __shared__ int posv[NMAX];
  __shared__ int piv_s;
  __shared__ double red[NT / 64];

  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const MatDesc d = descs[b];
  const double* h = hbuf + d.hoff;

  // assemble A = z I - H = z I + t K - diag(h); track max |a| (|Re|+|Im|)
  double amax = 0.0;
  for (int e = tid; e < N * N; e += NT) {
    int r = e / N, c = e % N;
    double re, im;
    if (r == c) { re = d.zr - h[r]; im = d.zi; }
    else { re = d.t * (double)kmult(r, c, L); im = 0.0; }
    ar[lidx<NMAX>(r, c)] = re;
    ai[lidx<NMAX>(r, c)] = im;
    amax = fmax(amax, fabs(re) + fabs(im));
  }
  if (tid < N) perm[tid] = tid;
  __syncthreads();

  double umax = 0.0;  // max |u| over the U factor, for the growth factor
  for (int k = 0; k < N; ++k) {
    if (tid < 64) {
      double mag = -1.0;
      int row = 0x7fffffff;
      for (int r = k + tid; r < N; r += 64) {
        double m = fabs(ar[lidx<NMAX>(r, k)]) + fabs(ai[lidx<NMAX>(r, k)]);
        if (m > mag || (m == mag && r < row)) { mag = m; row = r; }
      }
      argmax_wave(mag, row);
      // a column with no comparable entry (all NaN) keeps the diagonal
      // row; the NaN then reaches ln|det| and is reported as non-finite
      if (row >= N) row = k;
      if (tid == 0) {
        piv_s = row;
        int tp = perm[k]; perm[k] = perm[row]; perm[row] = tp;
      }
    }
    __syncthreads();
    const int p = piv_s;
    if (p != k) {
      for (int c = tid; c < N; c += NT) {
        double tr = ar[lidx<NMAX>(k, c)], ti = ai[lidx<NMAX>(k, c)];
        ar[lidx<NMAX>(k, c)] = ar[lidx<NMAX>(p, c)];
        ai[lidx<NMAX>(k, c)] = ai[lidx<NMAX>(p, c)];
        ar[lidx<NMAX>(p, c)] = tr;
        ai[lidx<NMAX>(p, c)] = ti;
      }
    }
    __syncthreads();
    const double pr = ar[lidx<NMAX>(k, k)], pi = ai[lidx<NMAX>(k, k)];
    const double den = pr * pr + pi * pi;
    const double ir = pr / den, ii = -pi / den;   // 1 / pivot
    for (int r = k + 1 + tid; r < N; r += NT) {
      double xr = ar[lidx<NMAX>(r, k)], xi = ai[lidx<NMAX>(r, k)];
      ar[lidx<NMAX>(r, k)] = xr * ir - xi * ii;
      ai[lidx<NMAX>(r, k)] = xr * ii + xi * ir;
    }
    for (int c = k + tid; c < N; c += NT)
      umax = fmax(umax, fabs(ar[lidx<NMAX>(k, c)]) + fabs(ai[lidx<NMAX>(k, c)]));
    __syncthreads();
    const int m = N - k - 1;
    for (int e = tid; e < m * m; e += NT) {
      int r = k + 1 + e / m, c = k + 1 + e % m;
      double lr = ar[lidx<NMAX>(r, k)], li = ai[lidx<NMAX>(r, k)];
      double ur = ar[lidx<NMAX>(k, c)], ui = ai[lidx<NMAX>(k, c)];
      ar[lidx<NMAX>(r, c)] -= lr * ur - li * ui;
      ai[lidx<NMAX>(r, c)] -= lr * ui + li * ur;
    }
    __syncthreads();
  }

  // ln|det| (fixed order, one lane) and the pivot growth factor
  if (tid == 0) {
    double s = 0.0;
    for (int k = 0; k < N; ++k)
      s += log(hypot(ar[lidx<NMAX>(k, k)], ai[lidx<NMAX>(k, k)]));
    lad[b] = s;
  }
  for (int off = 32; off >= 1; off >>= 1) umax = fmax(umax, __shfl_xor(umax, off));
  for (int off = 32; off >= 1; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off));
  if ((tid & 63) == 0) red[tid >> 6] = umax / amax;
  if (tid < N) posv[perm[tid]] = tid;
  __syncthreads();
  if (tid == 0) {
    double g = 0.0;
    for (int w = 0; w < NT / 64; ++w) g = fmax(g, red[w]);
    growth[b] = g;
  }

  // W = U^-1 (rows from the bottom) and V = L^-1 (rows from the top), one
  // row of each per step; lanes [0, HALF) own a W column, [HALF, 2 HALF) a
  // V column (N <= HALF).  W lives on/above the diagonal, V below it.
  constexpr int HALF = (NT == 64) ? 32 : 64;
  for (int s = 0; s < N; ++s) {
    const int iw = N - 1 - s;   // W row
    const int iv = s;           // V row
    double xr = 0.0, xi = 0.0;
    const bool wlane = tid < HALF && tid >= iw && tid < N;
    const int jv = tid - HALF;
    const bool vlane = tid >= HALF && tid < 2 * HALF && jv < iv;
    if (wlane) {
      // W[iw][j] = (delta_ij - sum_{k=iw+1}^{j} U[iw][k] W[k][j]) / U[iw][iw]
      const int j = tid;
      double sr = (j == iw) ? 1.0 : 0.0, si = 0.0;
      for (int k = iw + 1; k <= j; ++k) {
        double ur = ar[lidx<NMAX>(iw, k)], ui = ai[lidx<NMAX>(iw, k)];
        double wr = ar[lidx<NMAX>(k, j)], wi = ai[lidx<NMAX>(k, j)];
        sr -= ur * wr - ui * wi;
        si -= ur * wi + ui * wr;
      }
      double pr = ar[lidx<NMAX>(iw, iw)], pi = ai[lidx<NMAX>(iw, iw)];
      double den = pr * pr + pi * pi;
      xr = (sr * pr + si * pi) / den;
      xi = (si * pr - sr * pi) / den;
    } else if (vlane) {
      // V[iv][j] = -(L[iv][j] + sum_{k=j+1}^{iv-1} L[iv][k] V[k][j])
      const int j = jv;
      double sr = ar[lidx<NMAX>(iv, j)], si = ai[lidx<NMAX>(iv, j)];
      for (int k = j + 1; k < iv; ++k) {
        double lr = ar[lidx<NMAX>(iv, k)], li = ai[lidx<NMAX>(iv, k)];
        double vr = ar[lidx<NMAX>(k, j)], vi = ai[lidx<NMAX>(k, j)];
        sr += lr * vr - li * vi;
        si += lr * vi + li * vr;
      }
      xr = -sr; xi = -si;
    }
    __syncthreads();
    if (wlane) { ar[lidx<NMAX>(iw, tid)] = xr; ai[lidx<NMAX>(iw, tid)] = xi; }
    if (vlane) { ar[lidx<NMAX>(iv, jv)] = xr; ai[lidx<NMAX>(iv, jv)] = xi; }
    __syncthreads();
  }

  // (A^-1)_ii = sum_{k >= max(i, pos(i))} W[i][k] V[k][pos(i)], V_kk = 1
  for (int i = tid; i < N; i += NT) {
    const int q = posv[i];
    double sr = 0.0, si = 0.0;
    for (int k = (i > q ? i : q); k < N; ++k) {
      double xr = ar[lidx<NMAX>(i, k)], xi = ai[lidx<NMAX>(i, k)];
      double yr, yi;
      if (k == q) { yr = 1.0; yi = 0.0; }
      else { yr = ar[lidx<NMAX>(k, q)]; yi = ai[lidx<NMAX>(k, q)]; }
      sr += xr * yr - xi * yi;
      si += xr * yi + xi * yr;
    }
    dg[((size_t)b * N + i) * 2 + 0] = sr;
    dg[((size_t)b * N + i) * 2 + 1] = si;
  }
}

hipError_t launch_small_factor(const MatDesc* descs, const double* hbuf, int B,
                               int N, int L, double* lad, double* dg,
                               double* growth, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  struct Mark {
    hipStream_t s;
    explicit Mark(hipStream_t s_) : s(s_) { mark_begin(K_SMALL, s); }
    ~Mark() { mark_end(K_SMALL, s); }
  } mark(st);
  if (N <= 16) {
    hipLaunchKernelGGL((small_factor_kernel<16, 64>), dim3(B), dim3(64), 0, st,
                       descs, hbuf, N, L, lad, dg, growth);
  } else if (N <= 64) {
    hipLaunchKernelGGL((small_factor_kernel<64, 256>), dim3(B), dim3(256), 0, st,
                       descs, hbuf, N, L, lad, dg, growth);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace sca
