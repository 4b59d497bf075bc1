// Matsubara tail by moments: the frequencies w_n >= w_c of a problem are not
// factorised; their ln|det(i w_n - H)| and Re diag((i w_n - H)^-1) come from
// the moments of H (series in sca_common.h).
//
//   moments_kernel    diag(H^p), p = 1 .. kTailP, of both spins: one
//                     workgroup per (site i, spin, problem) applies the
//                     lattice stencil of H to e_i p times (vector in LDS).
//   tail_sums_kernel  per problem: sum_{n=Me}^{M-1} ln w_n and
//                     S_{2m} = sum_{n=Me}^{M-1} w_n^{-2m}, m = 1 .. kTailK+1
//                     (fixed summation order).
//   absmax_kernel     max_i |x_i| of one vector (host-side choice of w_c).
#include <math.h>
#include "sca_common.h"
#include "sca_kernels.h"
#include "sca_profile.h"

namespace sca {

namespace {
constexpr double kPi = 3.14159265358979323846;
constexpr int kMomThreads = 256;
}  // namespace

__global__ void __launch_bounds__(kMomThreads)
moments_kernel(const ProbDesc* __restrict__ probs, int N,
               const double* __restrict__ hbuf, double* __restrict__ mom) {
  const int i = blockIdx.x, sidx = blockIdx.y, p = blockIdx.z;
  const ProbDesc P = probs[p];
  if (P.Me >= P.M) return;   // no tail in this problem
  extern __shared__ double v_s[];   // two vectors of N
  const double* h = hbuf + P.hoff + sidx * N;
  double* out = mom + ((size_t)p * 2 + sidx) * kTailP * N + i;
  const int L = P.L;
  const double t = P.t;
  for (int j = threadIdx.x; j < N; j += kMomThreads) v_s[j] = (j == i) ? 1.0 : 0.0;
  __syncthreads();
  int cur = 0;
  for (int q = 0; q < kTailP; ++q) {
    const double* a = v_s + cur * N;
    double* b = v_s + (1 - cur) * N;
    // (H v)_j = h_j v_j - t sum over the four directions (K_jk counts them)
    for (int j = threadIdx.x; j < N; j += kMomThreads) {
      const int x = j % L, y = j / L;
      const double s = a[(x + 1) % L + L * y] + a[(x + L - 1) % L + L * y] +
                       a[x + L * ((y + 1) % L)] + a[x + L * ((y + L - 1) % L)];
      b[j] = h[j] * a[j] - t * s;
    }
    __syncthreads();
    cur = 1 - cur;
    if (threadIdx.x == 0) out[(size_t)q * N] = v_s[cur * N + i];
  }
}

// One workgroup per problem: thread k takes n = Me + k, Me + k + 256, ..
// (w^-2m by successive products), then a fixed-order tree over the threads.
__global__ void __launch_bounds__(256)
tail_sums_kernel(const ProbDesc* __restrict__ probs,
                 double* __restrict__ tsum) {
  const int p = blockIdx.x, tid = threadIdx.x;
  const ProbDesc P = probs[p];
  if (P.Me >= P.M) return;
  __shared__ double red[kTailS][256];
  double acc[kTailS];
#pragma unroll
  for (int m = 0; m < kTailS; ++m) acc[m] = 0.0;
  for (int n = P.Me + tid; n < P.M; n += 256) {
    const double w = (2.0 * n + 1.0) * kPi * P.T;
    const double x = 1.0 / (w * w);
    acc[0] += log(w);
    double y = 1.0;
#pragma unroll
    for (int m = 1; m < kTailS; ++m) { y *= x; acc[m] += y; }
  }
#pragma unroll
  for (int m = 0; m < kTailS; ++m) red[m][tid] = acc[m];
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (tid < w)
#pragma unroll
      for (int m = 0; m < kTailS; ++m) red[m][tid] += red[m][tid + w];
    __syncthreads();
  }
  if (tid < kTailS) tsum[(size_t)p * kTailS + tid] = red[tid][0];
}

__global__ void __launch_bounds__(256)
absmax_kernel(const double* __restrict__ x, int n, double* __restrict__ out) {
  __shared__ double r[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) m = max_nan(m, fabs(x[i]));
  r[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) r[threadIdx.x] = max_nan(r[threadIdx.x], r[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = r[0];
}

hipError_t launch_tail(const ProbDesc* probs, int nprob, int N,
                       const double* hbuf, double* mom, double* tsum,
                       hipStream_t st) {
  if (nprob <= 0) return hipSuccess;
  mark_begin(K_TAIL, st);
  hipLaunchKernelGGL(moments_kernel, dim3(N, 2, nprob), dim3(kMomThreads),
                     sizeof(double) * 2 * N, st, probs, N, hbuf, mom);
  hipLaunchKernelGGL(tail_sums_kernel, dim3(nprob), dim3(256), 0, st, probs,
                     tsum);
  mark_end(K_TAIL, st);
  return hipGetLastError();
}

size_t tail_workspace_bytes(int nprob, int N) {
  return sizeof(double) * (size_t)nprob * (2 * (size_t)kTailP * N + kTailS);
}

hipError_t launch_absmax(const double* x, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(absmax_kernel, dim3(1), dim3(256), 0, st, x, n, out);
  return hipGetLastError();
}

}  // namespace sca
