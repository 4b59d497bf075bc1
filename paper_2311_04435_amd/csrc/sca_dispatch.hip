// Factorisation path selection.
//   N <= 64  : fused small kernel (matrix in LDS), FP64 for both precisions
//              (these matrices are too small for the FP32 route to pay).
//   FP64, N <= 1024: blocked LU, then U^-1 / L^-1, then the diagonal.
//   FP32 refined, N <= 2304: blocked complex64 LU and U^-1 / L^-1, the
//              product X = W V, then the FP64 Newton diagonal and the
//              refined log-determinant.
#include "sca_blocked.h"
#include "sca_common.h"
#include "sca_kernels.h"
#include "sca_runtime.h"

namespace sca {

namespace {
constexpr int kSmallMax = 64;
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
}  // namespace

bool path_supported(int N, int precision) {
  if (N < 1) return false;
  if (N <= kSmallMax) return true;
  return blocked_plan(N, precision != 0).cfg >= 0;
}

namespace {

size_t refine_extra_bytes(const BlockedPlan& p, int B) {
  return align256(sizeof(float) * 2 * (size_t)B * p.Np * p.Np)        // X
       + align256(sizeof(double) * (size_t)B * refine_blocks(p.Np));  // parts
}

}  // namespace

size_t factor_workspace_bytes(int N, int B, int precision) {
  if (N <= kSmallMax) return 0;
  const BlockedPlan p = blocked_plan(N, precision != 0);
  if (p.cfg < 0) return 0;
  if (precision == 0) return blocked_factor_bytes(p, B, sizeof(double));
  return blocked_factor_bytes(p, B, sizeof(float)) + refine_extra_bytes(p, B);
}

namespace {

// F (planar re/im factors, B x 2 x Np x Np), perm (B x Np), tri (inverted
// diagonal blocks); the FP32 route adds X (B x 2 x Np x Np) and the
// per-block log-det parts.
template <typename T>
struct BlockedBufs { T* F; int* perm; T* tri; float* X; double* parts; };

template <typename T>
BlockedBufs<T> carve_blocked(void* fact, const BlockedPlan& p, int B) {
  char* c = static_cast<char*>(fact);
  BlockedBufs<T> r{};
  r.F = reinterpret_cast<T*>(c);
  c += align256(sizeof(T) * 2 * (size_t)B * p.Np * p.Np);
  r.perm = reinterpret_cast<int*>(c);
  c += align256(sizeof(int) * (size_t)B * p.Np);
  r.tri = reinterpret_cast<T*>(c);
  c += align256(sizeof(T) * (size_t)B * (p.Np / p.NB) * 4 * p.NB * p.NB);
  r.X = reinterpret_cast<float*>(c);
  c += align256(sizeof(float) * 2 * (size_t)B * p.Np * p.Np);
  r.parts = reinterpret_cast<double*>(c);
  return r;
}

hipError_t fp32r_batch(const BlockedPlan& p, const MatDesc* descs,
                       const double* hbuf, int B, int N, int L, double* lad,
                       double* dg, double* growth, void* fact,
                       hipStream_t st) {
  BlockedBufs<float> bb = carve_blocked<float>(fact, p, B);
  hipError_t e = blocked_lu_f32(p, descs, hbuf, B, N, L, bb.F, bb.perm,
                                bb.tri, lad, growth, st);
  if (e == hipSuccess) e = blocked_trtri_f32(p, B, bb.F, bb.perm, bb.tri, st);
  if (e == hipSuccess) e = launch_wv_gemm(B, p.Np, bb.F, bb.perm, bb.X, st);
  if (e == hipSuccess)
    e = launch_refine(B, N, p.Np, L, descs, hbuf, bb.F, bb.perm, bb.X, dg,
                      bb.parts, lad, st);
  return e;
}

}  // namespace

hipError_t factor_batch(const MatDesc* descs, const double* hbuf, int B, int N,
                        int L, int precision, double* lad, double* dg,
                        double* growth, void* fact, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  if (N <= kSmallMax)
    return launch_small_factor(descs, hbuf, B, N, L, lad, dg, growth, st);
  const BlockedPlan p = blocked_plan(N, precision != 0);
  if (p.cfg < 0) return hipErrorInvalidValue;
  if (precision != 0)
    return fp32r_batch(p, descs, hbuf, B, N, L, lad, dg, growth, fact, st);
  BlockedBufs<double> bb = carve_blocked<double>(fact, p, B);
  hipError_t e = blocked_lu_f64(p, descs, hbuf, B, N, L, bb.F, bb.perm, bb.tri,
                                lad, growth, st);
  if (e != hipSuccess) return e;
  return blocked_inv_f64(p, B, N, bb.F, bb.perm, bb.tri, dg, st);
}

bool factor_backward_consumes(int N, int precision) {
  return N > kSmallMax && precision == 0;
}

size_t autograd_factor_bytes(int N, int B, int precision) {
  size_t bytes = align256(sizeof(FactorHeader))
               + align256(sizeof(double) * (size_t)B)        // lad
               + align256(sizeof(double) * (size_t)B)        // growth
               + align256(sizeof(double) * 2 * (size_t)B * N)  // dg
               + factor_workspace_bytes(N, B, precision);   // LU factors
  return bytes;
}

AutogradLayout autograd_layout(void* base, int N, int B, int precision) {
  (void)precision;
  char* p = static_cast<char*>(base);
  AutogradLayout a;
  a.head = reinterpret_cast<FactorHeader*>(p);
  p += align256(sizeof(FactorHeader));
  a.lad = reinterpret_cast<double*>(p);
  p += align256(sizeof(double) * (size_t)B);
  a.growth = reinterpret_cast<double*>(p);
  p += align256(sizeof(double) * (size_t)B);
  a.dg = reinterpret_cast<double*>(p);
  p += align256(sizeof(double) * 2 * (size_t)B * N);
  a.fact = factor_workspace_bytes(N, B, precision) ? p : nullptr;
  return a;
}

hipError_t factor_forward(const MatDesc* descs, const double* hbuf, int B,
                          int N, int L, int precision, double* lad, double* dg,
                          double* growth, void* fact, hipStream_t st) {
  // the small path forms diag(A^-1) in the same pass as the LU; the FP32
  // route needs W and V for the refined log-determinant, so it completes
  // the diagonal in the forward as well
  if (N <= kSmallMax || precision != 0)
    return factor_batch(descs, hbuf, B, N, L, precision, lad, dg, growth, fact,
                        st);
  const BlockedPlan p = blocked_plan_f64(N);
  if (p.cfg < 0) return hipErrorInvalidValue;
  BlockedBufs<double> bb = carve_blocked<double>(fact, p, B);
  return blocked_lu_f64(p, descs, hbuf, B, N, L, bb.F, bb.perm, bb.tri, lad,
                        growth, st);
}

hipError_t factor_backward(int B, int N, int precision, const double* lad,
                           double* dg, void* fact, hipStream_t st) {
  (void)lad;
  if (N <= kSmallMax || precision != 0) return hipSuccess;   // dg complete
  const BlockedPlan p = blocked_plan_f64(N);
  if (p.cfg < 0) return hipErrorInvalidValue;
  BlockedBufs<double> bb = carve_blocked<double>(fact, p, B);
  return blocked_inv_f64(p, B, N, bb.F, bb.perm, bb.tri, dg, st);
}

__global__ void make_shifts_kernel(const double* __restrict__ w, int n_w,
                                   double eta, double* __restrict__ z) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_w) return;
  z[2 * j] = w[j];
  z[2 * j + 1] = eta;
}

hipError_t launch_make_shifts(const double* w, int n_w, double eta, double* z,
                              hipStream_t st) {
  if (n_w <= 0) return hipSuccess;
  hipLaunchKernelGGL(make_shifts_kernel, dim3((n_w + 255) / 256), dim3(256), 0,
                     st, w, n_w, eta, z);
  return hipGetLastError();
}

hipError_t launch_reduce_omega(ProbDesc* probs, int nprob, int N,
                               const double* lad, const double* growth,
                               ProbStats* stats, void* ws, hipStream_t st) {
  return launch_reduce(probs, nprob, N, lad, nullptr, growth, stats, false, ws,
                       st);
}

}  // namespace sca
