// Factorisation path selection.  `mode` is the route code of
// sca_runtime.h: bit 0 FP32 refined, bit 1 symmetric (unpivoted L D L^T).
//   N <= 64  : fused small kernel (matrix in LDS), FP64 pivoted LU for every
//              mode (these matrices are too small for the other routes to
//              pay).
//   FP64, N <= 1024: blocked LU, then U^-1 / L^-1, then the diagonal.
//   FP64 symmetric, N <= 1024: blocked L D L^T, L^-T, the diagonal; the
//              matrices whose growth check fails are redone by the LU.
//   FP32 refined, N <= 2304: blocked complex64 LU and U^-1 / L^-1, the
//              product X = W V, then the FP64 Newton diagonal and the
//              refined log-determinant.
//   spectral (FP64), any N: one eigendecomposition per h vector, every
//              matrix from the spectrum (k_eig.hip).
#include "sca_blocked.h"
#include "sca_common.h"
#include "sca_kernels.h"
#include "sca_runtime.h"

namespace sca {

namespace {
constexpr int kSmallMax = 64;
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
bool fp32_mode(int mode) { return (mode & kModeFp32) != 0; }
bool sym_mode(int mode) { return (mode & kModeSym) != 0; }
}  // namespace

bool path_supported(int N, int mode) {
  if (mode == kModeEig) return N >= 1;
  if (N < 1 || mode < 0 || mode > 3) return false;
  if (N <= kSmallMax) return true;
  if (fp32_mode(mode) && sym_mode(mode)) return false;
  return blocked_plan(N, fp32_mode(mode)).cfg >= 0;
}

namespace {

size_t refine_extra_bytes(const BlockedPlan& p, int B) {
  return align256(sizeof(float) * 2 * (size_t)B * p.Np * p.Np)        // X
       + align256(sizeof(double) * (size_t)B * refine_parts(p.Np));  // parts
}

size_t sym_extra_bytes(const BlockedPlan& p, int B) {
  return align256(sizeof(double) * 2 * (size_t)B * p.Np)   // 1/d
       + align256(sizeof(int) * (size_t)B);                // fallback flags
}

}  // namespace

size_t factor_workspace_bytes(int N, int B, int mode, int nH) {
  if (mode == kModeEig) return eig_workspace_bytes(N, nH);
  if (N <= kSmallMax) return 0;
  const BlockedPlan p = blocked_plan(N, fp32_mode(mode));
  if (p.cfg < 0) return 0;
  if (fp32_mode(mode))
    return blocked_factor_bytes(p, B, sizeof(float)) + refine_extra_bytes(p, B);
  size_t bytes = blocked_factor_bytes(p, B, sizeof(double));
  if (sym_mode(mode)) bytes += sym_extra_bytes(p, B);
  return bytes;
}

namespace {

// F (planar re/im factors, B x 2 x Np x Np), perm (B x Np), tri (inverted
// diagonal blocks), then the route's extra buffers.
template <typename T>
struct BlockedBufs { T* F; int* perm; T* tri; char* extra; };

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
  r.extra = c;
  return r;
}

hipError_t fp32r_batch(const BlockedPlan& p, const MatDesc* descs,
                       const double* hbuf, int B, int N, int L, double* lad,
                       double* dg, double* growth, void* fact,
                       hipStream_t st) {
  BlockedBufs<float> bb = carve_blocked<float>(fact, p, B);
  float* X = reinterpret_cast<float*>(bb.extra);
  double* parts = reinterpret_cast<double*>(
      bb.extra + align256(sizeof(float) * 2 * (size_t)B * p.Np * p.Np));
  hipError_t e = blocked_lu_f32(p, descs, hbuf, B, N, L, bb.F, bb.perm,
                                bb.tri, lad, growth, st);
  if (e == hipSuccess) e = blocked_trtri_f32(p, B, bb.F, bb.perm, bb.tri, st);
  if (e == hipSuccess)
    e = launch_wv_gemm(B, N, p.Np, L, descs, hbuf, bb.F, bb.perm, X, parts,
                       st);
  if (e == hipSuccess)
    e = launch_refine(B, N, p.Np, L, descs, hbuf, bb.F, bb.perm, X, dg,
                      parts, lad, st);
  return e;
}

// Symmetric route; the matrices the L D L^T kernel flags are redone by the
// pivoted LU (predicated launches that skip every other matrix).
hipError_t sym_batch(const BlockedPlan& p, const MatDesc* descs,
                     const double* hbuf, int B, int N, int L, double* lad,
                     double* dg, double* growth, void* fact, hipStream_t st) {
  BlockedBufs<double> bb = carve_blocked<double>(fact, p, B);
  double* invd = reinterpret_cast<double*>(bb.extra);
  int* flags = reinterpret_cast<int*>(
      bb.extra + align256(sizeof(double) * 2 * (size_t)B * p.Np));
  hipError_t e = blocked_ldlt_f64(p, descs, hbuf, B, N, L, bb.F, bb.perm,
                                  bb.tri, invd, lad, growth, flags, st);
  if (e == hipSuccess)
    e = blocked_trtri_upper_f64(p, B, bb.F, bb.perm, bb.tri, st, flags, 0);
  if (e == hipSuccess)
    e = launch_symdiag_f64(B, N, p.Np, bb.F, invd, dg, st, flags, 0);
  if (e == hipSuccess)
    e = blocked_lu_f64(p, descs, hbuf, B, N, L, bb.F, bb.perm, bb.tri, lad,
                       growth, st, flags, 1);
  if (e == hipSuccess)
    e = blocked_inv_f64(p, B, N, bb.F, bb.perm, bb.tri, dg, st, flags, 1);
  return e;
}

}  // namespace

hipError_t factor_batch(const MatDesc* descs, const double* hbuf, int B, int N,
                        int L, int mode, double* lad, double* dg,
                        double* growth, void* fact, hipStream_t st,
                        const ProbDesc* probs, int nH) {
  if (B <= 0) return hipSuccess;
  if (mode == kModeEig)
    return spectral_batch(probs, nH, descs, hbuf, B, N, L, lad, dg, growth,
                          fact, st);
  if (N <= kSmallMax)
    return launch_small_factor(descs, hbuf, B, N, L, lad, dg, growth, st);
  const BlockedPlan p = blocked_plan(N, fp32_mode(mode));
  if (p.cfg < 0 || (fp32_mode(mode) && sym_mode(mode)))
    return hipErrorInvalidValue;
  if (fp32_mode(mode))
    return fp32r_batch(p, descs, hbuf, B, N, L, lad, dg, growth, fact, st);
  if (sym_mode(mode))
    return sym_batch(p, descs, hbuf, B, N, L, lad, dg, growth, fact, st);
  BlockedBufs<double> bb = carve_blocked<double>(fact, p, B);
  hipError_t e = blocked_lu_f64(p, descs, hbuf, B, N, L, bb.F, bb.perm, bb.tri,
                                lad, growth, st);
  if (e != hipSuccess) return e;
  return blocked_inv_f64(p, B, N, bb.F, bb.perm, bb.tri, dg, st);
}

bool factor_backward_consumes(int N, int mode) {
  return N > kSmallMax && mode == 0;
}

size_t autograd_factor_bytes(int N, int B, int mode) {
  size_t bytes = align256(sizeof(FactorHeader))
               + align256(sizeof(double) * (size_t)B)        // lad
               + align256(sizeof(double) * (size_t)B)        // growth
               + align256(sizeof(double) * 2 * (size_t)B * N)  // dg
               + factor_workspace_bytes(N, B, mode);   // factors
  return bytes;
}

AutogradLayout autograd_layout(void* base, int N, int B, int mode) {
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
  a.fact = factor_workspace_bytes(N, B, mode) ? p : nullptr;
  return a;
}

hipError_t factor_forward(const MatDesc* descs, const double* hbuf, int B,
                          int N, int L, int mode, double* lad, double* dg,
                          double* growth, void* fact, hipStream_t st) {
  // only the FP64 pivoted route splits: the small path forms diag(A^-1) in
  // the same pass as the LU, the FP32 route needs W and V for the refined
  // log-determinant, the symmetric route's fallback needs both halves
  if (!factor_backward_consumes(N, mode))
    return factor_batch(descs, hbuf, B, N, L, mode, lad, dg, growth, fact, st);
  const BlockedPlan p = blocked_plan_f64(N);
  if (p.cfg < 0) return hipErrorInvalidValue;
  BlockedBufs<double> bb = carve_blocked<double>(fact, p, B);
  return blocked_lu_f64(p, descs, hbuf, B, N, L, bb.F, bb.perm, bb.tri, lad,
                        growth, st);
}

hipError_t factor_backward(int B, int N, int mode, const double* lad,
                           double* dg, void* fact, hipStream_t st) {
  (void)lad;
  if (!factor_backward_consumes(N, mode)) return hipSuccess;   // dg complete
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
                               ProbStats* stats, void* ws, const double* mom,
                               const double* tsum, hipStream_t st) {
  return launch_reduce(probs, nprob, N, lad, nullptr, growth, stats, false, ws,
                       mom, tsum, st);
}

}  // namespace sca
