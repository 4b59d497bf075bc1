// Dispatch layer between the C ABI and the kernels: picks the factorisation
// path from N and the route (precision and factorisation) and sizes its
// scratch memory.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include "sca_common.h"

namespace sca {

constexpr int kMaxL = 64;           // N <= 4096 sites
constexpr int kMaxNmax = 1 << 16;   // Matsubara frequencies per spin
constexpr int kMaxShifts = 1 << 20; // shifts per sca_dos / sca_shifted_terms

// Route code of a parameter point (the `mode` argument of the functions
// below): bit 0 = FP32 refined, bit 1 = symmetric L D L^T, bit 2 = spectral
// (one eigendecomposition per h vector instead of a factorisation per
// matrix; FP64 only).
constexpr int kModeFp32 = 1;
constexpr int kModeSym = 2;
constexpr int kModeEig = 4;

// Whether a factorisation path exists for N sites on route `mode`.
bool path_supported(int N, int mode);

// Scratch (bytes) the factorisation of B matrices of N sites needs beyond
// the per-matrix outputs (0 for the fused small path).  The spectral route's
// scratch depends on the number nH of h vectors instead of B.
size_t factor_workspace_bytes(int N, int B, int mode, int nH = 2);

// ln|det A_b| -> lad[b], diag(A_b^-1) -> dg[b][N][2] (re, im), pivot growth
// -> growth[b], for the B matrices described by descs.  `fact` is the
// scratch of factor_workspace_bytes(N, B, mode, nH) bytes.  The spectral
// route also needs the problems (probs: hopping of problem hv / 2) and the
// number nH of h vectors in hbuf (vector hv at hbuf + hv N).
hipError_t factor_batch(const MatDesc* descs, const double* hbuf, int B, int N,
                        int L, int mode, double* lad, double* dg,
                        double* growth, void* fact, hipStream_t st,
                        const ProbDesc* probs = nullptr, int nH = 0);

// Spectral route (k_eig.hip): the outputs of factor_batch from one
// eigendecomposition per h vector; growth is 1 (no pivoting).
size_t eig_workspace_bytes(int N, int nH);
hipError_t spectral_batch(const ProbDesc* probs, int nH, const MatDesc* descs,
                          const double* hbuf, int B, int N, int L, double* lad,
                          double* dg, double* growth, void* fact,
                          hipStream_t st);

// Autograd split of factor_batch.  The forward writes lad and growth and
// keeps in `fact` (and, for the fused small path and the FP32 route, in dg)
// what the backward needs; the backward completes dg from it.  The buffer
// starts with a header naming the problem shape and whether the factors are
// still usable: the FP64 blocked backward inverts them in place.
struct FactorHeader {
  uint32_t state; int32_t L, n_max, mode;
  int32_t tail, Me;    // tail option and frequencies factorised (n < Me)
  double tail_guard;
};
constexpr uint32_t kFactorsReady = 0x5CA10001u;
constexpr uint32_t kFactorsConsumed = 0x5CA10002u;
struct AutogradLayout {
  FactorHeader* head; double* lad; double* growth; double* dg; void* fact;
};
// Whether factor_backward overwrites the factors it reads.
bool factor_backward_consumes(int N, int mode);
size_t autograd_factor_bytes(int N, int B, int mode);
AutogradLayout autograd_layout(void* base, int N, int B, int mode);
hipError_t factor_forward(const MatDesc* descs, const double* hbuf, int B,
                          int N, int L, int mode, double* lad, double* dg,
                          double* growth, void* fact, hipStream_t st);
hipError_t factor_backward(int B, int N, int mode, const double* lad,
                           double* dg, void* fact, hipStream_t st);

// Omega, Omega~ of every problem without the gradient (dg not read).
hipError_t launch_reduce_omega(ProbDesc* probs, int nprob, int N,
                               const double* lad, const double* growth,
                               ProbStats* stats, void* ws, const double* mom,
                               const double* tsum, hipStream_t st);

// z[2j] = w[j], z[2j+1] = eta.
hipError_t launch_make_shifts(const double* w, int n_w, double eta, double* z,
                              hipStream_t st);

size_t footprint(int N, int M, int mode);

}  // namespace sca
