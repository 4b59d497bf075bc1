// Host-side pieces shared by the context calls (sca_api.cpp) and the
// request server (sca_serve.cpp): error reporting, validation, the
// workspace carve-up of one batch and one evaluation pass over it.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "../../include/sca.h"
#include "sca_common.h"

namespace sca {

// Sets the calling thread's message (sca_last_error) and returns s.
sca_status fail(sca_status s, const char* fmt, ...);

#define SCA_HIP_TRY(expr)                                                    \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess)                                                    \
      return ::sca::fail(SCA_EDEVICE, "%s failed: %s", #expr,                \
                         hipGetErrorString(e_));                             \
  } while (0)

sca_status validate_params(const sca_params* p);
// Route code (kModeFp32 | kModeSym bits) of a parameter point.
int route_of(const sca_params* p);
sca_status validate_adam_opts(const sca_adam_opts* o);
// ptr must be device (or managed) memory of `device`; NULL only if allowed.
sca_status check_device_ptr(int device, const void* ptr, const char* name,
                            bool allow_null);

// Problem descriptor of one parameter point (no ADAM state, offsets 0;
// every frequency factorised).
ProbDesc make_prob(const sca_params* p, const double* phi, double* grad);

// SCA_TAIL_MOMENTS split of a parameter point, from max|phi| and
// max|onsite|: P.Me = the frequencies factorised, P.tail_guard = the
// spectral bound above which a pass is flagged (see include/sca.h).
void tail_split(const sca_params* p, double phi_max, double onsite_max,
                ProbDesc& P);

// Workspace carve-up for one batch of `nprob` problems of N sites with B
// matrices in total (base == nullptr: sizes only, in `total`).
struct Carve {
  ProbDesc* probs; MatDesc* descs; double* hbuf; double* lad; double* growth;
  double* dg; void* rws; ProbStats* stats; void* fact;
  double* mom; double* tsum;   // Matsubara tail (moments, frequency sums)
  bool tail_on;                // some problem of the batch has Me < M
  bool hmc_on;                 // leapfrog updates in the reduction
  size_t total;
};
Carve carve(char* base, int nprob, int N, int B, int precision, bool own_dg,
            bool own_lad, size_t fact_bytes);

// One evaluation pass over a batch whose problem and matrix descriptors are
// on the device: h vectors, factorisation and inverse diagonal of all B
// matrices, reduction (+ the ADAM update of problems with steps left).
hipError_t enqueue_pass(const Carve& c, int nprob, int L, int B,
                        int precision, bool adam, hipStream_t st);

}  // namespace sca
