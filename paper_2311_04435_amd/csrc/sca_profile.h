// Per-kernel timing with HIP events on the launching stream.  The API layer
// installs a Profiler for the duration of a call on the calling thread; the
// launch sites bracket each kernel with mark_begin / mark_end.
#pragma once
#include <hip/hip_runtime.h>
#include <vector>

namespace sca {

enum KernelClass {
  K_SMALL = 0,    // fused small-lattice factor + inverse
  K_LU = 1,       // blocked LU
  K_TRTRI = 2,    // blocked U^-1 / L^-1
  K_DIAGDOT = 3,  // diagonal of the inverse from U^-1, L^-1
  K_REDUCE = 4,   // Matsubara/spin reduction + ADAM
  K_SETUP = 5,    // descriptors and diagonal vectors
  K_REFINE = 6,   // FP64 refinement of the FP32 route
  K_WVGEMM = 7,   // X = U^-1 L^-1 of the FP32 route
  K_LDLT = 8,     // symmetric route: L D L^T
  K_TRTRI_SYM = 9,  // symmetric route: L^-T
  K_SYMDIAG = 10,   // symmetric route: diagonal of A^-1
  K_FALLBACK = 11,  // symmetric route: pivoted LU of flagged matrices
  K_TAIL = 12,      // Matsubara tail: moments of H and frequency sums
  K_TRIDIAG = 13,   // spectral route: Householder tridiagonalisation
  K_SPECTRUM = 14,  // spectral route: eigenvalues, eigenvectors, psi^2
  K_EXPAND = 15,    // spectral route: per-matrix terms from the spectrum
  K_COUNT = 16
};

struct Profiler {
  bool on = false;
  double total_ms[K_COUNT] = {};
  long long launches[K_COUNT] = {};
  struct Pending { int k; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;

  hipEvent_t get();
  void begin(int k, hipStream_t st);
  void end(int k, hipStream_t st);
  // after the stream has drained: fold pending events into the totals
  void resolve();
  void reset();
  void release();
};

// Profiler of the current call on this thread (nullptr: not timing).
Profiler*& current_profiler();

// roctx ranges (SCA_ROCTX=1 in the environment, read once): every kernel
// class's launches are bracketed on the host by a range named after the
// class (rocprofv3 --marker-trace records them).
bool roctx_enabled();
void roctx_push(int k);
void roctx_pop();

inline void mark_begin(int k, hipStream_t st) {
  if (roctx_enabled()) roctx_push(k);
  Profiler* p = current_profiler();
  if (p && p->on) p->begin(k, st);
}
inline void mark_end(int k, hipStream_t st) {
  Profiler* p = current_profiler();
  if (p && p->on) p->end(k, st);
  if (roctx_enabled()) roctx_pop();
}

}  // namespace sca
