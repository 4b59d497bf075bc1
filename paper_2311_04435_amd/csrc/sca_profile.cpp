#include "sca_profile.h"

#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstdlib>
#include <cstring>

namespace sca {

bool roctx_enabled() {
  static const bool on = [] {
    const char* v = std::getenv("SCA_ROCTX");
    return v && std::strcmp(v, "0") != 0 && v[0] != '\0';
  }();
  return on;
}

void roctx_push(int k) {
  static const char* const names[K_COUNT] = {
      "sca:small", "sca:lu", "sca:trtri", "sca:diagdot", "sca:reduce",
      "sca:setup", "sca:refine", "sca:wvgemm", "sca:ldlt", "sca:trtri_sym",
      "sca:symdiag", "sca:fallback", "sca:tail", "sca:tridiag",
      "sca:spectrum", "sca:expand"};
  roctxRangePushA(k >= 0 && k < K_COUNT ? names[k] : "sca:?");
}

void roctx_pop() { (void)roctxRangePop(); }

Profiler*& current_profiler() {
  static thread_local Profiler* p = nullptr;
  return p;
}

hipEvent_t Profiler::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void Profiler::begin(int k, hipStream_t st) {
  hipEvent_t a = get();
  if (!a) return;
  (void)hipEventRecord(a, st);
  pending.push_back(Pending{k, a, nullptr});
}

void Profiler::end(int k, hipStream_t st) {
  for (auto it = pending.rbegin(); it != pending.rend(); ++it) {
    if (it->k == k && it->b == nullptr) {
      hipEvent_t b = get();
      if (!b) return;
      (void)hipEventRecord(b, st);
      it->b = b;
      return;
    }
  }
}

void Profiler::resolve() {
  for (auto& p : pending) {
    if (p.a && p.b) {
      float ms = 0.0f;
      if (hipEventSynchronize(p.b) == hipSuccess &&
          hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        total_ms[p.k] += ms;
        launches[p.k] += 1;
      }
    }
    if (p.a) pool.push_back(p.a);
    if (p.b) pool.push_back(p.b);
  }
  pending.clear();
}

void Profiler::reset() {
  for (int k = 0; k < K_COUNT; ++k) { total_ms[k] = 0.0; launches[k] = 0; }
}

void Profiler::release() {
  resolve();
  for (auto e : pool) (void)hipEventDestroy(e);
  pool.clear();
}

}  // namespace sca
