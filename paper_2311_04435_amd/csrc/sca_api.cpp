// Host runtime and C ABI of the SCA library (see include/sca.h).
//
// A context owns one growable device workspace and a small pinned staging
// buffer, and enqueues everything on the caller's stream.  One evaluation
// of a problem set runs, all on the device:
//   descriptors (once per call) -> h vectors -> batched factor + inverse
//   diagonal -> Matsubara/spin reduction (+ fused ADAM update)
// The host only reads back the per-problem statistics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sca.h"
#include "sca_common.h"
#include "sca_engine.h"
#include "sca_kernels.h"
#include "sca_profile.h"
#include "sca_runtime.h"

namespace sca {

thread_local std::string g_err;

sca_status fail(sca_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

}  // namespace sca

#define HIP_TRY SCA_HIP_TRY


struct sca_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t budget = 0;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  double* dscalar = nullptr;   // one device double (tail planning)
  double growth_limit = 1e3;   // SCA_OPT_FP32_GROWTH_LIMIT
  void* scratch = nullptr;     // this device's fixed scratch (sca_grad_noalloc)
  sca::Profiler prof;
};

// ---------------------------------------------- fixed scratch (no-alloc) --
// sca_grad_noalloc works in this array instead of the context's workspace:
// one copy per device, allocated by the code-object loader with the library
// and held until the process ends.  Host code never uses the array's name as
// an address: sca_create takes each device's address once, with that device
// current (hipGetSymbolAddress), and passes that pointer on.
namespace {
constexpr size_t kNoAllocBytes = size_t(16) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

// The device's scratch address; `device` must be the current device.
sca_status scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices)
    return sca::fail(SCA_EDEVICE, "device %d beyond the %d this library "
                     "tracks", device, kMaxDevices);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return sca::fail(SCA_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s",
                       hipGetErrorString(e));
    }
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return SCA_OK;
}

// Writes one problem descriptor to device memory from the kernel argument
// (no staging buffer on the host).
__global__ void store_desc_kernel(sca::ProbDesc* dst, sca::ProbDesc P) {
  *dst = P;
}
}  // namespace

namespace sca {

sca_status validate_params(const sca_params* p) {
  if (!p) return fail(SCA_EINVAL, "params is NULL");
  if (p->L < 2 || p->L > kMaxL || (p->L & 1))
    return fail(SCA_EINVAL, "L=%d: must be even and in [2, %d]", p->L, kMaxL);
  if (p->n_max < 1 || p->n_max > kMaxNmax)
    return fail(SCA_EINVAL, "n_max=%d: must be in [1, %d]", p->n_max, kMaxNmax);
  if (p->precision != SCA_FP64 && p->precision != SCA_FP32_REFINED)
    return fail(SCA_EINVAL, "precision=%d: unknown", p->precision);
  if (p->factor != SCA_FACTOR_LU && p->factor != SCA_FACTOR_LDLT &&
      p->factor != SCA_FACTOR_EIGH)
    return fail(SCA_EINVAL, "factor=%d: unknown", p->factor);
  if (p->tail != SCA_TAIL_NONE && p->tail != SCA_TAIL_MOMENTS)
    return fail(SCA_EINVAL, "tail=%d: unknown", p->tail);
  if (p->reserved != 0) return fail(SCA_EINVAL, "reserved must be 0");
  if (!std::isfinite(p->t) || !std::isfinite(p->delta))
    return fail(SCA_EINVAL, "t and delta must be finite");
  if (!(p->U > 0.0) || !std::isfinite(p->U))
    return fail(SCA_EINVAL, "U=%g: must be finite and > 0", p->U);
  if (!(p->T > 0.0) || !std::isfinite(p->T))
    return fail(SCA_EINVAL, "T=%g: must be finite and > 0", p->T);
  const int N = p->L * p->L;
  if (!path_supported(N, route_of(p)))
    return fail(SCA_EUNSUPPORTED, "N=%d with precision %d and factor %d is "
                "not built", N, p->precision, p->factor);
  return SCA_OK;
}

int route_of(const sca_params* p) {
  return (p->precision == SCA_FP32_REFINED ? kModeFp32 : 0) |
         (p->factor == SCA_FACTOR_LDLT ? kModeSym : 0) |
         (p->factor == SCA_FACTOR_EIGH ? kModeEig : 0);
}

sca_status check_device_ptr(int device, const void* ptr, const char* name,
                            bool allow_null) {
  if (!ptr) {
    if (allow_null) return SCA_OK;
    return fail(SCA_EINVAL, "%s is NULL", name);
  }
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(SCA_EINVAL, "%s is not a device pointer", name);
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    return fail(SCA_EINVAL, "%s is not device memory", name);
  if (attr.device != device)
    return fail(SCA_EINVAL, "%s lives on device %d, expected %d", name,
                attr.device, device);
  return SCA_OK;
}

sca_status validate_adam_opts(const sca_adam_opts* o) {
  if (!o) return fail(SCA_EINVAL, "opts is NULL");
  if (o->n_steps < 0 || o->check_every < 0 || o->t0 < 0)
    return fail(SCA_EINVAL, "n_steps, check_every, t0 must be >= 0");
  if (o->flags & ~SCA_ADAM_NO_FINAL_EVAL)
    return fail(SCA_EINVAL, "unknown ADAM flags 0x%x", o->flags);
  if (!(o->lr > 0.0) || !(o->beta1 >= 0.0 && o->beta1 < 1.0) ||
      !(o->beta2 >= 0.0 && o->beta2 < 1.0) || !(o->eps >= 0.0) ||
      !(o->grad_tol >= 0.0))
    return fail(SCA_EINVAL, "invalid ADAM hyper-parameters");
  return SCA_OK;
}

void tail_split(const sca_params* p, double phi_max, double onsite_max,
                ProbDesc& P) {
  constexpr double kPi = 3.14159265358979323846;
  P.Me = p->n_max;
  P.tail_guard = 0.0;
  if (p->tail != SCA_TAIL_MOMENTS) return;
  const double phib = std::max(phi_max, 0.5 * p->U) + 0.5;
  const double rho = 4.0 * std::fabs(p->t) + 0.5 * std::fabs(p->delta) +
                     onsite_max + phib;
  const double x = (4.0 * rho / (kPi * p->T) - 1.0) / 2.0;
  const int me = x >= (double)p->n_max ? p->n_max
                                       : std::max(1, (int)std::ceil(x));
  P.Me = me;
  P.tail_guard = (2.0 * me + 1.0) * kPi * p->T / 3.0;
}

ProbDesc make_prob(const sca_params* p, const double* phi, double* grad) {
  ProbDesc P{};
  P.phi = phi;
  P.onsite = p->onsite;
  P.grad = grad;
  P.t = p->t; P.U = p->U; P.delta = p->delta; P.T = p->T;
  P.L = p->L; P.N = p->L * p->L; P.M = p->n_max;
  P.Me = p->n_max;
  P.tail_guard = 0.0;
  P.mat_begin = 0;
  P.hoff = 0;
  return P;
}

hipError_t enqueue_pass(const Carve& c, int nprob, int L, int B,
                        int precision, bool adam, hipStream_t st) {
  const int N = L * L;
  hipError_t e = launch_hvec(c.probs, nprob, N, c.hbuf, st);
  if (e == hipSuccess && c.tail_on)
    e = launch_tail(c.probs, nprob, N, c.hbuf, c.mom, c.tsum, st);
  if (e == hipSuccess)
    e = factor_batch(c.descs, c.hbuf, B, N, L, precision, c.lad, c.dg,
                     c.growth, c.fact, st, c.probs, 2 * nprob);
  if (e == hipSuccess)
    e = launch_reduce(c.probs, nprob, N, c.lad, c.dg, c.growth, c.stats, adam,
                      c.rws, c.mom, c.tsum, st, c.hmc_on);
  return e;
}

}  // namespace sca

using namespace sca;

namespace {

sca_status check_dev_ptr(const sca_ctx* ctx, const void* ptr, const char* name,
                         bool allow_null = false) {
  return check_device_ptr(ctx->device, ptr, name, allow_null);
}

sca_status ensure_ws(sca_ctx* ctx, size_t bytes) {
  if (ctx->budget && bytes > ctx->budget)
    return fail(SCA_ENOMEM, "workspace of %zu bytes exceeds the budget of %zu",
                bytes, ctx->budget);
  if (bytes <= ctx->ws_bytes) return SCA_OK;
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  if (ctx->ws) HIP_TRY(hipFree(ctx->ws));
  ctx->ws = nullptr;
  ctx->ws_bytes = 0;
  hipError_t e = hipMalloc(&ctx->ws, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(SCA_ENOMEM, "hipMalloc(%zu) failed: %s", bytes,
                hipGetErrorString(e));
  }
  ctx->ws_bytes = bytes;
  return SCA_OK;
}

sca_status ensure_pinned(sca_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->pinned_bytes) return SCA_OK;
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  if (ctx->pinned) HIP_TRY(hipHostFree(ctx->pinned));
  ctx->pinned = nullptr;
  ctx->pinned_bytes = 0;
  HIP_TRY(hipHostMalloc(&ctx->pinned, bytes, hipHostMallocDefault));
  ctx->pinned_bytes = bytes;
  return SCA_OK;
}

sca_status device_absmax(sca_ctx* ctx, const double* x, int n, double* out) {
  if (!ctx->dscalar) HIP_TRY(hipMalloc(&ctx->dscalar, sizeof(double)));
  sca_status s = ensure_pinned(ctx, sizeof(double));
  if (s) return s;
  HIP_TRY(launch_absmax(x, n, ctx->dscalar, ctx->stream));
  HIP_TRY(hipMemcpyAsync(ctx->pinned, ctx->dscalar, sizeof(double),
                         hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  std::memcpy(out, ctx->pinned, sizeof(double));
  return SCA_OK;
}

// Frequencies factorised under SCA_TAIL_MOMENTS: n < Me, the first n with
// w_n >= 4 rho_b (rho_b: Gershgorin bound with a margin for phi to grow);
// each pass flags a bound above w_Me / 3.
sca_status plan_tail(sca_ctx* ctx, const sca_params* p, const double* phi,
                     ProbDesc& P) {
  P.Me = p->n_max;
  P.tail_guard = 0.0;
  if (p->tail != SCA_TAIL_MOMENTS) return SCA_OK;
  const int N = p->L * p->L;
  double pmax = 0.0, omax = 0.0;
  sca_status s = device_absmax(ctx, phi, N, &pmax);
  if (s) return s;
  if (p->onsite && (s = device_absmax(ctx, p->onsite, N, &omax))) return s;
  if (!std::isfinite(pmax) || !std::isfinite(omax))
    return fail(SCA_ENUMERIC, "phi or onsite is not finite");
  tail_split(p, pmax, omax, P);
  return SCA_OK;
}

// Per-call scope: selects the context's device and installs its profiler
// for the launches of this call; pending kernel timings are folded in when
// the call ends (every call drains its stream before returning).
struct DeviceGuard {
  int prev = -1;
  sca_ctx* ctx = nullptr;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  DeviceGuard(sca_ctx* c, int dev) : DeviceGuard(dev) {
    ctx = c;
    current_profiler() = &c->prof;
  }
  ~DeviceGuard() {
    if (ctx) {
      current_profiler() = nullptr;
      if (ctx->prof.on) {
        (void)hipStreamSynchronize(ctx->stream);
        ctx->prof.resolve();
      }
    }
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

}  // namespace

// ------------------------------------------------------------- engine ----

namespace sca {

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

Carve carve(char* base, int nprob, int N, int B, int precision,
                   bool own_dg, bool own_lad, size_t fact_bytes) {
  Carve c{};
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return base ? base + o : nullptr; };
  c.probs = (ProbDesc*)take(sizeof(ProbDesc) * nprob);
  c.descs = (MatDesc*)take(sizeof(MatDesc) * (size_t)B);
  c.hbuf = (double*)take(sizeof(double) * 2 * (size_t)nprob * N);
  c.lad = own_lad ? (double*)take(sizeof(double) * (size_t)B) : nullptr;
  c.growth = (double*)take(sizeof(double) * (size_t)B);
  c.dg = own_dg ? (double*)take(sizeof(double) * 2 * (size_t)B * N) : nullptr;
  c.rws = take(reduce_workspace_bytes(nprob));
  c.stats = (ProbStats*)take(sizeof(ProbStats) * nprob);
  c.mom = (double*)take(tail_workspace_bytes(nprob, N));
  c.tsum = c.mom ? c.mom + (size_t)nprob * 2 * kTailP * N : nullptr;
  c.tail_on = false;
  c.hmc_on = false;
  c.fact = fact_bytes ? (void*)take(fact_bytes) : nullptr;
  (void)precision;
  c.total = off;
  return c;
}

size_t footprint(int N, int M, int precision) {
  const int B = 2 * M;
  Carve c = carve(nullptr, 1, N, B, precision, true, true,
                  factor_workspace_bytes(N, B, precision));
  return c.total;
}

}  // namespace sca

namespace {

// Evaluate the terms of `nprob` problems (same L) described in host_probs;
// with `adam`, every problem with steps left takes one fused ADAM update
// (its counters advance on the device).  With `upload` the descriptors are
// copied to the device first; otherwise the device copies (and counters)
// of the previous pass are used.
sca_status run_batch(sca_ctx* ctx, Carve& c, const ProbDesc* host_probs,
                     int nprob, int L, int B, int max2M, int precision,
                     bool adam, bool upload) {
  const int N = L * L;
  hipStream_t st = ctx->stream;
  if (upload) {
    sca_status s = ensure_pinned(ctx, sizeof(ProbDesc) * nprob);
    if (s) return s;
    HIP_TRY(hipStreamSynchronize(st));
    std::memcpy(ctx->pinned, host_probs, sizeof(ProbDesc) * nprob);
    HIP_TRY(hipMemcpyAsync(c.probs, ctx->pinned, sizeof(ProbDesc) * nprob,
                           hipMemcpyHostToDevice, st));
    HIP_TRY(launch_matsubara_descs(c.probs, nprob, max2M, c.descs, st));
  }
  (void)N;
  HIP_TRY(enqueue_pass(c, nprob, L, B, precision, adam, st));
  return SCA_OK;
}

sca_status read_stats(sca_ctx* ctx, const Carve& c, int nprob,
                      ProbStats* out) {
  sca_status s = ensure_pinned(ctx, sizeof(ProbStats) * nprob);
  if (s) return s;
  HIP_TRY(hipMemcpyAsync(ctx->pinned, c.stats, sizeof(ProbStats) * nprob,
                         hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  std::memcpy(out, ctx->pinned, sizeof(ProbStats) * nprob);
  return SCA_OK;
}

sca_status begin_call(sca_ctx* ctx, const sca_params* p) {
  g_err.clear();
  if (!ctx) return fail(SCA_EINVAL, "context is NULL");
  sca_status s = validate_params(p);
  if (s) return s;
  return check_dev_ptr(ctx, p->onsite, "params.onsite", true);
}

// Pivot growth above which a complex64 factorisation is not trusted (the
// context's SCA_OPT_FP32_GROWTH_LIMIT, 1e3 by default): the backward error
// of an LU grows with it, and the FP64 refinement only corrects an error of
// FP32 size.
bool growth_exceeded(const sca_ctx* ctx, int mode, double growth) {
  return (mode & kModeFp32) && !(growth <= ctx->growth_limit);
}

// The limit a pass of route `mode` checks on the device: the context's, if
// an FP64 route can take over for N, else 0 (the growth is only reported).
double device_growth_limit(const sca_ctx* ctx, int N, int mode) {
  return ((mode & kModeFp32) && path_supported(N, mode & ~kModeFp32))
             ? ctx->growth_limit : 0.0;
}

sca_status eval_single(sca_ctx* ctx, const sca_params* p, const double* phi,
                       double* grad, double* omega2, ProbStats* st_out) {
  const int N = p->L * p->L;
  ProbDesc P = make_prob(p, phi, grad);
  sca_status s = plan_tail(ctx, p, phi, P);
  if (s) return s;
  P.growth_limit = device_growth_limit(ctx, N, route_of(p));
  const int B = 2 * P.Me;
  Carve c0 = carve(nullptr, 1, N, B, route_of(p), true, true,
                   factor_workspace_bytes(N, B, route_of(p)));
  if ((s = ensure_ws(ctx, c0.total))) return s;
  Carve c = carve((char*)ctx->ws, 1, N, B, route_of(p), true, true,
                  factor_workspace_bytes(N, B, route_of(p)));
  c.tail_on = P.Me < P.M;
  s = run_batch(ctx, c, &P, 1, p->L, B, B, route_of(p), false, true);
  if (s) return s;
  ProbStats S;
  s = read_stats(ctx, c, 1, &S);
  if (s) return s;
  if (S.tail_range) {
    // the spectral bound left the tail's range: evaluate every frequency
    sca_params q = *p;
    q.tail = SCA_TAIL_NONE;
    return eval_single(ctx, &q, phi, grad, omega2, st_out);
  }
  if (growth_exceeded(ctx, route_of(p), S.pivot_growth)) {
    if (!path_supported(N, route_of(p) & ~kModeFp32))
      return fail(SCA_ENUMERIC, "FP32 pivot growth %.3g above %.3g and no "
                  "FP64 path for N=%d", S.pivot_growth, ctx->growth_limit, N);
    sca_params q = *p;
    q.precision = SCA_FP64;
    return eval_single(ctx, &q, phi, grad, omega2, st_out);
  }
  if (omega2) {
    double o2[2] = {S.omega, S.omega_tilde};
    HIP_TRY(hipMemcpyAsync(omega2, o2, sizeof o2, hipMemcpyHostToDevice,
                           ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
  }
  if (st_out) *st_out = S;
  if (S.nonfinite)
    return fail(SCA_ENUMERIC, "non-finite potential or gradient");
  return SCA_OK;
}

// eval_single in the device's fixed scratch: nothing is allocated on the
// device or the host (descriptors go up as kernel arguments, statistics come
// back into the caller's stack through the stream).  Layout of the scratch:
// one double for the tail planning at 0, the batch's carve from 256.
sca_status eval_single_noalloc(sca_ctx* ctx, const sca_params* p,
                               const double* phi, double* grad,
                               double* omega2) {
  const int N = p->L * p->L;
  const int mode = route_of(p);
  hipStream_t st = ctx->stream;
  char* base = static_cast<char*>(ctx->scratch);
  ProbDesc P = make_prob(p, phi, grad);
  if (p->tail == SCA_TAIL_MOMENTS) {
    double pmax = 0.0, omax = 0.0;
    double* dsc = reinterpret_cast<double*>(base);
    HIP_TRY(launch_absmax(phi, N, dsc, st));
    HIP_TRY(hipMemcpyAsync(&pmax, dsc, sizeof pmax, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (p->onsite) {
      HIP_TRY(launch_absmax(p->onsite, N, dsc, st));
      HIP_TRY(hipMemcpyAsync(&omax, dsc, sizeof omax, hipMemcpyDeviceToHost,
                             st));
      HIP_TRY(hipStreamSynchronize(st));
    }
    if (!std::isfinite(pmax) || !std::isfinite(omax))
      return fail(SCA_ENUMERIC, "phi or onsite is not finite");
    tail_split(p, pmax, omax, P);
  }
  P.growth_limit = device_growth_limit(ctx, N, mode);
  const int B = 2 * P.Me;
  const size_t fb = factor_workspace_bytes(N, B, mode);
  const Carve c0 = carve(nullptr, 1, N, B, mode, true, true, fb);
  if (256 + c0.total > kNoAllocBytes)
    return fail(SCA_ENOMEM, "L=%d, n_max=%d needs %zu bytes of scratch; the "
                "fixed scratch of sca_grad_noalloc holds %zu", p->L,
                p->n_max, 256 + c0.total, kNoAllocBytes);
  Carve c = carve(base + 256, 1, N, B, mode, true, true, fb);
  c.tail_on = P.Me < P.M;
  hipLaunchKernelGGL(store_desc_kernel, dim3(1), dim3(1), 0, st, c.probs, P);
  HIP_TRY(hipGetLastError());
  HIP_TRY(launch_matsubara_descs(c.probs, 1, B, c.descs, st));
  HIP_TRY(enqueue_pass(c, 1, p->L, B, mode, false, st));
  ProbStats S;
  HIP_TRY(hipMemcpyAsync(&S, c.stats, sizeof S, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (S.tail_range) {
    sca_params q = *p;
    q.tail = SCA_TAIL_NONE;
    return eval_single_noalloc(ctx, &q, phi, grad, omega2);
  }
  if (growth_exceeded(ctx, mode, S.pivot_growth)) {
    if (!path_supported(N, mode & ~kModeFp32))
      return fail(SCA_ENUMERIC, "FP32 pivot growth %.3g above %.3g and no "
                  "FP64 path for N=%d", S.pivot_growth, ctx->growth_limit, N);
    sca_params q = *p;
    q.precision = SCA_FP64;
    return eval_single_noalloc(ctx, &q, phi, grad, omega2);
  }
  if (omega2) {
    // Omega and Omega~ lead ProbStats
    HIP_TRY(hipMemcpyAsync(omega2, c.stats, 2 * sizeof(double),
                           hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  if (S.nonfinite)
    return fail(SCA_ENUMERIC, "non-finite potential or gradient");
  return SCA_OK;
}

}  // namespace

// ------------------------------------------------------------- C ABI -----

extern "C" {

sca_status sca_create(int device, void* hip_stream, size_t hbm_budget_bytes,
                      sca_ctx** out) {
  g_err.clear();
  if (!out) return fail(SCA_EINVAL, "out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0) {
    (void)hipGetLastError();
    return fail(SCA_EDEVICE, "no HIP device available");
  }
  if (device < 0 || device >= n)
    return fail(SCA_EINVAL, "device %d out of range [0, %d)", device, n);
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(SCA_EDEVICE, "device %d is %s; this library is built for gfx950",
                device, prop.gcnArchName);
  void* scr = nullptr;
  {
    DeviceGuard g(device);
    sca_status s = scratch_address(device, &scr);
    if (s) return s;
  }
  sca_ctx* ctx = new sca_ctx;
  ctx->device = device;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  ctx->budget = hbm_budget_bytes;
  ctx->scratch = scr;
  *out = ctx;
  return SCA_OK;
}

void sca_destroy(sca_ctx* ctx) {
  if (!ctx) return;
  DeviceGuard g(ctx, ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->dscalar) (void)hipFree(ctx->dscalar);
  delete ctx;
}

size_t sca_footprint_bytes(const sca_params* p) {
  std::string saved = g_err;
  if (validate_params(p) != SCA_OK) return 0;
  g_err = saved;
  return footprint(p->L * p->L, p->n_max, route_of(p));
}

sca_status sca_potential(sca_ctx* ctx, const sca_params* p, const double* phi,
                         double* omega2) {
  sca_status s = begin_call(ctx, p);
  if (s) return s;
  DeviceGuard g(ctx, ctx->device);
  if ((s = check_dev_ptr(ctx, phi, "phi"))) return s;
  if ((s = check_dev_ptr(ctx, omega2, "omega2"))) return s;
  return eval_single(ctx, p, phi, nullptr, omega2, nullptr);
}

sca_status sca_grad(sca_ctx* ctx, const sca_params* p, const double* phi,
                    double* grad, double* omega2) {
  sca_status s = begin_call(ctx, p);
  if (s) return s;
  DeviceGuard g(ctx, ctx->device);
  if ((s = check_dev_ptr(ctx, phi, "phi"))) return s;
  if ((s = check_dev_ptr(ctx, grad, "grad"))) return s;
  if ((s = check_dev_ptr(ctx, omega2, "omega2", true))) return s;
  return eval_single(ctx, p, phi, grad, omega2, nullptr);
}

sca_status sca_grad_noalloc(sca_ctx* ctx, const sca_params* p,
                            const double* phi, double* grad, double* omega2) {
  sca_status s = begin_call(ctx, p);
  if (s) return s;
  if (!ctx->scratch)
    return fail(SCA_EDEVICE, "the context has no fixed scratch");
  DeviceGuard g(ctx, ctx->device);
  if ((s = check_dev_ptr(ctx, phi, "phi"))) return s;
  if ((s = check_dev_ptr(ctx, grad, "grad"))) return s;
  if ((s = check_dev_ptr(ctx, omega2, "omega2", true))) return s;
  return eval_single_noalloc(ctx, p, phi, grad, omega2);
}

sca_status sca_adam_solve(sca_ctx* ctx, const sca_params* p,
                          const sca_adam_opts* o, double* phi, double* m,
                          double* v, sca_result* res) {
  sca_status s = begin_call(ctx, p);
  if (s) return s;
  if (!o) return fail(SCA_EINVAL, "opts is NULL");
  if (!res) return fail(SCA_EINVAL, "result is NULL");
  if ((s = validate_adam_opts(o))) return s;
  DeviceGuard g(ctx, ctx->device);
  if ((s = check_dev_ptr(ctx, phi, "phi"))) return s;
  if ((s = check_dev_ptr(ctx, m, "m"))) return s;
  if ((s = check_dev_ptr(ctx, v, "v"))) return s;

  const int N = p->L * p->L;
  int prec = route_of(p);
  ProbDesc P = make_prob(p, phi, nullptr);
  if ((s = plan_tail(ctx, p, phi, P))) return s;
  int B = 2 * P.Me;
  Carve c;
  auto setup = [&]() -> sca_status {
    const size_t fb = factor_workspace_bytes(N, B, prec);
    Carve c0 = carve(nullptr, 1, N, B, prec, true, true, fb);
    sca_status r = ensure_ws(ctx, c0.total);
    if (r) return r;
    c = carve((char*)ctx->ws, 1, N, B, prec, true, true, fb);
    c.tail_on = P.Me < P.M;
    return SCA_OK;
  };
  if ((s = setup())) return s;
  P.m = m; P.v = v; P.phi_out = phi;
  P.lr = o->lr; P.beta1 = o->beta1; P.beta2 = o->beta2; P.eps = o->eps;
  P.adam_t = o->t0;
  P.steps_left = o->n_steps;
  P.growth_limit = device_growth_limit(ctx, N, prec);
  std::memset(res, 0, sizeof *res);

  // The passes run in chunks; the host reads the statistics of each chunk's
  // last pass.  A pass whose guard fires applies no update (the device
  // counters say how many were applied), so re-planning the problem at the
  // chunk's end and resuming from the device's step count gives the same
  // trajectory as a switch at that very pass, whatever the chunk length.
  const bool final_eval = !(o->flags & SCA_ADAM_NO_FINAL_EVAL);
  constexpr double kChunkMs = 50.0;   // aim of one chunk when check_every = 0
  int target = o->n_steps;   // updates to apply (lowered on convergence)
  int applied = 0;           // updates applied in this call
  double gmax = 0.0, pass_ms = 0.0;
  bool converged = false, upload = true;
  ProbStats S{};
  for (;;) {
    int need = target - applied + (final_eval ? 1 : 0);
    if (need < 1) need = 1;
    int K = need;
    if (o->check_every > 0) K = std::min(K, o->check_every);
    else K = std::min(K, pass_ms > 0.0 ? std::max(1, (int)(kChunkMs / pass_ms)) : 1);
    const auto t_start = std::chrono::steady_clock::now();
    for (int k = 0; k < K; ++k) {
      s = run_batch(ctx, c, &P, 1, p->L, B, B, prec, true, upload);
      if (s) return s;
      upload = false;
    }
    if ((s = read_stats(ctx, c, 1, &S))) return s;
    pass_ms = 1e3 * std::chrono::duration<double>(
                        std::chrono::steady_clock::now() - t_start).count() / K;
    applied = S.adam_t - o->t0;
    gmax = max_nan(gmax, S.growth_run);
    if (S.nonfinite) {
      res->steps_done = applied;
      res->max_pivot_growth = gmax;
      res->flags |= SCA_FLAG_NONFINITE;
      return fail(SCA_ENUMERIC, "non-finite value at step %d", S.adam_t);
    }
    if (!converged && o->grad_tol > 0.0 && o->check_every > 0 && S.updated &&
        S.max_abs_grad < o->grad_tol) {
      // stop here; with final_eval one more pass evaluates the returned phi
      converged = true;
      target = applied;
      upload = true;
    }
    // done: the last pass evaluated the returned phi (final_eval), or
    // applied the last update (its statistics describe that update's input)
    const bool done = final_eval
        ? (applied == target && !S.updated && S.guard == 0)
        : (applied == target && (S.updated || S.guard == 0));
    if (done) break;
    if (S.guard & kGuardTail) {
      // the remaining steps factorise every frequency
      res->flags |= SCA_FLAG_TAIL_RANGE;
      P.Me = P.M;
      P.tail_guard = 0.0;
      B = 2 * P.M;
      if ((s = setup())) return s;
      upload = true;
    }
    if (S.guard & kGuardGrowth) {
      // the remaining steps run in FP64 (the guard is only armed when that
      // path is built for N)
      res->flags |= SCA_FLAG_PIVOT_GROWTH;
      prec &= ~kModeFp32;
      P.growth_limit = 0.0;
      if ((s = setup())) return s;
      upload = true;
    }
    if (upload) {
      P.adam_t = S.adam_t;
      P.steps_left = target - applied;
      P.growth_run = 0.0;
    }
  }
  if (growth_exceeded(ctx, route_of(p), gmax))
    res->flags |= SCA_FLAG_PIVOT_GROWTH;
  res->omega = S.omega;
  res->omega_tilde = S.omega_tilde;
  res->af_order = S.af_order;
  res->max_abs_grad = S.max_abs_grad;
  res->max_pivot_growth = gmax;
  res->steps_done = applied;
  if (converged) res->flags |= SCA_FLAG_CONVERGED;
  return SCA_OK;
}

sca_status sca_hmc(sca_ctx* ctx, const sca_params* p, const sca_hmc_opts* o,
                   double* phi, const double* momenta, const double* uniforms,
                   int32_t* accepted, double* h_old, double* h_new) {
  sca_status s = begin_call(ctx, p);
  if (s) return s;
  if (!o) return fail(SCA_EINVAL, "opts is NULL");
  if (!(o->eps > 0.0) || !std::isfinite(o->eps) || o->n_leap < 1 ||
      o->n_traj < 0)
    return fail(SCA_EINVAL, "eps > 0, n_leap >= 1 and n_traj >= 0 required");
  if (o->n_traj > 0 && (!uniforms || !accepted || !h_old || !h_new))
    return fail(SCA_EINVAL, "uniforms, accepted, h_old, h_new must be host "
                "arrays of n_traj");
  DeviceGuard g(ctx, ctx->device);
  if ((s = check_dev_ptr(ctx, phi, "phi"))) return s;
  if (o->n_traj > 0 && (s = check_dev_ptr(ctx, momenta, "momenta"))) return s;
  const int N = p->L * p->L;
  const int prec = route_of(p);
  ProbDesc P = make_prob(p, phi, nullptr);
  if ((s = plan_tail(ctx, p, phi, P))) return s;
  const int B = 2 * P.Me;
  const size_t fb = factor_workspace_bytes(N, B, prec);
  Carve c0 = carve(nullptr, 1, N, B, prec, true, true, fb);
  // momentum and the trajectory's starting phi after the carve
  const size_t extra = 2 * ((sizeof(double) * N + 255) & ~size_t(255));
  if ((s = ensure_ws(ctx, c0.total + extra))) return s;
  Carve c = carve((char*)ctx->ws, 1, N, B, prec, true, true, fb);
  c.tail_on = P.Me < P.M;
  c.hmc_on = true;
  double* pmom = (double*)((char*)ctx->ws + c0.total);
  double* phi0 = (double*)((char*)pmom + extra / 2);
  P.phi_out = phi;
  P.pmom = pmom;
  P.hmc_eps = o->eps;
  P.hmc_L = o->n_leap;
  hipStream_t st = ctx->stream;
  if ((s = ensure_pinned(ctx, 2 * sizeof(ProbStats) + sizeof(ProbDesc))))
    return s;
  ProbStats* pin = (ProbStats*)ctx->pinned;
  for (int t = 0; t < o->n_traj; ++t) {
    HIP_TRY(hipMemcpyAsync(pmom, momenta + (size_t)t * N, sizeof(double) * N,
                           hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(phi0, phi, sizeof(double) * N,
                           hipMemcpyDeviceToDevice, st));
    // pass 0 (descriptors uploaded, hmc_k = 0), then passes 1 .. L
    P.hmc_k = 0;
    HIP_TRY(hipStreamSynchronize(st));
    std::memcpy(pin + 2, &P, sizeof P);
    HIP_TRY(hipMemcpyAsync(c.probs, pin + 2, sizeof P, hipMemcpyHostToDevice, st));
    HIP_TRY(launch_matsubara_descs(c.probs, 1, B, c.descs, st));
    for (int k = 0; k <= o->n_leap; ++k) {
      HIP_TRY(enqueue_pass(c, 1, p->L, B, prec, false, st));
      if (k == 0)
        HIP_TRY(hipMemcpyAsync(pin, c.stats, sizeof(ProbStats),
                               hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(hipMemcpyAsync(pin + 1, c.stats, sizeof(ProbStats),
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const ProbStats S0 = pin[0], S1 = pin[1];
    if (S0.nonfinite || S1.nonfinite)
      return fail(SCA_ENUMERIC, "non-finite value in trajectory %d", t);
    if (S0.tail_range || S1.tail_range)
      return fail(SCA_ENUMERIC, "trajectory %d left the Matsubara tail's "
                  "range: sample with tail = SCA_TAIL_NONE", t);
    h_old[t] = S0.omega_tilde / p->T + S0.kin0;
    h_new[t] = S1.omega_tilde / p->T + S1.kin;
    const double dh = h_new[t] - h_old[t];
    accepted[t] = (dh <= 0.0 || uniforms[t] < std::exp(-dh)) ? 1 : 0;
    if (!accepted[t])
      HIP_TRY(hipMemcpyAsync(phi, phi0, sizeof(double) * N,
                             hipMemcpyDeviceToDevice, st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  return SCA_OK;
}

sca_status sca_tail_split(sca_ctx* ctx, const sca_params* p,
                          const double* phi, int32_t* n_factorised) {
  sca_status s = begin_call(ctx, p);
  if (s) return s;
  if (!n_factorised) return fail(SCA_EINVAL, "n_factorised is NULL");
  DeviceGuard g(ctx, ctx->device);
  if ((s = check_dev_ptr(ctx, phi, "phi"))) return s;
  ProbDesc P = make_prob(p, phi, nullptr);
  if ((s = plan_tail(ctx, p, phi, P))) return s;
  *n_factorised = P.Me;
  return SCA_OK;
}

sca_status sca_shifted_terms(sca_ctx* ctx, const sca_params* p,
                             const double* phi, const double* z, int32_t n_z,
                             double* logabsdet, double* diag) {
  sca_status s = begin_call(ctx, p);
  if (s) return s;
  if (n_z < 1 || n_z > kMaxShifts)
    return fail(SCA_EINVAL, "n_z=%d: must be in [1, %d]", n_z, kMaxShifts);
  DeviceGuard g(ctx, ctx->device);
  if ((s = check_dev_ptr(ctx, phi, "phi"))) return s;
  if ((s = check_dev_ptr(ctx, z, "z"))) return s;
  if ((s = check_dev_ptr(ctx, logabsdet, "logabsdet"))) return s;
  if ((s = check_dev_ptr(ctx, diag, "diag"))) return s;
  const int N = p->L * p->L, B = 2 * n_z;
  const size_t fb = factor_workspace_bytes(N, B, route_of(p));
  Carve c0 = carve(nullptr, 1, N, B, route_of(p), false, false, fb);
  if ((s = ensure_ws(ctx, c0.total))) return s;
  Carve c = carve((char*)ctx->ws, 1, N, B, route_of(p), false, false, fb);
  ProbDesc P = make_prob(p, phi, nullptr);
  hipStream_t st = ctx->stream;
  if ((s = ensure_pinned(ctx, sizeof P))) return s;
  HIP_TRY(hipStreamSynchronize(st));
  std::memcpy(ctx->pinned, &P, sizeof P);
  HIP_TRY(hipMemcpyAsync(c.probs, ctx->pinned, sizeof P, hipMemcpyHostToDevice, st));
  HIP_TRY(launch_hvec(c.probs, 1, N, c.hbuf, st));
  HIP_TRY(launch_shift_descs(z, n_z, p->t, 0, N, c.descs, st));
  HIP_TRY(factor_batch(c.descs, c.hbuf, B, N, p->L, route_of(p), logabsdet,
                       diag, c.growth, c.fact, st, c.probs, 2));
  HIP_TRY(hipStreamSynchronize(st));
  return SCA_OK;
}

sca_status sca_dos(sca_ctx* ctx, const sca_params* p, const double* phi,
                   const double* w, int32_t n_w, double eta, double* rho) {
  sca_status s = begin_call(ctx, p);
  if (s) return s;
  if (n_w < 1 || n_w > kMaxShifts)
    return fail(SCA_EINVAL, "n_w=%d: must be in [1, %d]", n_w, kMaxShifts);
  if (!(eta > 0.0) || !std::isfinite(eta))
    return fail(SCA_EINVAL, "eta=%g: must be finite and > 0", eta);
  DeviceGuard g(ctx, ctx->device);
  if ((s = check_dev_ptr(ctx, phi, "phi"))) return s;
  if ((s = check_dev_ptr(ctx, w, "w"))) return s;
  if ((s = check_dev_ptr(ctx, rho, "rho"))) return s;
  const int N = p->L * p->L, B = 2 * n_w;
  const size_t fb = factor_workspace_bytes(N, B, route_of(p));
  // shifts z_j = w_j + i eta live after the carve
  Carve c0 = carve(nullptr, 1, N, B, route_of(p), true, true, fb);
  const size_t zoff = c0.total;
  if ((s = ensure_ws(ctx, zoff + align256(sizeof(double) * 2 * n_w)))) return s;
  Carve c = carve((char*)ctx->ws, 1, N, B, route_of(p), true, true, fb);
  double* zbuf = (double*)((char*)ctx->ws + zoff);
  ProbDesc P = make_prob(p, phi, nullptr);
  hipStream_t st = ctx->stream;
  if ((s = ensure_pinned(ctx, sizeof P))) return s;
  HIP_TRY(hipStreamSynchronize(st));
  std::memcpy(ctx->pinned, &P, sizeof P);
  HIP_TRY(hipMemcpyAsync(c.probs, ctx->pinned, sizeof P, hipMemcpyHostToDevice, st));
  HIP_TRY(launch_make_shifts(w, n_w, eta, zbuf, st));
  HIP_TRY(launch_hvec(c.probs, 1, N, c.hbuf, st));
  HIP_TRY(launch_shift_descs(zbuf, n_w, p->t, 0, N, c.descs, st));
  HIP_TRY(factor_batch(c.descs, c.hbuf, B, N, p->L, route_of(p), c.lad, c.dg,
                       c.growth, c.fact, st, c.probs, 2));
  HIP_TRY(launch_dos_reduce(c.dg, n_w, N, rho, st));
  HIP_TRY(hipStreamSynchronize(st));
  return SCA_OK;
}

size_t sca_factor_bytes(const sca_params* p) {
  std::string saved = g_err;
  if (validate_params(p) != SCA_OK) return 0;
  g_err = saved;
  if (p->factor == SCA_FACTOR_EIGH) return 0;   // no factors to keep
  const int N = p->L * p->L, B = 2 * p->n_max;
  const int mode = route_of(p);
  size_t bytes = autograd_factor_bytes(N, B, mode);
  // the FP32 route refactorises in FP64 (same layout up to the factors)
  // when its pivot growth is too large
  if ((mode & kModeFp32) && path_supported(N, mode & ~kModeFp32))
    bytes = std::max(bytes, autograd_factor_bytes(N, B, mode & ~kModeFp32));
  return bytes;
}

sca_status sca_factorize(sca_ctx* ctx, const sca_params* p, const double* phi,
                         void* factors, double* omega2) {
  sca_status s = begin_call(ctx, p);
  if (s) return s;
  if (p->factor == SCA_FACTOR_EIGH)
    return fail(SCA_EUNSUPPORTED, "the spectral route keeps no factors: use "
                "sca_potential / sca_grad");
  DeviceGuard g(ctx, ctx->device);
  if ((s = check_dev_ptr(ctx, phi, "phi"))) return s;
  if ((s = check_dev_ptr(ctx, factors, "factors"))) return s;
  if ((s = check_dev_ptr(ctx, omega2, "omega2"))) return s;
  const int N = p->L * p->L, B = 2 * p->n_max;
  ProbDesc P = make_prob(p, phi, nullptr);
  if ((s = plan_tail(ctx, p, phi, P))) return s;
  const int Be = 2 * P.Me;   // matrices factorised (the layout holds B)
  Carve c0 = carve(nullptr, 1, N, Be, route_of(p), false, false, 0);
  if ((s = ensure_ws(ctx, c0.total))) return s;
  Carve c = carve((char*)ctx->ws, 1, N, Be, route_of(p), false, false, 0);
  c.tail_on = P.Me < P.M;
  hipStream_t st = ctx->stream;
  if ((s = ensure_pinned(ctx, 512))) return s;
  HIP_TRY(hipStreamSynchronize(st));
  std::memcpy(ctx->pinned, &P, sizeof P);
  FactorHeader* hh = reinterpret_cast<FactorHeader*>(
      static_cast<char*>(ctx->pinned) + 256);
  HIP_TRY(hipMemcpyAsync(c.probs, ctx->pinned, sizeof P, hipMemcpyHostToDevice, st));
  HIP_TRY(launch_matsubara_descs(c.probs, 1, Be, c.descs, st));
  HIP_TRY(launch_hvec(c.probs, 1, N, c.hbuf, st));
  if (c.tail_on) HIP_TRY(launch_tail(c.probs, 1, N, c.hbuf, c.mom, c.tsum, st));
  // the FP32 route's factors are redone in FP64 when their pivot growth is
  // above the context's limit (the header records the route that was kept)
  int mode = route_of(p);
  ProbStats S;
  for (;;) {
    AutogradLayout lay = autograd_layout(factors, N, B, mode);
    HIP_TRY(factor_forward(c.descs, c.hbuf, Be, N, p->L, mode, lay.lad,
                           lay.dg, lay.growth, lay.fact, st));
    HIP_TRY(launch_reduce_omega(c.probs, 1, N, lay.lad, lay.growth, c.stats,
                                c.rws, c.mom, c.tsum, st));
    if ((s = read_stats(ctx, c, 1, &S))) return s;
    if (!growth_exceeded(ctx, mode, S.pivot_growth)) break;
    if (!path_supported(N, mode & ~kModeFp32))
      return fail(SCA_ENUMERIC, "FP32 pivot growth %.3g above %.3g and no "
                  "FP64 path for N=%d", S.pivot_growth, ctx->growth_limit, N);
    mode &= ~kModeFp32;
  }
  *hh = FactorHeader{kFactorsReady, p->L, p->n_max, mode, p->tail, P.Me,
                     P.tail_guard};
  HIP_TRY(hipMemcpyAsync(autograd_layout(factors, N, B, mode).head, hh,
                         sizeof *hh, hipMemcpyHostToDevice, st));
  double o2[2] = {S.omega, S.omega_tilde};
  HIP_TRY(hipMemcpyAsync(omega2, o2, sizeof o2, hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (!std::isfinite(S.omega) || !std::isfinite(S.omega_tilde))
    return fail(SCA_ENUMERIC, "non-finite potential");
  return SCA_OK;
}

sca_status sca_grad_from_factors(sca_ctx* ctx, const sca_params* p,
                                 const double* phi, void* factors,
                                 double* grad) {
  sca_status s = begin_call(ctx, p);
  if (s) return s;
  if (p->factor == SCA_FACTOR_EIGH)
    return fail(SCA_EUNSUPPORTED, "the spectral route keeps no factors: use "
                "sca_grad");
  DeviceGuard g(ctx, ctx->device);
  if ((s = check_dev_ptr(ctx, phi, "phi"))) return s;
  if ((s = check_dev_ptr(ctx, factors, "factors"))) return s;
  if ((s = check_dev_ptr(ctx, grad, "grad"))) return s;
  const int N = p->L * p->L, B = 2 * p->n_max;
  ProbDesc P = make_prob(p, phi, grad);
  hipStream_t st = ctx->stream;
  if ((s = ensure_pinned(ctx, 512))) return s;
  HIP_TRY(hipStreamSynchronize(st));
  FactorHeader* hh = reinterpret_cast<FactorHeader*>(
      static_cast<char*>(ctx->pinned) + 256);
  // the header sits at the start of every route's layout
  HIP_TRY(hipMemcpyAsync(hh, factors, sizeof *hh, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (hh->state == kFactorsConsumed)
    return fail(SCA_EINVAL, "factors were consumed by an earlier "
                "sca_grad_from_factors (this path inverts them in place); "
                "call sca_factorize again");
  // the FP32 route may have kept FP64 factors (pivot growth fallback)
  const int mode = hh->mode;
  const bool mode_ok = mode == route_of(p) ||
      ((route_of(p) & kModeFp32) && mode == (route_of(p) & ~kModeFp32));
  if (hh->state != kFactorsReady || hh->L != p->L || hh->n_max != p->n_max ||
      !mode_ok || hh->tail != p->tail || hh->Me < 1 || hh->Me > p->n_max)
    return fail(SCA_EINVAL, "factors do not hold a factorisation of these "
                "params (sca_factorize not called with them)");
  AutogradLayout lay = autograd_layout(factors, N, B, mode);
  // the frequencies the forward factorised; the tail again from phi
  P.Me = hh->Me;
  P.tail_guard = hh->tail_guard;
  const int Be = 2 * P.Me;
  Carve c0 = carve(nullptr, 1, N, Be, route_of(p), false, false, 0);
  if ((s = ensure_ws(ctx, c0.total))) return s;
  Carve c = carve((char*)ctx->ws, 1, N, Be, route_of(p), false, false, 0);
  c.tail_on = P.Me < P.M;
  std::memcpy(ctx->pinned, &P, sizeof P);
  HIP_TRY(hipMemcpyAsync(c.probs, ctx->pinned, sizeof P, hipMemcpyHostToDevice, st));
  if (c.tail_on) {
    HIP_TRY(launch_hvec(c.probs, 1, N, c.hbuf, st));
    HIP_TRY(launch_tail(c.probs, 1, N, c.hbuf, c.mom, c.tsum, st));
  }
  HIP_TRY(factor_backward(Be, N, mode, lay.lad, lay.dg, lay.fact, st));
  HIP_TRY(launch_reduce(c.probs, 1, N, lay.lad, lay.dg, lay.growth, c.stats,
                        false, c.rws, c.mom, c.tsum, st));
  if (factor_backward_consumes(N, mode)) {
    hh->state = kFactorsConsumed;
    HIP_TRY(hipMemcpyAsync(lay.head, hh, sizeof *hh, hipMemcpyHostToDevice,
                           st));
  }
  ProbStats S;
  if ((s = read_stats(ctx, c, 1, &S))) return s;
  if (S.nonfinite) return fail(SCA_ENUMERIC, "non-finite gradient");
  return SCA_OK;
}

sca_status sca_set_option(sca_ctx* ctx, int32_t option, double value) {
  g_err.clear();
  if (!ctx) return fail(SCA_EINVAL, "context is NULL");
  switch (option) {
    case SCA_OPT_FP32_GROWTH_LIMIT:
      if (!(value >= 1.0) || !std::isfinite(value))
        return fail(SCA_EINVAL, "growth limit %g: must be finite and >= 1",
                    value);
      ctx->growth_limit = value;
      return SCA_OK;
    default:
      return fail(SCA_EINVAL, "unknown option %d", option);
  }
}

sca_status sca_profile(sca_ctx* ctx, int enable) {
  g_err.clear();
  if (!ctx) return fail(SCA_EINVAL, "context is NULL");
  DeviceGuard g(ctx->device);
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  ctx->prof.resolve();
  if (enable) ctx->prof.reset();
  ctx->prof.on = enable != 0;
  return SCA_OK;
}

sca_status sca_profile_read(sca_ctx* ctx, double* total_ms,
                            int64_t* launches) {
  g_err.clear();
  if (!ctx) return fail(SCA_EINVAL, "context is NULL");
  if (!total_ms || !launches) return fail(SCA_EINVAL, "output is NULL");
  DeviceGuard g(ctx->device);
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  ctx->prof.resolve();
  for (int k = 0; k < SCA_PROFILE_SLOTS; ++k) {
    total_ms[k] = ctx->prof.total_ms[k];
    launches[k] = ctx->prof.launches[k];
  }
  return SCA_OK;
}

const char* sca_last_error(void) { return g_err.c_str(); }

}  // extern "C"
