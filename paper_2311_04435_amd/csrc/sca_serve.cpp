// Request server: continuous batching of SCA+ADAM solves (see include/sca.h).
//
// Requests with the same (L, n_max, precision) share a group: one device
// workspace, one HIP stream, one batched evaluation pass per ADAM step over
// all of the group's problems (their matrices side by side in one launch;
// each problem keeps its own phi, moments, step counter and
// hyper-parameters on the device).  Groups of different shapes run
// concurrently on their own streams.  Membership only changes between
// chunks of passes, when the group's stream is idle: finished requests
// leave, queued ones join (first come, first served, as long as the group
// has room and its workspace fits the HBM budget).
//
// Every pass of a problem is computed exactly as in a batch of its own:
// each matrix is factorised by its own workgroup, and each problem's
// reductions run in a fixed order over its own matrices only, so a
// request's result does not depend on which others shared its batches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/sca.h"
#include "sca_common.h"
#include "sca_engine.h"
#include "sca_kernels.h"
#include "sca_runtime.h"

using namespace sca;

namespace {

constexpr double kChunkTargetMs = 2.0;   // aim of one chunk of passes
constexpr int kMaxChunk = 64;

// Batching more problems into one pass only pays while a pass is short
// (launch- and latency-bound): every matrix already has a workgroup of its
// own, so once one problem fills the GPU a bigger batch only makes all of
// its members wait for each other.  A group therefore takes as many
// problems as keep one pass near kPassFlops of factorisation work (about
// 2 ms at the rate the FP64 kernels reach on these sizes), at least one.
constexpr double kPassFlops = 3e10;
// The spectral route factorises nothing: a pass is one Householder
// reduction per spin (N dependent launches shared by every member) whose
// traffic, about 2 x 16 N^3 / 3 bytes per problem, bounds it once the
// launches are full; a group takes as many problems as keep that near
// kPassBytes.
constexpr double kPassBytes = 5e10;

int group_cap(int N, int M, int mode, int max_batch) {
  double cap;
  if (mode == kModeEig) {
    cap = std::floor(kPassBytes / (2.0 * 16.0 / 3.0 * (double)N * N * N));
  } else {
    const double per_problem = 2.0 * M * (16.0 / 3.0) * (double)N * N * N;
    cap = std::floor(kPassFlops / per_problem);
  }
  return (int)std::max(1.0, std::min((double)max_batch, cap));
}

struct Group;

struct Request {
  int64_t id = 0;
  sca_params p{};
  sca_adam_opts o{};
  double* phi = nullptr;
  double* m = nullptr;
  double* v = nullptr;
  int Me = 0;              // frequencies factorised (tail: < n_max)
  double tail_guard = 0.0;
  int applied = 0;        // ADAM updates applied (device count, last chunk)
  double gmax = 0.0;      // largest pivot growth seen
  Group* group = nullptr;
  bool done = false;
  double t_submit = 0.0, t_done = 0.0;
  sca_result res{};
};

struct Group {
  int L = 0, M = 0, precision = 0, N = 0, cap = 0;   // precision: route code
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  void* ws = nullptr;
  size_t bytes = 0;
  Carve c{};
  std::vector<Request*> mem;
  ProbDesc* pin_probs = nullptr;   // pinned staging, cap entries
  ProbStats* pin_stats = nullptr;
  bool dirty = true;
  bool inflight = false;
  int chunk = 0;                   // passes in flight
  double t_launch = 0.0;
  double pass_ms = 0.0;            // measured cost of one pass (0: unknown)

  Group() = default;
  Group(const Group&) = delete;
  Group& operator=(const Group&) = delete;
  ~Group() {
    if (st) (void)hipStreamSynchronize(st);
    if (ws) (void)hipFree(ws);
    if (pin_probs) (void)hipHostFree(pin_probs);
    if (pin_stats) (void)hipHostFree(pin_stats);
    if (ev) (void)hipEventDestroy(ev);
    if (st) (void)hipStreamDestroy(st);
  }
};

size_t group_bytes(int N, int M, int precision, int cap) {
  const int B = 2 * M * cap;
  return carve(nullptr, cap, N, B, precision, true, true,
               factor_workspace_bytes(N, B, precision, 2 * cap)).total;
}

}  // namespace

struct sca_server {
  int device = 0;
  size_t budget = 0;
  size_t used = 0;
  int max_batch = 1;
  std::chrono::steady_clock::time_point t0;
  int64_t next_id = 1;
  std::deque<Request*> queue;
  std::vector<std::unique_ptr<Group>> groups;
  std::unordered_map<int64_t, std::unique_ptr<Request>> reqs;
  double* dscalar = nullptr;   // device scratch of the tail planning
  bool broken = false;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0)
        .count();
  }
};

namespace {

struct DevScope {
  int prev = -1;
  explicit DevScope(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DevScope() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// Frees idle, empty groups until `need` more bytes fit the budget.
bool make_room(sca_server* s, size_t need) {
  if (s->used + need <= s->budget) return true;
  for (size_t k = 0; k < s->groups.size();) {
    Group* g = s->groups[k].get();
    if (!g->inflight && g->mem.empty()) {
      s->used -= g->bytes;
      s->groups.erase(s->groups.begin() + k);   // releases its memory
      if (s->used + need <= s->budget) return true;
    } else {
      ++k;
    }
  }
  return s->used + need <= s->budget;
}

// A new group for the shape of r, with as many problem slots as the budget
// allows (up to max_batch); nullptr if not even one fits now.
sca_status new_group(sca_server* s, const Request* r, Group** out) {
  *out = nullptr;
  const int N = r->p.L * r->p.L, M = r->p.n_max, prec = route_of(&r->p);
  auto fits = [&](int cap) {
    return s->used + group_bytes(N, M, prec, cap) <= s->budget;
  };
  int cap = group_cap(N, M, prec, s->max_batch);
  if (!fits(cap)) make_room(s, group_bytes(N, M, prec, cap));
  while (cap > 1 && !fits(cap)) cap /= 2;
  if (!fits(cap)) return SCA_OK;   // wait until a group frees its memory
  const size_t bytes = group_bytes(N, M, prec, cap);
  auto g = std::make_unique<Group>();
  g->L = r->p.L; g->M = M; g->precision = prec; g->N = N; g->cap = cap;
  g->bytes = bytes;
  SCA_HIP_TRY(hipStreamCreateWithFlags(&g->st, hipStreamNonBlocking));
  SCA_HIP_TRY(hipEventCreateWithFlags(&g->ev, hipEventDisableTiming));
  hipError_t e = hipMalloc(&g->ws, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    g->ws = nullptr;
    return fail(SCA_ENOMEM, "hipMalloc(%zu) for a request group failed: %s",
                bytes, hipGetErrorString(e));
  }
  SCA_HIP_TRY(hipHostMalloc((void**)&g->pin_probs, sizeof(ProbDesc) * cap,
                            hipHostMallocDefault));
  SCA_HIP_TRY(hipHostMalloc((void**)&g->pin_stats, sizeof(ProbStats) * cap,
                            hipHostMallocDefault));
  g->c = carve(static_cast<char*>(g->ws), cap, N, 2 * M * cap, prec, true,
               true, factor_workspace_bytes(N, 2 * M * cap, prec, 2 * cap));
  s->used += bytes;
  *out = g.get();
  s->groups.push_back(std::move(g));
  return SCA_OK;
}

Group* find_group(sca_server* s, const Request* r) {
  for (auto& g : s->groups)
    if (g->L == r->p.L && g->M == r->p.n_max &&
        g->precision == route_of(&r->p))
      return g.get();
  return nullptr;
}

// Queued requests join idle groups of their shape (first come, first
// served within each shape; a full or busy shape does not block others).
sca_status admit(sca_server* s) {
  for (auto it = s->queue.begin(); it != s->queue.end();) {
    Request* r = *it;
    Group* g = find_group(s, r);
    if (!g) {
      sca_status st = new_group(s, r, &g);
      if (st) return st;
      if (!g) { ++it; continue; }
    }
    if (g->inflight || (int)g->mem.size() >= g->cap) { ++it; continue; }
    r->group = g;
    g->mem.push_back(r);
    g->dirty = true;
    it = s->queue.erase(it);
  }
  return SCA_OK;
}

// Enqueue the next chunk of passes of an idle group with members.
sca_status launch(sca_server* s, Group* g) {
  const int n = (int)g->mem.size();
  int B = 0, max2M = 0;
  for (const Request* r : g->mem) { B += 2 * r->Me; max2M = std::max(max2M, 2 * r->Me); }
  g->c.tail_on = false;
  for (const Request* r : g->mem) g->c.tail_on |= r->Me < r->p.n_max;
  if (g->dirty) {
    int mb = 0;   // members' matrices side by side
    for (int k = 0; k < n; ++k) {
      const Request* r = g->mem[k];
      ProbDesc P = make_prob(&r->p, r->phi, nullptr);
      P.m = r->m; P.v = r->v; P.phi_out = r->phi;
      P.lr = r->o.lr; P.beta1 = r->o.beta1; P.beta2 = r->o.beta2;
      P.eps = r->o.eps;
      P.adam_t = r->o.t0 + r->applied;
      P.steps_left = r->o.n_steps - r->applied;
      P.Me = r->Me;
      P.tail_guard = r->tail_guard;
      P.mat_begin = mb;
      mb += 2 * r->Me;
      P.hoff = 2 * g->N * k;
      g->pin_probs[k] = P;
    }
    // the group is idle: no copy from pin_probs is pending
    SCA_HIP_TRY(hipMemcpyAsync(g->c.probs, g->pin_probs, sizeof(ProbDesc) * n,
                               hipMemcpyHostToDevice, g->st));
    SCA_HIP_TRY(launch_matsubara_descs(g->c.probs, n, max2M, g->c.descs,
                                       g->st));
    g->dirty = false;
  }
  // passes each member still needs if no guard holds one back; a chunk
  // never runs a member past its last one
  int left = kMaxChunk;
  for (const Request* r : g->mem) {
    const bool fe = !(r->o.flags & SCA_ADAM_NO_FINAL_EVAL);
    left = std::min(left, std::max(1, r->o.n_steps - r->applied + (fe ? 1 : 0)));
  }
  int K = 1;
  if (g->pass_ms > 0.0)
    K = std::max(1, std::min(left, (int)(kChunkTargetMs / g->pass_ms)));
  for (int k = 0; k < K; ++k)
    SCA_HIP_TRY(enqueue_pass(g->c, n, g->L, B, g->precision, true, g->st));
  SCA_HIP_TRY(hipMemcpyAsync(g->pin_stats, g->c.stats, sizeof(ProbStats) * n,
                             hipMemcpyDeviceToHost, g->st));
  SCA_HIP_TRY(hipEventRecord(g->ev, g->st));
  g->chunk = K;
  g->inflight = true;
  g->t_launch = s->now();
  return SCA_OK;
}

// A finished chunk.  The device counters say how many updates each member
// has applied (a pass whose tail guard fired applied none), so the switch
// of a tail member to every frequency happens at the pass where its guard
// fired, whatever the chunk length and whoever shares the group.  Members
// that reached their last pass retire with the statistics of that pass:
// the evaluation at the returned phi, or (SCA_ADAM_NO_FINAL_EVAL) the pass
// that applied the last update.
void complete(sca_server* s, Group* g) {
  const double t = s->now();
  const double ms = 1e3 * (t - g->t_launch) / g->chunk;
  g->pass_ms = g->pass_ms > 0.0 ? 0.5 * (g->pass_ms + ms) : ms;
  g->inflight = false;
  std::vector<Request*> keep;
  for (size_t k = 0; k < g->mem.size(); ++k) {
    Request* r = g->mem[k];
    const ProbStats& S = g->pin_stats[k];
    r->applied = S.adam_t - r->o.t0;
    r->gmax = max_nan(r->gmax, S.growth_run);
    const bool fe = !(r->o.flags & SCA_ADAM_NO_FINAL_EVAL);
    const bool finished =
        S.nonfinite ||
        (fe ? (r->applied == r->o.n_steps && !S.updated && S.guard == 0)
            : (r->applied == r->o.n_steps && (S.updated || S.guard == 0)));
    if (!finished && (S.guard & kGuardTail) && r->Me < r->p.n_max) {
      // the spectral bound left the tail's range: the following passes
      // factorise every frequency, from the step the guard held back
      r->res.flags |= SCA_FLAG_TAIL_RANGE;
      r->Me = r->p.n_max;
      r->tail_guard = 0.0;
      g->dirty = true;
    }
    if (!finished) { keep.push_back(r); continue; }
    r->res.omega = S.omega;
    r->res.omega_tilde = S.omega_tilde;
    r->res.af_order = S.af_order;
    r->res.max_abs_grad = S.max_abs_grad;
    r->res.max_pivot_growth = r->gmax;
    r->res.steps_done = r->applied;
    r->res.flags &= SCA_FLAG_TAIL_RANGE;
    if (S.nonfinite) r->res.flags |= SCA_FLAG_NONFINITE;
    if ((route_of(&r->p) & kModeFp32) && !(r->gmax <= 1e3))
      r->res.flags |= SCA_FLAG_PIVOT_GROWTH;
    r->done = true;
    r->t_done = t;
    r->group = nullptr;
  }
  if (keep.size() != g->mem.size()) {
    g->mem.swap(keep);
    g->dirty = true;
  }
}

// One scheduling round: retire finished chunks, admit, launch.
sca_status pump(sca_server* s, bool* progressed) {
  *progressed = false;
  for (auto& g : s->groups) {
    if (!g->inflight) continue;
    hipError_t e = hipEventQuery(g->ev);
    if (e == hipErrorNotReady) continue;
    if (e != hipSuccess) {
      s->broken = true;
      return fail(SCA_EDEVICE, "request group failed: %s",
                  hipGetErrorString(e));
    }
    complete(s, g.get());
    *progressed = true;
  }
  sca_status st = admit(s);
  if (st) return st;
  for (auto& g : s->groups) {
    if (g->inflight || g->mem.empty()) continue;
    st = launch(s, g.get());
    if (st) { s->broken = true; return st; }
  }
  return SCA_OK;
}

}  // namespace

extern "C" {

sca_status sca_server_create(int device, size_t hbm_budget_bytes,
                             int32_t max_batch, sca_server** out) {
  if (!out) return fail(SCA_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_batch < 1 || max_batch > 4096)
    return fail(SCA_EINVAL, "max_batch=%d: must be in [1, 4096]", max_batch);
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    (void)hipGetLastError();
    return fail(SCA_EDEVICE, "device %d not present", device);
  }
  DevScope d(device);
  hipDeviceProp_t prop;
  SCA_HIP_TRY(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(SCA_EDEVICE, "device %d is %s, not gfx950", device,
                prop.gcnArchName);
  size_t free_b = 0, total_b = 0;
  SCA_HIP_TRY(hipMemGetInfo(&free_b, &total_b));
  auto s = std::make_unique<sca_server>();
  s->device = device;
  s->budget = hbm_budget_bytes ? hbm_budget_bytes : free_b / 10 * 9;
  s->max_batch = max_batch;
  s->t0 = std::chrono::steady_clock::now();
  *out = s.release();
  return SCA_OK;
}

void sca_server_destroy(sca_server* s) {
  if (!s) return;
  DevScope d(s->device);
  s->groups.clear();
  if (s->dscalar) (void)hipFree(s->dscalar);
  delete s;
}

double sca_server_clock(const sca_server* s) { return s ? s->now() : 0.0; }

sca_status sca_server_submit(sca_server* s, const sca_params* p,
                             const sca_adam_opts* o, double* phi, double* m,
                             double* v, int64_t* ticket) {
  if (!s) return fail(SCA_EINVAL, "server is NULL");
  if (!ticket) return fail(SCA_EINVAL, "ticket is NULL");
  sca_status st = validate_params(p);
  if (st) return st;
  if ((st = validate_adam_opts(o))) return st;
  if (o->grad_tol != 0.0 || o->check_every != 0)
    return fail(SCA_EINVAL, "grad_tol and check_every are not supported by "
                "the server (requests run a fixed number of steps)");
  if ((st = check_device_ptr(s->device, p->onsite, "params.onsite", true)))
    return st;
  if ((st = check_device_ptr(s->device, phi, "phi", false))) return st;
  if ((st = check_device_ptr(s->device, m, "m", false))) return st;
  if ((st = check_device_ptr(s->device, v, "v", false))) return st;
  const size_t one = group_bytes(p->L * p->L, p->n_max, route_of(p), 1);
  if (one > s->budget)
    return fail(SCA_ENOMEM, "a request of L=%d needs %zu bytes, above the "
                "server budget of %zu", p->L, one, s->budget);
  auto r = std::make_unique<Request>();
  r->Me = p->n_max;
  if (p->tail == SCA_TAIL_MOMENTS) {
    // max|phi| (and max|onsite|) of the starting point; phi is ready (the
    // caller's contract), read on the null stream
    DevScope d(s->device);
    if (!s->dscalar) SCA_HIP_TRY(hipMalloc(&s->dscalar, sizeof(double)));
    double pm = 0.0, om = 0.0;
    SCA_HIP_TRY(launch_absmax(phi, p->L * p->L, s->dscalar, nullptr));
    SCA_HIP_TRY(hipMemcpy(&pm, s->dscalar, sizeof pm, hipMemcpyDeviceToHost));
    if (p->onsite) {
      SCA_HIP_TRY(launch_absmax(p->onsite, p->L * p->L, s->dscalar, nullptr));
      SCA_HIP_TRY(hipMemcpy(&om, s->dscalar, sizeof om, hipMemcpyDeviceToHost));
    }
    if (!std::isfinite(pm) || !std::isfinite(om))
      return fail(SCA_ENUMERIC, "phi or onsite is not finite");
    ProbDesc P{};
    tail_split(p, pm, om, P);
    r->Me = P.Me;
    r->tail_guard = P.tail_guard;
  }
  r->id = s->next_id++;
  r->p = *p;
  r->o = *o;
  r->phi = phi; r->m = m; r->v = v;
  r->t_submit = s->now();
  *ticket = r->id;
  s->queue.push_back(r.get());
  s->reqs.emplace(r->id, std::move(r));
  return SCA_OK;
}

sca_status sca_server_progress(sca_server* s, double wait_s,
                               int32_t* n_active, int32_t* n_queued) {
  if (!s) return fail(SCA_EINVAL, "server is NULL");
  if (s->broken) return fail(SCA_EDEVICE, "server stopped after a failure");
  DevScope d(s->device);
  bool prog = false;
  sca_status st = pump(s, &prog);
  if (st) return st;
  if (!prog && wait_s > 0.0) {
    const double until = s->now() + wait_s;
    bool any = false;
    for (auto& g : s->groups) any |= g->inflight;
    while (any && !prog && s->now() < until) {
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      if ((st = pump(s, &prog))) return st;
    }
  }
  int act = 0;
  for (auto& g : s->groups) act += (int)g->mem.size();
  if (n_active) *n_active = act;
  if (n_queued) *n_queued = (int32_t)s->queue.size();
  return SCA_OK;
}

sca_status sca_server_poll(sca_server* s, int64_t ticket, int32_t* done,
                           sca_result* res, double* t_done) {
  if (!s) return fail(SCA_EINVAL, "server is NULL");
  if (!done) return fail(SCA_EINVAL, "done is NULL");
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end())
    return fail(SCA_EINVAL, "unknown ticket %lld", (long long)ticket);
  Request* r = it->second.get();
  *done = r->done ? 1 : 0;
  if (!r->done) return SCA_OK;
  if (res) *res = r->res;
  if (t_done) *t_done = r->t_done;
  s->reqs.erase(it);
  return SCA_OK;
}

}  // extern "C"
