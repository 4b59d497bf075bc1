// Host emulation of the HIP execution model for the library's kernels (test
// infrastructure: tests/test_kernel_emu.py).  A launch runs its workgroups
// one after another; in a workgroup every thread is a fiber with its own
// stack, and the scheduler resumes them in a chosen order until each blocks
// at a workgroup barrier, blocks in a cross-lane operation or returns.
//
//   * __syncthreads releases when every thread that has not returned waits
//     at it.
//   * The cross-lane operations of a 64-lane wave (MFMA, readlane,
//     readfirstlane, shfl, shfl_up, shfl_xor, ballot, DPP, wave_barrier) are
//     rendezvous: all 64 lanes of the wave deposit their operands and the
//     last to arrive computes every lane's result.  Lanes of one wave that
//     arrive at different operations, a non-uniform readlane index, a
//     barrier that not all threads reach: each is reported as an error.
//   * Between two synchronisation points the lanes and waves run one after
//     the other in the scheduler's order (forward, reverse, or a seeded
//     random order re-drawn at every pass).  A kernel whose results differ
//     between orders reads shared memory that another thread writes without
//     a barrier between them.
//
// Memory: dynamic LDS is a heap block of exactly the launch's size, filled
// with 0xFF bytes (NaN for floating point, -1 for integers), so that under
// AddressSanitizer any access outside it is reported and reads of LDS the
// kernel never wrote show up as NaN in its results.  Static __shared__
// arrays become function-local statics (one workgroup runs at a time).
//
// Not modelled: the lockstep of a wave between synchronisation points (a
// kernel relying on it without a wave barrier shows up as order-dependent
// here), memory ordering beyond program order, and timing.
#pragma once
#include <sys/mman.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <random>
#include <tuple>
#include <vector>

#if defined(__has_feature)
#if __has_feature(address_sanitizer)
#define EMU_ASAN 1
#endif
#endif
#ifdef EMU_ASAN
extern "C" {
void __sanitizer_start_switch_fiber(void** fake_stack_save, const void* bottom,
                                    size_t size);
void __sanitizer_finish_switch_fiber(void* fake_stack_save,
                                     const void** bottom_old, size_t* size_old);
void __asan_unpoison_memory_region(void const volatile* addr, size_t size);
}
#endif

// x86-64 System V context switch: saves the callee-saved registers on the
// current stack, stores the stack pointer to *save, continues on `to`
// (weak: every translation unit that includes this header defines it).
extern "C" void emu_ctx_switch(void** save, void* to);
asm(R"(
  .text
  .weak emu_ctx_switch
  .type emu_ctx_switch, @function
emu_ctx_switch:
  pushq %rbp
  pushq %rbx
  pushq %r12
  pushq %r13
  pushq %r14
  pushq %r15
  movq %rsp, (%rdi)
  movq %rsi, %rsp
  popq %r15
  popq %r14
  popq %r13
  popq %r12
  popq %rbx
  popq %rbp
  ret
  .size emu_ctx_switch, .-emu_ctx_switch
)");

struct dim3 {
  unsigned x, y, z;
  constexpr dim3(unsigned x_ = 1, unsigned y_ = 1, unsigned z_ = 1)
      : x(x_), y(y_), z(z_) {}
};

namespace emu {

[[noreturn]] inline void fail(const char* what) {
  std::fprintf(stderr, "EMU ERROR: %s\n", what);
  std::fflush(stderr);
  std::abort();
}

enum State { kReady, kWaveOp, kBarrier, kDone };
enum Op {
  kNone, kReadlane, kReadfirstlane, kShfl, kShflUp, kShflXor, kBallot, kDpp,
  kMfmaF32, kMfmaF64, kWaveBarrier
};

constexpr size_t kStackBytes = size_t(512) << 10;
constexpr size_t kMaxLds = size_t(160) << 10;   // LDS of one gfx950 CU

struct Fiber {
  void* sp = nullptr;
  char* base = nullptr;   // mapping: guard page, then the stack
  State st = kReady;
  void* fake = nullptr;
  dim3 tidx;
  int lane = 0, wave = 0;
};

struct Wave {
  int arrived = 0;
  int op[64];
  int ip[64];                  // per-lane integer parameter
  uint64_t in[64][4], in2[64]; // operands (bit patterns)
  double acc[64][4];           // MFMA accumulators in / out
  uint64_t out[64];
};

struct Block {
  std::vector<Fiber> fibers;
  std::vector<Wave> waves;
  dim3 bidx, bdim, gdim;
  void* lds = nullptr;
  size_t lds_bytes = 0;
  std::function<void()> body;
  void* sched_sp = nullptr;
  void* sched_fake = nullptr;
  const void* main_bottom = nullptr;
  size_t main_size = 0;
  int nthreads = 0;
  long long barriers = 0, waveops = 0;
};

inline Block*& blk() { static Block* b = nullptr; return b; }
inline Fiber*& cur() { static Fiber* f = nullptr; return f; }
// scheduling order: 0 forward, 1 reverse, 2 seeded random per pass
inline int& order_mode() { static int m = 0; return m; }
inline std::mt19937_64& order_rng() { static std::mt19937_64 r(12345); return r; }
inline long long& total_waveops() { static long long n = 0; return n; }
inline long long& total_barriers() { static long long n = 0; return n; }

inline char* stack_pool(size_t i) {
  static std::vector<char*> pool;
  while (pool.size() <= i) {
    const size_t page = 4096;
    void* m = mmap(nullptr, kStackBytes + page, PROT_READ | PROT_WRITE,
                   MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
    if (m == MAP_FAILED) fail("cannot map a fiber stack");
    mprotect(m, page, PROT_NONE);   // overflow guard below the stack
    pool.push_back(static_cast<char*>(m));
  }
  return pool[i];
}

// back to the scheduler (from a fiber)
inline void yield_to_sched(bool exiting = false) {
  Block* b = blk();
  Fiber* f = cur();
#ifdef EMU_ASAN
  __sanitizer_start_switch_fiber(exiting ? nullptr : &f->fake, b->main_bottom,
                                 b->main_size);
#else
  (void)exiting;
#endif
  emu_ctx_switch(&f->sp, b->sched_sp);
#ifdef EMU_ASAN
  __sanitizer_finish_switch_fiber(f->fake, &b->main_bottom, &b->main_size);
#endif
}

extern "C" inline void emu_fiber_entry() {
  Block* b = blk();
#ifdef EMU_ASAN
  __sanitizer_finish_switch_fiber(nullptr, &b->main_bottom, &b->main_size);
#endif
  b->body();
  cur()->st = kDone;
  yield_to_sched(true);
  fail("a finished fiber was resumed");
}

inline void resume(Block* b, Fiber* f) {
  cur() = f;
#ifdef EMU_ASAN
  __sanitizer_start_switch_fiber(&b->sched_fake, f->base + 4096, kStackBytes);
#endif
  emu_ctx_switch(&b->sched_sp, f->sp);
#ifdef EMU_ASAN
  __sanitizer_finish_switch_fiber(b->sched_fake, nullptr, nullptr);
#endif
  cur() = nullptr;
}

inline void init_fiber(Fiber& f, char* base) {
  f.base = base;
#ifdef EMU_ASAN
  // a reused stack may still carry the poisoned redzones of earlier frames
  __asan_unpoison_memory_region(base + 4096, kStackBytes);
#endif
  char* top = base + 4096 + kStackBytes;
  uintptr_t s = (reinterpret_cast<uintptr_t>(top) - 64) & ~uintptr_t(15);
  void** slot = reinterpret_cast<void**>(s);
  slot[0] = reinterpret_cast<void*>(&emu_fiber_entry);   // popped by ret
  slot[1] = nullptr;                                      // entry's return
  for (int r = 1; r <= 6; ++r) slot[-r] = nullptr;        // saved registers
  f.sp = slot - 6;
  f.st = kReady;
  f.fake = nullptr;
}

inline void report_deadlock(Block* b) {
  std::fprintf(stderr, "EMU ERROR: no thread can proceed in block (%u,%u,%u)\n",
               b->bidx.x, b->bidx.y, b->bidx.z);
  for (size_t w = 0; w < b->waves.size(); ++w) {
    int cnt[4] = {0, 0, 0, 0};
    for (int l = 0; l < 64; ++l) {
      const size_t t = w * 64 + l;
      if (t < b->fibers.size()) ++cnt[b->fibers[t].st];
    }
    std::fprintf(stderr, "  wave %zu: ready %d, in a wave op %d (arrived %d), "
                 "at the barrier %d, returned %d\n", w, cnt[0], cnt[1],
                 b->waves[w].arrived, cnt[2], cnt[3]);
  }
  fail("deadlock (divergent barrier or cross-lane operation)");
}

inline void run_block(Block* b) {
  const int nt = b->nthreads;
  const int nw = (nt + 63) / 64;
  b->fibers.assign(nt, Fiber{});
  b->waves.assign(nw, Wave{});
  for (int t = 0; t < nt; ++t) {
    init_fiber(b->fibers[t], stack_pool(t));
    b->fibers[t].tidx = dim3(t % b->bdim.x, (t / b->bdim.x) % b->bdim.y,
                             t / (b->bdim.x * b->bdim.y));
    b->fibers[t].lane = t % 64;
    b->fibers[t].wave = t / 64;
  }
  std::vector<int> wo(nw), lo(64);
  for (;;) {
    for (int i = 0; i < nw; ++i) wo[i] = i;
    for (int i = 0; i < 64; ++i) lo[i] = i;
    if (order_mode() == 1) {
      std::reverse(wo.begin(), wo.end());
      std::reverse(lo.begin(), lo.end());
    } else if (order_mode() == 2) {
      std::shuffle(wo.begin(), wo.end(), order_rng());
      std::shuffle(lo.begin(), lo.end(), order_rng());
    }
    bool progress = false;
    for (int wi : wo)
      for (int li : lo) {
        const int t = wi * 64 + li;
        if (t < nt && b->fibers[t].st == kReady) {
          resume(b, &b->fibers[t]);
          progress = true;
        }
      }
    if (progress) continue;
    int done = 0, at_bar = 0;
    for (const Fiber& f : b->fibers) {
      done += f.st == kDone;
      at_bar += f.st == kBarrier;
    }
    if (done == nt) break;
    if (done + at_bar == nt) {   // the barrier releases
      for (Fiber& f : b->fibers)
        if (f.st == kBarrier) f.st = kReady;
      ++b->barriers;
      continue;
    }
    report_deadlock(b);
  }
}

template <class... P, class... A>
void launch(void (*k)(P...), dim3 grid, dim3 block, size_t lds, A... args) {
  const unsigned nt = block.x * block.y * block.z;
  if (nt == 0 || nt > 1024) fail("workgroup size outside 1..1024");
  if (lds > kMaxLds) fail("dynamic LDS above 160 KiB");
  std::tuple<P...> tp(static_cast<P>(args)...);
  for (unsigned z = 0; z < grid.z; ++z)
    for (unsigned y = 0; y < grid.y; ++y)
      for (unsigned x = 0; x < grid.x; ++x) {
        Block b;
        b.bidx = dim3(x, y, z);
        b.bdim = block;
        b.gdim = grid;
        b.nthreads = (int)nt;
        b.lds_bytes = lds;
        b.lds = lds ? std::malloc(lds) : nullptr;
        if (lds) std::memset(b.lds, 0xFF, lds);
        b.body = [&]() { std::apply(k, tp); };
        blk() = &b;
        run_block(&b);
        blk() = nullptr;
        total_barriers() += b.barriers;
        total_waveops() += b.waveops;
        std::free(b.lds);
      }
}

inline void* lds() {
  Block* b = blk();
  if (!b->lds) fail("dynamic LDS used by a launch that requested none");
  return b->lds;
}

// ---- cross-lane operations -------------------------------------------------

inline Wave& my_wave() { return blk()->waves[cur()->wave]; }

// Deposit this lane's operands (already stored in the wave), then wait for
// the wave.  The last lane to arrive checks that every lane is at the same
// operation and computes all results with `finish`.
template <class F>
inline void arrive(Op op, F finish) {
  Block* b = blk();
  Fiber* f = cur();
  Wave& w = b->waves[f->wave];
  w.op[f->lane] = op;
  int live = 0;
  for (int l = 0; l < 64; ++l) {
    const size_t t = (size_t)f->wave * 64 + l;
    live += t < b->fibers.size() && b->fibers[t].st != kDone;
  }
  if (live != 64) fail("cross-lane operation in a wave with returned lanes");
  if (++w.arrived == 64) {
    for (int l = 0; l < 64; ++l)
      if (w.op[l] != op) fail("lanes of a wave at different cross-lane operations");
    finish(w);
    w.arrived = 0;
    ++b->waveops;
    for (int l = 0; l < 64; ++l) {
      Fiber& g = b->fibers[(size_t)f->wave * 64 + l];
      if (g.st == kWaveOp) g.st = kReady;
    }
  } else {
    f->st = kWaveOp;
    yield_to_sched();
  }
}

template <class T> inline uint64_t bits(T v) {
  static_assert(sizeof(T) <= 8, "cross-lane value wider than 8 bytes");
  uint64_t u = 0;
  std::memcpy(&u, &v, sizeof(T));
  return u;
}
template <class T> inline T from_bits(uint64_t u) {
  T v;
  std::memcpy(&v, &u, sizeof(T));
  return v;
}

inline void syncthreads() {
  cur()->st = kBarrier;
  yield_to_sched();
}

inline void wave_barrier() {
  arrive(kWaveBarrier, [](Wave&) {});
}

template <class T> inline T readlane(T v, int src) {
  Wave& w = my_wave();
  const int me = cur()->lane;
  w.in[me][0] = bits(v);
  w.ip[me] = src;
  arrive(kReadlane, [](Wave& w) {
    for (int l = 1; l < 64; ++l)
      if (w.ip[l] != w.ip[0]) fail("readlane with a non-uniform lane index");
    if (w.ip[0] < 0 || w.ip[0] > 63) fail("readlane index outside 0..63");
    for (int l = 0; l < 64; ++l) w.out[l] = w.in[w.ip[0]][0];
  });
  return from_bits<T>(w.out[me]);
}

template <class T> inline T readfirstlane(T v) {
  Wave& w = my_wave();
  const int me = cur()->lane;
  w.in[me][0] = bits(v);
  arrive(kReadfirstlane, [](Wave& w) {
    for (int l = 0; l < 64; ++l) w.out[l] = w.in[0][0];
  });
  return from_bits<T>(w.out[me]);
}

template <class T> inline T shfl(T v, int src, int width = 64) {
  Wave& w = my_wave();
  const int me = cur()->lane;
  if (width != 64) fail("shfl width other than 64");
  w.in[me][0] = bits(v);
  w.ip[me] = src & 63;
  arrive(kShfl, [](Wave& w) {
    for (int l = 0; l < 64; ++l) w.out[l] = w.in[w.ip[l]][0];
  });
  return from_bits<T>(w.out[me]);
}

template <class T> inline T shfl_up(T v, unsigned delta, int width = 64) {
  Wave& w = my_wave();
  const int me = cur()->lane;
  if (width != 64) fail("shfl_up width other than 64");
  w.in[me][0] = bits(v);
  w.ip[me] = me >= (int)delta ? me - (int)delta : me;   // below 0: own value
  arrive(kShflUp, [](Wave& w) {
    for (int l = 0; l < 64; ++l) w.out[l] = w.in[w.ip[l]][0];
  });
  return from_bits<T>(w.out[me]);
}

template <class T> inline T shfl_xor(T v, int mask, int width = 64) {
  Wave& w = my_wave();
  const int me = cur()->lane;
  if (width != 64) fail("shfl_xor width other than 64");
  w.in[me][0] = bits(v);
  w.ip[me] = (me ^ mask) & 63;
  arrive(kShflXor, [](Wave& w) {
    for (int l = 0; l < 64; ++l) w.out[l] = w.in[w.ip[l]][0];
  });
  return from_bits<T>(w.out[me]);
}

inline unsigned long long ballot(int pred) {
  Wave& w = my_wave();
  const int me = cur()->lane;
  w.ip[me] = pred != 0;
  arrive(kBallot, [](Wave& w) {
    uint64_t m = 0;
    for (int l = 0; l < 64; ++l) m |= uint64_t(w.ip[l]) << l;
    for (int l = 0; l < 64; ++l) w.out[l] = m;
  });
  return w.out[me];
}

// v_mov_dpp with all rows and banks enabled: quad permutations (controls
// 0x00-0xFF), row mirror (0x140) and half-row mirror (0x141).
inline int update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask,
                      bool bound_ctrl) {
  (void)old;
  (void)bound_ctrl;
  if (row_mask != 0xF || bank_mask != 0xF) fail("DPP with masked rows or banks");
  Wave& w = my_wave();
  const int me = cur()->lane;
  w.in[me][0] = bits(src);
  w.ip[me] = ctrl;
  arrive(kDpp, [](Wave& w) {
    const int c = w.ip[0];
    for (int l = 1; l < 64; ++l)
      if (w.ip[l] != c) fail("DPP control not uniform");
    for (int l = 0; l < 64; ++l) {
      int s;
      if (c <= 0xFF) s = (l & ~3) | ((c >> (2 * (l & 3))) & 3);
      else if (c == 0x140) s = (l & ~15) | (15 - (l & 15));
      else if (c == 0x141) s = (l & ~7) | (7 - (l & 7));
      else fail("DPP control not modelled");
      w.out[l] = w.in[s][0];
    }
  });
  return from_bits<int>(w.out[me]);
}

// v_mfma_{f32,f64}_16x16x4: A[m][k] from lane (k<<4 | m), B[k][n] from lane
// (k<<4 | n); lane (g<<4 | n) holds accumulator rows g + 4i (f64) or 4g + i
// (f32), i = 0..3, of column n.
template <class V, class S, bool kF64>
inline V mfma(S a, S b, V c) {
  Wave& w = my_wave();
  const int me = cur()->lane;
  w.in[me][0] = bits(a);
  w.in[me][1] = bits(b);
  for (int i = 0; i < 4; ++i) w.acc[me][i] = (double)c[i];
  arrive(kF64 ? kMfmaF64 : kMfmaF32, [](Wave& w) {
    S A[16][4], B[4][16];
    for (int l = 0; l < 64; ++l) {
      A[l & 15][l >> 4] = from_bits<S>(w.in[l][0]);
      B[l >> 4][l & 15] = from_bits<S>(w.in[l][1]);
    }
    double out[64][4];
    for (int l = 0; l < 64; ++l) {
      const int g = l >> 4, n = l & 15;
      for (int i = 0; i < 4; ++i) {
        const int m = kF64 ? g + 4 * i : 4 * g + i;
        S s = (S)w.acc[l][i];
        for (int k = 0; k < 4; ++k) s = std::fma(A[m][k], B[k][n], s);
        out[l][i] = (double)s;
      }
    }
    std::memcpy(w.acc, out, sizeof out);
  });
  V r;
  for (int i = 0; i < 4; ++i) r[i] = (S)w.acc[me][i];
  return r;
}

}  // namespace emu
