// Driver of the host emulation of the blocked factor kernels (k_factor.hip:
// pivoted LU, triangular inverses, diagonal of the inverse; k_refine.hip:
// the W V product and the FP64 refinement).  The kernel sources are
// included after a mechanical rewrite (tests/test_kernel_emu.py: dynamic
// LDS declarations become pointers to the emulator's LDS block,
// register-pinning asm statements and occupancy attributes are dropped), and
// launched through the library's own dispatch, so the launch configuration
// is the product's.
//
//   factor_emu <config> <input> <output> <order>
//
// config: f64:<cfg> or f32:<cfg> (the instance blocked_lu_f64/_f32 run for
// that cfg), or f32:16x9 (16 waves x 9 row tiles, block width 16: an
// instance the library does not ship); f32r:<cfg> runs the refined route
// (k_refine.hip) in place of the plain diagonal.  order: 0 forward,
// 1 reverse, 2 random scheduling of lanes and waves.
// input (little endian): int32 B, N, L, Np; double t; B x (zr, zi);
// B x N doubles h.  output: double lad[B], growth[B], dg[B][N][2]; int32
// perm[B][Np].
#include "k_factor_emu.cc"
#include "k_refine_emu.cc"

#include <cstdio>
#include <string>
#include <vector>

namespace sca {
bool roctx_enabled() { return false; }
void roctx_push(int) {}
void roctx_pop() {}
Profiler*& current_profiler() {
  static Profiler* p = nullptr;
  return p;
}
void Profiler::begin(int, hipStream_t) {}
void Profiler::end(int, hipStream_t) {}
}  // namespace sca

namespace {

template <class T>
std::vector<T> poisoned(size_t n) {
  std::vector<T> v(n);
  std::memset(v.data(), 0xFF, n * sizeof(T));   // NaN / -1
  return v;
}

template <class T>
int run(const std::string& inst, bool refined, int B, int N, int L, int Np,
        const std::vector<sca::MatDesc>& descs, const std::vector<double>& h,
        std::vector<double>& lad, std::vector<double>& growth,
        std::vector<double>& dg, std::vector<int>& perm) {
  const bool f32 = std::is_same<T, float>::value;
  int cfg = -1;
  int NB = 16;
  if (inst != "16x9") {
    cfg = std::stoi(inst);
    NB = (cfg == 0 || cfg == 1 || (f32 && (cfg == 2 || cfg == 4))) ? 32 : 16;
  }
  if (Np % NB || Np < N) {
    std::fprintf(stderr, "Np %d does not fit block width %d\n", Np, NB);
    return 2;
  }
  const sca::BlockedPlan plan{cfg, NB, Np};
  auto F = poisoned<T>((size_t)B * 2 * Np * Np);
  auto tri = poisoned<T>((size_t)B * (Np / NB) * 4 * NB * NB);
  perm = poisoned<int>((size_t)B * Np);
  lad = poisoned<double>(B);
  growth = poisoned<double>(B);
  dg = poisoned<double>((size_t)B * N * 2);
  hipError_t e;
  if constexpr (std::is_same<T, double>::value) {
    e = sca::blocked_lu_f64(plan, descs.data(), h.data(), B, N, L, F.data(),
                            perm.data(), tri.data(), lad.data(), growth.data(),
                            nullptr);
    if (e == hipSuccess)
      e = sca::blocked_inv_f64(plan, B, N, F.data(), perm.data(), tri.data(),
                               dg.data(), nullptr);
  } else {
    if (inst == "16x9") {
      e = sca::run_lu<float, 16, 9, 1>(descs.data(), h.data(), B, N, Np, L,
                                        F.data(), perm.data(), tri.data(),
                                        lad.data(), growth.data(), nullptr);
      if (e == hipSuccess)
        e = sca::run_trtri<float, 16, 9, 1>(B, Np, F.data(), perm.data(),
                                             tri.data(), nullptr);
    } else {
      e = sca::blocked_lu_f32(plan, descs.data(), h.data(), B, N, L, F.data(),
                              perm.data(), tri.data(), lad.data(),
                              growth.data(), nullptr);
      if (e == hipSuccess)
        e = sca::blocked_trtri_f32(plan, B, F.data(), perm.data(), tri.data(),
                                   nullptr);
    }
    if (e == hipSuccess && !refined)
      e = sca::run_diagdot<float>(B, N, Np, F.data(), perm.data(), dg.data(),
                                  nullptr);
    if (e == hipSuccess && refined) {
      // the refined route: X = fl32(W V) stored transposed, the FP64 Newton
      // diagonal and the refined log-determinant
      auto XT = poisoned<float>((size_t)B * 2 * Np * Np);   // re, im planes
      auto parts = poisoned<double>((size_t)B * sca::refine_parts(Np));
      e = sca::launch_wv_gemm(B, N, Np, L, descs.data(), h.data(), F.data(),
                              perm.data(), XT.data(), parts.data(), nullptr);
      if (e == hipSuccess)
        e = sca::launch_refine(B, N, Np, L, descs.data(), h.data(), F.data(),
                               perm.data(), XT.data(), dg.data(), parts.data(),
                               lad.data(), nullptr);
    }
  }
  (void)f32;
  return e == hipSuccess ? 0 : 3;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 5) {
    std::fprintf(stderr, "usage: factor_emu config input output order\n");
    return 2;
  }
  const std::string config = argv[1];
  const auto colon = config.find(':');
  if (colon == std::string::npos) return 2;
  const std::string prec = config.substr(0, colon), inst = config.substr(colon + 1);
  emu::order_mode() = std::stoi(argv[4]);

  FILE* in = std::fopen(argv[2], "rb");
  if (!in) return 2;
  int32_t hdr[4];
  double t = 0.0;
  if (std::fread(hdr, sizeof hdr, 1, in) != 1 || std::fread(&t, 8, 1, in) != 1)
    return 2;
  const int B = hdr[0], N = hdr[1], L = hdr[2], Np = hdr[3];
  std::vector<double> z(2 * (size_t)B), h((size_t)B * N);
  if (std::fread(z.data(), 8, z.size(), in) != z.size() ||
      std::fread(h.data(), 8, h.size(), in) != h.size())
    return 2;
  std::fclose(in);
  std::vector<sca::MatDesc> descs(B);
  for (int b = 0; b < B; ++b) {
    descs[b].zr = z[2 * b];
    descs[b].zi = z[2 * b + 1];
    descs[b].t = t;
    descs[b].hoff = b * N;
    descs[b].prob = 0;
  }
  std::vector<double> lad, growth, dg;
  std::vector<int> perm;
  const int rc = prec == "f64"
                     ? run<double>(inst, false, B, N, L, Np, descs, h, lad, growth, dg, perm)
                 : prec == "f32" || prec == "f32r"
                     ? run<float>(inst, prec == "f32r", B, N, L, Np, descs, h, lad, growth, dg, perm)
                     : 2;
  if (rc) return rc;
  FILE* out = std::fopen(argv[3], "wb");
  if (!out) return 2;
  std::fwrite(lad.data(), 8, lad.size(), out);
  std::fwrite(growth.data(), 8, growth.size(), out);
  std::fwrite(dg.data(), 8, dg.size(), out);
  std::fwrite(perm.data(), 4, perm.size(), out);
  std::fclose(out);
  std::printf("barriers %lld wave-ops %lld\n", emu::total_barriers(),
              emu::total_waveops());
  return 0;
}
