// Host-side exercise of the C ABI's validation and error paths, for a build
// of the library's host code under AddressSanitizer and
// UndefinedBehaviorSanitizer (tests/test_abi_sanitize.py).  Needs no GPU:
// every call below is refused before any device work, or reports that no
// usable device exists.  Prints "OK" when every expectation held.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>

#include "sca.h"

static int failures = 0;

#define EXPECT(cond)                                                        \
  do {                                                                      \
    if (!(cond)) {                                                          \
      std::fprintf(stderr, "FAILED %s:%d: %s (last error: %s)\n", __FILE__,  \
                   __LINE__, #cond, sca_last_error());                      \
      ++failures;                                                           \
    }                                                                       \
  } while (0)

static sca_params params(int L, int n_max) {
  sca_params p;
  std::memset(&p, 0, sizeof p);
  p.L = L; p.n_max = n_max; p.precision = SCA_FP64; p.factor = SCA_FACTOR_LU;
  p.t = 1.0; p.U = 4.0; p.delta = 0.5; p.T = 0.1; p.onsite = nullptr;
  p.tail = SCA_TAIL_NONE; p.reserved = 0;
  return p;
}

int main(int argc, char** argv) {
  const bool no_gpu = argc > 1 && std::strcmp(argv[1], "--no-gpu") == 0;
  // sizes of valid parameter points on every route
  for (int L : {2, 4, 8, 10, 20, 32, 48, 64}) {
    for (int prec : {SCA_FP64, SCA_FP32_REFINED}) {
      for (int fac : {SCA_FACTOR_LU, SCA_FACTOR_LDLT, SCA_FACTOR_EIGH}) {
        sca_params p = params(L, 64);
        p.precision = prec;
        p.factor = fac;
        const size_t fb = sca_footprint_bytes(&p);
        const size_t ab = sca_factor_bytes(&p);
        (void)fb;
        (void)ab;
      }
    }
  }
  EXPECT(sca_footprint_bytes(nullptr) == 0);
  EXPECT(sca_factor_bytes(nullptr) == 0);

  // invalid parameter points: rejected (0 bytes, EINVAL with a message)
  const double nan = std::nan("");
  for (int k = 0; k < 14; ++k) {
    sca_params p = params(10, 32);
    switch (k) {
      case 0: p.L = 3; break;
      case 1: p.L = 0; break;
      case 2: p.L = 66; break;
      case 3: p.n_max = 0; break;
      case 4: p.n_max = -5; break;
      case 5: p.U = 0.0; break;
      case 6: p.U = nan; break;
      case 7: p.T = -1.0; break;
      case 8: p.t = INFINITY; break;
      case 9: p.precision = 9; break;
      case 10: p.factor = -1; break;
      case 11: p.tail = 7; break;
      case 12: p.reserved = 1; break;
      default: p.delta = nan; break;
    }
    EXPECT(sca_footprint_bytes(&p) == 0);
    EXPECT(sca_factor_bytes(&p) == 0);
  }

  // NULL context: every call refuses before touching a device
  sca_params p = params(10, 32);
  double d2[2];
  int32_t n = 0;
  sca_result res;
  sca_adam_opts o;
  std::memset(&o, 0, sizeof o);
  o.lr = 0.01; o.beta1 = 0.9; o.beta2 = 0.999; o.eps = 1e-8; o.n_steps = 3;
  sca_hmc_opts ho = {0.01, 2, 1};
  EXPECT(sca_potential(nullptr, &p, nullptr, d2) == SCA_EINVAL);
  EXPECT(std::string(sca_last_error()).find("context") != std::string::npos);
  EXPECT(sca_grad(nullptr, &p, nullptr, nullptr, nullptr) == SCA_EINVAL);
  EXPECT(sca_adam_solve(nullptr, &p, &o, nullptr, nullptr, nullptr, &res) ==
         SCA_EINVAL);
  EXPECT(sca_hmc(nullptr, &p, &ho, nullptr, nullptr, nullptr, nullptr, nullptr,
                 nullptr) == SCA_EINVAL);
  EXPECT(sca_dos(nullptr, &p, nullptr, nullptr, 4, 0.05, nullptr) == SCA_EINVAL);
  EXPECT(sca_shifted_terms(nullptr, &p, nullptr, nullptr, 2, nullptr,
                           nullptr) == SCA_EINVAL);
  EXPECT(sca_tail_split(nullptr, &p, nullptr, &n) == SCA_EINVAL);
  EXPECT(sca_factorize(nullptr, &p, nullptr, nullptr, nullptr) == SCA_EINVAL);
  EXPECT(sca_grad_from_factors(nullptr, &p, nullptr, nullptr, nullptr) ==
         SCA_EINVAL);
  EXPECT(sca_set_option(nullptr, SCA_OPT_FP32_GROWTH_LIMIT, 10.0) ==
         SCA_EINVAL);
  EXPECT(sca_profile(nullptr, 1) == SCA_EINVAL);
  double ms[SCA_PROFILE_SLOTS];
  int64_t cnt[SCA_PROFILE_SLOTS];
  EXPECT(sca_profile_read(nullptr, ms, cnt) == SCA_EINVAL);
  sca_destroy(nullptr);

  // server calls without a server
  sca_server* srv = nullptr;
  int64_t ticket = 0;
  int32_t a = 0, q = 0, done = 0;
  double td = 0.0;
  EXPECT(sca_server_create(0, 0, 0, &srv) == SCA_EINVAL);
  EXPECT(sca_server_create(0, 0, 5000, &srv) == SCA_EINVAL);
  EXPECT(sca_server_create(0, 0, 4, nullptr) == SCA_EINVAL);
  EXPECT(sca_server_submit(nullptr, &p, &o, nullptr, nullptr, nullptr,
                           &ticket) == SCA_EINVAL);
  EXPECT(sca_server_progress(nullptr, 0.0, &a, &q) == SCA_EINVAL);
  EXPECT(sca_server_poll(nullptr, 1, &done, &res, &td) == SCA_EINVAL);
  EXPECT(sca_server_clock(nullptr) == 0.0);
  sca_server_destroy(nullptr);

  // without a GPU: no context can be created, and nothing is written
  if (no_gpu) {
    sca_ctx* ctx = reinterpret_cast<sca_ctx*>(0x1);
    const sca_status st = sca_create(0, nullptr, 0, &ctx);
    EXPECT(st == SCA_EDEVICE || st == SCA_EINVAL);
    EXPECT(ctx == nullptr);
    EXPECT(sca_create(0, nullptr, 0, nullptr) == SCA_EINVAL);
    EXPECT(sca_server_create(0, 0, 4, &srv) == SCA_EDEVICE);
  }

  // the message is per thread
  (void)sca_grad(nullptr, &p, nullptr, nullptr, nullptr);
  std::string other;
  std::thread th([&] { other = sca_last_error(); });
  th.join();
  EXPECT(other.empty());
  EXPECT(!std::string(sca_last_error()).empty());

  if (failures) {
    std::fprintf(stderr, "%d expectation(s) failed\n", failures);
    return 1;
  }
  std::printf("OK\n");
  return 0;
}
