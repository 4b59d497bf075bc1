// Shared device/host definitions of the SCA library (gfx950).
//
// A batch is a list of complex matrices A_b = z_b I - H_b, where
//   H_b = -t_b K + diag(h_b),   K = periodic nearest-neighbour adjacency of
// the L x L lattice (site i = x + L*y; K_ij counts the directions +-x, +-y
// that map i to j, so K_ij = 2 on L = 2).  h_b is the real diagonal
// (Delta/2) (-1)^(x+y) - s phi_i (+ onsite_i) of spin s (Sec. II, Eq. (1)
// after the static Hubbard-Stratonovich decoupling of Eqs. (5)-(7)).
// A is generated on chip from (z_b, t_b, h_b); it is never read from HBM.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sca {

struct MatDesc {
  double zr, zi;   // shift z_b
  double t;        // hopping
  int32_t hoff;    // offset (doubles) of h_b in the diagonal buffer
  int32_t prob;    // owning problem
};

struct ProbDesc {
  const double* phi;     // [N] field
  const double* onsite;  // [N] extra site potential or nullptr
  double* grad;          // [N] gradient output (may be nullptr)
  double* m;             // [N] ADAM first moment (adam only)
  double* v;             // [N] ADAM second moment (adam only)
  double* phi_out;       // [N] updated field (adam only; may alias phi)
  double t, U, delta, T;
  double lr, beta1, beta2, eps;   // ADAM hyper-parameters
  int32_t L, N, M;       // lattice side, sites, Matsubara count
  int32_t mat_begin;     // matrices [mat_begin, mat_begin + 2M): up then down
  int32_t hoff;          // h vectors: up at hoff, down at hoff + N
  int32_t adam_t;        // ADAM updates applied so far (next uses adam_t + 1)
  int32_t steps_left;    // updates still to apply; 0: evaluate only
  int32_t Me;            // frequencies factorised (n < Me); n in [Me, M) by
                         // the moment expansion of the tail (Me == M: none)
  double tail_guard;     // tail only: flag a pass whose Gershgorin bound on
                         // the spectral radius of H exceeds this
  // Hybrid Monte Carlo (hmc_L > 0): pass k of a trajectory evaluates the
  // force at phi_k, then p -= c_k grad/T (c_0 = c_L = eps/2, else eps) and,
  // for k < L, phi += eps p
  double* pmom;          // [N] momentum
  double hmc_eps;        // leapfrog step
  int32_t hmc_L;         // leapfrog steps per trajectory (0: no HMC)
  int32_t hmc_k;         // passes done in the current trajectory
  // Guards.  A pass is out of range when the Gershgorin bound of its H
  // exceeds tail_guard (tail only) or, when growth_limit > 0, when the
  // largest pivot growth of the problem's matrices exceeds growth_limit
  // (or is not finite).  Such a pass applies no ADAM update and advances
  // no counter, so the caller can re-plan the problem and resume from the
  // same step, whatever number of passes it had queued behind it.
  double growth_limit;
  double growth_run;     // running max of the pivot growth over passes
};

// ProbStats::guard bits
constexpr int32_t kGuardTail = 1;     // tail's spectral bound exceeded
constexpr int32_t kGuardGrowth = 2;   // pivot growth above growth_limit

// Matsubara tail by moments.  For w > rho(H),
//   ln|det(i w - H)| = N ln w + 1/2 sum_{m>=1} (-1)^(m+1)/m tr(H^2m) / w^2m,
//   Re[(i w - H)^-1]_ii = -sum_{m>=0} (-1)^m (H^(2m+1))_ii / w^(2m+2);
// the series are cut after kTailK terms (powers of H up to kTailP).
constexpr int kTailK = 14;
constexpr int kTailP = 2 * kTailK + 1;
constexpr int kTailS = kTailK + 2;   // sum of ln w_n, then S_2 .. S_{2K+2}

// Per-problem statistics written by the reduction kernel.
struct ProbStats {
  double omega, omega_tilde, max_abs_grad, af_order, pivot_growth;
  int32_t nonfinite;
  int32_t tail_range;   // the tail's spectral bound exceeded its guard
  double kin0, kin;     // HMC: 1/2 sum p^2 before and after this pass's kick
  double growth_run;    // largest pivot growth since the descriptor upload
  int32_t guard;        // kGuard* bits of this pass
  int32_t updated;      // this pass applied an ADAM update
  int32_t adam_t;       // ADAM updates applied after this pass
  int32_t steps_left;   // updates still to apply after this pass
};

// Number of lattice directions d in {+x,-x,+y,-y} with j = i + d (mod L).
__host__ __device__ inline int kmult(int i, int j, int L) {
  int xi = i % L, yi = i / L, xj = j % L, yj = j / L;
  int dx = xj - xi; if (dx < 0) dx += L;
  int dy = yj - yi; if (dy < 0) dy += L;
  int c = 0;
  if (dy == 0) c += (dx == 1) + (dx == L - 1);
  if (dx == 0) c += (dy == 1) + (dy == L - 1);
  return c;
}

// max that keeps a NaN (fmax drops it): guards and absmax read a NaN as
// out of range.
__host__ __device__ inline double max_nan(double a, double b) {
  return (a != a || b != b) ? a + b : (a > b ? a : b);
}

__host__ __device__ inline int stagger_sign(int i, int L) {
  return (((i % L) + (i / L)) & 1) ? -1 : 1;
}

}  // namespace sca
