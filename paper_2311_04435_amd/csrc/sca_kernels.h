// Kernel launchers of the SCA library (internal C++ interface).
#pragma once
#include <hip/hip_runtime.h>
#include "sca_common.h"

namespace sca {

// h vectors of every problem: h[hoff + s_idx*N + i] =
//   (Delta/2)(-1)^(x+y) - s phi_i + onsite_i,  s_idx 0 -> s = +1, 1 -> s = -1
hipError_t launch_hvec(const ProbDesc* probs, int nprob, int N, double* hbuf,
                       hipStream_t st);

// Matsubara descriptors of every problem: for b in [mat_begin, +2 Me),
// z = i w_n (n = (b - mat_begin) mod Me), spin up for the first Me.
hipError_t launch_matsubara_descs(const ProbDesc* probs, int nprob,
                                  int max2M, MatDesc* descs, hipStream_t st);

// Small fused path, N <= 64: per matrix ln|det A_b| -> lad[b],
// diag(A_b^-1) -> dg[b][N][2], growth max|u|/max|a| -> growth[b].
hipError_t launch_small_factor(const MatDesc* descs, const double* hbuf, int B,
                               int N, int L, double* lad, double* dg,
                               double* growth, hipStream_t st);

// Reduction of the per-matrix terms into Omega, Omega~ and the gradient of
// every problem.  With `adam` set (and dg given), every problem whose
// steps_left is positive then takes one ADAM update with step count
// adam_t + 1 and its own hyper-parameters, and the kernel advances that
// problem's adam_t and steps_left in place; problems with steps_left == 0
// are only evaluated.  stats[p] receives Omega, Omega~, max|g|, |phi| (of
// the phi the terms were evaluated at) and the largest pivot growth of the
// problem's matrices.
// Problems with Me < M add their tail from mom / tsum (launch_tail).
// With `hmc`, problems with hmc_L > 0 take the leapfrog kick/drift of their
// pass hmc_k instead (and advance hmc_k).
hipError_t launch_reduce(ProbDesc* probs, int nprob, int N, const double* lad,
                         const double* dg, const double* growth,
                         ProbStats* stats, bool adam, void* ws,
                         const double* mom, const double* tsum,
                         hipStream_t st, bool hmc = false);
size_t reduce_workspace_bytes(int nprob);
int reduce_max_sites();

// Matsubara tail of every problem with Me < M: mom[p][s][q][i] =
// (H_s^(q+1))_ii for q < kTailP, tsum[p] = (sum ln w_n, S_2, .., S_{2K+2})
// over n in [Me, M).
hipError_t launch_tail(const ProbDesc* probs, int nprob, int N,
                       const double* hbuf, double* mom, double* tsum,
                       hipStream_t st);
size_t tail_workspace_bytes(int nprob, int N);
// *out = max_i |x_i| (device scalar).
hipError_t launch_absmax(const double* x, int n, double* out, hipStream_t st);

// Descriptors for arbitrary shifts: b = s_idx * n_z + j, z = (z[2j], z[2j+1]),
// h vector of spin s_idx at hoff0 + s_idx * N.
hipError_t launch_shift_descs(const double* z, int n_z, double t, int hoff0,
                              int N, MatDesc* descs, hipStream_t st);

// DOS reduction: rho[s][j] = -(1/(pi N)) sum_i Im dg[b][i][1] for the
// matrix b = s*n_w + j of a DOS batch.
hipError_t launch_dos_reduce(const double* dg, int n_w, int N, double* rho,
                             hipStream_t st);

}  // namespace sca
