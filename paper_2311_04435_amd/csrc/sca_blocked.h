// Blocked (N > 64) factorisation paths.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include "sca_common.h"

namespace sca {

// Launch configuration of the blocked FP64 path for N sites: cfg selects
// the (waves, row tiles per wave, block width) instance, Np is N rounded up
// to the block width NB.  cfg < 0: N too large for FP64.
struct BlockedPlan { int cfg, NB, Np; };
BlockedPlan blocked_plan_f64(int N);

// Bytes of the factor storage of B matrices: F [B][2][Np][Np] doubles,
// perm [B][Np] int32, diagonal-block inverses [B][Np/NB][2][2][NB][NB].
size_t blocked_factor_bytes_f64(const BlockedPlan& p, int B);

// P A = L U of every matrix into F/perm/tri; lad[b] = ln|det A_b|,
// growth[b] = max|u|/max|a|.
hipError_t blocked_lu_f64(const BlockedPlan& p, const MatDesc* descs,
                          const double* hbuf, int B, int N, int L, double* F,
                          int* perm, double* tri, double* lad, double* growth,
                          hipStream_t st);

// diag(A_b^-1) -> dg[b][N][2] from the factors (F is overwritten by
// U^-1 and L^-1).
hipError_t blocked_inv_f64(const BlockedPlan& p, int B, int N, double* F,
                           const int* perm, const double* tri, double* dg,
                           hipStream_t st);

}  // namespace sca
