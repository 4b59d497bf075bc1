// Blocked (N > 64) factorisation paths.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include "sca_common.h"

namespace sca {

// Launch configuration of a blocked path for N sites: cfg selects the
// (waves, row tiles per wave, block width) instance, Np is N rounded up to
// the block width NB.  cfg < 0: N too large for that precision.
struct BlockedPlan { int cfg, NB, Np; };
BlockedPlan blocked_plan(int N, bool fp32);
BlockedPlan blocked_plan_f64(int N);
size_t blocked_factor_bytes(const BlockedPlan& p, int B, size_t elem);

// Bytes of the factor storage of B matrices: F [B][2][Np][Np] doubles,
// perm [B][Np] int32, diagonal-block inverses [B][Np/NB][2][2][NB][NB].
size_t blocked_factor_bytes_f64(const BlockedPlan& p, int B);

// With `only` given, the FP64 kernels below act on the matrices b with
// only[b] == want and leave the others untouched.

// P A = L U of every matrix into F/perm/tri; lad[b] = ln|det A_b|,
// growth[b] = max|u|/max|a|.
hipError_t blocked_lu_f64(const BlockedPlan& p, const MatDesc* descs,
                          const double* hbuf, int B, int N, int L, double* F,
                          int* perm, double* tri, double* lad, double* growth,
                          hipStream_t st, const int* only = nullptr,
                          int want = 0);

// diag(A_b^-1) -> dg[b][N][2] from the factors (F is overwritten by
// U^-1 and L^-1).
hipError_t blocked_inv_f64(const BlockedPlan& p, int B, int N, double* F,
                           const int* perm, const double* tri, double* dg,
                           hipStream_t st, const int* only = nullptr,
                           int want = 0);

// Only the upper-triangle inverse W = U^-1 (in place), from tri's U slot.
hipError_t blocked_trtri_upper_f64(const BlockedPlan& p, int B, double* F,
                                   const int* perm, const double* tri,
                                   hipStream_t st, const int* only = nullptr,
                                   int want = 0);

// Symmetric route (k_ldlt.hip): A = L D L^T without pivoting into F (L^T
// row-major, d on the diagonal), perm (identity), tri, invd [B][2][Np]
// (1/d); lad, growth; fallback[b] = 1 where the pivoted LU must redo b.
hipError_t blocked_ldlt_f64(const BlockedPlan& p, const MatDesc* descs,
                            const double* hbuf, int B, int N, int L, double* F,
                            int* perm, double* tri, double* invd, double* lad,
                            double* growth, int* fallback, hipStream_t st);
// dg[b][i] = sum_k (L^-T)_ik^2 / d_k once F holds L^-T (trtri upper mode).
hipError_t launch_symdiag_f64(int B, int N, int Np, const double* F,
                              const double* invd, double* dg, hipStream_t st,
                              const int* only = nullptr, int want = 0);

// FP32 factor route (k_factor.hip, k_refine.hip).
hipError_t blocked_lu_f32(const BlockedPlan& p, const MatDesc* descs,
                          const double* hbuf, int B, int N, int L, float* F,
                          int* perm, float* tri, double* lad, double* growth,
                          hipStream_t st);
hipError_t blocked_trtri_f32(const BlockedPlan& p, int B, float* F,
                             const int* perm, const float* tri,
                             hipStream_t st);
// X = fl32(W V) for every matrix (Np a multiple of 16), and the tiles'
// shares of Re tr(A W V P) into ldpart (B * refine_parts(Np) doubles).
hipError_t launch_wv_gemm(int B, int N, int Np, int L, const MatDesc* descs,
                          const double* hbuf, const float* F, const int* perm,
                          float* X, double* ldpart, hipStream_t st);
// FP64 Newton diagonal -> dg[b][N][2] and refined ln|det| -> lad[b] (after
// launch_wv_gemm on the same ldpart).
int refine_parts(int Np);
hipError_t launch_refine(int B, int N, int Np, int L, const MatDesc* descs,
                         const double* hbuf, const float* F, const int* perm,
                         const float* X, double* dg, double* ldpart,
                         double* lad, hipStream_t st);

}  // namespace sca
