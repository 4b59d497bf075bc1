/*
 * sca.h -- C ABI of the MI355X (gfx950) SCA library.
 *
 * The library evaluates the semiclassical-approximation (SCA) potential of the
 * half-filled ionic Hubbard model on an L x L periodic square lattice, its
 * gradient, its ADAM minimisation and the density of states at the optimum
 * (Sec. II of the paper: Hamiltonian Eq. (1), potential Eq. (7), DOS Eq. (8);
 * the ADAM/autograd procedure described after Eq. (7) and in Sec. III).
 *
 *   N = L*L sites, site i = x + L*y, t the hopping, U > 0, Delta the ionic
 *   amplitude (site potential +Delta/2 on (-1)^(x+y) = +1 sites, -Delta/2 on
 *   the others), T > 0 the temperature, M = n_max Matsubara frequencies
 *   w_n = (2n+1) pi T, n = 0..M-1 (the negative ones enter as the complex
 *   conjugates of these, so each contributes twice).
 *
 *   H_s(phi) = -t K + (Delta/2) S - s diag(phi) [+ diag(onsite)],  s = +1, -1
 *   A_ns     = i w_n I - H_s(phi)                       (complex symmetric)
 *   Omega    = sum_i phi_i^2/U - 2T sum_s sum_n ln|det A_ns|
 *   Omega~   = Omega + 2 N T sum_n ln w_n^2            (constant removed)
 *   dOmega/dphi_i = 2 phi_i/U - 2T sum_s s sum_n Re (A_ns^-1)_ii
 *   rho_s(w) = -(1/(pi N)) Im sum_i ((w + i eta) I - H_s)^-1_ii
 *   |phi|    = |N^-1 sum_i (-1)^(x+y) phi_i|          (AF order parameter)
 *
 * Every ln|det| and diagonal of an inverse comes from a batched complex LU
 * with partial pivoting (largest |Re|+|Im| in the column) on the GPU.
 *
 * Conventions common to all calls
 *   - Array arguments are DEVICE pointers on the context's device, allocated
 *     and owned by the caller (e.g. torch tensors).  Struct arguments
 *     (params, options, results) are HOST pointers.
 *   - Work is enqueued on the context's stream; each call returns only after
 *     that stream has drained, so the returned status covers the device work.
 *   - Parameters are validated before any device work; on error nothing is
 *     written.  sca_last_error() gives a message for the calling thread.
 *   - A context is not thread-safe; use one context per host thread/stream.
 *   - All values are float64; `precision` selects the arithmetic of the LU
 *     (SCA_FP64, or SCA_FP32_REFINED: complex64 factorisation with float64
 *     refinement of ln|det| and diag(A^-1)).
 */
#ifndef SCA_H
#define SCA_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define SCA_API __attribute__((visibility("default")))
#else
#define SCA_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sca_ctx sca_ctx;

typedef enum {
  SCA_OK = 0,
  SCA_EINVAL = -1,       /* invalid argument (message in sca_last_error) */
  SCA_ENOMEM = -2,       /* workspace would exceed the context's HBM budget */
  SCA_EDEVICE = -3,      /* HIP runtime error or no usable gfx950 device */
  SCA_ENUMERIC = -4,     /* non-finite Omega/gradient/phi or a singular matrix */
  SCA_EUNSUPPORTED = -5  /* size/precision/factor combination not built */
} sca_status;

typedef enum { SCA_FP64 = 0, SCA_FP32_REFINED = 1 } sca_precision;

/* Factorisation of each A = z I - H (lattices with L*L > 64; smaller ones
 * always use the fused pivoted LU, except under SCA_FACTOR_EIGH).
 *   SCA_FACTOR_LU    complex LU with partial pivoting (the default).
 *   SCA_FACTOR_LDLT  A is complex symmetric: A = L D L^T without pivoting,
 *                    half the flops and one triangular inverse instead of
 *                    two.  Exists and is stable for Im z > 0 (every shift
 *                    used here); each matrix whose growth max(max|D L^T| /
 *                    max|A|, max|L|) exceeds 64 or whose pivots are not
 *                    finite is redone by the pivoted LU on the device.
 *                    FP64 only (SCA_EUNSUPPORTED with SCA_FP32_REFINED). */
/*   SCA_FACTOR_EIGH  spectral route, any L: no matrix is factorised.  Each
 *                    H_s is real symmetric; H_s = sum_k e_k psi_k psi_k^T
 *                    is computed once per spin and evaluation (Householder
 *                    tridiagonalisation, bisection, inverse iteration), and
 *                    every shift then follows from the spectrum:
 *                    ln|det(z - H_s)| = sum_k ln|z - e_k|,
 *                    (z - H_s)^-1_ii = sum_k psi_k(i)^2 / (z - e_k).
 *                    O(N^3 + n_max N^2) per spin instead of O(n_max N^3).
 *                    FP64 only (SCA_EUNSUPPORTED with SCA_FP32_REFINED and
 *                    in sca_factorize / sca_grad_from_factors, whose buffer
 *                    holds factors).  max_pivot_growth reads 1.  An
 *                    eigenvector cluster that loses rank in its
 *                    orthogonalisation is reported as non-finite
 *                    (SCA_ENUMERIC / SCA_FLAG_NONFINITE). */
typedef enum { SCA_FACTOR_LU = 0, SCA_FACTOR_LDLT = 1,
               SCA_FACTOR_EIGH = 2 } sca_factor;

/* Matsubara frequencies that are factorised.
 *   SCA_TAIL_NONE     all n < n_max (the default).
 *   SCA_TAIL_MOMENTS  only n < n_c; for n_c <= n < n_max the terms come from
 *                     the moments of H: for w > rho(H),
 *                       ln|det(i w - H)| = N ln w
 *                           + 1/2 sum_{m>=1} (-1)^(m+1)/m tr(H^2m) w^-2m,
 *                       Re (i w - H)^-1_ii = -sum_{m>=0} (-1)^m (H^(2m+1))_ii
 *                           w^-(2m+2),
 *                     each cut after 14 terms.  n_c is the first n with
 *                     w_n >= 4 rho_b, rho_b = 4|t| + |delta|/2 + max|onsite|
 *                     + max(max|phi|, U/2) + 1/2 (a Gershgorin bound with a
 *                     margin for phi to grow during a solve), at least 1.
 *                     While every pass's Gershgorin bound stays below
 *                     w_{n_c}/3 the truncation error of each term is below
 *                     9^-15 of its scale; a pass above it sets
 *                     SCA_FLAG_TAIL_RANGE (sca_potential and sca_grad then
 *                     re-evaluate without the tail; in sca_adam_solve and
 *                     the request server that pass applies no update and
 *                     the solve goes on without the tail from that step:
 *                     see "Guards of a solve").  The same sums are computed, only the
 *                     evaluation of the high frequencies differs.
 *                     sca_factorize keeps the split it chose in the factor
 *                     buffer and sca_grad_from_factors uses it. */
typedef enum { SCA_TAIL_NONE = 0, SCA_TAIL_MOMENTS = 1 } sca_tail;

/* One SCA problem.  onsite: optional DEVICE array of N extra site
 * potentials (a disordered lattice), or NULL (the paper's ionic model). */
typedef struct {
  int32_t L;          /* even, 2 <= L <= 64 */
  int32_t n_max;      /* M >= 1 */
  int32_t precision;  /* sca_precision */
  int32_t factor;     /* sca_factor */
  double t, U, delta, T;
  const double* onsite;
  int32_t tail;       /* sca_tail */
  int32_t reserved;   /* 0 */
} sca_params;

typedef struct {
  double lr, beta1, beta2, eps;  /* ADAM (Kingma-Ba) hyper-parameters */
  double grad_tol;     /* stop early once max|g| < grad_tol (0: never) */
  int32_t n_steps;     /* maximum number of ADAM updates */
  int32_t check_every; /* host reads the statistics every k passes (0: by
                          elapsed time); convergence is tested only if > 0 */
  int32_t t0;          /* ADAM step count already taken (resume); 0 fresh */
  int32_t flags;       /* SCA_ADAM_* bits, 0 by default */
} sca_adam_opts;

/* Skip the evaluation at the returned phi: the result then describes the
 * last phi the loop evaluated (the input of the final update). */
#define SCA_ADAM_NO_FINAL_EVAL 1

typedef struct {
  double omega;         /* Omega at the returned phi */
  double omega_tilde;   /* Omega~ at the returned phi */
  double af_order;      /* |phi| */
  double max_abs_grad;  /* max_i |dOmega/dphi_i| at the returned phi */
  double max_pivot_growth; /* max over matrices of max|u|/max|a| */
  int32_t steps_done;   /* ADAM updates applied in this call */
  int32_t flags;        /* SCA_FLAG_* bits */
} sca_result;

/* SCA_FLAG_PIVOT_GROWTH: under SCA_FP32_REFINED a factorisation had pivot
 * growth max|u|/max|a| above the context's limit (SCA_OPT_FP32_GROWTH_LIMIT,
 * 1e3 by default).  Where an FP64 path is built for N (L*L <= 1024) the
 * pass that saw it applies no update and the solve continues in FP64 from
 * that step (sca_potential, sca_grad and sca_factorize redo the evaluation
 * in FP64); where it is not, sca_adam_solve and the server report the flag
 * and sca_potential / sca_grad / sca_factorize return SCA_ENUMERIC. */
#define SCA_FLAG_NONFINITE 1    /* a non-finite value was produced */
#define SCA_FLAG_PIVOT_GROWTH 2 /* FP32 growth above 1e3 (see above) */
#define SCA_FLAG_CONVERGED 4    /* stopped by grad_tol */
#define SCA_FLAG_TAIL_RANGE 8   /* a pass exceeded the tail's spectral guard */

/* Guards of a solve.  Every pass of sca_adam_solve checks on the device,
 * before its update, the Gershgorin bound of the tail (SCA_TAIL_MOMENTS)
 * and, under SCA_FP32_REFINED, the pivot growth; a pass that fails either
 * applies no update and advances no step counter, and the host re-plans
 * the problem (every frequency; FP64) when it next reads the statistics
 * and resumes from the step that was held back.  The trajectory is
 * therefore the same as with the switch made at that very step, whatever
 * check_every is and whoever shares a server's batches. */

/* Create a context on `device` (HIP ordinal) that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  hbm_budget_bytes bounds the
 * workspace the context may hold (0 = no bound).  Returns SCA_EDEVICE if
 * the device is absent or not gfx950. */
SCA_API sca_status sca_create(int device, void* hip_stream, size_t hbm_budget_bytes,
                      sca_ctx** out);
SCA_API void sca_destroy(sca_ctx* ctx);

/* Context options (sca_set_option; SCA_EINVAL for an unknown option or an
 * invalid value).
 *   SCA_OPT_FP32_GROWTH_LIMIT  pivot growth above which a complex64 LU is
 *                              not trusted (see SCA_FLAG_PIVOT_GROWTH);
 *                              finite, >= 1; default 1e3. */
#define SCA_OPT_FP32_GROWTH_LIMIT 1
SCA_API sca_status sca_set_option(sca_ctx* ctx, int32_t option, double value);

/* Device workspace (bytes) one problem needs: admission control for
 * serving.  0 if the parameters are invalid. */
SCA_API size_t sca_footprint_bytes(const sca_params* p);

/* Omega and Omega~ at phi[N] -> omega2[2] = {Omega, Omega~}: the SCA
 * potential V(phi) of Eq. (7) (Sec. II), with the sum over the Matsubara
 * frequencies cut at n_max. */
SCA_API sca_status sca_potential(sca_ctx* ctx, const sca_params* p, const double* phi,
                         double* omega2);

/* Gradient dOmega/dphi -> grad[N]; omega2[2] as above, or NULL.  The
 * derivative of Eq. (7): d ln det A / d phi_i = -s (A^-1)_ii for the
 * diagonal coupling -s phi_i of H_s (Eq. (5) after the static
 * Hubbard-Stratonovich decoupling), which the paper takes by automatic
 * differentiation (Sec. III). */
SCA_API sca_status sca_grad(sca_ctx* ctx, const sca_params* p, const double* phi,
                    double* grad, double* omega2);

/* ADAM minimisation of Omega from phi (in: phi0, out: final phi), with the
 * first and second moments m[N], v[N] (in/out, zeros for a fresh start) so a
 * run can resume where another stopped (opts->t0 = steps already taken):
 * the optimiser the paper applies to Eq. (7) (Sec. II after Eq. (7), and
 * Sec. III), Kingma-Ba with bias correction.  Every step runs on the
 * device; the host reads the statistics of the last pass every check_every
 * passes (0: every ~50 ms of passes), acts on the guards above and, with
 * grad_tol > 0 and check_every > 0, stops once max|g| < grad_tol.
 * res->max_pivot_growth is the largest over the whole call; steps_done the
 * updates applied.  On SCA_ENUMERIC (a non-finite value) phi, m, v hold
 * the state the failing pass produced and res->steps_done says when. */
SCA_API sca_status sca_adam_solve(sca_ctx* ctx, const sca_params* p,
                          const sca_adam_opts* opts, double* phi, double* m,
                          double* v, sca_result* res);

/* Hybrid Monte Carlo sampling of the static-field weight exp(-Omega(phi)/T)
 * (the SCA partition function, Z = integral over phi of exp(-Omega/T),
 * Sec. II; Omega~ is used, which differs by a constant).  Trajectory t
 * starts from the current phi with momentum momenta[t][N] (device; the
 * caller draws it, normally standard normal), takes n_leap leapfrog steps
 * of size eps in H = Omega~/T + |p|^2/2 (every force evaluation is a full
 * pass over the Matsubara matrices on the device; the kick and drift are
 * fused into its reduction) and is accepted if
 * uniforms[t] < exp(-(H_new - H_old)) (uniforms: host array, the caller's
 * draws in [0, 1)); on rejection phi returns to the trajectory's start.
 * Outputs on the host: accepted[t] (0/1), h_old[t], h_new[t].  phi (device,
 * in/out) ends at the chain's last state.  With SCA_TAIL_MOMENTS a
 * trajectory whose end points leave the tail's range returns
 * SCA_ENUMERIC. */
typedef struct {
  double eps;       /* leapfrog step, > 0 */
  int32_t n_leap;   /* leapfrog steps per trajectory, >= 1 */
  int32_t n_traj;   /* trajectories, >= 0 */
} sca_hmc_opts;
SCA_API sca_status sca_hmc(sca_ctx* ctx, const sca_params* p,
                           const sca_hmc_opts* opts, double* phi,
                           const double* momenta, const double* uniforms,
                           int32_t* accepted, double* h_old, double* h_new);

/* Matsubara frequencies per spin that the calls above factorise for p at
 * phi (device array of N) -> *n_factorised (host): n_max, or under
 * SCA_TAIL_MOMENTS the split n_c described there, planned from max|phi|
 * and max|onsite| read on the device (SCA_ENUMERIC if either is not
 * finite).  The frequencies above n_c enter Eq. (7) through the moment
 * series of the same sums. */
SCA_API sca_status sca_tail_split(sca_ctx* ctx, const sca_params* p,
                                  const double* phi, int32_t* n_factorised);

/* Density of states per spin (Eq. (8), mu = 0; the spectral function of
 * the optimised field, Sec. II): rho[2][n_w] (spin up first) at the n_w
 * real frequencies w[n_w], broadening eta > 0. */
SCA_API sca_status sca_dos(sca_ctx* ctx, const sca_params* p, const double* phi,
                   const double* w, int32_t n_w, double eta, double* rho);

/* The per-matrix terms behind the calls above, for arbitrary complex shifts
 * z[n_z][2] (re, im): for both spins (up first) and every z_j,
 *   logabsdet[2][n_z] = ln|det(z_j I - H_s)|   (the ln det of Eq. (7) at
 *                       z = i w_n, of Eq. (8) at z = w + i eta)
 *   diag[2][n_z][N][2] = (z_j I - H_s)^-1_ii  (re, im interleaved; the
 *                       gradient's and the DOS's term). */
SCA_API sca_status sca_shifted_terms(sca_ctx* ctx, const sca_params* p,
                             const double* phi, const double* z, int32_t n_z,
                             double* logabsdet, double* diag);

/* sca_grad without any allocation, for callers that cannot allocate (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and errors as sca_grad, but every
 * intermediate lives in a fixed scratch array of 16 MiB compiled into the
 * library: one per device, held from the library's load until the process
 * ends (sca_create takes its address).  Nothing is allocated on the device
 * or the host: descriptors go up as kernel arguments and the statistics come
 * back through the context's stream.  A problem whose workspace exceeds the
 * scratch (sca_footprint_bytes gives it, plus 256 bytes) is refused with
 * SCA_ENOMEM before any device work (with SCA_TAIL_MOMENTS, after max|phi|
 * is read for the split).  That admits the fused path up to n_max = 7807 at
 * L = 8 (27568 at L = 4), small blocked lattices (L = 10 up to n_max = 21 in
 * FP64, 25 in refined FP32) and the spectral route up to L = 16 (n_max =
 * 1211).  Every call on one device shares that device's
 * scratch and leaves its last contents there (nothing in it needs to start
 * at zero): calls that overlap on one device, from any context or stream,
 * race and must be serialised by the caller. */
SCA_API sca_status sca_grad_noalloc(sca_ctx* ctx, const sca_params* p,
                                    const double* phi, double* grad,
                                    double* omega2);

/* Differentiable split of sca_grad (a custom autograd backward of Eq. (7),
 * in place of the automatic differentiation of the determinant the paper
 * uses in Sec. III): the
 * forward factorises every A_ns and keeps what the backward needs in the
 * caller's device buffer `factors` of sca_factor_bytes(p) bytes (0 for
 * invalid params); the backward then reads it instead of factorising
 * again.  phi and params must be the same in both calls.  On the FP64
 * blocked path (L*L > 64) the backward inverts the factors in place, so a
 * second sca_grad_from_factors on the same buffer returns SCA_EINVAL until
 * sca_factorize refills it; the other paths leave the buffer reusable.  A
 * buffer that sca_factorize did not fill for these params is refused with
 * SCA_EINVAL.  Under SCA_FP32_REFINED the buffer has room for FP64 factors
 * too: a factorisation whose pivot growth exceeds the context's limit is
 * redone in FP64 (SCA_ENUMERIC where no FP64 path is built), and the
 * backward uses whichever was kept. */
SCA_API size_t sca_factor_bytes(const sca_params* p);
SCA_API sca_status sca_factorize(sca_ctx* ctx, const sca_params* p, const double* phi,
                         void* factors, double* omega2);
SCA_API sca_status sca_grad_from_factors(sca_ctx* ctx, const sca_params* p,
                                 const double* phi, void* factors,
                                 double* grad);

/* Kernel timing (tracing).  With SCA_ROCTX=1 in the environment (read once
 * per process) the library also brackets every kernel class's launches
 * with a roctx range named "sca:<class>" (rocprofv3 --marker-trace).
 * sca_profile(ctx, 1) resets the counters and
 * brackets every later kernel launch of this context with HIP events on its
 * stream; sca_profile(ctx, 0) stops.  sca_profile_read fills HOST arrays of
 * SCA_PROFILE_SLOTS entries with the accumulated milliseconds and launch
 * counts per kernel class (SCA_K_*). */
#define SCA_PROFILE_SLOTS 16
#define SCA_K_SMALL 0   /* fused small-lattice factor + inverse diagonal */
#define SCA_K_LU 1      /* blocked LU with partial pivoting */
#define SCA_K_TRTRI 2   /* blocked U^-1 and L^-1 */
#define SCA_K_DIAGDOT 3 /* diagonal of A^-1 from U^-1 and L^-1 */
#define SCA_K_REDUCE 4  /* Matsubara/spin reduction and ADAM update */
#define SCA_K_SETUP 5   /* descriptors and diagonal vectors */
#define SCA_K_REFINE 6  /* FP64 refinement of the FP32 route */
#define SCA_K_WVGEMM 7  /* X = U^-1 L^-1 product of the FP32 route */
#define SCA_K_LDLT 8    /* symmetric route: L D L^T */
#define SCA_K_TRTRI_SYM 9  /* symmetric route: L^-T */
#define SCA_K_SYMDIAG 10   /* symmetric route: diagonal of A^-1 */
#define SCA_K_FALLBACK 11  /* symmetric route: pivoted LU of flagged matrices */
#define SCA_K_TAIL 12      /* Matsubara tail: moments of H, frequency sums */
#define SCA_K_TRIDIAG 13   /* spectral route: Householder tridiagonalisation */
#define SCA_K_SPECTRUM 14  /* spectral route: eigenpairs and psi^2 */
#define SCA_K_EXPAND 15    /* spectral route: per-shift terms from the spectrum */
SCA_API sca_status sca_profile(sca_ctx* ctx, int enable);
SCA_API sca_status sca_profile_read(sca_ctx* ctx, double* total_ms,
                                    int64_t* launches);

/* Serving (the request loop of continuous batching).  A server owns its
 * own HIP streams and device workspaces on `device` and runs many ADAM
 * solves at once: requests of the same (L, n_max, precision) are evaluated
 * together, one batched pass (every matrix of every member problem) per
 * ADAM step, and shapes run concurrently on separate streams.  Each request
 * keeps its own phi, moments, step counter and hyper-parameters on the
 * device; its result equals that of sca_adam_solve on the same inputs, bit
 * for bit, whatever else shared its batches.
 *
 * Admission: first come, first served per shape.  A shape's group takes up
 * to max_batch problems, fewer for large lattices (as many as keep one pass
 * near 3e10 flops of factorisation work, at least one: past that a bigger
 * batch adds latency, not throughput); its workspace (the footprint of that
 * many problems, fewer if the budget is short) must fit hbm_budget_bytes
 * (0 = 90% of the device memory free at creation) together with the other
 * groups; idle empty groups give their memory back when another shape
 * needs it.  Requests wait in the queue until they fit.
 *
 * The caller owns phi, m, v (device arrays of L*L float64: phi holds phi0
 * on submit and the solution when done; m, v the ADAM moments, zero for a
 * fresh start) and must keep them alive and untouched until the request is
 * done.  Work advances only inside sca_server_progress.  A server is not
 * thread-safe.
 *
 *   sca_server_create   max_batch in [1, 4096]; SCA_EDEVICE if the device
 *                       is absent or not gfx950.
 *   sca_server_submit   validates like sca_adam_solve (grad_tol and
 *                       check_every must be 0: requests run exactly
 *                       n_steps updates, then, unless SCA_ADAM_NO_FINAL_EVAL,
 *                       one evaluation at the returned phi); SCA_ENOMEM if
 *                       one request alone exceeds the budget.  *ticket
 *                       names the request.
 *   sca_server_progress retires finished passes, admits queued requests
 *                       and launches the next passes; with wait_s > 0 it
 *                       waits up to that long for a pass to finish.
 *                       Reports the running and queued request counts.
 *   sca_server_poll     *done = 1 once the request finished; then *res
 *                       (flags as for sca_adam_solve; a pivot growth above
 *                       1e3 under FP32 is flagged, not re-run; a tail
 *                       member whose guard fires continues with every
 *                       frequency from the step that was held back) and *t_done
 *                       (sca_server_clock time the server saw it finish)
 *                       are set and the ticket is released.
 *   sca_server_clock    seconds since the server was created. */
typedef struct sca_server sca_server;
SCA_API sca_status sca_server_create(int device, size_t hbm_budget_bytes,
                                     int32_t max_batch, sca_server** out);
SCA_API void sca_server_destroy(sca_server* s);
SCA_API double sca_server_clock(const sca_server* s);
SCA_API sca_status sca_server_submit(sca_server* s, const sca_params* p,
                                     const sca_adam_opts* o, double* phi,
                                     double* m, double* v, int64_t* ticket);
SCA_API sca_status sca_server_progress(sca_server* s, double wait_s,
                                       int32_t* n_active, int32_t* n_queued);
SCA_API sca_status sca_server_poll(sca_server* s, int64_t ticket,
                                   int32_t* done, sca_result* res,
                                   double* t_done);

/* Message for the last error on this thread ("" if none). */
SCA_API const char* sca_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SCA_H */
