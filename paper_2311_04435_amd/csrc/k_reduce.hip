// Set-up, Matsubara/spin accumulation and the fused ADAM update.
//
//   Omega    = sum_i phi_i^2/U - 2T sum_b ln|det A_b|
//   Omega~   = sum_i phi_i^2/U - 2T sum_b (ln|det A_b| - N ln w_n(b))
//   g_i      = 2 phi_i/U - 2T (sum_n Re dg_up[n][i] - sum_n Re dg_dn[n][i])
//
// (potential Eq. (7); the factor 2 pairs +w_n with -w_n).  Every sum runs
// in a fixed order that does not depend on the launch shape or on which
// other problems share the batch, so a problem's result is the same alone
// and in a mixed batch.  ADAM (Kingma & Ba, Algorithm 1; the paper's
// optimizer, Sec. II after Eq. (7)) updates phi, m, v in the same pass.
#include <math.h>
#include "sca_common.h"
#include "sca_kernels.h"
#include "sca_profile.h"

namespace sca {

namespace {
constexpr int kSitesPerBlock = 64;
constexpr int kBParts = 4;          // b-range split per site (fixed order)
constexpr int kReduceThreads = kSitesPerBlock * kBParts;
constexpr int kMaxChunks = 128;     // N <= 64 * 128 = 8192 sites
constexpr double kPi = 3.14159265358979323846;
}  // namespace

__global__ void hvec_kernel(const ProbDesc* __restrict__ probs, int N,
                            double* __restrict__ hbuf) {
  const int p = blockIdx.y >> 1;
  const int sidx = blockIdx.y & 1;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const ProbDesc P = probs[p];
  const double s = sidx ? -1.0 : 1.0;
  double h = 0.5 * P.delta * (double)stagger_sign(i, P.L) - s * P.phi[i];
  if (P.onsite) h += P.onsite[i];
  hbuf[P.hoff + sidx * N + i] = h;
}

hipError_t launch_hvec(const ProbDesc* probs, int nprob, int N, double* hbuf,
                       hipStream_t st) {
  if (nprob <= 0) return hipSuccess;
  mark_begin(K_SETUP, st);
  hipLaunchKernelGGL(hvec_kernel, dim3((N + 255) / 256, 2 * nprob), dim3(256),
                     0, st, probs, N, hbuf);
  mark_end(K_SETUP, st);
  return hipGetLastError();
}

__global__ void matsubara_desc_kernel(const ProbDesc* __restrict__ probs,
                                      MatDesc* __restrict__ descs) {
  const int p = blockIdx.y;
  const ProbDesc P = probs[p];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 2 * P.Me) return;
  const int sidx = k / P.Me, n = k % P.Me;
  MatDesc d;
  d.zr = 0.0;
  d.zi = (2.0 * n + 1.0) * kPi * P.T;
  d.t = P.t;
  d.hoff = P.hoff + sidx * P.N;
  d.prob = p;
  descs[P.mat_begin + k] = d;
}

hipError_t launch_matsubara_descs(const ProbDesc* probs, int nprob,
                                    int max2M, MatDesc* descs,
                                    hipStream_t st) {
  if (nprob <= 0) return hipSuccess;
  hipLaunchKernelGGL(matsubara_desc_kernel, dim3((max2M + 255) / 256, nprob),
                     dim3(256), 0, st, probs, descs);
  return hipGetLastError();
}

// Partial results of one 64-site chunk of one problem.
struct ChunkPartial {
  double phi2;      // sum phi_i^2 (phi at which the terms were evaluated)
  double stag;      // sum (-1)^(x+y) phi_i
  double gmax;      // max |g_i|
  double kin0, kin; // HMC: sum p^2 before / after the kick
  int32_t nonfinite;
  int32_t guard;    // kGuard* bits of the pass (the same in every chunk)
};

// Guard bits of a pass (see ProbDesc): the Gershgorin bound 4|t| +
// max_i (|Delta/2 + onsite_i| + |phi_i|) of H against tail_guard, and the
// largest pivot growth of the problem's matrices against growth_limit.
// Block-wide; every block of the problem computes the same bits (max is
// exact in any order, and a NaN stays a NaN).
__device__ int pass_guard(const ProbDesc& P, const double* __restrict__ growth,
                          double (*red)[kReduceThreads]) {
  const int tid = threadIdx.x;
  const bool tail = P.Me < P.M;
  const bool grow = P.growth_limit > 0.0 && growth != nullptr;
  if (!tail && !grow) return 0;
  double hm = 0.0, gm = 0.0;
  if (tail)
    for (int k = tid; k < P.N; k += kReduceThreads) {
      double a = 0.5 * P.delta * (double)stagger_sign(k, P.L);
      if (P.onsite) a += P.onsite[k];
      hm = max_nan(hm, fabs(a) + fabs(P.phi[k]));
    }
  if (grow)
    for (int k = tid; k < 2 * P.Me; k += kReduceThreads)
      gm = max_nan(gm, growth[P.mat_begin + k]);
  red[0][tid] = hm;
  red[1][tid] = gm;
  __syncthreads();
  for (int w = kReduceThreads / 2; w >= 1; w >>= 1) {
    if (tid < w) {
      red[0][tid] = max_nan(red[0][tid], red[0][tid + w]);
      red[1][tid] = max_nan(red[1][tid], red[1][tid + w]);
    }
    __syncthreads();
  }
  int guard = 0;
  if (tail && !(red[0][0] + 4.0 * fabs(P.t) <= P.tail_guard))
    guard |= kGuardTail;
  if (grow && !(red[1][0] <= P.growth_limit)) guard |= kGuardGrowth;
  return guard;
}

__global__ void __launch_bounds__(kReduceThreads)
site_reduce_kernel(const ProbDesc* __restrict__ probs, int N,
                   const double* __restrict__ dg,
                   const double* __restrict__ growth,
                   ChunkPartial* __restrict__ part,
                   int adam, const double* __restrict__ mom,
                   const double* __restrict__ tsum, int hmc) {
  const int p = blockIdx.y;
  const int chunk = blockIdx.x;
  const ProbDesc P = probs[p];
  const int tid = threadIdx.x;
  const int site_l = tid % kSitesPerBlock;
  const int bpart = tid / kSitesPerBlock;
  const int i = chunk * kSitesPerBlock + site_l;
  __shared__ double acc_s[kBParts][kSitesPerBlock];
  __shared__ double red_s[5][kSitesPerBlock];
  __shared__ int nf_s[kSitesPerBlock];
  __shared__ double guard_s[2][kReduceThreads];
  const int guard = pass_guard(P, growth, guard_s);

  // sum over the problem's 2 Me matrices, split in kBParts contiguous ranges
  // per spin; each range summed in increasing n
  double acc = 0.0;
  if (i < N && dg) {
    const int M = P.Me;
    const int per = (M + kBParts - 1) / kBParts;
    const int n0 = bpart * per, n1 = min(M, n0 + per);
    double su = 0.0, sd = 0.0;
    const double* up = dg + ((size_t)P.mat_begin * N + i) * 2;
    const double* dn = dg + ((size_t)(P.mat_begin + M) * N + i) * 2;
    for (int n = n0; n < n1; ++n) su += up[(size_t)n * N * 2];
    for (int n = n0; n < n1; ++n) sd += dn[(size_t)n * N * 2];
    acc = su - sd;
  }
  acc_s[bpart][site_l] = acc;
  __syncthreads();
  if (bpart == 0) {
    double phi2 = 0.0, stag = 0.0, ga = 0.0, k0 = 0.0, k1 = 0.0;
    int nf = 0;
    if (i < N) {
      double s = acc_s[0][site_l];
      for (int q = 1; q < kBParts; ++q) s += acc_s[q][site_l];
      const double ph = P.phi[i];
      if (P.Me < P.M && dg) {
        // tail: sum_{n >= Me} Re G_ii = -sum_m (-1)^m (H^(2m+1))_ii S_{2m+2},
        // up minus down
        const double* ts = tsum + (size_t)p * kTailS;
        const double* mu = mom + (size_t)p * 2 * kTailP * N + i;
        const double* md = mu + (size_t)kTailP * N;
        double tu = 0.0, td = 0.0;
        for (int m = kTailK; m >= 0; --m) {
          const double sg = (m & 1) ? -1.0 : 1.0;
          tu += sg * mu[(size_t)(2 * m) * N] * ts[m + 1];
          td += sg * md[(size_t)(2 * m) * N] * ts[m + 1];
        }
        s += td - tu;
      }
      const double g = dg ? 2.0 * ph / P.U - 2.0 * P.T * s : 0.0;
      if (P.grad && dg) P.grad[i] = g;
      phi2 = ph * ph;
      stag = (double)stagger_sign(i, P.L) * ph;
      ga = fabs(g);
      nf = !isfinite(g);
      if (hmc && dg && P.hmc_L > 0 && P.hmc_k <= P.hmc_L) {
        // leapfrog: kick with the force of this pass, drift unless last
        const double c = (P.hmc_k == 0 || P.hmc_k == P.hmc_L) ? 0.5 * P.hmc_eps
                                                              : P.hmc_eps;
        const double p0 = P.pmom[i];
        const double p1 = p0 - c * g / P.T;
        P.pmom[i] = p1;
        k0 = p0 * p0;
        k1 = p1 * p1;
        nf |= !isfinite(p1);
        if (P.hmc_k < P.hmc_L) {
          const double nphi = ph + P.hmc_eps * p1;
          nf |= !isfinite(nphi);
          P.phi_out[i] = nphi;
        }
      }
      if (adam && dg && P.steps_left > 0 && !guard) {
        const int t = P.adam_t + 1;
        const double m = P.beta1 * P.m[i] + (1.0 - P.beta1) * g;
        const double v = P.beta2 * P.v[i] + (1.0 - P.beta2) * g * g;
        const double bc1 = 1.0 - pow(P.beta1, (double)t);
        const double bc2 = 1.0 - pow(P.beta2, (double)t);
        const double upd = P.lr * (m / bc1) / (sqrt(v / bc2) + P.eps);
        P.m[i] = m;
        P.v[i] = v;
        const double nphi = ph - upd;
        nf |= !isfinite(nphi);
        P.phi_out[i] = nphi;
      }
    }
    red_s[0][site_l] = phi2;
    red_s[1][site_l] = stag;
    red_s[2][site_l] = ga;
    red_s[3][site_l] = k0;
    red_s[4][site_l] = k1;
    nf_s[site_l] = nf;
  }
  __syncthreads();
  if (tid == 0) {
    double a = 0.0, b = 0.0, c = 0.0, k0 = 0.0, k1 = 0.0;
    int nf = 0;
    for (int q = 0; q < kSitesPerBlock; ++q) {
      a += red_s[0][q];
      b += red_s[1][q];
      c = max_nan(c, red_s[2][q]);
      k0 += red_s[3][q];
      k1 += red_s[4][q];
      nf |= nf_s[q];
    }
    ChunkPartial cp;
    cp.phi2 = a; cp.stag = b; cp.gmax = c; cp.kin0 = k0; cp.kin = k1;
    cp.nonfinite = nf; cp.guard = guard;
    part[p * kMaxChunks + chunk] = cp;
  }
}

__global__ void __launch_bounds__(256)
problem_reduce_kernel(ProbDesc* __restrict__ probs, int N,
                      const double* __restrict__ lad,
                      const double* __restrict__ growth,
                      const ChunkPartial* __restrict__ part, int nchunks,
                      ProbStats* __restrict__ stats, int advance,
                      const double* __restrict__ mom,
                      const double* __restrict__ tsum, int hmc) {
  const int p = blockIdx.x;
  const ProbDesc P = probs[p];
  const int tid = threadIdx.x;
  __shared__ double s_full[256], s_red[256], s_gr[256];
  // each thread sums a strided subset of the 2M matrices in increasing b
  double full = 0.0, red = 0.0, gr = 0.0;
  for (int k = tid; k < 2 * P.Me; k += 256) {
    const int n = k % P.Me;
    const double w = (2.0 * n + 1.0) * kPi * P.T;
    const double l = lad[P.mat_begin + k];
    full += l;
    red += l - (double)N * log(w);
    gr = max_nan(gr, growth[P.mat_begin + k]);
  }
  if (P.Me < P.M) {
    // tail of both spins: 1/2 sum_m (-1)^(m+1)/m tr(H^2m) S_2m, plus
    // N sum_n ln w_n in the full sum
    const double* ts = tsum + (size_t)p * kTailS;
    const double* mb = mom + (size_t)p * 2 * kTailP * N;
    for (int i = tid; i < N; i += 256) {
      double r = 0.0;
      for (int sidx = 0; sidx < 2; ++sidx)
        for (int m = kTailK; m >= 1; --m)
          r += ((m & 1) ? 0.5 : -0.5) / m * ts[m] *
               mb[((size_t)sidx * kTailP + 2 * m - 1) * N + i];
      red += r;
      full += r;
    }
    if (tid == 0) full += 2.0 * (double)N * ts[0];
  }
  s_full[tid] = full; s_red[tid] = red; s_gr[tid] = gr;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (tid < w) {
      s_full[tid] += s_full[tid + w];
      s_red[tid] += s_red[tid + w];
      s_gr[tid] = max_nan(s_gr[tid], s_gr[tid + w]);
    }
    __syncthreads();
  }
  if (tid == 0) {
    double phi2 = 0.0, stag = 0.0, gmax = 0.0, k0 = 0.0, k1 = 0.0;
    int nf = 0;
    for (int c = 0; c < nchunks; ++c) {
      const ChunkPartial cp = part[p * kMaxChunks + c];
      phi2 += cp.phi2; stag += cp.stag; gmax = max_nan(gmax, cp.gmax);
      k0 += cp.kin0; k1 += cp.kin;
      nf |= cp.nonfinite;
    }
    const int guard = part[p * kMaxChunks].guard;
    ProbStats S;
    S.omega = phi2 / P.U - 2.0 * P.T * s_full[0];
    S.omega_tilde = phi2 / P.U - 2.0 * P.T * s_red[0];
    S.max_abs_grad = gmax;
    S.af_order = fabs(stag) / (double)N;
    S.pivot_growth = s_gr[0];
    nf |= !isfinite(S.omega) || !isfinite(S.omega_tilde);
    S.nonfinite = nf;
    S.tail_range = (guard & kGuardTail) ? 1 : 0;
    S.kin0 = 0.5 * k0;
    S.kin = 0.5 * k1;
    S.growth_run = max_nan(P.growth_run, s_gr[0]);
    S.guard = guard;
    // the site kernel of this pass has read adam_t and steps_left already;
    // it applied the update exactly when the same condition held
    const bool upd = advance && P.steps_left > 0 && !guard;
    S.updated = upd ? 1 : 0;
    S.adam_t = P.adam_t + (upd ? 1 : 0);
    S.steps_left = P.steps_left - (upd ? 1 : 0);
    stats[p] = S;
    probs[p].growth_run = S.growth_run;
    if (upd) {
      probs[p].adam_t = S.adam_t;
      probs[p].steps_left = S.steps_left;
    }
    if (hmc && P.hmc_L > 0) probs[p].hmc_k = P.hmc_k + 1;
  }
}

size_t reduce_workspace_bytes(int nprob) {
  return (size_t)nprob * kMaxChunks * sizeof(ChunkPartial);
}

int reduce_max_sites() { return kSitesPerBlock * kMaxChunks; }

hipError_t launch_reduce(ProbDesc* probs, int nprob, int N, const double* lad,
                         const double* dg, const double* growth,
                         ProbStats* stats, bool adam, void* ws,
                         const double* mom, const double* tsum,
                         hipStream_t st, bool hmc) {
  if (nprob <= 0) return hipSuccess;
  const int nchunks = (N + kSitesPerBlock - 1) / kSitesPerBlock;
  if (nchunks > kMaxChunks) return hipErrorInvalidValue;
  ChunkPartial* part = static_cast<ChunkPartial*>(ws);
  mark_begin(K_REDUCE, st);
  hipLaunchKernelGGL(site_reduce_kernel, dim3(nchunks, nprob),
                     dim3(kReduceThreads), 0, st, probs, N, dg, growth, part,
                     (int)adam, mom, tsum, (int)(hmc && dg != nullptr));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(problem_reduce_kernel, dim3(nprob), dim3(256), 0, st,
                     probs, N, lad, growth, part, nchunks, stats,
                     (int)(adam && dg != nullptr), mom, tsum,
                     (int)(hmc && dg != nullptr));
  mark_end(K_REDUCE, st);
  return hipGetLastError();
}

__global__ void dos_reduce_kernel(const double* __restrict__ dg, int n_w,
                                  int N, double* __restrict__ rho) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (j >= n_w) return;
  const double* x = dg + ((size_t)(s * n_w + j) * N) * 2;
  double acc = 0.0;
  for (int i = 0; i < N; ++i) acc += x[2 * i + 1];
  rho[s * n_w + j] = -acc / (kPi * (double)N);
}

hipError_t launch_dos_reduce(const double* dg, int n_w, int N, double* rho,
                             hipStream_t st) {
  if (n_w <= 0) return hipSuccess;
  hipLaunchKernelGGL(dos_reduce_kernel, dim3((n_w + 127) / 128, 2), dim3(128),
                     0, st, dg, n_w, N, rho);
  return hipGetLastError();
}

}  // namespace sca

namespace sca {

__global__ void shift_desc_kernel(const double* __restrict__ z, int n_z,
                                  double t, int hoff0, int N,
                                  MatDesc* __restrict__ descs) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int sidx = blockIdx.y;
  if (j >= n_z) return;
  MatDesc d;
  d.zr = z[2 * j];
  d.zi = z[2 * j + 1];
  d.t = t;
  d.hoff = hoff0 + sidx * N;
  d.prob = 0;
  descs[sidx * n_z + j] = d;
}

hipError_t launch_shift_descs(const double* z, int n_z, double t, int hoff0,
                              int N, MatDesc* descs, hipStream_t st) {
  if (n_z <= 0) return hipSuccess;
  hipLaunchKernelGGL(shift_desc_kernel, dim3((n_z + 255) / 256, 2), dim3(256),
                     0, st, z, n_z, t, hoff0, N, descs);
  return hipGetLastError();
}

}  // namespace sca
