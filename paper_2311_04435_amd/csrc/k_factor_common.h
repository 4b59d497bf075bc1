// Device helpers shared by the factorisation kernels (k_factor.hip,
// k_ldlt.hip): the MFMA of each element type, a double readlane, DPP moves
// inside rows of 16 lanes (also the spectral route's wave sums, k_eig.hip),
// and the inverses of the two triangles of a diagonal block.
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>

namespace sca {
namespace {

// MFMA of the element type: 16x16x4, A[m][k] from lane (k<<4 | m), B[k][n]
// from lane (k<<4 | n); accumulator element i of lane (g<<4 | n) holds row
// m(g, i) of column n (f64: g + 4i, f32: 4g + i, as measured on gfx950).
template <typename T> struct Mma;
template <> struct Mma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int m(int g, int i) { return g + 4 * i; }
};
template <> struct Mma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int m(int g, int i) { return 4 * g + i; }
};

__device__ inline void argmax_wave(double& mag, int& row) {
  for (int off = 32; off >= 1; off >>= 1) {
    double om = __shfl_xor(mag, off);
    int orow = __shfl_xor(row, off);
    if (om > mag || (om == mag && orow < row)) { mag = om; row = orow; }
  }
}

constexpr int LD(int NB) { return NB + 1; }

__device__ inline double readlane_d(double v, int lane) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Cross-lane moves inside a row of 16 lanes (DPP controls: 0xB1 and 0x4E
// are quad permutations [1,0,3,2] and [2,3,0,1], 0x141 mirrors each half
// row, 0x140 the whole row).  After the four steps in that order every lane
// of a row has combined all 16 of its row's values.
template <int C> __device__ inline double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), C, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), C, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int C> __device__ inline int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, C, 0xF, 0xF, false);
}
__device__ inline double dmax(double a, double b) { return a > b ? a : b; }

// Wave maximum of a value that is never NaN (uniform result).
__device__ inline double wave_max_d(double v) {
  v = dmax(v, dpp_d<0xB1>(v));
  v = dmax(v, dpp_d<0x4E>(v));
  v = dmax(v, dpp_d<0x141>(v));
  v = dmax(v, dpp_d<0x140>(v));
  return dmax(dmax(readlane_d(v, 0), readlane_d(v, 16)),
              dmax(readlane_d(v, 32), readlane_d(v, 48)));
}

// Wave minimum of an int (uniform result).
__device__ inline int wave_min_i(int v) {
  v = min(v, dpp_i<0xB1>(v));
  v = min(v, dpp_i<0x4E>(v));
  v = min(v, dpp_i<0x141>(v));
  v = min(v, dpp_i<0x140>(v));
  return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
             min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

// Calls f(integral_constant<int, J>) for J = J0 .. J1-1 in order: a loop over
// compile-time indices, so register arrays indexed by J stay in registers.
template <int J0, int J1> struct StaticFor {
  template <class F> static __device__ __forceinline__ void run(F& f) {
    f(std::integral_constant<int, J0>{});
    StaticFor<J0 + 1, J1>::run(f);
  }
};
template <int J1> struct StaticFor<J1, J1> {
  template <class F> static __device__ __forceinline__ void run(F&) {}
};

// Inverses of the unit lower and the upper triangle of the NB x NB block
// (xr, xi; leading dimension NB+1), by recursive doubling: 4x4 leaves by
// one thread each, then for s = 8, 16, .. NB
//   [A 0; C D]^-1 = [A^-1 0; -D^-1 C A^-1  D^-1]
//   [A B; 0 D]^-1 = [A^-1  -A^-1 B D^-1; 0 D^-1]
// with the products spread over all threads.  Outputs carry explicit zeros
// and the unit diagonal of L^-1.  kUpper = false inverts only the lower
// triangle (ur, ui untouched).
template <typename T, int NB, int NT, bool kUpper = true>
__device__ void block_tri_inverses(const T* xr, const T* xi, T* lr, T* li,
                                   T* ur, T* ui, T* tr, T* ti, int tid) {
  constexpr int LDB = NB + 1;
  constexpr int NTRI = kUpper ? 2 : 1;   // triangles inverted
  for (int e = tid; e < NB * NB; e += NT) {
    const int r = e / NB, c = e % NB;
    lr[r * LDB + c] = 0.0; li[r * LDB + c] = 0.0;
    if (kUpper) { ur[r * LDB + c] = 0.0; ui[r * LDB + c] = 0.0; }
  }
  __syncthreads();
  constexpr int NLEAF = NB / 4;
  if (tid < NTRI * NLEAF) {
    const int o = 4 * (tid % NLEAF);
    if (tid < NLEAF) {
      for (int c = 0; c < 4; ++c) {
        lr[(o + c) * LDB + o + c] = 1.0;
        for (int r = c + 1; r < 4; ++r) {
          double sr = xr[(o + r) * LDB + o + c], si = xi[(o + r) * LDB + o + c];
          for (int k = c + 1; k < r; ++k) {
            const double ar = xr[(o + r) * LDB + o + k], ai = xi[(o + r) * LDB + o + k];
            const double br = lr[(o + k) * LDB + o + c], bi = li[(o + k) * LDB + o + c];
            sr += ar * br - ai * bi;
            si += ar * bi + ai * br;
          }
          lr[(o + r) * LDB + o + c] = -sr;
          li[(o + r) * LDB + o + c] = -si;
        }
      }
    } else {
      for (int c = 0; c < 4; ++c) {
        for (int r = c; r >= 0; --r) {
          double sr = (r == c) ? 1.0 : 0.0, si = 0.0;
          for (int k = r + 1; k <= c; ++k) {
            const double ar = xr[(o + r) * LDB + o + k], ai = xi[(o + r) * LDB + o + k];
            const double br = ur[(o + k) * LDB + o + c], bi = ui[(o + k) * LDB + o + c];
            sr -= ar * br - ai * bi;
            si -= ar * bi + ai * br;
          }
          const double pr = xr[(o + r) * LDB + o + r], pi = xi[(o + r) * LDB + o + r];
          const double d = pr * pr + pi * pi;
          ur[(o + r) * LDB + o + c] = (sr * pr + si * pi) / d;
          ui[(o + r) * LDB + o + c] = (si * pr - sr * pi) / d;
        }
      }
    }
  }
  __syncthreads();
  for (int sz = 8; sz <= NB; sz *= 2) {
    const int h = sz / 2, npair = NB / sz, per = npair * h * h;
    // T = C A^-1 (lower) and T = A^-1 B (upper), h x h per pair
    for (int e = tid; e < NTRI * per; e += NT) {
      const int up = e >= per, rest = e - up * per;
      const int pr_ = rest / (h * h), r = (rest / h) % h, c = rest % h;
      const int o = pr_ * sz;
      double sr = 0.0, si = 0.0;
      if (!up) {
        for (int k = c; k < h; ++k) {   // C[r][k] A^-1[k][c], A^-1 lower
          const double ar = xr[(o + h + r) * LDB + o + k], ai = xi[(o + h + r) * LDB + o + k];
          const double br = lr[(o + k) * LDB + o + c], bi = li[(o + k) * LDB + o + c];
          sr += ar * br - ai * bi;
          si += ar * bi + ai * br;
        }
      } else {
        for (int k = r; k < h; ++k) {   // A^-1[r][k] B[k][c], A^-1 upper
          const double ar = ur[(o + r) * LDB + o + k], ai = ui[(o + r) * LDB + o + k];
          const double br = xr[(o + k) * LDB + o + h + c], bi = xi[(o + k) * LDB + o + h + c];
          sr += ar * br - ai * bi;
          si += ar * bi + ai * br;
        }
      }
      tr[e] = sr;
      ti[e] = si;
    }
    __syncthreads();
    for (int e = tid; e < NTRI * per; e += NT) {
      const int up = e >= per, rest = e - up * per;
      const int pr_ = rest / (h * h), r = (rest / h) % h, c = rest % h;
      const int o = pr_ * sz;
      const T* Tr = tr + up * per + pr_ * h * h;
      const T* Ti = ti + up * per + pr_ * h * h;
      double sr = 0.0, si = 0.0;
      if (!up) {
        for (int k = 0; k <= r; ++k) {   // -D^-1[r][k] T[k][c], D^-1 lower
          const double ar = lr[(o + h + r) * LDB + o + h + k], ai = li[(o + h + r) * LDB + o + h + k];
          const double br = Tr[k * h + c], bi = Ti[k * h + c];
          sr += ar * br - ai * bi;
          si += ar * bi + ai * br;
        }
        lr[(o + h + r) * LDB + o + c] = -sr;
        li[(o + h + r) * LDB + o + c] = -si;
      } else {
        for (int k = 0; k <= c; ++k) {   // -T[r][k] D^-1[k][c], D^-1 upper
          const double ar = Tr[r * h + k], ai = Ti[r * h + k];
          const double br = ur[(o + h + k) * LDB + o + h + c], bi = ui[(o + h + k) * LDB + o + h + c];
          sr += ar * br - ai * bi;
          si += ar * bi + ai * br;
        }
        ur[(o + r) * LDB + o + h + c] = -sr;
        ui[(o + r) * LDB + o + h + c] = -si;
      }
    }
    __syncthreads();
  }
}

}  // namespace
}  // namespace sca
