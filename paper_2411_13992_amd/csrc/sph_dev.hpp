// Device-side building blocks shared by the libsph kernels (gfx950).
//
// Particles live in (cell, id) order; a particle's position is its cell's
// origin plus a cell-local offset.  A sweep gives one thread to particle i and
// walks the 3^D cells around i's cell through the CSR array cell_start.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace sph {

constexpr int kBlock = 256;          // threads per block for every particle kernel
constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kNumPartials = 9;      // per-block diagnostic partials
constexpr double kPi = 3.14159265358979323846;

// Host-computed description of the grid, passed by value to kernels.
struct Grid {
  int n;            // particles
  int nc[3];        // cells per axis (nc[2] = 1 in 2-D)
  int ncells;
  double L[3];      // exact cell edges (box / nc)
  double box[3];    // periodic box edges
};

// Host-computed coefficients in the sweep precision T.
template <typename T>
struct Coeffs {
  T L[3];           // cell edges rounded towards zero into T
  T h, inv_h;       // uniform smoothing length (h_min when per-particle h is absent)
  T sup2;           // (2h)^2, squared support radius for uniform h
  T alpha;          // Wendland normalisation alpha_D(h)
  T fcoef;          // -5 alpha / h^2: F(r) = fcoef (1 - q/2)^3
  T mass;           // uniform mass
  T rho0, c0, c0sq, inv_c0, eta, riemann_eta;
  T inv_kappa;
  T dt, half_dt;
  double xi, lim_c, lim_s0, hmin2, band_tol, inv_dt;
};

// ---------------------------------------------------------------- math
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fsqrt(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }
// 1/sqrt(x); callers guarantee x > 0
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double frsq(double x) { return 1.0 / __builtin_sqrt(x); }

template <typename T>
__device__ __forceinline__ T tmin(T a, T b) { return a < b ? a : b; }
template <typename T>
__device__ __forceinline__ T tmax(T a, T b) { return a > b ? a : b; }

// Wendland C2 normalisation alpha_D(h) for a per-pair smoothing length
template <int D, typename T>
__device__ __forceinline__ T wendland_alpha(T inv_h) {
  if constexpr (D == 2) return T(7.0 / (4.0 * kPi)) * inv_h * inv_h;
  else return T(21.0 / (16.0 * kPi)) * inv_h * inv_h * inv_h;
}

// (1 - q/2)^4 (1 + 2q): W / alpha for q < 2
template <typename T>
__device__ __forceinline__ T wendland_shape(T q) {
  T t = T(1) - T(0.5) * q;
  T t2 = t * t;
  return t2 * t2 * (T(1) + T(2) * q);
}

// ---------------------------------------------------------------- sums
// Kahan-compensated accumulator (compensation on for FP32 sweeps).
template <typename T, bool COMP>
struct Acc {
  T s, c;
  __device__ __forceinline__ void init(T x) { s = x; c = T(0); }
  __device__ __forceinline__ void add(T x) {
    if constexpr (COMP) {
      T y = x - c;
      T t = s + y;
      c = (t - s) - y;
      s = t;
    } else {
      s += x;
    }
  }
  __device__ __forceinline__ T value() const { return COMP ? s - c : s; }
};

template <typename T>
struct UseKahan { static constexpr bool value = false; };
template <>
struct UseKahan<float> { static constexpr bool value = true; };

// ---------------------------------------------------------------- cells
__device__ __forceinline__ int wrap_index(int x, int n) {
  x += (x < 0) ? n : 0;
  x -= (x >= n) ? n : 0;
  return x;
}

template <int D>
__device__ __forceinline__ void decode_cell(const Grid& g, int cell, int c[3]) {
  c[0] = cell % g.nc[0];
  int rest = cell / g.nc[0];
  if constexpr (D == 3) {
    c[1] = rest % g.nc[1];
    c[2] = rest / g.nc[1];
  } else {
    c[1] = rest;
    c[2] = 0;
  }
}

// Calls body(j, shift) for every particle j of the 3^D cells around `cell`
// (the particle's own cell included, so j == i is visited once).  shift[k]
// is the offset of j's cell origin from i's cell origin: r_i - r_j =
// (o_i - o_j) - shift.
template <int D, typename T, typename Body>
__device__ __forceinline__ void for_each_candidate(const Grid& g, const Coeffs<T>& k, int cell,
                                                   const int* __restrict__ cs, Body&& body) {
  int c[3];
  decode_cell<D>(g, cell, c);
  constexpr int zlo = (D == 3) ? -1 : 0;
  constexpr int zhi = (D == 3) ? 1 : 0;
#pragma unroll
  for (int dz = zlo; dz <= zhi; ++dz) {
    int z = (D == 3) ? wrap_index(c[2] + dz, g.nc[2]) : 0;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      int y = wrap_index(c[1] + dy, g.nc[1]);
      int row = g.nc[0] * (y + g.nc[1] * z);
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        int x = wrap_index(c[0] + dx, g.nc[0]);
        int cc = row + x;
        int b = cs[cc];
        int e = cs[cc + 1];
        T shift[3] = {T(dx) * k.L[0], T(dy) * k.L[1], T(dz) * k.L[2]};
        for (int j = b; j < e; ++j) body(j, shift);
      }
    }
  }
}

// ---------------------------------------------------------------- reductions
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int m = kWave / 2; m > 0; m >>= 1) v += __shfl_xor(v, m, kWave);
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int m = kWave / 2; m > 0; m >>= 1) {
    T o = __shfl_xor(v, m, kWave);
    v = v > o ? v : o;
  }
  return v;
}

// Block-wide sum/max of one value per thread (blockDim.x == kBlock); the
// result is valid in thread 0.  Fixed order, hence deterministic.
template <typename T, bool MAX>
__device__ __forceinline__ T block_reduce(T v, T* lds /* kBlock / kWave entries */) {
  v = MAX ? wave_max(v) : wave_sum(v);
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  T r = lds[0];
  for (int w = 1; w < kBlock / kWave; ++w) r = MAX ? (r > lds[w] ? r : lds[w]) : r + lds[w];
  return r;
}

}  // namespace sph
