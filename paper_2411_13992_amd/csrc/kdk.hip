// Kick-drift-kick integration around the sweeps, and the FP64 diagnostics.
//
// The first half kick, the drift (with the transport correction added to the
// displacement) and the rebinning into cells are one elementwise pass that
// writes the moved particles into staging buffers and claims their cell
// slots; the cell build then gathers them back in (cell, id) order.  The
// second half kick is fused with the per-block FP64 partial sums.
#include "sph_internal.hpp"

namespace sph {

// ------------------------------------------------------------------ stage copy
template <int D, typename T>
__global__ __launch_bounds__(kBlock) void stage_copy_kernel(int n, PArrays<T> src, PArrays<T> stg,
                                                            int* __restrict__ counts,
                                                            int* __restrict__ slot) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int c = src.cell[i];
  stg.cell[i] = c;
  stg.id[i] = src.id[i];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    stg.off[d * n + i] = src.off[d * n + i];
    if (src.vel) stg.vel[d * n + i] = src.vel[d * n + i];
    if (src.acc) stg.acc[d * n + i] = src.acc[d * n + i];
  }
  if (src.rho) stg.rho[i] = src.rho[i];
  if (src.mass) stg.mass[i] = src.mass[i];
  if (src.h) stg.h[i] = src.h[i];
  slot[i] = atomicAdd(&counts[c], 1);
}

template <typename T>
void launch_stage_copy(const Launch& l, int n, const PArrays<T>& src, const PArrays<T>& stg,
                       int* counts, int* slot) {
  if (n == 0) return;
  if (l.dim == 2)
    hipLaunchKernelGGL((stage_copy_kernel<2, T>), dim3(blocks_for(n)), dim3(kBlock), 0, l.stream,
                       n, src, stg, counts, slot);
  else
    hipLaunchKernelGGL((stage_copy_kernel<3, T>), dim3(blocks_for(n)), dim3(kBlock), 0, l.stream,
                       n, src, stg, counts, slot);
}

// ------------------------------------------------------------------ kick + drift + rebin
// v' = v + dt/2 a;  o' = o + dt v' + dr;  a particle may cross at most one
// cell face per axis per step (else SPH_FLAG_CFL).  Offsets stay in
// [0, L_T): a value that rounds onto a face starts the next cell at 0.
template <int D, typename T, bool VAR>
__global__ __launch_bounds__(kBlock) void drift_kernel(Grid g, Coeffs<T> k, PArrays<T> p,
                                                       const T* __restrict__ dr, PArrays<T> stg,
                                                       int* __restrict__ counts,
                                                       int* __restrict__ slot,
                                                       unsigned* __restrict__ flags) {
  const int n = g.n;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int c[3];
  decode_cell<D>(g, p.cell[i], c);
  unsigned f = 0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const T v = p.vel[d * n + i] + k.half_dt * p.acc[d * n + i];
    T o = p.off[d * n + i] + k.dt * v + (dr ? dr[d * n + i] : T(0));
    if (!isfinite(v) || !isfinite(o)) {
      f |= kFlagNonfinite;
      o = T(0);
    } else if (o < T(0)) {
      const T m = (T)((double)o + g.L[d]);
      if (m >= k.L[d]) {
        o = T(0);                     // rounds back onto this cell's lower face
      } else {
        c[d] -= 1;
        o = m;
        if (o < T(0)) {
          f |= kFlagCfl;
          o = T(0);
        }
      }
    } else if (o >= k.L[d]) {
      T m = (T)((double)o - g.L[d]);
      c[d] += 1;
      if (m < T(0)) m = T(0);         // inside [L_T, L): next cell's lower face
      if (m >= k.L[d]) {
        f |= kFlagCfl;
        m = T(0);
      }
      o = m;
    }
    c[d] = wrap_index(c[d], g.nc[d]);
    stg.off[d * n + i] = o;
    stg.vel[d * n + i] = v;
  }
  const int lin = c[0] + g.nc[0] * (c[1] + g.nc[1] * c[2]);
  stg.cell[i] = lin;
  stg.id[i] = p.id[i];
  if constexpr (VAR) {
    stg.mass[i] = p.mass[i];
    stg.h[i] = p.h[i];
  }
  slot[i] = atomicAdd(&counts[lin], 1);
  if (f) atomicOr(flags, f);
}

template <typename T>
void launch_drift(const Launch& l, const Grid& g, const Coeffs<T>& k, const PArrays<T>& p,
                  const T* dr, const PArrays<T>& stg, int* counts, int* slot, unsigned* flags) {
  if (g.n == 0) return;
#define SPH_DRIFT(D, V)                                                                        \
  hipLaunchKernelGGL((drift_kernel<D, T, V>), dim3(l.nblk), dim3(kBlock), 0, l.stream, g, k, p, \
                     dr, stg, counts, slot, flags)
  if (l.dim == 2) { if (l.var) SPH_DRIFT(2, true); else SPH_DRIFT(2, false); }
  else { if (l.var) SPH_DRIFT(3, true); else SPH_DRIFT(3, false); }
#undef SPH_DRIFT
}

// ------------------------------------------------------------------ kick + partials
// v = v + dt/2 a (when `write`), then per-block FP64 partials of the kinetic
// energy, momentum and max |v| of the resulting velocity.
template <int D, typename T>
__global__ __launch_bounds__(kBlock) void kick_kernel(Coeffs<T> k, int n, T* __restrict__ vel,
                                                      const T* __restrict__ acc,
                                                      const T* __restrict__ mass,
                                                      double* __restrict__ partials, int write,
                                                      unsigned* __restrict__ flags) {
  __shared__ double red[kBlock / kWave];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  double ke = 0.0, mom[3] = {0.0, 0.0, 0.0}, vmax = 0.0;
  if (i < n) {
    const double m = mass ? (double)mass[i] : (double)k.mass;
    double v2 = 0.0;
    bool bad = false;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      T v = vel[d * n + i];
      if (write) {
        v = v + k.half_dt * acc[d * n + i];
        vel[d * n + i] = v;
      }
      bad |= !isfinite(v);
      v2 += (double)v * (double)v;
      mom[d] = m * (double)v;
    }
    ke = 0.5 * m * v2;
    vmax = sqrt(v2);
    if (bad) atomicOr(flags, kFlagNonfinite);
  }
  if (partials) {
    double a = block_reduce<double, false>(ke, red);
    double b = block_reduce<double, false>(mom[0], red);
    double c = block_reduce<double, false>(mom[1], red);
    double d = block_reduce<double, false>(mom[2], red);
    double e = block_reduce<double, true>(vmax, red);
    if (threadIdx.x == 0) {
      double* o = partials + blockIdx.x * kNumPartials;
      o[0] = a;
      o[1] = b;
      o[2] = c;
      o[3] = d;
      o[4] = e;
    }
  }
}

template <typename T>
void launch_kick(const Launch& l, const Coeffs<T>& k, int n, T* vel, const T* acc,
                 const T* mass, double* partials, bool write, unsigned* flags) {
  if (n == 0) return;
  if (l.dim == 2)
    hipLaunchKernelGGL((kick_kernel<2, T>), dim3(l.nblk), dim3(kBlock), 0, l.stream, k, n, vel,
                       acc, mass, partials, write ? 1 : 0, flags);
  else
    hipLaunchKernelGGL((kick_kernel<3, T>), dim3(l.nblk), dim3(kBlock), 0, l.stream, k, n, vel,
                       acc, mass, partials, write ? 1 : 0, flags);
}

// ------------------------------------------------------------------ final reduction
// One block folds the per-block partials in a fixed order: deterministic.
__global__ __launch_bounds__(kBlock) void diag_final_kernel(int nblk, const double* __restrict__ partials,
                                                            double* __restrict__ diag) {
  __shared__ double red[kBlock / kWave];
  for (int col = 0; col < kNumPartials; ++col) {
    const bool is_max = (col == 4 || col == 8);
    double v = 0.0;
    for (int r = threadIdx.x; r < nblk; r += kBlock) {
      const double x = partials[r * kNumPartials + col];
      v = is_max ? (x > v ? x : v) : v + x;
    }
    double t = is_max ? block_reduce<double, true>(v, red) : block_reduce<double, false>(v, red);
    if (threadIdx.x == 0) diag[col] = t;
  }
}

void launch_diag_final(hipStream_t s, int nblk, const double* partials, double* diag) {
  hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(kBlock), 0, s, nblk, partials, diag);
}

__global__ __launch_bounds__(kBlock) void zero_double_kernel(double* __restrict__ p, long n) {
  long i = (long)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

void launch_zero_partials(hipStream_t s, int nblk, double* partials) {
  long n = (long)(nblk > 0 ? nblk : 1) * kNumPartials;
  hipLaunchKernelGGL(zero_double_kernel, dim3(blocks_for(n)), dim3(kBlock), 0, s, partials, n);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void zero_kernel(T* __restrict__ p, long n) {
  long i = (long)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = T(0);
}

template <typename T>
void launch_zero(hipStream_t s, T* p, long n) {
  if (n <= 0) return;
  hipLaunchKernelGGL((zero_kernel<T>), dim3(blocks_for(n)), dim3(kBlock), 0, s, p, n);
}

#define SPH_INST(T)                                                                          \
  template void launch_zero<T>(hipStream_t, T*, long);                                       \
  template void launch_stage_copy<T>(const Launch&, int, const PArrays<T>&, const PArrays<T>&,\
                                     int*, int*);                                            \
  template void launch_drift<T>(const Launch&, const Grid&, const Coeffs<T>&,                \
                                const PArrays<T>&, const T*, const PArrays<T>&, int*, int*,  \
                                unsigned*);                                                  \
  template void launch_kick<T>(const Launch&, const Coeffs<T>&, int, T*, const T*, const T*, \
                               double*, bool, unsigned*);
SPH_INST(float)
SPH_INST(double)
#undef SPH_INST

}  // namespace sph
