// Neighbour sweeps of one TV-WCSPH step: density summation (Eq. 8), the
// transport-velocity correction with its limiter (Eq. 14-16) and the
// Riemann pressure + viscous accelerations (Eq. 2, 3b, 5-7).
//
// One thread per particle in (cell, id) order; each thread walks the 3^D
// cells around its own through cell_start.  Consecutive threads sit in the
// same or adjacent cells, so their neighbour reads hit the same cache lines.
// No floating-point atomics: every particle gathers its own sum.
#include "sph_internal.hpp"

namespace sph {

// ------------------------------------------------------------------ density
template <int D, typename T, bool VAR>
__global__ __launch_bounds__(kBlock) void density_kernel(
    Grid g, Coeffs<T> k, const int* __restrict__ cell, const int* __restrict__ cs,
    const T* __restrict__ off, const T* __restrict__ mass, const T* __restrict__ hh,
    T* __restrict__ rho, double* __restrict__ partials, int* __restrict__ counts,
    unsigned* __restrict__ flags) {
  __shared__ double red[kBlock / kWave];
  const int n = g.n;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  int cnt = 0;
  if (i < n) {
    T oi[3];
#pragma unroll
    for (int d = 0; d < D; ++d) oi[d] = off[d * n + i];
    const T hi = VAR ? hh[i] : k.h;
    Acc<T, UseKahan<T>::value> acc;
    if constexpr (VAR) acc.init(mass[i] * wendland_alpha<D>(frcp(hi)));
    else acc.init(T(1));
    for_each_candidate<D>(g, k, cell[i], cs, [&](int j, const T* sh) {
      T r2 = T(0);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        T rv = (oi[d] - off[d * n + j]) - sh[d];
        r2 += rv * rv;
      }
      if constexpr (VAR) {
        const T sup = hi + hh[j];
        if (r2 < sup * sup && j != i) {
          const T inv = frcp(T(0.5) * sup);
          acc.add(mass[j] * wendland_alpha<D>(inv) * wendland_shape(fsqrt(r2) * inv));
          ++cnt;
        }
      } else {
        if (r2 < k.sup2 && j != i) {
          acc.add(wendland_shape(fsqrt(r2) * k.inv_h));
          ++cnt;
        }
      }
    });
    // uniform: rho = m alpha (1 + sum shape) / kappa
    const T r = VAR ? acc.value() * k.inv_kappa : acc.value() * (k.mass * k.alpha * k.inv_kappa);
    rho[i] = r;
    if (counts) counts[i] = cnt;
    if (!isfinite(r)) atomicOr(flags, kFlagNonfinite);
  }
  if (partials) {
    double tot = block_reduce<double, false>((double)cnt, red);
    if (threadIdx.x == 0) partials[blockIdx.x * kNumPartials + 5] = tot;
  }
}

// ------------------------------------------------------------------ transport velocity
// g_i = sum_j V_j F_ij r_ij (V_j = m_j / rho_j); s_i = h_min^2 |g_i|^2 tested in
// FP64; beta_i = min(C s_i, 1) if s_i > s0 else 0; dr_i = xi beta_i h_min^2 g_i.
template <int D, typename T, bool VAR>
__global__ __launch_bounds__(kBlock) void tv_kernel(
    Grid g, Coeffs<T> k, const int* __restrict__ cell, const int* __restrict__ cs,
    const T* __restrict__ off, const T* __restrict__ rho, const T* __restrict__ mass,
    const T* __restrict__ hh, T* __restrict__ dr, T* __restrict__ beta_out,
    double* __restrict__ s_out, T* __restrict__ g_out, double* __restrict__ partials) {
  __shared__ double red[kBlock / kWave];
  const int n = g.n;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  double nbeta = 0.0, nband = 0.0, drmax = 0.0;
  if (i < n) {
    T oi[3];
#pragma unroll
    for (int d = 0; d < D; ++d) oi[d] = off[d * n + i];
    const T hi = VAR ? hh[i] : k.h;
    Acc<T, UseKahan<T>::value> acc[3];
#pragma unroll
    for (int d = 0; d < D; ++d) acc[d].init(T(0));
    for_each_candidate<D>(g, k, cell[i], cs, [&](int j, const T* sh) {
      T rv[3];
      T r2 = T(0);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        rv[d] = (oi[d] - off[d * n + j]) - sh[d];
        r2 += rv[d] * rv[d];
      }
      if constexpr (VAR) {
        const T sup = hi + hh[j];
        if (r2 < sup * sup && j != i) {
          const T inv = frcp(T(0.5) * sup);
          const T t = T(1) - T(0.5) * fsqrt(r2) * inv;
          // V_j F_ij = (m_j / rho_j) (-5 alpha_ij t^3 / h_ij^2)
          const T w = mass[j] * frcp(rho[j]) * T(-5) * wendland_alpha<D>(inv) * inv * inv *
                      (t * t * t);
#pragma unroll
          for (int d = 0; d < D; ++d) acc[d].add(w * rv[d]);
        }
      } else {
        if (r2 < k.sup2 && j != i) {
          const T t = T(1) - T(0.5) * fsqrt(r2) * k.inv_h;
          const T w = (t * t * t) * frcp(rho[j]);
#pragma unroll
          for (int d = 0; d < D; ++d) acc[d].add(w * rv[d]);
        }
      }
    });
    T gi[3];
    double g2 = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      gi[d] = VAR ? acc[d].value() : acc[d].value() * (k.fcoef * k.mass);
      g2 += (double)gi[d] * (double)gi[d];
    }
    const double s = k.hmin2 * g2;
    double b = 0.0;
    if (s > k.lim_s0) b = fmin(k.lim_c * s, 1.0);
    const double f = k.xi * b * k.hmin2;
    double d2 = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const T v = (T)(f * (double)gi[d]);
      dr[d * n + i] = v;
      d2 += (double)v * (double)v;
      if (g_out) g_out[d * n + i] = gi[d];
    }
    if (beta_out) beta_out[i] = (T)b;
    if (s_out) s_out[i] = s;
    nbeta = b > 0.0 ? 1.0 : 0.0;
    nband = fabs(s - k.lim_s0) <= k.band_tol * k.lim_s0 ? 1.0 : 0.0;
    drmax = sqrt(d2) * k.inv_dt;
  }
  if (partials) {
    double a = block_reduce<double, false>(nbeta, red);
    double b = block_reduce<double, false>(nband, red);
    double c = block_reduce<double, true>(drmax, red);
    if (threadIdx.x == 0) {
      partials[blockIdx.x * kNumPartials + 6] = a;
      partials[blockIdx.x * kNumPartials + 7] = b;
      partials[blockIdx.x * kNumPartials + 8] = c;
    }
  }
}

// ------------------------------------------------------------------ forces
// a_i = (2 / rho_i) sum_j (m_j / rho_j) F_ij (eta v_ij - P*_ij r_ij), with
// P* = (p_i + p_j)/2 + beta^R rhobar c0 dU / 2, dU = -(v_ij . r_ij) / r,
// beta^R = min(eta_R max(dU / c0, 0), 1), p = c0^2 (rho - rho0).
template <int D, typename T, bool VAR>
__global__ __launch_bounds__(kBlock) void forces_kernel(
    Grid g, Coeffs<T> k, const int* __restrict__ cell, const int* __restrict__ cs,
    const T* __restrict__ off, const T* __restrict__ vel, const T* __restrict__ rho,
    const T* __restrict__ mass, const T* __restrict__ hh, T* __restrict__ acc_out,
    unsigned* __restrict__ flags) {
  const int n = g.n;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  T oi[3], vi[3];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    oi[d] = off[d * n + i];
    vi[d] = vel[d * n + i];
  }
  const T rhoi = rho[i];
  const T pi = k.c0sq * (rhoi - k.rho0);
  const T hi = VAR ? hh[i] : k.h;
  Acc<T, UseKahan<T>::value> acc[3];
#pragma unroll
  for (int d = 0; d < D; ++d) acc[d].init(T(0));
  for_each_candidate<D>(g, k, cell[i], cs, [&](int j, const T* sh) {
    T rv[3];
    T r2 = T(0);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      rv[d] = (oi[d] - off[d * n + j]) - sh[d];
      r2 += rv[d] * rv[d];
    }
    T sup2, inv_h;
    if constexpr (VAR) {
      const T sup = hi + hh[j];
      sup2 = sup * sup;
      inv_h = frcp(T(0.5) * sup);
    } else {
      sup2 = k.sup2;
      inv_h = k.inv_h;
    }
    if (r2 < sup2 && j != i) {
      const T inv_r = r2 > T(0) ? frsq(r2) : T(0);
      const T t = T(1) - T(0.5) * (r2 * inv_r) * inv_h;
      T F;
      if constexpr (VAR) F = T(-5) * wendland_alpha<D>(inv_h) * inv_h * inv_h * (t * t * t);
      else F = k.fcoef * (t * t * t);
      T vij[3];
      T vr = T(0);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        vij[d] = vi[d] - vel[d * n + j];
        vr += vij[d] * rv[d];
      }
      const T du = -vr * inv_r;
      const T br = tmin(k.riemann_eta * tmax(du * k.inv_c0, T(0)), T(1));
      const T rhoj = rho[j];
      const T pj = k.c0sq * (rhoj - k.rho0);
      const T pstar = T(0.5) * (pi + pj) + T(0.25) * br * (rhoi + rhoj) * k.c0 * du;
      const T mj = VAR ? mass[j] : k.mass;
      const T coef = mj * F * frcp(rhoj);
#pragma unroll
      for (int d = 0; d < D; ++d) acc[d].add(coef * (k.eta * vij[d] - pstar * rv[d]));
    }
  });
  const T s = T(2) / rhoi;
  bool bad = false;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const T a = s * acc[d].value();
    acc_out[d * n + i] = a;
    bad |= !isfinite(a);
  }
  if (bad) atomicOr(flags, kFlagNonfinite);
}

// ------------------------------------------------------------------ launchers
template <typename T>
void launch_density(const Launch& l, const Grid& g, const Coeffs<T>& k, const PArrays<T>& p,
                    const int* cs, T* rho_out, double* partials, int* counts, unsigned* flags) {
  if (g.n == 0) return;
  dim3 grid(l.nblk), block(kBlock);
#define SPH_DENS(D, V)                                                                      \
  hipLaunchKernelGGL((density_kernel<D, T, V>), grid, block, 0, l.stream, g, k, p.cell, cs, \
                     p.off, p.mass, p.h, rho_out, partials, counts, flags)
  if (l.dim == 2) { if (l.var) SPH_DENS(2, true); else SPH_DENS(2, false); }
  else { if (l.var) SPH_DENS(3, true); else SPH_DENS(3, false); }
#undef SPH_DENS
}

template <typename T>
void launch_tv(const Launch& l, const Grid& g, const Coeffs<T>& k, const PArrays<T>& p,
               const int* cs, T* dr, T* beta, double* s_out, T* g_out, double* partials) {
  if (g.n == 0) return;
  dim3 grid(l.nblk), block(kBlock);
#define SPH_TV(D, V)                                                                        \
  hipLaunchKernelGGL((tv_kernel<D, T, V>), grid, block, 0, l.stream, g, k, p.cell, cs,      \
                     p.off, p.rho, p.mass, p.h, dr, beta, s_out, g_out, partials)
  if (l.dim == 2) { if (l.var) SPH_TV(2, true); else SPH_TV(2, false); }
  else { if (l.var) SPH_TV(3, true); else SPH_TV(3, false); }
#undef SPH_TV
}

template <typename T>
void launch_forces(const Launch& l, const Grid& g, const Coeffs<T>& k, const PArrays<T>& p,
                   const int* cs, const T* vel, T* acc_out, unsigned* flags) {
  if (g.n == 0) return;
  dim3 grid(l.nblk), block(kBlock);
#define SPH_FRC(D, V)                                                                       \
  hipLaunchKernelGGL((forces_kernel<D, T, V>), grid, block, 0, l.stream, g, k, p.cell, cs,  \
                     p.off, vel, p.rho, p.mass, p.h, acc_out, flags)
  if (l.dim == 2) { if (l.var) SPH_FRC(2, true); else SPH_FRC(2, false); }
  else { if (l.var) SPH_FRC(3, true); else SPH_FRC(3, false); }
#undef SPH_FRC
}

#define SPH_INST(T)                                                                          \
  template void launch_density<T>(const Launch&, const Grid&, const Coeffs<T>&,              \
                                  const PArrays<T>&, const int*, T*, double*, int*,          \
                                  unsigned*);                                                \
  template void launch_tv<T>(const Launch&, const Grid&, const Coeffs<T>&, const PArrays<T>&,\
                             const int*, T*, T*, double*, T*, double*);                      \
  template void launch_forces<T>(const Launch&, const Grid&, const Coeffs<T>&,               \
                                 const PArrays<T>&, const int*, const T*, T*, unsigned*);
SPH_INST(float)
SPH_INST(double)
#undef SPH_INST

}  // namespace sph
