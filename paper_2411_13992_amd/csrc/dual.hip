// Dual-criteria time stepping (Sec. 2.4, Eq. 9-11) with the continuity
// equation (Eq. 3a) and the Riemann solver (Eq. 5-6).
//
// One advection step of size dt_ad = CFL_ad h_min / max(|v|_max, nu / h_min,
// U_ref) on a sorted state:
//   density summation (Eq. 8; density_kernel)
//   prologue sweep: the viscous acceleration of Eq. 7 (held for the step),
//     the correction of Eq. 14/16 (written into the displacement accumulator
//     delta), and drho/dt of Eq. 3a at the step's start
//   K substeps, each two sweeps on the step's topology (the cells, offsets
//     and pairs of the step's start stay as they are; particles only
//     accumulate their displacement in delta):
//       pressure sweep:   rho' = rho + dt/2 drho/dt (of i and of each j),
//                         v+ = v + dt (a^p(rho', v) + a^visc)  (Eq. 3b, 5-6),
//                         delta += dt (v + v+) / 2
//       continuity sweep: drho/dt at (rho', v+) (Eq. 3a with U* of Eq. 5),
//                         rho+ = rho' + dt/2 drho/dt
//     with dt = min(CFL_ac h_min / (|v|_max + c0), dt_ad - t) (Eq. 11), 0
//     once the substeps cover dt_ad (the launch then only copies through)
//   move: offsets += delta, rebinning, staging for the next cell build.
// The step sizes live on the device: a clock of K + 1 slots per step holds
// each substep's start time and the largest speed at its start, the latter
// gathered with integer atomic maxima on the bits of non-negative doubles
// (exact and order-independent).  Every kernel derives dt_ad and its dt from
// the clock with the same FP64 arithmetic.  Velocity, density and its rate
// are double-buffered across the substeps (substep k reads buffer k & 1).
#include "sph_internal.hpp"

namespace sph {

__device__ __forceinline__ double bits_to_double(unsigned long long b) {
  return __builtin_bit_cast(double, b);
}
__device__ __forceinline__ unsigned long long double_to_bits(double x) {
  return __builtin_bit_cast(unsigned long long, x);
}

// Eq. 9-10
__device__ __forceinline__ double dt_advection(const DualCoeffs& q, const DualSlot* clk) {
  const double vmax = bits_to_double(clk[0].vmax_bits);
  const double vad = fmax(vmax, fmax(q.nu / q.h_min, q.u_ref));
  return q.cfl_ad * q.h_min / vad;
}

// Size of substep k (0 when the step is already covered), Eq. 11
__device__ __forceinline__ double substep_dt(const DualCoeffs& q, const DualSlot* clk, int k) {
  const double dt_ad = dt_advection(q, clk);
  const double t = k == 0 ? 0.0 : clk[k].t;
  if (!(t < dt_ad) || k >= q.cap) return 0.0;
  const double vk = bits_to_double(clk[k].vmax_bits);
  return fmin(q.cfl_ac * q.h_min / (vk + q.c0), dt_ad - t);
}

// Largest |v| of the block's valid lanes into slot->vmax_bits; every thread
// of the block calls it (it synchronises the block).  Requests to one address
// serialise where device-scope atomics are served, so the block reduces first
// (one request per block, not per wavefront), and as the slot only grows a
// block whose maximum is not above what the slot already holds skips its
// atomic.  A stale read only costs an unneeded atomic; the result is the same
// maximum.
__device__ __forceinline__ void block_vmax(double speed, DualSlot* slot) {
  __shared__ double red[kBlock / kWave];
  const double w = wave_max(speed);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int q = 1; q < kBlock / kWave; ++q) m = fmax(m, red[q]);
    if (m > 0.0) {
      const unsigned long long b = double_to_bits(m);
      if (__hip_atomic_load(&slot->vmax_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < b)
        atomicMax(&slot->vmax_bits, b);
    }
  }
}

// The listed neighbour walk of particle i on the step's topology: body(j,
// rv, r2, ph, pg, t3) for every neighbour j (r_ij = rv, |r_ij|^2 = r2), in the
// order of for_each_candidate.
template <int D, typename T, bool VAR, int G, int CAP, typename Body>
__device__ __forceinline__ void topology_walk(const Grid& g, const Coeffs<T>& k,
                                              const int* __restrict__ cell,
                                              const int* __restrict__ cs,
                                              const Cols<T, D>& offc, const Cols<T, 1>& hc,
                                              int i, int sub, const T* oi, T hi,
                                              Stage<D, T, D + (VAR ? 1 : 0),
                                                    StageCap<D, T>::value>& st,
                                              NeighbourList<CAP>& nl, Body&& body) {
  constexpr int NS = D + (VAR ? 1 : 0);
  auto srct = [&](int j, T* v) {
#pragma unroll
    for (int d = 0; d < D; ++d) v[d] = offc(d, j);
    if constexpr (VAR) v[D] = hc(0, j);
  };
  auto test = [&](int j, const T* v, const T* sh) -> bool {
    T r2 = T(0);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const T rv = (oi[d] - v[d]) - sh[d];
      r2 = tfma(rv, rv, r2);
    }
    return (j != i) & (r2 < pair_h<D, T, VAR>(k, hi, VAR ? v[D] : T(0)).sup2);
  };
  auto walk_body = [&](int j, const T* sh) {
    T rv[3] = {T(0), T(0), T(0)};
    T r2 = T(0);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      rv[d] = (oi[d] - offc(d, j)) - sh[d];
      r2 = tfma(rv[d], rv[d], r2);
    }
    const PairH<D, T, VAR> ph = pair_h<D, T, VAR>(k, hi, VAR ? hc(0, j) : T(0));
    const PairGeo<T> pg = pair_geo(r2);
    const T t = kernel_t(pg.r, ph.inv_h);
    body(j, rv, ph, pg, t * t * t);
  };
  for_each_neighbour_listed<D, G, T, NS, candidate_batch<D, T, VAR>()>(g, k, cell[i], cs, sub, st,
                                                                     nl, srct, test, walk_body);
}

template <int G>
struct DualCap { static constexpr int value = G == 2 ? 24 : (G == 4 ? 16 : 8); };

// ------------------------------------------------------------------ prologue
// At the advection step's start (density just reinitialised): the viscous
// acceleration a^visc_i = (2 eta / rho_i) sum_j (m_j / rho_j) F_ij v_ij
// (Eq. 7), the correction sum g_i and its correction dr_i (Eq. 14/16, into
// delta), and drho_i/dt = rho_i sum_j (m_j / rho_j) F_ij (v_ij . r_ij +
// (p_i - p_j) |r_ij| / (rhobar c0)) (Eq. 3a with U* of Eq. 5).  Also clears
// the next step's clock and writes the correction's diagnostics partials.
template <int D, typename T, bool VAR, int G>
__global__ __launch_bounds__(kBlock) void dual_prologue_kernel(
    Grid g, Coeffs<T> k, DualCoeffs q, const int* __restrict__ cell, const int* __restrict__ cs,
    const T* __restrict__ off, const T* __restrict__ vel, const T* __restrict__ rho,
    const T* __restrict__ mass, const T* __restrict__ hh, T* __restrict__ visc,
    T* __restrict__ delta, T* __restrict__ drho, const DualSlot* __restrict__ clk,
    DualSlot* __restrict__ clk_next, double* __restrict__ partials,
    unsigned* __restrict__ flags) {
  __shared__ NeighbourList<DualCap<G>::value> nl;
  constexpr int NS = D + (VAR ? 1 : 0);
  __shared__ Stage<D, T, NS, StageCap<D, T>::value> st;
  const int n = g.n;
  const Cols<T, D> offc(off, n), velc(vel, n);
  const Cols<T, 1> rhoc(rho, n), hc(hh, n), mc(mass, n);
  auto srct = [&](int j, T* v) {
#pragma unroll
    for (int d = 0; d < D; ++d) v[d] = offc(d, j);
    if constexpr (VAR) v[D] = hc(0, j);
  };
  stage_positions<D, G>(g, cell, cs, st, srct);
  if (blockIdx.x == 0 && threadIdx.x <= q.K) clk_next[threadIdx.x] = DualSlot{0.0, 0ull};
  const int i = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int sub = threadIdx.x % G;
  const bool valid = i < n;
  const bool lead = valid && sub == 0;
  T rhoi = T(1);
  Acc<T, UseKahan<T>::value> av[3], tv[3], cr;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    av[d].init(T(0));
    tv[d].init(T(0));
  }
  cr.init(T(0));
  if (valid) {
    T oi[3] = {T(0), T(0), T(0)}, vi[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int d = 0; d < D; ++d) {
      oi[d] = off[d * n + i];
      vi[d] = vel[d * n + i];
    }
    rhoi = rho[i];
    const T pi = k.c0sq * (rhoi - k.rho0);
    const T hi = VAR ? hh[i] : k.h;
    topology_walk<D, T, VAR, G>(
        g, k, cell, cs, offc, hc, i, sub, oi, hi, st, nl,
        [&](int j, const T* rv, const PairH<D, T, VAR>& ph, const PairGeo<T>& pg, T t3) {
          const T F = ph.fc * t3;
          const T rhoj = rhoc(0, j);
          const T rinv = frcp(rhoj);
          const T mj = VAR ? mc(0, j) : k.mass;
          const T vol = mj * rinv;
          T vr = T(0);
#pragma unroll
          for (int d = 0; d < D; ++d) {
            const T vij = vi[d] - velc(d, j);
            vr = tfma(vij, rv[d], vr);
            av[d].add(vol * F * vij);
          }
          const T w = tv_weight<D, T, VAR>(ph, t3, rinv, mj);
#pragma unroll
          for (int d = 0; d < D; ++d) tv[d].add(w * rv[d]);
          const T pj = k.c0sq * (rhoj - k.rho0);
          const T diff = (pi - pj) * pg.r * frcp(T(0.5) * (rhoi + rhoj) * k.c0);
          cr.add(vol * F * (vr + diff));
        });
  }
  T ai[3], gi[3], dri[3] = {T(0), T(0), T(0)};
  const T s2 = T(2) * k.eta / rhoi;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    ai[d] = s2 * group_sum<G>(av[d]);
    gi[d] = tv_finish<T, VAR>(k, group_sum<G>(tv[d]));
  }
  const T crs = group_sum<G>(cr);
  double v[3] = {0.0, 0.0, 0.0};   // beta > 0, in band, |dr| / dt_ad
  if (lead) {
    const Limited lim = limit_correction<D>(k, gi, rhoi, dri);
    double d2 = 0.0;
    bool bad = false;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      visc[d * n + i] = ai[d];
      delta[d * n + i] = dri[d];
      d2 += (double)dri[d] * (double)dri[d];
      bad |= !isfinite(ai[d]);
    }
    const T dr_i = rhoi * crs;
    drho[i] = dr_i;
    bad |= !isfinite(dr_i);
    if (bad) atomicOr(flags, kFlagNonfinite);
    v[0] = lim.beta > 0.0 ? 1.0 : 0.0;
    v[1] = fabs(lim.s - k.lim_s0) <= k.band_tol * k.lim_s0 ? 1.0 : 0.0;
    v[2] = sqrt(d2) / dt_advection(q, clk);
  }
  if (partials) {
    const int cols[3] = {6, 7, 8};
    wave_partials<3>(partials, cols, v, 1u << 2, 3u);
  }
}

// ------------------------------------------------------------------ pressure substep
// Substep k: rho'_x = rho_x + dt/2 drho_x for i and every j; a^p_i =
// -(2 / rho'_i) sum_j (m_j / rho'_j) P*_ij F_ij r_ij with P* of Eq. 5-6 from
// the velocities at the substep's start; v+ = v + dt (a^p + a^visc) into the
// other velocity buffer; delta += dt (v + v+) / 2; the largest |v+| into the
// next clock slot.  With dt = 0 the velocities are copied through.
template <int D, typename T, bool VAR, int G>
__global__ __launch_bounds__(kBlock) void dual_pressure_kernel(
    Grid g, Coeffs<T> k, DualCoeffs q, int sk, const int* __restrict__ cell,
    const int* __restrict__ cs, const T* __restrict__ off, const T* __restrict__ vel,
    const T* __restrict__ rho, const T* __restrict__ drho, const T* __restrict__ mass,
    const T* __restrict__ hh, const T* __restrict__ visc, T* __restrict__ vel_out,
    T* __restrict__ delta, DualSlot* __restrict__ clk, unsigned* __restrict__ flags) {
  const int n = g.n;
  const double dt = substep_dt(q, clk, sk);
  const int i = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int sub = threadIdx.x % G;
  const bool valid = i < n;
  const bool lead = valid && sub == 0;
  if (dt == 0.0) {
    if (lead) {
#pragma unroll
      for (int d = 0; d < D; ++d) vel_out[d * n + i] = vel[d * n + i];
    }
    return;
  }
  __shared__ NeighbourList<DualCap<G>::value> nl;
  constexpr int NS = D + (VAR ? 1 : 0);
  __shared__ Stage<D, T, NS, StageCap<D, T>::value> st;
  const Cols<T, D> offc(off, n), velc(vel, n);
  const Cols<T, 1> rhoc(rho, n), drc(drho, n), hc(hh, n), mc(mass, n);
  auto srct = [&](int j, T* v) {
#pragma unroll
    for (int d = 0; d < D; ++d) v[d] = offc(d, j);
    if constexpr (VAR) v[D] = hc(0, j);
  };
  stage_positions<D, G>(g, cell, cs, st, srct);
  const T hdt = (T)(0.5 * dt);
  T vi[3] = {T(0), T(0), T(0)};
  T rhoi = T(1);
  Acc<T, UseKahan<T>::value> ap[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) ap[d].init(T(0));
  if (valid) {
    T oi[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int d = 0; d < D; ++d) {
      oi[d] = off[d * n + i];
      vi[d] = vel[d * n + i];
    }
    rhoi = tfma(hdt, drho[i], rho[i]);
    const T pi = k.c0sq * (rhoi - k.rho0);
    const T hi = VAR ? hh[i] : k.h;
    topology_walk<D, T, VAR, G>(
        g, k, cell, cs, offc, hc, i, sub, oi, hi, st, nl,
        [&](int j, const T* rv, const PairH<D, T, VAR>& ph, const PairGeo<T>& pg, T t3) {
          const T F = ph.fc * t3;
          T vr = T(0);
#pragma unroll
          for (int d = 0; d < D; ++d) vr = tfma(vi[d] - velc(d, j), rv[d], vr);
          const T du = -vr * pg.inv_r;
          const T br = tmin(k.riemann_eta * tmax(du * k.inv_c0, T(0)), T(1));
          const T rhoj = tfma(hdt, drc(0, j), rhoc(0, j));
          const T pj = k.c0sq * (rhoj - k.rho0);
          const T pstar = tfma(T(0.25) * br * (rhoi + rhoj) * k.c0, du, T(0.5) * (pi + pj));
          const T mj = VAR ? mc(0, j) : k.mass;
          const T coef = mj * F * frcp(rhoj) * pstar;
#pragma unroll
          for (int d = 0; d < D; ++d) ap[d].add(coef * rv[d]);
        });
  }
  const T s = T(-2) / rhoi;
  T a[3];
#pragma unroll
  for (int d = 0; d < D; ++d) a[d] = s * group_sum<G>(ap[d]);
  double speed = 0.0;
  if (lead) {
    const T tdt = (T)dt;
    double v2 = 0.0;
    bool bad = false;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const T vn = tfma(tdt, a[d] + visc[d * n + i], vi[d]);
      vel_out[d * n + i] = vn;
      delta[d * n + i] = tfma(hdt, vi[d] + vn, delta[d * n + i]);
      v2 += (double)vn * (double)vn;
      bad |= !isfinite(vn);
    }
    speed = sqrt(v2);
    if (bad) atomicOr(flags, kFlagNonfinite);
  }
  block_vmax(speed, &clk[sk + 1]);
}

// ------------------------------------------------------------------ continuity substep
// Substep k: drho+_i = rho'_i sum_j (m_j / rho'_j) F_ij (v+_ij . r_ij +
// (p'_i - p'_j) |r_ij| / (rhobar' c0)) (Eq. 3a with U* of Eq. 5) into the
// other rate buffer, rho+ = rho' + dt/2 drho+ into the other density buffer,
// and the next substep's start time t + dt into the clock.  With dt = 0 the
// density and its rate are copied through.
template <int D, typename T, bool VAR, int G>
__global__ __launch_bounds__(kBlock) void dual_continuity_kernel(
    Grid g, Coeffs<T> k, DualCoeffs q, int sk, const int* __restrict__ cell,
    const int* __restrict__ cs, const T* __restrict__ off, const T* __restrict__ vel,
    const T* __restrict__ rho, const T* __restrict__ drho, const T* __restrict__ mass,
    const T* __restrict__ hh, T* __restrict__ rho_out, T* __restrict__ drho_out,
    DualSlot* __restrict__ clk, unsigned* __restrict__ flags) {
  const int n = g.n;
  const double dt = substep_dt(q, clk, sk);
  const int i = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int sub = threadIdx.x % G;
  const bool valid = i < n;
  const bool lead = valid && sub == 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) clk[sk + 1].t = (sk == 0 ? 0.0 : clk[sk].t) + dt;
  if (dt == 0.0) {
    if (lead) {
      rho_out[i] = rho[i];
      drho_out[i] = drho[i];
    }
    return;
  }
  __shared__ NeighbourList<DualCap<G>::value> nl;
  constexpr int NS = D + (VAR ? 1 : 0);
  __shared__ Stage<D, T, NS, StageCap<D, T>::value> st;
  const Cols<T, D> offc(off, n), velc(vel, n);
  const Cols<T, 1> rhoc(rho, n), drc(drho, n), hc(hh, n), mc(mass, n);
  auto srct = [&](int j, T* v) {
#pragma unroll
    for (int d = 0; d < D; ++d) v[d] = offc(d, j);
    if constexpr (VAR) v[D] = hc(0, j);
  };
  stage_positions<D, G>(g, cell, cs, st, srct);
  const T hdt = (T)(0.5 * dt);
  T rhoi = T(1);
  Acc<T, UseKahan<T>::value> cr;
  cr.init(T(0));
  if (valid) {
    T oi[3] = {T(0), T(0), T(0)}, vi[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int d = 0; d < D; ++d) {
      oi[d] = off[d * n + i];
      vi[d] = vel[d * n + i];
    }
    rhoi = tfma(hdt, drho[i], rho[i]);
    const T pi = k.c0sq * (rhoi - k.rho0);
    const T hi = VAR ? hh[i] : k.h;
    topology_walk<D, T, VAR, G>(
        g, k, cell, cs, offc, hc, i, sub, oi, hi, st, nl,
        [&](int j, const T* rv, const PairH<D, T, VAR>& ph, const PairGeo<T>& pg, T t3) {
          const T F = ph.fc * t3;
          T vr = T(0);
#pragma unroll
          for (int d = 0; d < D; ++d) vr = tfma(vi[d] - velc(d, j), rv[d], vr);
          const T rhoj = tfma(hdt, drc(0, j), rhoc(0, j));
          const T pj = k.c0sq * (rhoj - k.rho0);
          const T diff = (pi - pj) * pg.r * frcp(T(0.5) * (rhoi + rhoj) * k.c0);
          const T mj = VAR ? mc(0, j) : k.mass;
          cr.add(mj * frcp(rhoj) * F * (vr + diff));
        });
  }
  const T crs = group_sum<G>(cr);
  if (lead) {
    const T dr = rhoi * crs;
    drho_out[i] = dr;
    const T r = tfma(hdt, dr, rhoi);
    rho_out[i] = r;
    if (!isfinite(r)) atomicOr(flags, kFlagNonfinite);
  }
}

// ------------------------------------------------------------------ move
// End of the advection step: offsets += delta with rebinning (a particle may
// cross one cell face per axis, else SPH_FLAG_CFL), staged for the cell
// build with the final velocity and density; kinetic energy, momentum and
// max |v| partials; the largest speed into the next step's clock; the step's
// record (dt_ad, substeps, time covered).  A step whose substeps did not
// cover dt_ad with the automatic substep budget sets SPH_FLAG_CFL.
template <int D, typename T, bool VAR, int G>
__global__ __launch_bounds__(kBlock) void dual_move_kernel(
    Grid g, Coeffs<T> k, DualCoeffs q, PArrays<T> a, const T* __restrict__ delta,
    PArrays<T> stg, int* __restrict__ counts, int* __restrict__ slot_out,
    const DualSlot* __restrict__ clk, DualSlot* __restrict__ clk_next,
    double* __restrict__ partials, double* __restrict__ record, unsigned* __restrict__ flags) {
  const int n = g.n;
  const int i = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int sub = threadIdx.x % G;
  const bool lead = i < n && sub == 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int used = 0;
    for (int s = 0; s < q.K; ++s) used += substep_dt(q, clk, s) > 0.0 ? 1 : 0;
    const double dt_ad = dt_advection(q, clk);
    const double t = clk[q.K].t;
    if (record) {
      record[0] = dt_ad;
      record[1] = (double)used;
      record[2] = t;
    }
    if (!q.capped && t < dt_ad) atomicOr(flags, kFlagCfl);
  }
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  int lin = 0;
  if (lead) {
    const double m = VAR ? (double)a.mass[i] : (double)k.mass;
    T o[3] = {T(0), T(0), T(0)}, dl[3] = {T(0), T(0), T(0)};
    const T zero[3] = {T(0), T(0), T(0)};
    double v2 = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      o[d] = a.off[d * n + i];
      dl[d] = delta[d * n + i];
      const T vd = a.vel[d * n + i];
      stg.vel[d * n + i] = vd;
      v2 += (double)vd * (double)vd;
      v[1 + d] = m * (double)vd;
    }
    v[0] = 0.5 * m * v2;
    v[4] = sqrt(v2);
    unsigned f = 0;
    lin = drift_rebin<D>(g, k, a.cell[i], o, zero, dl, f);
#pragma unroll
    for (int d = 0; d < D; ++d) stg.off[d * n + i] = o[d];
    stg.cell[i] = lin;
    stg.id[i] = a.id[i];
    stg.rho[i] = a.rho[i];
    if constexpr (VAR) {
      stg.mass[i] = a.mass[i];
      stg.h[i] = a.h[i];
    }
    if (f) atomicOr(flags, f);
  }
  block_vmax(v[4], &clk_next[0]);
  if (counts) {
    const int slot = wave_claim_slot(lead, lin, counts);
    if (lead) slot_out[i] = slot;
  }
  if (partials) {
    const int cols[5] = {0, 1, 2, 3, 4};
    wave_partials<5>(partials, cols, v, 1u << 4);
  }
}

// Largest |v| of the state into clk[0] (for the first advection step of a
// run; the clocks are cleared before).
template <typename T>
__global__ __launch_bounds__(kBlock) void dual_start_kernel(int n, int dim, const T* __restrict__ vel,
                                                            DualSlot* __restrict__ clk) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  double v2 = 0.0;
  if (i < n)
    for (int d = 0; d < dim; ++d) v2 += (double)vel[(size_t)d * n + i] * (double)vel[(size_t)d * n + i];
  block_vmax(sqrt(v2), &clk[0]);
}

// ------------------------------------------------------------------ launchers
template <typename T>
void launch_dual_start(hipStream_t s, int n, int dim, const T* vel, DualSlot* clk) {
  if (n == 0) return;
  hipLaunchKernelGGL(dual_start_kernel<T>, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, dim, vel,
                     clk);
}

template <typename T>
void launch_dual_prologue(const Launch& l, const Grid& g, const Coeffs<T>& k, const DualCoeffs& q,
                          const PArrays<T>& p, const int* cs, T* visc, T* delta, T* drho,
                          const DualSlot* clk, DualSlot* clk_next, double* partials,
                          unsigned* flags) {
  if (g.n == 0) return;
  SPH_SWEEP(dual_prologue_kernel, SPH_ARGS(g, k, q, p.cell, cs, p.off, p.vel, p.rho, p.mass, p.h,
                                           visc, delta, drho, clk, clk_next, partials, flags));
}

template <typename T>
void launch_dual_pressure(const Launch& l, const Grid& g, const Coeffs<T>& k,
                          const DualCoeffs& q, int sk, const PArrays<T>& p, const int* cs,
                          const T* vel, const T* rho, const T* drho, const T* visc, T* vel_out,
                          T* delta, DualSlot* clk, unsigned* flags) {
  if (g.n == 0) return;
  SPH_SWEEP(dual_pressure_kernel, SPH_ARGS(g, k, q, sk, p.cell, cs, p.off, vel, rho, drho, p.mass,
                                           p.h, visc, vel_out, delta, clk, flags));
}

template <typename T>
void launch_dual_continuity(const Launch& l, const Grid& g, const Coeffs<T>& k,
                            const DualCoeffs& q, int sk, const PArrays<T>& p, const int* cs,
                            const T* vel, const T* rho, const T* drho, T* rho_out, T* drho_out,
                            DualSlot* clk, unsigned* flags) {
  if (g.n == 0) return;
  SPH_SWEEP(dual_continuity_kernel, SPH_ARGS(g, k, q, sk, p.cell, cs, p.off, vel, rho, drho,
                                             p.mass, p.h, rho_out, drho_out, clk, flags));
}

template <typename T>
void launch_dual_move(const Launch& l, const Grid& g, const Coeffs<T>& k, const DualCoeffs& q,
                      const PArrays<T>& p, const T* delta, const PArrays<T>& stg, int* counts,
                      int* slot, const DualSlot* clk, DualSlot* clk_next, double* partials,
                      double* record, unsigned* flags) {
  if (g.n == 0) return;
  SPH_SWEEP(dual_move_kernel, SPH_ARGS(g, k, q, p, delta, stg, counts, slot, clk, clk_next,
                                       partials, record, flags));
}

#define SPH_INST(T)                                                                           \
  template void launch_dual_start<T>(hipStream_t, int, int, const T*, DualSlot*);             \
  template void launch_dual_prologue<T>(const Launch&, const Grid&, const Coeffs<T>&,         \
                                        const DualCoeffs&, const PArrays<T>&, const int*, T*, \
                                        T*, T*, const DualSlot*, DualSlot*, double*,          \
                                        unsigned*);                                           \
  template void launch_dual_pressure<T>(const Launch&, const Grid&, const Coeffs<T>&,         \
                                        const DualCoeffs&, int, const PArrays<T>&,            \
                                        const int*, const T*, const T*, const T*, const T*,   \
                                        T*, T*, DualSlot*, unsigned*);                        \
  template void launch_dual_continuity<T>(const Launch&, const Grid&, const Coeffs<T>&,       \
                                          const DualCoeffs&, int, const PArrays<T>&,          \
                                          const int*, const T*, const T*, const T*, T*, T*,   \
                                          DualSlot*, unsigned*);                              \
  template void launch_dual_move<T>(const Launch&, const Grid&, const Coeffs<T>&,             \
                                    const DualCoeffs&, const PArrays<T>&, const T*,           \
                                    const PArrays<T>&, int*, int*, const DualSlot*,           \
                                    DualSlot*, double*, double*, unsigned*);
SPH_INST(float)
SPH_INST(double)
#undef SPH_INST

}  // namespace sph
