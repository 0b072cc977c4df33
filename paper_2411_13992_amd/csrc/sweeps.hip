// Neighbour sweeps of one TV-WCSPH step: density summation (Eq. 8), the
// transport-velocity correction with its limiter (Eq. 14-16) and the
// Riemann pressure + viscous accelerations (Eq. 2, 3b, 5-7).
//
// A group of G consecutive lanes per particle (G = 2, 4 or 8, by size), the
// particles in (cell, id) order; the group walks the 3^D cells around the
// particle's own through cell_start, each lane every G-th candidate.
// Consecutive groups sit in the same or adjacent cells, so their neighbour
// reads hit the same cache lines.  No floating-point atomics: every particle
// gathers its own sum.  Wall particles (told by id) take part as neighbours
// and get the wall state of wall_state_kernel instead of their own sums.
//
// The force sweep has a fused form used inside multi-step runs: it also
// accumulates the transport-velocity sum g at the same positions and
// densities (the correction of the next step), applies the second half kick,
// the next step's first half kick, correction and drift, and claims the
// particle's cell slot for the next cell build.  Pair terms come from the
// shared helpers in sph_dev.hpp, so the fused and standalone sweeps produce
// bit-identical results.
#include "sph_internal.hpp"

namespace sph {

// ------------------------------------------------------------------ density
// Entries of the stored neighbour list each density thread holds in LDS
template <int D, int G>
constexpr int kDensityListCap = list_cap(D, G);

// LIST: also record each lane's neighbours into the stored list sl
template <int D, typename T, bool VAR, int G, bool LIST>
__device__ __forceinline__ void density_impl(
    const Grid& g, const Coeffs<T>& k, const int* __restrict__ cell, const int* __restrict__ cs,
    const T* __restrict__ off, const T* __restrict__ mass, const T* __restrict__ hh,
    T* __restrict__ rho, double* __restrict__ partials, int* __restrict__ counts,
    unsigned* __restrict__ flags, const StoredList& sl) {
  const int n = g.n;
  const Cols<T, D> offc(off, n);
  const Cols<T, 1> hc(hh, n), mc(mass, n);
  // candidate-test values: offsets, then h (variable resolution); staged in
  // LDS for the 2-D FP32 sweeps
  constexpr int NS = D + (VAR ? 1 : 0);
  auto srct = [&](int j, T* v) {
#pragma unroll
    for (int d = 0; d < D; ++d) v[d] = offc(d, j);
    if constexpr (VAR) v[D] = hc(0, j);
  };
  __shared__ Stage<D, T, NS, StageCap<D, T>::value> st;
  __shared__ NeighbourList<LIST ? kDensityListCap<D, G> : 1> nl;
  const int i = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int sub = threadIdx.x % G;
  const bool valid = i < n;
  // the particle's own values, read before the stage so that their round
  // trip overlaps the stage's
  T oi[3] = {T(0), T(0), T(0)};
  T hi = k.h, mi = T(0);
  int celli = 0;
  if (valid) {
    celli = cell[i];
#pragma unroll
    for (int d = 0; d < D; ++d) oi[d] = off[d * n + i];
    if constexpr (VAR) {
      hi = hh[i];
      mi = mass[i];
    }
  }
  stage_positions<D, G>(g, cell, cs, st, srct);
  if constexpr (LIST && D == 2 && StageCap<D, T>::value > 0) {
    // the stage's runs, for the force sweep's body stage over the same state
    if (sl.runs && threadIdx.x < 3) {
      sl.runs[blockIdx.x * 6 + threadIdx.x] = st.pstart[threadIdx.x];
      sl.runs[blockIdx.x * 6 + 3 + threadIdx.x] = st.plen[threadIdx.x];
    }
  }
  int cnt = 0;
  Acc<T, UseKahan<T>::value> acc;
  acc.init(T(0));
  if (valid) {
    if (sub == 0) {
      if constexpr (VAR) acc.init(mi * wendland_alpha<D>(frcp(hi)));
      else acc.init(T(1));
    }
    // lane L's neighbours go to the stored list (for the force sweep), first
    // into this thread's column of the LDS list
    auto record = [&](int j, unsigned code) {
      if (LIST && cnt < kDensityListCap<D, G>)
        nl.slot[cnt][threadIdx.x] = (unsigned)j | (code << list_jbits<D>());
      ++cnt;
    };
    // one candidate j with test values v (offsets, then h_j)
    auto pair = [&](int j, const T* v, const T* sh, bool live, unsigned code) {
      T r2 = T(0);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        T rv = (oi[d] - v[d]) - sh[d];
        r2 = tfma(rv, rv, r2);
      }
      if constexpr (VAR) {
        const T sup = hi + v[D];
        if (live && r2 < sup * sup && j != i) {
          const T inv = frcp(T(0.5) * sup);
          acc.add(mc(0, j) * wendland_alpha<D>(inv) * wendland_shape(fsqrt(r2) * inv));
          record(j, code);
        }
      } else {
        if (live && r2 < k.sup2 && j != i) {
          acc.add(wendland_shape(fsqrt(r2) * k.inv_h));
          record(j, code);
        }
      }
    };
    for_each_candidate_values<D, G, T, VAR>(g, k, celli, cs, sub, st, srct, pair);
  }
  if constexpr (LIST) {
    // the LDS list out to the stored list, row by row: a row's stores cover
    // consecutive lanes (coalesced); rows past a lane's count are not written
    const int L = blockIdx.x * kBlock + threadIdx.x;
    sl.count[L] = cnt;
    const int rows = min(cnt, (int)kDensityListCap<D, G>);
    int wave_rows = rows;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) wave_rows = max(wave_rows, __shfl_xor(wave_rows, o, kWave));
    unsigned* __restrict__ col = sl.entry + L;
    // eight rows at a time: their LDS reads first, then their stores
    constexpr int CAP = kDensityListCap<D, G>;
    for (int q0 = 0; q0 < wave_rows; q0 += 8) {
      unsigned ev[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (q0 + u < CAP) ev[u] = nl.slot[min(q0 + u, CAP - 1)][threadIdx.x];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (q0 + u < rows) col[(size_t)(q0 + u) * sl.stride] = ev[u];
    }
  }
  const T sum = group_sum<G>(acc);
  cnt = group_sum_int<G>(cnt);
  const bool lead = valid && sub == 0;
  if (lead) {
    // uniform: rho = m alpha (1 + sum shape) / kappa
    const T r = VAR ? sum * k.inv_kappa : sum * (k.mass * k.alpha * k.inv_kappa);
    rho[i] = r;
    if (counts) counts[i] = cnt;
    if (!isfinite(r) && flags) atomicOr(flags, kFlagNonfinite);
  }
  if (partials) {
    const int cols[1] = {5};
    double v[1] = {lead ? (double)cnt : 0.0};
    wave_partials<1>(partials, cols, v, 0u, 0u, 1u);
  }
}

template <int D, typename T, bool VAR, int G>
__global__ __launch_bounds__(kBlock) void density_kernel(
    Grid g, Coeffs<T> k, const int* __restrict__ cell, const int* __restrict__ cs,
    const T* __restrict__ off, const T* __restrict__ mass, const T* __restrict__ hh,
    T* __restrict__ rho, double* __restrict__ partials, int* __restrict__ counts,
    unsigned* __restrict__ flags) {
  density_impl<D, T, VAR, G, false>(g, k, cell, cs, off, mass, hh, rho, partials, counts, flags,
                                    StoredList{});
}

template <int D, typename T, bool VAR, int G>
__global__ __launch_bounds__(kBlock) void density_list_kernel(
    Grid g, Coeffs<T> k, const int* __restrict__ cell, const int* __restrict__ cs,
    const T* __restrict__ off, const T* __restrict__ mass, const T* __restrict__ hh,
    T* __restrict__ rho, double* __restrict__ partials, int* __restrict__ counts,
    unsigned* __restrict__ flags, StoredList sl) {
  density_impl<D, T, VAR, G, true>(g, k, cell, cs, off, mass, hh, rho, partials, counts, flags,
                                   sl);
}

// ------------------------------------------------------------------ transport velocity
// g_i = sum_j V_j F_ij r_ij (V_j = m_j / rho_j), then the correction of the
// chosen formulation from g_i (limit_correction, FP64).
template <int D, typename T, bool VAR, int G>
__global__ __launch_bounds__(kBlock) void tv_kernel(
    Grid g, Coeffs<T> k, const int* __restrict__ cell, const int* __restrict__ cs,
    const T* __restrict__ off, const T* __restrict__ rho, const T* __restrict__ mass,
    const T* __restrict__ hh, const int* __restrict__ id, T* __restrict__ dr,
    T* __restrict__ beta_out, double* __restrict__ s_out, T* __restrict__ g_out,
    double* __restrict__ partials, TvDrift<T> td) {
  const int n = g.n;
  if (td.clear) {
    for (long x = (long)blockIdx.x * kBlock + threadIdx.x; x < td.clear_n;
         x += (long)gridDim.x * kBlock)
      td.clear[x] = 0;
  }
  const Cols<T, D> offc(off, n);
  const Cols<T, 1> rhoc(rho, n), hc(hh, n), mc(mass, n);
  const int i = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int sub = threadIdx.x % G;
  const bool valid = i < n;
  const bool fluid = valid && !wall_at(k, n, id, i);   // walls get no correction
  Acc<T, UseKahan<T>::value> acc[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) acc[d].init(T(0));
  if (fluid) {
    T oi[3];
#pragma unroll
    for (int d = 0; d < D; ++d) oi[d] = off[d * n + i];
    const T hi = VAR ? hh[i] : k.h;
    auto load = [&](int j) { return candidate_of<D, T, VAR>(offc, hc, k, j); };
    for_each_candidate_batched<D, G, candidate_batch<D, T, VAR>()>(
        g, k, cell[i], cs, sub, load, [&](const Candidate<D, T>& cj, int j, const T* sh,
                                          bool live) {
          T rv[3];
          T r2 = T(0);
#pragma unroll
          for (int d = 0; d < D; ++d) {
            rv[d] = (oi[d] - cj.o[d]) - sh[d];
            r2 = tfma(rv[d], rv[d], r2);
          }
          if (!live || j == i) return;
          const PairH<D, T, VAR> ph = pair_h<D, T, VAR>(k, hi, cj.h);
          if (!(r2 < ph.sup2)) return;
          const PairGeo<T> pg = pair_geo(r2);
          const T t = kernel_t(pg.r, ph.inv_h);
          const T t3 = t * t * t;
          const T w = tv_weight<D, T, VAR>(ph, t3, frcp(rhoc(0, j)), VAR ? mc(0, j) : k.mass);
#pragma unroll
          for (int d = 0; d < D; ++d) acc[d].add(w * rv[d]);
        });
  }
  T gi[3], dri[3];
#pragma unroll
  for (int d = 0; d < D; ++d) gi[d] = tv_finish<T, VAR>(k, group_sum<G>(acc[d]));
  double v[3] = {0.0, 0.0, 0.0};   // beta > 0, in band, |dr| / dt
  if (valid && sub == 0) {
    Limited lim = limit_correction<D>(k, gi, rho[i], dri);
    if (!fluid) {
      // walls: no correction; g written as +0, as the fused sweep does
      lim = Limited{};
#pragma unroll
      for (int d = 0; d < D; ++d) {
        dri[d] = T(0);
        gi[d] = T(0);
      }
    }
    double d2 = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      dr[d * n + i] = dri[d];
      d2 += (double)dri[d] * (double)dri[d];
      if (g_out) g_out[d * n + i] = gi[d];
    }
    if (beta_out) beta_out[i] = (T)lim.beta;
    if (s_out) s_out[i] = lim.s;
    if (td.stg.off) {
      // v' = v + dt/2 a, o' = o + dt v' + dr, rebinned; walls stay in place
      const PArrays<T>& p = td.src;
      T o[3], vh[3];
#pragma unroll
      for (int d = 0; d < D; ++d) {
        vh[d] = !fluid ? p.vel[d * n + i] : tfma(k.half_dt, p.acc[d * n + i], p.vel[d * n + i]);
        o[d] = p.off[d * n + i];
      }
      unsigned f = 0;
      const int lin = !fluid ? p.cell[i] : drift_rebin<D>(g, k, p.cell[i], o, vh, dri, f);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        td.stg.off[d * n + i] = o[d];
        td.stg.vel[d * n + i] = vh[d];
      }
      td.stg.cell[i] = lin;
      td.stg.id[i] = p.id[i];
      if constexpr (VAR) {
        td.stg.mass[i] = p.mass[i];
        td.stg.h[i] = p.h[i];
      }
      if (f) atomicOr(td.flags, f);
    }
    v[0] = lim.beta > 0.0 ? 1.0 : 0.0;
    v[1] = fabs(lim.s - k.lim_s0) <= k.band_tol * k.lim_s0 ? 1.0 : 0.0;
    v[2] = sqrt(d2) * k.inv_dt;
  }
  if (partials) {
    const int cols[3] = {6, 7, 8};
    wave_partials<3>(partials, cols, v, 1u << 2, 3u);
  }
}

// ------------------------------------------------------------------ forces
// a_i = (2 / rho_i) sum_j (m_j / rho_j) F_ij (eta v_ij - P*_ij r_ij), with
// P* = (p_i + p_j)/2 + beta^R rhobar c0 dU / 2, dU = -(v_ij . r_ij) / r,
// beta^R = min(eta_R max(dU / c0, 0), 1), p = c0^2 (rho - rho0).
// The pair body is long, so the sweep walks its neighbours through a
// per-thread LDS list (for_each_neighbour_listed): positions are tested for
// every candidate, the body runs for neighbours only.
template <int G>
struct ForceCap { static constexpr int value = G == 2 ? 24 : (G == 4 ? 16 : 8); };

// LIST: the neighbours come from the stored list of the step's density sweep
// (no candidate tests, no LDS), else from the compacted walk.
template <int D, typename T, bool VAR, bool FUSED, int G, bool LIST>
__device__ __forceinline__ void forces_impl(
    const Grid& g, const Coeffs<T>& k, const int* __restrict__ cell, const int* __restrict__ cs,
    const T* __restrict__ off, const T* __restrict__ vel, const T* __restrict__ rho,
    const T* __restrict__ mass, const T* __restrict__ hh, const int* __restrict__ id,
    T* __restrict__ acc_out, unsigned* __restrict__ flags, const FusedOut<T>& fo,
    const StoredList& sl) {
  __shared__ NeighbourList<LIST ? 1 : ForceCap<G>::value> nl;
  const int n = g.n;
  if constexpr (FUSED) {
    if (fo.clear) {
      for (long x = (long)blockIdx.x * kBlock + threadIdx.x; x < fo.clear_n;
           x += (long)gridDim.x * kBlock)
        fo.clear[x] = 0;
    }
  }
  const Cols<T, D> offc(off, n), velc(vel, n);
  const Cols<T, 1> rhoc(rho, n), hc(hh, n), mc(mass, n);
  // candidate-test values: offsets, then h (variable resolution)
  constexpr int NS = D + (VAR ? 1 : 0);
  auto srct = [&](int j, T* v) {
#pragma unroll
    for (int d = 0; d < D; ++d) v[d] = offc(d, j);
    if constexpr (VAR) v[D] = hc(0, j);
  };
  __shared__ Stage<D, T, NS, LIST ? 0 : StageCap<D, T>::value> st;
  const int i = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int sub = threadIdx.x % G;
  const bool valid = i < n;
  const bool lead = valid && sub == 0;
  // the particle's own values, read before the stages so that their round
  // trip overlaps the stages'
  T oi[3] = {T(0), T(0), T(0)}, vi[3] = {T(0), T(0), T(0)};
  T ai[3] = {T(0), T(0), T(0)}, gi[3] = {T(0), T(0), T(0)};
  int celli = 0;
  T rhoi = T(1);
  if (valid) {
    celli = cell[i];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      oi[d] = off[d * n + i];
      vi[d] = vel[d * n + i];
    }
    rhoi = rho[i];
  }
  // wall particles: no acceleration, correction, kick or drift
  const bool wall = valid && wall_at(k, n, id, i);
  stage_positions<D, G>(g, cell, cs, st, srct);
  // with stored lists in uniform 2-D FP32, the neighbours' body values in LDS
  // (in FP64 the twice larger stage costs more occupancy than it saves)
  constexpr bool BSTAGE = LIST && body_stage_on<D, T, VAR>();
  constexpr int BCAP = BSTAGE ? 256 : 1;
  static_assert(!BSTAGE || BCAP == StageCap<D, T>::value, "runs found with the density's cap");
  __shared__ BodyStage<T, BCAP> bst;
  if constexpr (BSTAGE) stage_bodies<G>(g, cell, cs, off, vel, rho, bst, sl.runs);
  Acc<T, UseKahan<T>::value> acc[3], tv[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    acc[d].init(T(0));
    tv[d].init(T(0));
  }
  if (valid) {
    const T pi = k.c0sq * (rhoi - k.rho0);
    const T hi = VAR ? hh[i] : k.h;
    // branch-free, so a batch's loads are not moved behind a test
    auto test = [&](int j, const T* v, const T* sh) -> bool {
      T r2 = T(0);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const T rv = (oi[d] - v[d]) - sh[d];
        r2 = tfma(rv, rv, r2);
      }
      return (j != i) & (r2 < pair_h<D, T, VAR>(k, hi, VAR ? v[D] : T(0)).sup2);
    };
    // the pair body in two parts: fetch reads what it needs of neighbour j,
    // compute adds the pair's terms (the stored-list walk issues several
    // neighbours' fetches before their computes)
    auto fetch = [&](int j) {
      PairIn<D, T> nb;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        nb.o[d] = offc(d, j);
        nb.v[d] = velc(d, j);
      }
      nb.rho = rhoc(0, j);
      nb.m = VAR ? mc(0, j) : k.mass;
      nb.h = VAR ? hc(0, j) : T(0);
      return nb;
    };
    auto compute = [&](const PairIn<D, T>& nb, const T* sh) {
      T rv[3];
      T r2 = T(0);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        rv[d] = (oi[d] - nb.o[d]) - sh[d];
        r2 = tfma(rv[d], rv[d], r2);
      }
      const PairH<D, T, VAR> ph = pair_h<D, T, VAR>(k, hi, nb.h);
      const PairGeo<T> pg = pair_geo(r2);
      const T t = kernel_t(pg.r, ph.inv_h);
      const T t3 = t * t * t;
      const T F = ph.fc * t3;
      T vij[3];
      T vr = T(0);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        vij[d] = vi[d] - nb.v[d];
        vr = tfma(vij[d], rv[d], vr);
      }
      const T du = -vr * pg.inv_r;
      const T br = tmin(k.riemann_eta * tmax(du * k.inv_c0, T(0)), T(1));
      const T rhoj = nb.rho;
      const T rinv = frcp(rhoj);
      const T pj = k.c0sq * (rhoj - k.rho0);
      const T pstar = tfma(T(0.25) * br * (rhoi + rhoj) * k.c0, du, T(0.5) * (pi + pj));
      const T mj = nb.m;
      const T coef = mj * F * rinv;
#pragma unroll
      for (int d = 0; d < D; ++d) acc[d].add(coef * tfma(-pstar, rv[d], k.eta * vij[d]));
      if constexpr (FUSED) {
        const T w = tv_weight<D, T, VAR>(ph, t3, rinv, mj);
#pragma unroll
        for (int d = 0; d < D; ++d) tv[d].add(w * rv[d]);
      }
    };
    auto body = [&](int j, const T* sh) { compute(fetch(j), sh); };
    // a stored-list entry's values: from the body stage when its row's run
    // holds it (2-D), else through fetch; an entry without code bits (the
    // overflow walk) has row code 0 and is found in row 0's run or fetched
    auto fetch_entry = [&](unsigned e) {
      constexpr unsigned JM = (1u << list_jbits<D>()) - 1u;
      const int j = (int)(e & JM);
      if constexpr (BSTAGE) {
        const int r = (int)(e >> (list_jbits<D>() + 2));
        int o = j - bst.pstart[r];
        o += o < 0 ? n : 0;
        if (o < bst.plen[r]) {
          PairIn<D, T> nb;
          const auto v = bst.ov[r * BCAP + o];
          nb.o[0] = v.ox;
          nb.o[1] = v.oy;
          nb.v[0] = v.vx;
          nb.v[1] = v.vy;
          nb.rho = bst.rho[r * BCAP + o];
          nb.m = k.mass;
          nb.h = T(0);
          return nb;
        }
      }
      return fetch(j);
    };
    if (!wall) {
      if constexpr (LIST)
        for_each_neighbour_stored<D, G, T, NS>(g, k, celli, cs, sub, sl, srct, test, fetch_entry,
                                               compute);
      else
        for_each_neighbour_listed<D, G, T, NS, candidate_batch<D, T, VAR>()>(
            g, k, celli, cs, sub, st, nl, srct, test, body);
    }
  }
  const T s = T(2) / rhoi;
  bool bad = false;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    ai[d] = s * group_sum<G>(acc[d]);
    bad |= !isfinite(ai[d]);
    if (FUSED) gi[d] = tv_finish<T, VAR>(k, group_sum<G>(tv[d]));
  }
  if (lead) {
#pragma unroll
    for (int d = 0; d < D; ++d) acc_out[d * n + i] = ai[d];
    if (bad) atomicOr(flags, kFlagNonfinite);
  }
  if constexpr (FUSED) {
    // second half kick of this step, then the next step's half kick, correction
    // and drift; the moved particle goes to the staging buffers
    double v[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // ke, mom x3, vmax, nbeta, nband, drmax
    int lin = 0;
    if (lead && wall) {
      // a wall particle stays in place with its velocity; its cell slot is
      // claimed like any other
      lin = celli;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        fo.stg.off[d * n + i] = oi[d];
        fo.stg.vel[d * n + i] = vi[d];
        if (fo.kick_vel) fo.kick_vel[d * n + i] = vi[d];
        if (fo.g_next) fo.g_next[d * n + i] = T(0);
      }
      if (fo.g_next) fo.beta_next[i] = T(0);
      fo.stg.cell[i] = lin;
      fo.stg.id[i] = id[i];
      if constexpr (VAR) {
        fo.stg.mass[i] = mass[i];
        fo.stg.h[i] = hh[i];
      }
    } else if (lead) {
      const double m = VAR ? (double)mass[i] : (double)k.mass;
      T vh[3], dr[3] = {T(0), T(0), T(0)};
      double v2 = 0.0;
      bool badv = false;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const T vn = tfma(k.half_dt, ai[d], vi[d]);
        if (fo.kick_vel) fo.kick_vel[d * n + i] = vn;
        badv |= !isfinite(vn);
        v2 += (double)vn * (double)vn;
        v[1 + d] = m * (double)vn;
        vh[d] = tfma(k.half_dt, ai[d], vn);
      }
      if (badv) atomicOr(flags, kFlagNonfinite);
      v[0] = 0.5 * m * v2;
      v[4] = sqrt(v2);
      if (fo.apply_next) {
        const Limited lim = limit_correction<D>(k, gi, rhoi, dr);
        if (fo.g_next) {
#pragma unroll
          for (int d = 0; d < D; ++d) fo.g_next[d * n + i] = gi[d];
          fo.beta_next[i] = (T)lim.beta;
        }
        double d2 = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) d2 += (double)dr[d] * (double)dr[d];
        v[5] = lim.beta > 0.0 ? 1.0 : 0.0;
        v[6] = fabs(lim.s - k.lim_s0) <= k.band_tol * k.lim_s0 ? 1.0 : 0.0;
        v[7] = sqrt(d2) * k.inv_dt;
      }
      unsigned f = 0;
      T o2[3] = {oi[0], oi[1], oi[2]};
      lin = drift_rebin<D>(g, k, celli, o2, vh, dr, f);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        fo.stg.off[d * n + i] = o2[d];
        fo.stg.vel[d * n + i] = vh[d];
      }
      fo.stg.cell[i] = lin;
      fo.stg.id[i] = id[i];
      if constexpr (VAR) {
        fo.stg.mass[i] = mass[i];
        fo.stg.h[i] = hh[i];
      }
      if (f) atomicOr(flags, f);
    }
    // with counts given, the slot claim's atomic overlaps the diagnostics
    // reductions (the one-launch rebuild needs no slots)
    SlotClaim sc{};
    if (fo.counts) sc = slot_claim_issue(lead, lin, fo.counts);
    if (fo.part_cur) {
      const int cur_cols[5] = {0, 1, 2, 3, 4};
      wave_partials<5>(fo.part_cur, cur_cols, v, 1u << 4);
    }
    if (fo.part_next) {
      const int next_cols[3] = {6, 7, 8};
      wave_partials<3>(fo.part_next, next_cols, v + 5, 1u << 2, 3u);
    }
    if (fo.counts) {
      const int slot = slot_claim_finish(sc);
      if (lead) fo.slot[i] = slot;
    }
  }
}

template <int D, typename T, bool VAR, int G>
__global__ __launch_bounds__(kBlock) void forces_kernel(
    Grid g, Coeffs<T> k, const int* __restrict__ cell, const int* __restrict__ cs,
    const T* __restrict__ off, const T* __restrict__ vel, const T* __restrict__ rho,
    const T* __restrict__ mass, const T* __restrict__ hh, const int* __restrict__ id,
    T* __restrict__ acc_out, unsigned* __restrict__ flags, FusedOut<T> fo) {
  forces_impl<D, T, VAR, false, G, false>(g, k, cell, cs, off, vel, rho, mass, hh, id, acc_out,
                                          flags, fo, StoredList{});
}

template <int D, typename T, bool VAR, int G>
__global__ __launch_bounds__(kBlock) void forces_fused_kernel(
    Grid g, Coeffs<T> k, const int* __restrict__ cell, const int* __restrict__ cs,
    const T* __restrict__ off, const T* __restrict__ vel, const T* __restrict__ rho,
    const T* __restrict__ mass, const T* __restrict__ hh, const int* __restrict__ id,
    T* __restrict__ acc_out, unsigned* __restrict__ flags, FusedOut<T> fo) {
  forces_impl<D, T, VAR, true, G, false>(g, k, cell, cs, off, vel, rho, mass, hh, id, acc_out,
                                         flags, fo, StoredList{});
}

// the force sweep over the density sweep's stored lists
template <int D, typename T, bool VAR, int G>
__global__ __launch_bounds__(kBlock) void forces_list_kernel(
    Grid g, Coeffs<T> k, const int* __restrict__ cell, const int* __restrict__ cs,
    const T* __restrict__ off, const T* __restrict__ vel, const T* __restrict__ rho,
    const T* __restrict__ mass, const T* __restrict__ hh, const int* __restrict__ id,
    T* __restrict__ acc_out, unsigned* __restrict__ flags, FusedOut<T> fo, StoredList sl) {
  forces_impl<D, T, VAR, false, G, true>(g, k, cell, cs, off, vel, rho, mass, hh, id, acc_out,
                                         flags, fo, sl);
}

// the fused sweep over the density sweep's stored lists
template <int D, typename T, bool VAR, int G>
__global__ __launch_bounds__(kBlock) void forces_fused_list_kernel(
    Grid g, Coeffs<T> k, const int* __restrict__ cell, const int* __restrict__ cs,
    const T* __restrict__ off, const T* __restrict__ vel, const T* __restrict__ rho,
    const T* __restrict__ mass, const T* __restrict__ hh, const int* __restrict__ id,
    T* __restrict__ acc_out, unsigned* __restrict__ flags, FusedOut<T> fo, StoredList sl) {
  forces_impl<D, T, VAR, true, G, true>(g, k, cell, cs, off, vel, rho, mass, hh, id, acc_out,
                                        flags, fo, sl);
}

// ------------------------------------------------------------------ wall state
// For each wall particle a, from its fluid neighbours f (kernel-weighted
// averages): p_a = sum p_f W / sum W, rho_a = rho0 + p_a / c0^2 and the
// no-slip mirror velocity v_a = 2 u_a - sum v_f W / sum W (u_a prescribed);
// p_a = 0 and v_a = u_a without fluid neighbours.  Only wall entries of rho
// and vel are written and only fluid entries are read.  Wavefronts without a
// wall particle leave at once.
template <int D, typename T, bool VAR, int G>
__global__ __launch_bounds__(kBlock) void wall_state_kernel(
    Grid g, Coeffs<T> k, const int* __restrict__ cell, const int* __restrict__ cs,
    const T* __restrict__ off, const T* __restrict__ hh, const int* __restrict__ id,
    const T* __restrict__ wall_vel, int n_wall, T* __restrict__ rho, T* __restrict__ vel,
    T* __restrict__ wsum_out, T* __restrict__ wavg_out) {
  const int n = g.n;
  const int i = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int sub = threadIdx.x % G;
  const int idi = i < n ? id[i] : 0;
  const bool wall = i < n && is_wall(k, idi);
  if (!__any(wall)) return;     // whole wavefront: no lane needs a group sum
  const Cols<T, D> offc(off, n), velc(vel, n);
  const Cols<T, 1> rhoc(rho, n), hc(hh, n);
  Acc<T, UseKahan<T>::value> sw, sp, sv[3];
  sw.init(T(0));
  sp.init(T(0));
#pragma unroll
  for (int d = 0; d < 3; ++d) sv[d].init(T(0));
  if (wall) {
    T oi[3];
#pragma unroll
    for (int d = 0; d < D; ++d) oi[d] = off[d * n + i];
    const T hi = VAR ? hh[i] : k.h;
    auto load = [&](int j) { return candidate_of<D, T, VAR>(offc, hc, k, j); };
    for_each_candidate_batched<D, G, candidate_batch<D, T, VAR>()>(
        g, k, cell[i], cs, sub, load, [&](const Candidate<D, T>& cj, int j, const T* sh,
                                          bool live) {
          T r2 = T(0);
#pragma unroll
          for (int d = 0; d < D; ++d) {
            const T rv = (oi[d] - cj.o[d]) - sh[d];
            r2 = tfma(rv, rv, r2);
          }
          if (!live) return;
          T w;
          if constexpr (VAR) {
            const T sup = hi + cj.h;
            if (!(r2 < sup * sup)) return;
            const T inv = frcp(T(0.5) * sup);
            w = wendland_alpha<D>(inv) * wendland_shape(fsqrt(r2) * inv);
          } else {
            if (!(r2 < k.sup2)) return;
            w = wendland_shape(fsqrt(r2) * k.inv_h);   // alpha cancels in the ratios
          }
          if (is_wall(k, id[j])) return;               // fluid neighbours only
          sw.add(w);
          sp.add(k.c0sq * (rhoc(0, j) - k.rho0) * w);
#pragma unroll
          for (int d = 0; d < D; ++d) sv[d].add(velc(d, j) * w);
        });
  }
  const T S = group_sum<G>(sw);
  const T P = group_sum<G>(sp);
  T V[3];
#pragma unroll
  for (int d = 0; d < D; ++d) V[d] = group_sum<G>(sv[d]);
  if (wall && sub == 0) {
    const int w = idi - k.nfluid;      // < n_wall for ids below n
    const bool any = S > T(0);
    const T inv = any ? T(1) / S : T(0);
    rho[i] = k.rho0 + (any ? P * inv : T(0)) / k.c0sq;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const T ua = w < n_wall ? wall_vel[(size_t)d * n_wall + w] : T(0);
      vel[d * n + i] = T(2) * ua - (any ? V[d] * inv : ua);
    }
    // for the adjoint: sum W (with alpha) and the averaged fluid velocity
    if (wsum_out && w < n_wall) {
      wsum_out[w] = VAR ? S : S * k.alpha;
#pragma unroll
      for (int d = 0; d < D; ++d) wavg_out[(size_t)d * n_wall + w] = any ? V[d] * inv : T(0);
    }
  }
}

// ------------------------------------------------------------------ launchers


template <typename T>
void launch_density(const Launch& l, const Grid& g, const Coeffs<T>& k, const PArrays<T>& p,
                    const int* cs, T* rho_out, double* partials, int* counts, unsigned* flags,
                    const StoredList& sl) {
  if (g.n == 0) return;
  if (sl.entry)
    SPH_SWEEP(density_list_kernel, SPH_ARGS(g, k, p.cell, cs, p.off, p.mass, p.h, rho_out,
                                            partials, counts, flags, sl));
  else
    SPH_SWEEP(density_kernel, SPH_ARGS(g, k, p.cell, cs, p.off, p.mass, p.h, rho_out, partials,
                                       counts, flags));
}

template <typename T>
void launch_tv(const Launch& l, const Grid& g, const Coeffs<T>& k, const PArrays<T>& p,
               const int* cs, T* dr, T* beta, double* s_out, T* g_out, double* partials,
               const TvDrift<T>& td) {
  if (g.n == 0) return;
  SPH_SWEEP(tv_kernel, SPH_ARGS(g, k, p.cell, cs, p.off, p.rho, p.mass, p.h, p.id, dr, beta,
                                s_out, g_out, partials, td));
}

template <typename T>
void launch_forces(const Launch& l, const Grid& g, const Coeffs<T>& k, const PArrays<T>& p,
                   const int* cs, const T* vel, T* acc_out, unsigned* flags,
                   const StoredList& sl) {
  if (g.n == 0) return;
  FusedOut<T> none{};
  if (sl.entry)
    SPH_SWEEP(forces_list_kernel, SPH_ARGS(g, k, p.cell, cs, p.off, vel, p.rho, p.mass, p.h,
                                           p.id, acc_out, flags, none, sl));
  else
    SPH_SWEEP(forces_kernel, SPH_ARGS(g, k, p.cell, cs, p.off, vel, p.rho, p.mass, p.h, p.id,
                                      acc_out, flags, none));
}

template <typename T>
void launch_forces_fused(const Launch& l, const Grid& g, const Coeffs<T>& k, const PArrays<T>& p,
                         const int* cs, const FusedOut<T>& fo, unsigned* flags,
                         const StoredList& sl) {
  if (g.n == 0) return;
  if (sl.entry)
    SPH_SWEEP(forces_fused_list_kernel, SPH_ARGS(g, k, p.cell, cs, p.off, p.vel, p.rho, p.mass,
                                                 p.h, p.id, p.acc, flags, fo, sl));
  else
    SPH_SWEEP(forces_fused_kernel, SPH_ARGS(g, k, p.cell, cs, p.off, p.vel, p.rho, p.mass, p.h,
                                            p.id, p.acc, flags, fo));
}

template <typename T>
void launch_wall_state(const Launch& l, const Grid& g, const Coeffs<T>& k, const PArrays<T>& p,
                       const int* cs, const T* wall_vel, int n_wall, T* wsum_out, T* wavg_out) {
  if (g.n == 0 || n_wall == 0) return;
  SPH_SWEEP(wall_state_kernel, SPH_ARGS(g, k, p.cell, cs, p.off, p.h, p.id, wall_vel, n_wall,
                                        p.rho, p.vel, wsum_out, wavg_out));
}

#define SPH_INST(T)                                                                          \
  template void launch_wall_state<T>(const Launch&, const Grid&, const Coeffs<T>&,           \
                                     const PArrays<T>&, const int*, const T*, int, T*, T*);  \
  template void launch_density<T>(const Launch&, const Grid&, const Coeffs<T>&,              \
                                  const PArrays<T>&, const int*, T*, double*, int*,          \
                                  unsigned*, const StoredList&);                             \
  template void launch_tv<T>(const Launch&, const Grid&, const Coeffs<T>&, const PArrays<T>&,\
                             const int*, T*, T*, double*, T*, double*, const TvDrift<T>&);   \
  template void launch_forces<T>(const Launch&, const Grid&, const Coeffs<T>&,               \
                                 const PArrays<T>&, const int*, const T*, T*, unsigned*,     \
                                 const StoredList&);                                         \
  template void launch_forces_fused<T>(const Launch&, const Grid&, const Coeffs<T>&,         \
                                       const PArrays<T>&, const int*, const FusedOut<T>&,    \
                                       unsigned*, const StoredList&);
SPH_INST(float)
SPH_INST(double)
#undef SPH_INST

}  // namespace sph
