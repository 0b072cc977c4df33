// Reverse (vector-Jacobian) sweeps of one TV-WCSPH step.
//
// Every pair term of the forward sweeps is antisymmetric under i <-> j up to
// the mass ratio (m_i f_ij = -m_j f_ji for the accelerations; the kernel sum
// of Eq. 8 and the gradient sum of Eq. 14 are symmetric / antisymmetric), so
// the reverse sweeps are gathers too: particle i collects the derivative of
// every pair term it takes part in from its own and its neighbours'
// cotangents, and writes only its own entries.  No atomics.
//
// Notation per pair: r = r_i - r_j, q = |r| / h_ij, t = 1 - q/2,
// F = W'(|r|)/|r| = fc t^3 with fc = -5 alpha / h^2, and
// F'(|r|) / |r| = -1.5 fc t^2 / (h |r|).
//
// The cotangent sums are plain (uncompensated) in FP32 as in FP64: the FP32
// gradient's error is set by the FP32 forward recompute, and compensating
// these sums changed directional derivatives of a 200-step rollout by ~1e-8
// relative while costing ~8% of the reverse step.
#include "sph_internal.hpp"

namespace sph {

template <typename T>
using VjpAcc = Acc<T, false>;

template <int D, typename T>
struct PairKernel {
  T F;        // W'/r
  T Fpr;      // F'(r)/r
};

template <int D, typename T, bool VAR>
__device__ __forceinline__ bool pair_kernel(const Coeffs<T>& k, T r2, T hi, T hj,
                                            PairKernel<D, T>& pk, T& inv_r) {
  const PairH<D, T, VAR> ph = pair_h<D, T, VAR>(k, hi, hj);
  if (!(r2 < ph.sup2)) return false;
  const PairGeo<T> pg = pair_geo(r2);
  inv_r = pg.inv_r;
  const T t = kernel_t(pg.r, ph.inv_h);
  pk.F = ph.fc * (t * t * t);
  pk.Fpr = T(-1.5) * ph.fc * (t * t) * ph.inv_h * pg.inv_r;
  return true;
}

// ------------------------------------------------------------------ forces^T
// Accumulates, for each i, over its neighbours j with w = abar_i - (m_i/m_j) abar_j:
//   rbar_i   += (B.w) Cp r + Cc (-P* w + dP (r.w) v_perp / |r|)
//   vbar_i   += Cc (eta w + dP (r.w) r / |r|)
//   rhobar_i += -(f.w) / rho_i - Cc (c0^2/2 + beta c0 dU / 4) (r.w)
// with Cc = 2 m_j F / (rho_i rho_j), Cp = 2 m_j (F'/|r|) / (rho_i rho_j),
// B = eta v_ij - P* r, f = Cc B, dP = dP*/dU = rhobar c0 (beta + dU beta') / 2,
// v_perp = v_ij - (v_ij . r) r / |r|^2.  The long pair body runs over a
// per-thread neighbour list (positions are tested first).
template <int G>
struct VjpCap { static constexpr int value = G == 2 ? 24 : (G == 4 ? 16 : 8); };

// LIST: over the stored lists of the same state (no candidate tests)
template <int D, typename T, bool VAR, int G, bool LIST>
__device__ __forceinline__ void force_vjp_impl(
    const Grid& g, const Coeffs<T>& k, const int* __restrict__ cell, const int* __restrict__ cs,
    const T* __restrict__ off, const T* __restrict__ vel, const T* __restrict__ rho,
    const T* __restrict__ mass, const T* __restrict__ hh, const T* __restrict__ a_bar,
    T* __restrict__ r_bar, T* __restrict__ v_bar, T* __restrict__ rho_bar,
    const StoredList& sl) {
  __shared__ NeighbourList<LIST ? 1 : VjpCap<G>::value> nl;
  const int n = g.n;
  const Cols<T, D> offc(off, n), velc(vel, n), abarc(a_bar, n);
  const Cols<T, 1> rhoc(rho, n), hc(hh, n), mc(mass, n);
  // candidate-test values: offsets, then h (variable resolution)
  constexpr int NS = D + (VAR ? 1 : 0);
  auto srct = [&](int j, T* v) {
#pragma unroll
    for (int d = 0; d < D; ++d) v[d] = offc(d, j);
    if constexpr (VAR) v[D] = hc(0, j);
  };
  __shared__ Stage<D, T, NS, LIST ? 0 : StageCap<D, T>::value> st;
  stage_positions<D, G>(g, cell, cs, st, srct);
  const int i = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int sub = threadIdx.x % G;
  const bool valid = i < n;
  VjpAcc<T> rb[3], vb[3], pb;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    rb[d].init(T(0));
    vb[d].init(T(0));
  }
  pb.init(T(0));
  if (valid) {
    T oi[3], vi[3], ai[3];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      oi[d] = off[d * n + i];
      vi[d] = vel[d * n + i];
      ai[d] = a_bar[d * n + i];
    }
    const T rhoi = rho[i];
    const T inv_rhoi = T(1) / rhoi;
    const T pi = k.c0sq * (rhoi - k.rho0);
    const T hi = VAR ? hh[i] : k.h;
    const T mi = VAR ? mass[i] : k.mass;
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
    auto body = [&](int j, const T* sh) {
      T r[3];
      T r2 = T(0);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        r[d] = (oi[d] - offc(d, j)) - sh[d];
        r2 = tfma(r[d], r[d], r2);
      }
      PairKernel<D, T> pk;
      T inv_r;
      pair_kernel<D, T, VAR>(k, r2, hi, VAR ? hc(0, j) : k.h, pk, inv_r);
      const T mj = VAR ? mc(0, j) : k.mass;
      const T rhoj = rhoc(0, j);
      const T pj = k.c0sq * (rhoj - k.rho0);
      T vij[3], w[3];
      T vr = T(0);
      const T mratio = VAR ? mi * frcp(mj) : T(1);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        vij[d] = vi[d] - velc(d, j);
        vr = tfma(vij[d], r[d], vr);
        w[d] = tfma(-mratio, abarc(d, j), ai[d]);
      }
      const T du = -vr * inv_r;
      const T x = k.riemann_eta * du * k.inv_c0;
      const T br = tmin(tmax(x, T(0)), T(1));
      const T bprime = (x > T(0) && x < T(1)) ? k.riemann_eta * k.inv_c0 : T(0);
      const T rhobar = T(0.5) * (rhoi + rhoj);
      const T pstar = T(0.5) * (pi + pj) + T(0.5) * br * rhobar * k.c0 * du;
      const T dP = T(0.5) * rhobar * k.c0 * (br + du * bprime);
      const T base = T(2) * mj * inv_rhoi * frcp(rhoj);
      const T Cc = base * pk.F;
      const T Cp = base * pk.Fpr;
      T Bw = T(0), rw = T(0);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const T B = tfma(-pstar, r[d], k.eta * vij[d]);
        Bw = tfma(B, w[d], Bw);
        rw = tfma(r[d], w[d], rw);
      }
      const T vperp_coef = vr * inv_r * inv_r;   // (v_ij . r) / |r|^2
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const T vperp = vij[d] - vperp_coef * r[d];
        rb[d].add(Bw * Cp * r[d] + Cc * (-pstar * w[d] + dP * rw * vperp * inv_r));
        vb[d].add(Cc * (k.eta * w[d] + dP * inv_r * rw * r[d]));
      }
      pb.add(-Cc * Bw * inv_rhoi - Cc * (T(0.5) * k.c0sq + T(0.25) * br * k.c0 * du) * rw);
    };
    if constexpr (LIST)
      for_each_stored_entry<D, G, T, NS>(g, k, cell[i], cs, sub, sl, srct, test, body);
    else   // the plain candidate walk: batching costs this long body's occupancy
      for_each_neighbour_listed<D, G, T, NS, 1>(g, k, cell[i], cs, sub, st, nl, srct, test, body);
  }
  T rbs[3], vbs[3];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    rbs[d] = group_sum<G>(rb[d]);
    vbs[d] = group_sum<G>(vb[d]);
  }
  const T pbs = group_sum<G>(pb);
  if (valid && sub == 0) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      r_bar[d * n + i] += rbs[d];
      v_bar[d * n + i] += vbs[d];
    }
    rho_bar[i] += pbs;
  }
}

template <int D, typename T, bool VAR, int G>
__global__ __launch_bounds__(kBlock) void force_vjp_kernel(
    Grid g, Coeffs<T> k, const int* __restrict__ cell, const int* __restrict__ cs,
    const T* __restrict__ off, const T* __restrict__ vel, const T* __restrict__ rho,
    const T* __restrict__ mass, const T* __restrict__ hh, const T* __restrict__ a_bar,
    T* __restrict__ r_bar, T* __restrict__ v_bar, T* __restrict__ rho_bar) {
  force_vjp_impl<D, T, VAR, G, false>(g, k, cell, cs, off, vel, rho, mass, hh, a_bar, r_bar,
                                      v_bar, rho_bar, StoredList{});
}

template <int D, typename T, bool VAR, int G>
__global__ __launch_bounds__(kBlock) void force_vjp_list_kernel(
    Grid g, Coeffs<T> k, const int* __restrict__ cell, const int* __restrict__ cs,
    const T* __restrict__ off, const T* __restrict__ vel, const T* __restrict__ rho,
    const T* __restrict__ mass, const T* __restrict__ hh, const T* __restrict__ a_bar,
    T* __restrict__ r_bar, T* __restrict__ v_bar, T* __restrict__ rho_bar, StoredList sl) {
  force_vjp_impl<D, T, VAR, G, true>(g, k, cell, cs, off, vel, rho, mass, hh, a_bar, r_bar,
                                     v_bar, rho_bar, sl);
}

// ------------------------------------------------------------------ density^T
// rbar_i += sum_j (rhobar_i m_j + rhobar_j m_i) F_ij r_ij / kappa, then
// vbar_i += vcoef * rbar_i (the drift r' = r + dt v' of the same step; wall
// particles, told by id when id is given, do not drift).
template <int D, typename T, bool VAR, int G, bool LIST>
__device__ __forceinline__ void density_vjp_impl(
    const Grid& g, const Coeffs<T>& k, const int* __restrict__ cell, const int* __restrict__ cs,
    const T* __restrict__ off, const T* __restrict__ mass, const T* __restrict__ hh,
    const int* __restrict__ id, const T* __restrict__ rho_bar, T* __restrict__ r_bar,
    T* __restrict__ v_bar, T vcoef, const StoredList& sl) {
  const int n = g.n;
  const Cols<T, D> offc(off, n);
  const Cols<T, 1> rbarc(rho_bar, n), hc(hh, n), mc(mass, n);
  // candidate-test values: offsets, then h (variable resolution); staged in
  // LDS for the 2-D FP32 sweeps
  constexpr int NS = D + (VAR ? 1 : 0);
  auto srct = [&](int j, T* v) {
#pragma unroll
    for (int d = 0; d < D; ++d) v[d] = offc(d, j);
    if constexpr (VAR) v[D] = hc(0, j);
  };
  __shared__ Stage<D, T, NS, LIST ? 0 : StageCap<D, T>::value> st;
  stage_positions<D, G>(g, cell, cs, st, srct);
  const int i = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int sub = threadIdx.x % G;
  const bool valid = i < n;
  VjpAcc<T> acc[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) acc[d].init(T(0));
  if (valid) {
    T oi[3];
#pragma unroll
    for (int d = 0; d < D; ++d) oi[d] = off[d * n + i];
    const T hi = VAR ? hh[i] : k.h;
    const T mi = VAR ? mass[i] : k.mass;
    const T pbi = rho_bar[i];
    // one candidate j with test values v (offsets, then h_j)
    auto pair = [&](int j, const T* v, const T* sh, bool live) {
      T r[3];
      T r2 = T(0);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        r[d] = (oi[d] - v[d]) - sh[d];
        r2 = tfma(r[d], r[d], r2);
      }
      if (!live || j == i) return;
      PairKernel<D, T> pk;
      T inv_r;
      if (!pair_kernel<D, T, VAR>(k, r2, hi, VAR ? v[D] : k.h, pk, inv_r)) return;
      const T mj = VAR ? mc(0, j) : k.mass;
      const T c = (pbi * mj + rbarc(0, j) * mi) * pk.F;
#pragma unroll
      for (int d = 0; d < D; ++d) acc[d].add(c * r[d]);
    };
    if constexpr (LIST) {
      // every stored entry is a neighbour; the pair repeats the (passing) test
      auto always = [](int, const T*, const T*) { return true; };
      for_each_stored_entry<D, G, T, NS>(g, k, cell[i], cs, sub, sl, srct, always,
                                         [&](int j, const T* sh) {
                                           T v[NS];
                                           srct(j, v);
                                           pair(j, v, sh, true);
                                         });
    } else {
      for_each_candidate_values<D, G, T, VAR>(g, k, cell[i], cs, sub, st, srct, pair);
    }
  }
  T sums[3];
#pragma unroll
  for (int d = 0; d < D; ++d) sums[d] = group_sum<G>(acc[d]);
  if (valid && sub == 0) {
    const bool drifts = v_bar && !(id && is_wall(k, id[i]));
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const T rb = r_bar[d * n + i] + sums[d] * k.inv_kappa;
      r_bar[d * n + i] = rb;
      if (drifts) v_bar[d * n + i] += vcoef * rb;
    }
  }
}

template <int D, typename T, bool VAR, int G>
__global__ __launch_bounds__(kBlock) void density_vjp_kernel(
    Grid g, Coeffs<T> k, const int* __restrict__ cell, const int* __restrict__ cs,
    const T* __restrict__ off, const T* __restrict__ mass, const T* __restrict__ hh,
    const int* __restrict__ id, const T* __restrict__ rho_bar, T* __restrict__ r_bar,
    T* __restrict__ v_bar, T vcoef) {
  density_vjp_impl<D, T, VAR, G, false>(g, k, cell, cs, off, mass, hh, id, rho_bar, r_bar, v_bar,
                                        vcoef, StoredList{});
}

template <int D, typename T, bool VAR, int G>
__global__ __launch_bounds__(kBlock) void density_vjp_list_kernel(
    Grid g, Coeffs<T> k, const int* __restrict__ cell, const int* __restrict__ cs,
    const T* __restrict__ off, const T* __restrict__ mass, const T* __restrict__ hh,
    const int* __restrict__ id, const T* __restrict__ rho_bar, T* __restrict__ r_bar,
    T* __restrict__ v_bar, T vcoef, StoredList sl) {
  density_vjp_impl<D, T, VAR, G, true>(g, k, cell, cs, off, mass, hh, id, rho_bar, r_bar, v_bar,
                                       vcoef, sl);
}

// ------------------------------------------------------------------ wall state^T
// The wall state (sph_wall_state) for wall a over its fluid neighbours f:
//   S_a = sum W_af,  rho_a = rho0 + sum (rho_f - rho0) W_af / S_a,
//   v_a = 2 u_a - Vbar_a,  Vbar_a = sum v_f W_af / S_a.
// S_a and Vbar_a per wall particle (by id - nfluid) come from the forward
// wall state recorded in the tape, or, for the initial state, from pass 1;
// the cells that hold walls are marked first.  Pass 2 is a gather over the
// fluid-wall pairs (particles whose 3^D cells hold no wall skip it): with
//   c_af = (rhobar_a (rho_f - rho_a) - vbar_a . (v_f - Vbar_a)) / S_a,
// a fluid particle f collects rhobar_f += rhobar_a W_af / S_a,
// vbar_f -= vbar_a W_af / S_a and rbar_f += c_af F_af (r_f - r_a); a wall
// particle a collects rbar_a += c_af F_af (r_a - r_f).  Pass 3 clears the
// walls' rhobar and vbar (consumed; the walls' summation densities and
// earlier velocities feed nothing).
template <int D, typename T, bool VAR, int G>
__global__ __launch_bounds__(kBlock) void wall_sums_kernel(
    Grid g, Coeffs<T> k, const int* __restrict__ cell, const int* __restrict__ cs,
    const T* __restrict__ off, const T* __restrict__ hh, const int* __restrict__ id,
    const T* __restrict__ vel, T* __restrict__ wsum, T* __restrict__ wavg, int n_wall,
    int* __restrict__ wall_cells) {
  const int n = g.n;
  const int i = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int sub = threadIdx.x % G;
  const bool wall = i < n && is_wall(k, id[i]);
  if (!__any(wall)) return;     // whole wavefront: no lane needs a group sum
  const Cols<T, D> offc(off, n), velc(vel, n);
  const Cols<T, 1> hc(hh, n);
  VjpAcc<T> sw, sv[3];
  sw.init(T(0));
#pragma unroll
  for (int d = 0; d < 3; ++d) sv[d].init(T(0));
  if (wall) {
    T oi[3];
#pragma unroll
    for (int d = 0; d < D; ++d) oi[d] = off[d * n + i];
    const T hi = VAR ? hh[i] : k.h;
    for_each_candidate<D, G>(g, k, cell[i], cs, sub, [&](int j, const T* sh) {
      T r2 = T(0);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const T rv = (oi[d] - offc(d, j)) - sh[d];
        r2 = tfma(rv, rv, r2);
      }
      const PairH<D, T, VAR> ph = pair_h<D, T, VAR>(k, hi, VAR ? hc(0, j) : T(0));
      if (!(r2 < ph.sup2) || is_wall(k, id[j])) return;
      const T w = wendland_alpha<D>(ph.inv_h) * wendland_shape(fsqrt(r2) * ph.inv_h);
      sw.add(w);
#pragma unroll
      for (int d = 0; d < D; ++d) sv[d].add(velc(d, j) * w);
    });
  }
  const T S = group_sum<G>(sw);
  T V[3];
#pragma unroll
  for (int d = 0; d < D; ++d) V[d] = group_sum<G>(sv[d]);
  const int iw = wall ? id[i] - k.nfluid : 0;
  if (wall && sub == 0 && iw < n_wall) {
    wsum[iw] = S;
#pragma unroll
    for (int d = 0; d < D; ++d) wavg[(size_t)d * n_wall + iw] = S > T(0) ? V[d] / S : T(0);
  }
}

// LIST: over the stored lists of the same state (entries are the pairs
// inside the support; the fluid-wall test stays)
template <int D, typename T, bool VAR, int G, bool LIST>
__device__ __forceinline__ void wall_vjp_impl(
    const Grid& g, const Coeffs<T>& k, const int* __restrict__ cell, const int* __restrict__ cs,
    const T* __restrict__ off, const T* __restrict__ hh, const int* __restrict__ id,
    const T* __restrict__ vel, const T* __restrict__ rho, const T* __restrict__ wsum,
    const T* __restrict__ wavg, int n_wall, const int* __restrict__ wall_cells,
    T* __restrict__ r_bar, T* __restrict__ v_bar, T* __restrict__ rho_bar,
    const StoredList& sl) {
  const int n = g.n;
  const int i = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int sub = threadIdx.x % G;
  const bool valid = i < n;
  const bool wall_i = valid && is_wall(k, id[i]);
  // a fluid particle takes part only if a cell around it holds a wall
  bool near = wall_i;
  if (valid && !wall_i) {
    int c[3];
    decode_cell<D>(g, cell[i], c);
    constexpr int zlo = (D == 3) ? -1 : 0;
    constexpr int zhi = (D == 3) ? 1 : 0;
#pragma unroll
    for (int dz = zlo; dz <= zhi; ++dz) {
      const int z = (D == 3) ? wrap_index(c[2] + dz, g.nc[2]) : 0;
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
        const int row = g.nc[0] * (wrap_index(c[1] + dy, g.nc[1]) + g.nc[1] * z);
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) near |= wall_cells[row + wrap_index(c[0] + dx, g.nc[0])] != 0;
      }
    }
  }
  if (!__any(near)) return;       // whole wavefront: no lane needs a group sum
  const Cols<T, D> offc(off, n), velc(vel, n), vbarc(v_bar, n);
  const Cols<T, 1> hc(hh, n), rhoc(rho, n), rbarc(rho_bar, n);
  VjpAcc<T> ra[3], va[3], pa;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    ra[d].init(T(0));
    va[d].init(T(0));
  }
  pa.init(T(0));
  if (valid && near) {
    // a wall's own sums, by wall index (id - nfluid < n_wall for ids below n)
    const int iw = wall_i ? min(id[i] - k.nfluid, n_wall - 1) : 0;
    T oi[3], vi[3], vbi[3], avi[3];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      oi[d] = off[d * n + i];
      vi[d] = vel[d * n + i];
      vbi[d] = wall_i ? v_bar[d * n + i] : T(0);
      avi[d] = wall_i ? wavg[(size_t)d * n_wall + iw] : T(0);
    }
    const T rhoi = rho[i];
    const T pbi = wall_i ? rho_bar[i] : T(0);
    const T si = wall_i ? wsum[iw] : T(0);
    const T hi = VAR ? hh[i] : k.h;
    auto pair = [&](int j, const T* sh) {
      T r[3];
      T r2 = T(0);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        r[d] = (oi[d] - offc(d, j)) - sh[d];
        r2 = tfma(r[d], r[d], r2);
      }
      const PairH<D, T, VAR> ph = pair_h<D, T, VAR>(k, hi, VAR ? hc(0, j) : T(0));
      const int idj = id[j];
      if (!(r2 < ph.sup2) || is_wall(k, idj) == wall_i) return;     // fluid-wall pairs
      const PairGeo<T> pg = pair_geo(r2);
      const T t = kernel_t(pg.r, ph.inv_h);
      const T F = ph.fc * (t * t * t);
      if (!wall_i) {
        // i = f (fluid), j = a (wall)
        const int jw = min(idj - k.nfluid, n_wall - 1);
        const T sa = wsum[jw];
        if (!(sa > T(0))) return;
        const T inv = T(1) / sa;
        const T w = wendland_alpha<D>(ph.inv_h) * wendland_shape(pg.r * ph.inv_h);
        const T pbj = rbarc(0, j);
        T c = pbj * (rhoi - rhoc(0, j));
#pragma unroll
        for (int d = 0; d < D; ++d) {
          const T vbj = vbarc(d, j);
          c -= vbj * (vi[d] - wavg[(size_t)d * n_wall + jw]);
          va[d].add(-vbj * w * inv);
        }
        pa.add(pbj * w * inv);
        c *= inv;
#pragma unroll
        for (int d = 0; d < D; ++d) ra[d].add(c * F * r[d]);
      } else {
        // i = a (wall), j = f (fluid)
        if (!(si > T(0))) return;
        T c = pbi * (rhoc(0, j) - rhoi);
#pragma unroll
        for (int d = 0; d < D; ++d) c -= vbi[d] * (velc(d, j) - avi[d]);
        c /= si;
#pragma unroll
        for (int d = 0; d < D; ++d) ra[d].add(c * F * r[d]);
      }
    };
    if constexpr (LIST)
      for_each_stored_entry<D, G, T, 1>(
          g, k, cell[i], cs, sub, sl, [](int, T*) {},
          [](int, const T*, const T*) { return true; }, pair);
    else
      for_each_candidate<D, G>(g, k, cell[i], cs, sub, pair);
  }
  T rs[3], vs[3];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    rs[d] = group_sum<G>(ra[d]);
    vs[d] = group_sum<G>(va[d]);
  }
  const T ps = group_sum<G>(pa);
  if (valid && near && sub == 0) {
#pragma unroll
    for (int d = 0; d < D; ++d) r_bar[d * n + i] += rs[d];
    if (!wall_i) {
#pragma unroll
      for (int d = 0; d < D; ++d) v_bar[d * n + i] += vs[d];
      rho_bar[i] += ps;
    }
  }
}

template <int D, typename T, bool VAR, int G>
__global__ __launch_bounds__(kBlock) void wall_vjp_kernel(
    Grid g, Coeffs<T> k, const int* __restrict__ cell, const int* __restrict__ cs,
    const T* __restrict__ off, const T* __restrict__ hh, const int* __restrict__ id,
    const T* __restrict__ vel, const T* __restrict__ rho, const T* __restrict__ wsum,
    const T* __restrict__ wavg, int n_wall, const int* __restrict__ wall_cells,
    T* __restrict__ r_bar, T* __restrict__ v_bar, T* __restrict__ rho_bar) {
  wall_vjp_impl<D, T, VAR, G, false>(g, k, cell, cs, off, hh, id, vel, rho, wsum, wavg, n_wall,
                                     wall_cells, r_bar, v_bar, rho_bar, StoredList{});
}

template <int D, typename T, bool VAR, int G>
__global__ __launch_bounds__(kBlock) void wall_vjp_list_kernel(
    Grid g, Coeffs<T> k, const int* __restrict__ cell, const int* __restrict__ cs,
    const T* __restrict__ off, const T* __restrict__ hh, const int* __restrict__ id,
    const T* __restrict__ vel, const T* __restrict__ rho, const T* __restrict__ wsum,
    const T* __restrict__ wavg, int n_wall, const int* __restrict__ wall_cells,
    T* __restrict__ r_bar, T* __restrict__ v_bar, T* __restrict__ rho_bar, StoredList sl) {
  wall_vjp_impl<D, T, VAR, G, true>(g, k, cell, cs, off, hh, id, vel, rho, wsum, wavg, n_wall,
                                    wall_cells, r_bar, v_bar, rho_bar, sl);
}

// x[c][i] = 0 (c < ncomp) and, when given, y[i] = 0 for the wall particles i
template <typename T>
__global__ __launch_bounds__(kBlock) void zero_walls_kernel(Coeffs<T> k, int n, int ncomp,
                                                            const int* __restrict__ id,
                                                            T* __restrict__ x,
                                                            T* __restrict__ y) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n || !is_wall(k, id[i])) return;
  for (int c = 0; c < ncomp; ++c) x[(size_t)c * n + i] = T(0);
  if (y) y[i] = T(0);
}

// ------------------------------------------------------------------ correction^T, pass 1
// The cell build's permutation reversed, and the first pass of the
// correction's VJP, in one pass over the new order q: i = perm[q] is q's
// index in order n; r_n[i] and vh_n[i] take r_bar[q] and v_bar[q], and
// ghat_i = d(dr_i)/dg_i ^T rbar_i for the chosen formulation (beta_i from the
// tape is 0 on steps without correction, which zeroes every term):
//   limited:    xi h^2 (beta_i rbar_i + 2 C h^2 (g_i . rbar_i) g_i [ramp branch only])
//   scaled:     xi h^2 beta_i rbar_i
//   background: -(rho0 c0^2 dt^2 / rho_i) beta_i rbar_i
// with per-wavefront partials (q order) of the xi derivative
// sum_i h^2 beta_i g_i . rbar_i (none for the background formulation, which
// has no xi).
template <int D, typename T>
__global__ __launch_bounds__(kBlock) void unpermute_ghat_kernel(
    Coeffs<T> k, int n, const int* __restrict__ perm, const T* __restrict__ r_bar,
    const T* __restrict__ v_bar, const T* __restrict__ gsum, const T* __restrict__ beta,
    const T* __restrict__ rho, T* __restrict__ r_n, T* __restrict__ vh_n, T* __restrict__ ghat,
    double* __restrict__ partials) {
  const int q = blockIdx.x * kBlock + threadIdx.x;
  double xi_part = 0.0;
  if (q < n) {
    const int i = perm[q];
    double gg = 0.0, gr = 0.0;
    double gi[3], ri[3];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const T rq = r_bar[d * n + q];
      r_n[d * n + i] = rq;
      vh_n[d * n + i] = v_bar[d * n + q];
      gi[d] = (double)gsum[d * n + i];
      ri[d] = (double)rq;
      gg += gi[d] * gi[d];
      gr += gi[d] * ri[d];
    }
    const double b = (double)beta[i];
    double f, two_c_h2 = 0.0;
    if (k.tv_mode == kTvBackground) {
      f = -k.bg / (double)rho[i] * b;
    } else {
      f = k.xi * k.hmin2 * b;
      xi_part = k.hmin2 * b * gr;
      if (k.tv_mode == kTvLimited) {
        const double s = k.hmin2 * gg;
        const bool ramp = (s > k.lim_s0) && (k.lim_c * s < 1.0);
        if (ramp) two_c_h2 = 2.0 * k.lim_c * k.hmin2 * k.xi * k.hmin2;
      }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) ghat[d * n + i] = (T)(f * ri[d] + two_c_h2 * gr * gi[d]);
  }
  const int cols[1] = {0};
  double v[1] = {xi_part};
  wave_partials<1>(partials, cols, v, 0u);
}

// ------------------------------------------------------------------ correction^T, pass 2
// r_out_i = r_in_i + sum_j H_ij (V_j ghat_i - V_i ghat_j),  H = F I + (F'/r) r r^T
// rho_out_i = (m_i / rho_i^2) sum_j F_ij (ghat_j . r_ij), plus for the
// background formulation the derivative of its 1/rho_i factor,
// (rho0 c0^2 dt^2 / rho_i^2) beta_i (g_i . r_in_i) (FP64).
template <int D, typename T, bool VAR, int G>
__global__ __launch_bounds__(kBlock) void tv_vjp_kernel(
    Grid g, Coeffs<T> k, const int* __restrict__ cell, const int* __restrict__ cs,
    const T* __restrict__ off, const T* __restrict__ rho, const T* __restrict__ mass,
    const T* __restrict__ hh, const T* __restrict__ ghat, const T* __restrict__ gsum,
    const T* __restrict__ beta, const T* __restrict__ r_in, T* __restrict__ r_out,
    T* __restrict__ rho_out, AdjFinish<T> fin) {
  if (fin.xi_bar && (int)blockIdx.x == (int)gridDim.x - 1) {
    // the extra last block folds the xi partials of the ghat pass (fixed order)
    __shared__ double red[kBlock / kWave];
    const double t = block_reduce<double, false>(fold_rows<false>(fin.xi_partials, fin.xi_rows), red);
    if (threadIdx.x == 0) fin.xi_bar[0] += t;
    return;
  }
  const int n = g.n;
  const Cols<T, D> offc(off, n), ghatc(ghat, n);
  const Cols<T, 1> rhoc(rho, n), hc(hh, n), mc(mass, n);
  // candidate-test values: offsets, then h (variable resolution); staged in
  // LDS for the 2-D FP32 sweeps
  constexpr int NS = D + (VAR ? 1 : 0);
  auto srct = [&](int j, T* v) {
#pragma unroll
    for (int d = 0; d < D; ++d) v[d] = offc(d, j);
    if constexpr (VAR) v[D] = hc(0, j);
  };
  __shared__ Stage<D, T, NS, StageCap<D, T>::value> st;
  stage_positions<D, G>(g, cell, cs, st, srct);
  const int i = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int sub = threadIdx.x % G;
  const bool valid = i < n;
  VjpAcc<T> acc[3], pb;
#pragma unroll
  for (int d = 0; d < 3; ++d) acc[d].init(T(0));
  pb.init(T(0));
  T mi = T(1), rhoi = T(1);
  if (valid) {
    T oi[3], gi[3];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      oi[d] = off[d * n + i];
      gi[d] = ghat[d * n + i];
    }
    const T hi = VAR ? hh[i] : k.h;
    mi = VAR ? mass[i] : k.mass;
    rhoi = rho[i];
    const T Vi = mi / rhoi;
    for_each_candidate_values<D, G, T, VAR>(
        g, k, cell[i], cs, sub, st, srct, [&](int j, const T* v, const T* sh, bool live) {
          T r[3];
          T r2 = T(0);
#pragma unroll
          for (int d = 0; d < D; ++d) {
            r[d] = (oi[d] - v[d]) - sh[d];
            r2 = tfma(r[d], r[d], r2);
          }
          if (!live || j == i) return;
          PairKernel<D, T> pk;
          T inv_r;
          if (!pair_kernel<D, T, VAR>(k, r2, hi, VAR ? v[D] : k.h, pk, inv_r)) return;
          const T mj = VAR ? mc(0, j) : k.mass;
          const T Vj = mj * frcp(rhoc(0, j));
          T u[3], gj[3];
          T ur = T(0), gjr = T(0);
#pragma unroll
          for (int d = 0; d < D; ++d) {
            gj[d] = ghatc(d, j);
            u[d] = Vj * gi[d] - Vi * gj[d];
            ur = tfma(u[d], r[d], ur);
            gjr = tfma(gj[d], r[d], gjr);
          }
#pragma unroll
          for (int d = 0; d < D; ++d) acc[d].add(pk.F * u[d] + pk.Fpr * ur * r[d]);
          pb.add(pk.F * gjr);
        });
  }
  T sums[3];
#pragma unroll
  for (int d = 0; d < D; ++d) sums[d] = group_sum<G>(acc[d]);
  const T pbs = group_sum<G>(pb);
  if (valid && sub == 0) {
    double direct = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      if (k.tv_mode == kTvBackground)
        direct += (double)gsum[d * n + i] * (double)r_in[d * n + i];
      r_out[d * n + i] = r_in[d * n + i] + sums[d];
    }
    T rb = pbs * mi / (rhoi * rhoi);
    if (k.tv_mode == kTvBackground)
      rb = (T)((double)rb + k.bg * (double)beta[i] / ((double)rhoi * (double)rhoi) * direct);
    rho_out[i] = rb;
    // 2^T: v' = v^n + dt/2 a^n (fluid): v_bar^n = v'_bar, a_bar^n = dt/2 v'_bar
    if (fin.v_bar) {
      const bool wall = fin.id && fin.id[i] >= k.nfluid;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const T v = wall ? T(0) : fin.vh_bar[d * n + i];
        fin.v_bar[d * n + i] = v;
        fin.a_bar[d * n + i] = k.half_dt * v;
      }
    }
  }
}

// ------------------------------------------------------------------ elementwise
// Wall particles (told by id when id is given) are not kicked: their
// velocity cotangent is that of the wall state, not of a kick, and their
// acceleration is not an output (its cotangent is cleared).
template <typename T>
__global__ __launch_bounds__(kBlock) void adj_kick_kernel(long dn, int n, T half_dt, int nfluid,
                                                          const int* __restrict__ id,
                                                          const T* __restrict__ v_bar,
                                                          T* __restrict__ a_bar) {
  const long i = (long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= dn) return;
  if (id && id[i % n] >= nfluid) a_bar[i] = T(0);
  else a_bar[i] += half_dt * v_bar[i];
}

// ------------------------------------------------------------------ launchers
template <typename T>
void launch_force_vjp(const Launch& l, const Grid& g, const Coeffs<T>& k, const PArrays<T>& p,
                      const int* cs, const T* vel, const T* a_bar, T* r_bar, T* v_bar,
                      T* rho_bar, const StoredList& sl) {
  if (g.n == 0) return;
  if (sl.entry)
    SPH_SWEEP(force_vjp_list_kernel, SPH_ARGS(g, k, p.cell, cs, p.off, vel, p.rho, p.mass, p.h,
                                              a_bar, r_bar, v_bar, rho_bar, sl));
  else
    SPH_SWEEP(force_vjp_kernel, SPH_ARGS(g, k, p.cell, cs, p.off, vel, p.rho, p.mass, p.h, a_bar,
                                         r_bar, v_bar, rho_bar));
}

template <typename T>
void launch_density_vjp(const Launch& l, const Grid& g, const Coeffs<T>& k, const PArrays<T>& p,
                        const int* cs, const T* rho_bar, T* r_bar, T* v_bar, T vcoef,
                        const StoredList& sl) {
  if (g.n == 0) return;
  if (sl.entry)
    SPH_SWEEP(density_vjp_list_kernel, SPH_ARGS(g, k, p.cell, cs, p.off, p.mass, p.h, p.id,
                                                rho_bar, r_bar, v_bar, vcoef, sl));
  else
    SPH_SWEEP(density_vjp_kernel, SPH_ARGS(g, k, p.cell, cs, p.off, p.mass, p.h, p.id, rho_bar,
                                           r_bar, v_bar, vcoef));
}

template <typename T>
void launch_tv_vjp(const Launch& l, const Grid& g, const Coeffs<T>& k, const PArrays<T>& p,
                   const int* cs, const T* ghat, const T* gsum, const T* beta, const T* r_in,
                   T* r_out, T* rho_out, const AdjFinish<T>& fin) {
  if (g.n == 0) return;
  // with xi_bar, one extra block folds the xi partials
  Launch lx = l;
  if (fin.xi_bar) lx.nblk = l.nblk + 1;
  {
    const Launch& l = lx;
    SPH_SWEEP(tv_vjp_kernel, SPH_ARGS(g, k, p.cell, cs, p.off, p.rho, p.mass, p.h, ghat, gsum,
                                      beta, r_in, r_out, rho_out, fin));
  }
}

template <typename T>
void launch_unpermute_ghat(const Launch& l, const Coeffs<T>& k, int n, const int* perm,
                           const T* r_bar, const T* v_bar, const T* gsum, const T* beta,
                           const T* rho, T* r_n, T* vh_n, T* ghat, double* partials) {
  if (n == 0) return;
  const dim3 grid(blocks_for(n));
  if (l.dim == 2)
    hipLaunchKernelGGL((unpermute_ghat_kernel<2, T>), grid, dim3(kBlock), 0, l.stream, k, n, perm,
                       r_bar, v_bar, gsum, beta, rho, r_n, vh_n, ghat, partials);
  else
    hipLaunchKernelGGL((unpermute_ghat_kernel<3, T>), grid, dim3(kBlock), 0, l.stream, k, n, perm,
                       r_bar, v_bar, gsum, beta, rho, r_n, vh_n, ghat, partials);
}

template <typename T>
void launch_adj_kick(const Launch& l, const Coeffs<T>& k, int n, const int* id, const T* v_bar,
                     T* a_bar) {
  const long dn = (long)l.dim * n;
  if (dn == 0) return;
  hipLaunchKernelGGL((adj_kick_kernel<T>), dim3(blocks_for(dn)), dim3(kBlock), 0, l.stream, dn,
                     n, k.half_dt, k.nfluid, id, v_bar, a_bar);
}

// wall_cells[c] = 1 for the cells holding a wall particle (cells cleared first)
template <typename T>
__global__ __launch_bounds__(kBlock) void mark_wall_cells_kernel(Coeffs<T> k, int n,
                                                                 const int* __restrict__ id,
                                                                 const int* __restrict__ cell,
                                                                 int* __restrict__ wall_cells) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n && is_wall(k, id[i])) wall_cells[cell[i]] = 1;   // every writer stores 1
}

template <typename T>
void launch_wall_vjp(const Launch& l, const Grid& g, const Coeffs<T>& k, const PArrays<T>& p,
                     const int* cs, const T* vel, T* wsum, T* wavg, int n_wall, bool sums_given,
                     int* wall_cells, T* r_bar, T* v_bar, T* rho_bar, const StoredList& sl) {
  if (g.n == 0 || n_wall == 0) return;
  launch_fill(l.stream, wall_cells, g.ncells, 0);
  hipLaunchKernelGGL((mark_wall_cells_kernel<T>), dim3(blocks_for(g.n)), dim3(kBlock), 0,
                     l.stream, k, g.n, p.id, p.cell, wall_cells);
  if (!sums_given)
    SPH_SWEEP(wall_sums_kernel, SPH_ARGS(g, k, p.cell, cs, p.off, p.h, p.id, vel, wsum, wavg,
                                         n_wall, wall_cells));
  if (sl.entry)
    SPH_SWEEP(wall_vjp_list_kernel, SPH_ARGS(g, k, p.cell, cs, p.off, p.h, p.id, vel, p.rho, wsum,
                                             wavg, n_wall, wall_cells, r_bar, v_bar, rho_bar, sl));
  else
    SPH_SWEEP(wall_vjp_kernel, SPH_ARGS(g, k, p.cell, cs, p.off, p.h, p.id, vel, p.rho, wsum,
                                        wavg, n_wall, wall_cells, r_bar, v_bar, rho_bar));
  launch_zero_walls<T>(l, k, g.n, p.id, l.dim, v_bar, rho_bar);
}

template <typename T>
void launch_zero_walls(const Launch& l, const Coeffs<T>& k, int n, const int* id, int ncomp,
                       T* x, T* y) {
  if (n == 0) return;
  hipLaunchKernelGGL((zero_walls_kernel<T>), dim3(blocks_for(n)), dim3(kBlock), 0, l.stream, k,
                     n, ncomp, id, x, y);
}

#define SPH_INST(T)                                                                          \
  template void launch_force_vjp<T>(const Launch&, const Grid&, const Coeffs<T>&,            \
                                    const PArrays<T>&, const int*, const T*, const T*, T*,   \
                                    T*, T*, const StoredList&);                              \
  template void launch_density_vjp<T>(const Launch&, const Grid&, const Coeffs<T>&,          \
                                      const PArrays<T>&, const int*, const T*, T*, T*, T,    \
                                      const StoredList&);                                    \
  template void launch_tv_vjp<T>(const Launch&, const Grid&, const Coeffs<T>&,               \
                                 const PArrays<T>&, const int*, const T*, const T*,          \
                                 const T*, const T*, T*, T*, const AdjFinish<T>&);           \
  template void launch_unpermute_ghat<T>(const Launch&, const Coeffs<T>&, int, const int*,   \
                                         const T*, const T*, const T*, const T*, const T*,   \
                                         T*, T*, T*, double*);                               \
  template void launch_adj_kick<T>(const Launch&, const Coeffs<T>&, int, const int*,          \
                                   const T*, T*);                                            \
  template void launch_wall_vjp<T>(const Launch&, const Grid&, const Coeffs<T>&,             \
                                   const PArrays<T>&, const int*, const T*, T*, T*, int,     \
                                   bool, int*, T*, T*, T*, const StoredList&);               \
  template void launch_zero_walls<T>(const Launch&, const Coeffs<T>&, int, const int*, int,  \
                                     T*, T*);
SPH_INST(float)
SPH_INST(double)
#undef SPH_INST

}  // namespace sph
