// Device-side building blocks shared by the libsph kernels (gfx950).
//
// Particles live in (cell, id) order; a particle's position is its cell's
// origin plus a cell-local offset.  A sweep gives one thread to particle i and
// walks the 3^D cells around i's cell through the CSR array cell_start.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <type_traits>

namespace sph {

constexpr int kBlock = 256;          // threads per block for every particle kernel
constexpr int kTvLimited = 0, kTvScaled = 1, kTvBackground = 2;   // SPH_TV_*
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
  int tv_mode;      // SPH_TV_LIMITED / SPH_TV_SCALED / SPH_TV_BACKGROUND
  double bg;        // rho0 c0^2 dt^2, the background-pressure coefficient
  int nfluid;       // particles with id >= nfluid are walls (nfluid = n: none)
};

template <typename T>
__device__ __forceinline__ bool is_wall(const Coeffs<T>& k, int id) { return id >= k.nfluid; }

// Whether particle i (of n) is a wall particle; reads its id only when the
// run has walls (a uniform branch), so wall-free sweeps load no ids.
template <typename T>
__device__ __forceinline__ bool wall_at(const Coeffs<T>& k, int n, const int* __restrict__ id,
                                        int i) {
  return k.nfluid < n && id[i] >= k.nfluid;
}

// ---------------------------------------------------------------- math
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fsqrt(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }
// 1/sqrt(x); callers guarantee x > 0
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double frsq(double x) { return 1.0 / __builtin_sqrt(x); }

// Fused multiply-add written out: the library is built without automatic
// contraction, so every FMA is explicit and the same expression rounds the
// same way in every kernel that evaluates it.
__device__ __forceinline__ float tfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double tfma(double a, double b, double c) { return __builtin_fma(a, b, c); }

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
  const T t = tfma(q, T(-0.5), T(1));
  const T t2 = t * t;
  return t2 * t2 * tfma(q, T(2), T(1));
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

// Neighbour reads through raw buffer resources.  Cols<T, NC> views NC
// consecutive components of n elements each (component c starts at p + c n),
// one 128-bit resource per component in scalar registers; a read takes the
// element index in one VGPR (byte offset j * sizeof(T) < 2^31 since
// n < 2^28), so every array a pair touches is read with the same offset and
// no 64-bit address arithmetic.  A read past a component's n elements
// returns 0 instead of touching memory.
constexpr int kBufferWord3 = 0x00020000;   // raw untyped dword access (gfx9 family)

template <typename T, int NC>
struct Cols {
  __amdgpu_buffer_rsrc_t r[NC];
  __device__ __forceinline__ Cols(const T* p, int n) {
#pragma unroll
    for (int c = 0; c < NC; ++c)
      r[c] = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(p) + (long)c * n, 0,
                                               n * (int)sizeof(T), kBufferWord3);
  }
  __device__ __forceinline__ T operator()(int c, int j) const {
    if constexpr (sizeof(T) == 4)
      return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r[c], j * 4, 0, 0));
    else
      return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r[c], j * 8, 0, 0));
  }
};

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

// ---------------------------------------------------------------- cell codes
// Which of the 3^D cells around a particle's own holds a neighbour, as a small
// code stored beside the neighbour's index: (dx+1) | (dy+1) << 2 in 2-D (four
// bits), (dx+1) + 3 (dy+1) + 9 (dz+1) in 3-D (five bits).  An entry is
// j | code << list_jbits: j < 2^28 in 2-D, 2^27 in 3-D.
template <int D>
constexpr int list_jbits() { return D == 3 ? 27 : 28; }

// Whether the force sweep over stored lists stages its neighbours' body values
// in LDS: uniform 2-D FP32 (in FP64 the twice larger stage costs more
// occupancy than it saves).
template <int D, typename T, bool VAR>
constexpr bool body_stage_on() { return D == 2 && !VAR && sizeof(T) == 4; }

template <int D>
constexpr unsigned cell_code(int dx, int dy, int dz) {
  return D == 3 ? (unsigned)((dx + 1) + 3 * (dy + 1) + 9 * (dz + 1))
                : (unsigned)((dx + 1) | ((dy + 1) << 2));
}

// The offset of the coded cell's origin from the particle's cell origin:
// (c - 1) L computed as c L - L, exact for c in {0, 1, 2}.
template <int D, typename T>
__device__ __forceinline__ void code_shift(const Coeffs<T>& k, unsigned code, T* shift) {
  unsigned cx, cy, cz = 0;
  if constexpr (D == 3) {
    cz = (code * 57u) >> 9;          // code / 9 for code < 27
    const unsigned r = code - 9u * cz;
    cy = (r * 11u) >> 5;             // r / 3 for r < 9
    cx = r - 3u * cy;
  } else {
    cx = code & 3u;
    cy = code >> 2;
  }
  shift[0] = tfma(T(cx), k.L[0], -k.L[0]);
  shift[1] = tfma(T(cy), k.L[1], -k.L[1]);
  shift[2] = D == 3 ? tfma(T(cz), k.L[2], -k.L[2]) : T(0);
}

// Calls body(j, shift) for the particles j of the 3^D cells around `cell`
// (the particle's own cell included, so j == i is visited).  A particle may be
// served by a group of G consecutive lanes: lane `sub` of the group takes
// every G-th particle of each cell, starting at the cell's sub-th.  shift[k]
// is the offset of j's cell origin from i's cell origin: r_i - r_j =
// (o_i - o_j) - shift.  Order: z, then y, then x rows of cells, ascending j.
template <int D, int G, typename T, typename Body>
__device__ __forceinline__ void for_each_candidate(const Grid& g, const Coeffs<T>& k, int cell,
                                                   const int* __restrict__ cs, int sub,
                                                   Body&& body) {
  int c[3];
  decode_cell<D>(g, cell, c);
  constexpr int zlo = (D == 3) ? -1 : 0;
  constexpr int zhi = (D == 3) ? 1 : 0;
#pragma unroll
  for (int dz = zlo; dz <= zhi; ++dz) {
    const int z = (D == 3) ? wrap_index(c[2] + dz, g.nc[2]) : 0;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int y = wrap_index(c[1] + dy, g.nc[1]);
      const int row = g.nc[0] * (y + g.nc[1] * z);
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int cc = row + wrap_index(c[0] + dx, g.nc[0]);
        const int b = cs[cc];
        const int e = cs[cc + 1];
        const T shift[3] = {T(dx) * k.L[0], T(dy) * k.L[1], T(dz) * k.L[2]};
        for (int j = b + sub; j < e; j += G) body(j, shift);
      }
    }
  }
}

// What a candidate test reads of j: its offsets and its h (the uniform h
// without per-particle resolution).
template <int D, typename T>
struct Candidate {
  T o[D], h;
};
template <int D, typename T, bool VAR>
__device__ __forceinline__ Candidate<D, T> candidate_of(const Cols<T, D>& offc,
                                                        const Cols<T, 1>& hc,
                                                        const Coeffs<T>& k, int j) {
  Candidate<D, T> c;
#pragma unroll
  for (int d = 0; d < D; ++d) c.o[d] = offc(d, j);
  c.h = VAR ? hc(0, j) : k.h;
  return c;
}

// Candidates per lane and batch for the sweeps with short pair bodies: 4 in
// FP32 with many candidates per lane and cell (3-D, or cells sized by the
// largest h), 1 (the plain walk) otherwise, where a batch's unused slots
// cost more than the overlap gains.
template <int D, typename T, bool VAR>
constexpr int candidate_batch() { return (sizeof(T) == 4 && (D == 3 || VAR)) ? 4 : 1; }

// The same walk with the candidates of a cell taken B at a time per lane:
// load(j) reads what the body needs of candidate j (through buffer resources,
// so any j is safe: past a component's end a read returns 0), the B loads of
// a batch are issued together, then body(values, j, shift, live) runs for
// each in order, live = false for the batch's slots past the cell's end.  The
// visiting order and the bodies run with live = true are those of
// for_each_candidate, so sums are bit-identical to it.  A body that takes a
// fifth argument also gets the candidate's cell code.
template <int D, int G, int B, typename T, typename Load, typename Body>
__device__ __forceinline__ void for_each_candidate_batched(const Grid& g, const Coeffs<T>& k,
                                                           int cell, const int* __restrict__ cs,
                                                           int sub, Load&& load, Body&& body) {
  int c[3];
  decode_cell<D>(g, cell, c);
  constexpr int zlo = (D == 3) ? -1 : 0;
  constexpr int zhi = (D == 3) ? 1 : 0;
#pragma unroll
  for (int dz = zlo; dz <= zhi; ++dz) {
    const int z = (D == 3) ? wrap_index(c[2] + dz, g.nc[2]) : 0;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int y = wrap_index(c[1] + dy, g.nc[1]);
      const int row = g.nc[0] * (y + g.nc[1] * z);
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int cc = row + wrap_index(c[0] + dx, g.nc[0]);
        const int b = cs[cc];
        const int e = cs[cc + 1];
        const T shift[3] = {T(dx) * k.L[0], T(dy) * k.L[1], T(dz) * k.L[2]};
        const unsigned code = cell_code<D>(dx, dy, dz);
        for (int j0 = b + sub; j0 < e; j0 += B * G) {
          decltype(load(0)) v[B];
#pragma unroll
          for (int u = 0; u < B; ++u) v[u] = load(j0 + u * G);
#pragma unroll
          for (int u = 0; u < B; ++u) {
            if constexpr (std::is_invocable_v<Body&, decltype(v[u])&, int, const T*, bool,
                                              unsigned>)
              body(v[u], j0 + u * G, shift, j0 + u * G < e, code);
            else
              body(v[u], j0 + u * G, shift, j0 + u * G < e);
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------- lane moves
// DPP (data-parallel primitive) moves: a lane reads a register of another
// lane in its row of 16 with one VALU instruction per 32-bit half, instead of
// a round trip through the LDS crossbar (ds_bpermute, which __shfl uses).
// A source lane that is switched off reads as 0; every caller runs with the
// whole wavefront on.  Control codes of the GFX9 DPP encoding: a quad
// permutation [p0, p1, p2, p3] is p0 | p1 << 2 | p2 << 4 | p3 << 6.
constexpr int kDppQuadXor1 = 0xB1;        // [1, 0, 3, 2]
constexpr int kDppQuadXor2 = 0x4E;        // [2, 3, 0, 1]
constexpr int kDppRowHalfMirror = 0x141;  // lane l of 8 reads lane 7 - l
constexpr int kDppRowMirror = 0x140;      // lane l of 16 reads lane 15 - l

template <int CTRL, typename T>
__device__ __forceinline__ T dpp_move(T v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(
        T, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
  } else {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, true);
    return __builtin_bit_cast(T, (long long)(((unsigned long long)(unsigned)hi << 32) |
                                             (unsigned)lo));
  }
}

// Lane `LANE`'s value of a double, in every lane (a wave-uniform read).
template <int LANE>
__device__ __forceinline__ double read_lane(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)b, LANE);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), LANE);
  return __builtin_bit_cast(double,
                            (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Quad permutation by which every lane of a group of G (2 or 4) consecutive
// lanes reads the group's lane Q.
template <int G, int Q>
constexpr int quad_group_read() {
  static_assert((G == 2 || G == 4) && Q < G, "groups of 2 or 4 lanes");
  return G == 4 ? Q * 0x55 : (Q | Q << 2 | (2 + Q) << 4 | (2 + Q) << 6);
}

// Combines the partial sums of a lane group (G consecutive lanes) in a fixed
// order (lane 0 of the group first), compensated when the accumulator is:
// the result is the same in every lane of the group and does not depend on
// timing.
template <int G, typename T, bool COMP>
__device__ __forceinline__ T group_sum(const Acc<T, COMP>& a) {
  const T v = a.value();
  if constexpr (G == 1) {
    return v;
  } else if constexpr (G == 2 || G == 4) {
    Acc<T, COMP> tot;
    tot.init(dpp_move<quad_group_read<G, 0>()>(v));
    tot.add(dpp_move<quad_group_read<G, 1>()>(v));
    if constexpr (G == 4) {
      tot.add(dpp_move<quad_group_read<G, 2>()>(v));
      tot.add(dpp_move<quad_group_read<G, 3>()>(v));
    }
    return tot.value();
  } else {
    const int lane = threadIdx.x % kWave;
    const int base = lane - lane % G;
    Acc<T, COMP> tot;
    tot.init(__shfl(v, base, kWave));
#pragma unroll
    for (int q = 1; q < G; ++q) tot.add(__shfl(v, base + q, kWave));
    return tot.value();
  }
}

// Integer sum over a lane group of G = 1, 2, 4 or 8 (exact, so the pairing
// does not matter): pairs, then quads, then the two quads of eight lanes.
template <int G>
__device__ __forceinline__ int group_sum_int(int v) {
  static_assert(G == 1 || G == 2 || G == 4 || G == 8, "lane groups of 1, 2, 4 or 8");
  if constexpr (G >= 2) v += dpp_move<kDppQuadXor1>(v);
  if constexpr (G >= 4) v += dpp_move<kDppQuadXor2>(v);
  if constexpr (G >= 8) v += dpp_move<kDppRowHalfMirror>(v);
  return v;
}

// ---------------------------------------------------------------- pair terms
// Per-pair kernel quantities shared by every sweep, so that the same pair
// gives bit-identical values wherever it is evaluated.
template <typename T>
struct PairGeo {
  T inv_r;   // 1/|r| (0 for coincident particles)
  T r;       // |r|
};

template <typename T>
__device__ __forceinline__ PairGeo<T> pair_geo(T r2) {
  PairGeo<T> pg;
  pg.inv_r = r2 > T(0) ? frsq(r2) : T(0);
  pg.r = r2 * pg.inv_r;
  return pg;
}

// Smoothing-length data of a pair: uniform h, or h_ij = (h_i + h_j)/2.
template <int D, typename T, bool VAR>
struct PairH {
  T sup2;    // (2 h_ij)^2
  T inv_h;   // 1/h_ij
  T fc;      // -5 alpha(h_ij) / h_ij^2, so that W'(r)/r = fc (1 - q/2)^3
};

template <int D, typename T, bool VAR>
__device__ __forceinline__ PairH<D, T, VAR> pair_h(const Coeffs<T>& k, T hi, T hj) {
  PairH<D, T, VAR> ph;
  if constexpr (VAR) {
    const T sup = hi + hj;
    ph.sup2 = sup * sup;
    ph.inv_h = frcp(T(0.5) * sup);
    ph.fc = T(-5) * wendland_alpha<D>(ph.inv_h) * ph.inv_h * ph.inv_h;
  } else {
    ph.sup2 = k.sup2;
    ph.inv_h = k.inv_h;
    ph.fc = k.fcoef;
  }
  return ph;
}

// t = 1 - q/2 for q = |r| / h
template <typename T>
__device__ __forceinline__ T kernel_t(T r, T inv_h) { return tfma(r * T(-0.5), inv_h, T(1)); }

// Term of the transport-velocity sum g_i = sum_j V_j F_ij r_ij, as the weight
// multiplying r_ij.  Uniform resolution leaves out the constant fcoef * m,
// applied once per particle (tv_finish).
template <int D, typename T, bool VAR>
__device__ __forceinline__ T tv_weight(const PairH<D, T, VAR>& ph, T t3, T rinv_rhoj, T mj) {
  if constexpr (VAR) return mj * rinv_rhoj * (ph.fc * t3);
  else return t3 * rinv_rhoj;
}

template <typename T, bool VAR>
__device__ __forceinline__ T tv_finish(const Coeffs<T>& k, T acc) {
  return VAR ? acc : acc * (k.fcoef * k.mass);
}

// ---------------------------------------------------------------- drift
// o' = o + dt v' + dr per axis, then rebinning: a particle may cross at most
// one cell face per axis (else flag bit 2).  Offsets stay in [0, L_T): a
// value that rounds onto a face starts the next cell at 0.  Returns the new
// linear cell; `o` is updated in place.  Flag bit 1: non-finite.
template <int D, typename T>
__device__ __forceinline__ int drift_rebin(const Grid& g, const Coeffs<T>& k, int cell, T* o,
                                           const T* vh, const T* dr, unsigned& f) {
  int c[3];
  decode_cell<D>(g, cell, c);
#pragma unroll
  for (int d = 0; d < D; ++d) {
    T x = tfma(k.dt, vh[d], o[d]) + dr[d];
    if (!isfinite(vh[d]) || !isfinite(x)) {
      f |= 1u;
      x = T(0);
    } else if (x < T(0)) {
      const T m = (T)((double)x + g.L[d]);
      if (m >= k.L[d]) {
        x = T(0);                   // rounds back onto this cell's lower face
      } else {
        c[d] -= 1;
        x = m;
        if (x < T(0)) {
          f |= 2u;                  // moved more than one cell
          x = T(0);
        }
      }
    } else if (x >= k.L[d]) {
      T m = (T)((double)x - g.L[d]);
      c[d] += 1;
      if (m < T(0)) m = T(0);       // inside [L_T, L): next cell's lower face
      if (m >= k.L[d]) {
        f |= 2u;
        m = T(0);
      }
      x = m;
    }
    c[d] = wrap_index(c[d], g.nc[d]);
    o[d] = x;
  }
  return c[0] + g.nc[0] * (c[1] + g.nc[1] * c[2]);
}

// ---------------------------------------------------------------- correction
struct Limited {
  double s, beta;
};

// The correction of one particle from its sum g (FP64 arithmetic):
//   limited (Eq. 15-16): beta = min(C s, 1) if s > s0 else 0, dr = xi beta h^2 g
//   scaled (Eq. 14):     beta = 1, dr = xi h^2 g
//   background (Eq. 12 in the drift): beta = 1, dr = -(rho0 c0^2 dt^2 / rho_i) g
// with s = h_min^2 |g|^2.
template <int D, typename T>
__device__ __forceinline__ Limited limit_correction(const Coeffs<T>& k, const T* gi, T rhoi,
                                                    T* dr) {
  double g2 = 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) g2 += (double)gi[d] * (double)gi[d];
  Limited out;
  out.s = k.hmin2 * g2;
  double f;
  if (k.tv_mode == kTvLimited) {
    out.beta = out.s > k.lim_s0 ? fmin(k.lim_c * out.s, 1.0) : 0.0;
    f = k.xi * out.beta * k.hmin2;
  } else if (k.tv_mode == kTvScaled) {
    out.beta = 1.0;
    f = k.xi * k.hmin2;
  } else {
    out.beta = 1.0;
    f = -k.bg / (double)rhoi;
  }
#pragma unroll
  for (int d = 0; d < D; ++d) dr[d] = (T)(f * (double)gi[d]);
  return out;
}

// ---------------------------------------------------------------- histogram
// Claims a slot in counts[c] for every valid lane.  Lanes are split into runs
// of consecutive lanes with the same cell (particles arrive sorted by their
// previous cell and move by at most one, so runs are long); the first lane of
// each run adds the run length to the cell's counter, all runs of the wave in
// one atomic instruction, and the run's lanes take consecutive slots.  In two
// halves: slot_claim_issue issues the atomic, slot_claim_finish reads its
// result, so a caller can put independent work between them and overlap the
// atomic's round trip (device-scope atomics are served far from the CU).
struct SlotClaim {
  int base;    // the run's first slot (valid in the run's first lane)
  int start;   // lane holding the run's base
  int lane;
};

__device__ __forceinline__ SlotClaim slot_claim_issue(bool valid, int c, int* __restrict__ counts) {
  const int lane = threadIdx.x % kWave;
  const int key = valid ? c : -1 - lane;             // invalid lanes form their own runs
  const int prev = __shfl_up(key, 1, kWave);
  const bool lead = (lane == 0) || (key != prev);
  const unsigned long long leaders = __ballot(lead);
  const unsigned long long upto = (lane == kWave - 1) ? ~0ull : ((2ull << lane) - 1);
  const int start = 63 - __clzll((long long)(leaders & upto));
  const unsigned long long after = (lane == kWave - 1) ? 0ull : (leaders >> (lane + 1));
  const int next = after ? lane + __ffsll((long long)after) : kWave;
  int base = 0;
  if (lead && valid) base = atomicAdd(&counts[c], next - lane);
  return SlotClaim{base, start, lane};
}

__device__ __forceinline__ int slot_claim_finish(const SlotClaim& sc) {
  return __shfl(sc.base, sc.start, kWave) + (sc.lane - sc.start);
}

__device__ __forceinline__ int wave_claim_slot(bool valid, int c, int* __restrict__ counts) {
  return slot_claim_finish(slot_claim_issue(valid, c, counts));
}

// ---------------------------------------------------------------- position staging
// A block serves kBlock / G consecutive particles of the (cell, id) order, so
// their cells form one range [cf, cl] of linear cell indices.  For each
// stencil offset (dy, dz) the cells they reach lie in the circular range
// [cf + o - 1, cl + o + 1], o = dy nx + dz nx ny (except cells reached across
// the periodic x seam), and the particles of a circular cell range are one
// circular run of particle indices.  stage_positions copies each run that
// fits in CAP slots into LDS once, with coalesced reads, as records of the NS
// values the candidate test needs; the compacted walk's test phase then reads
// LDS when every lane's cell of the wavefront is staged, global memory
// otherwise.  The values are the same either way.
template <int D>
struct Ranges { static constexpr int value = D == 3 ? 9 : 3; };

// Slots per staged range, 0 to stage nothing.  Staging pays for the 2-D FP32
// force sweeps (a block of 128 particles reaches ~21 cells of ~7 particles per
// range, ~150 particles, up to ~220); larger FP64 and 3-D stages would cut
// occupancy.
template <int D, typename T>
struct StageCap { static constexpr int value = (D == 2 && sizeof(T) == 4) ? 256 : 0; };

template <int D, typename T, int NS, int CAP_>
struct Stage {
  static constexpr int R = Ranges<D>::value;
  static constexpr int CAP = CAP_;
  static constexpr int W = NS == 3 ? 4 : NS;          // record width (power of 2)
  struct alignas(W * sizeof(T)) Rec { T w[W]; };
  Rec rec[CAP > 0 ? R * CAP : 1];
  int pstart[R];   // first particle of range r's run
  int plen[R];     // particles staged for range r (0: not staged)
  int clo[R];      // first cell of range r
  int cspan[R];    // (last cell - first cell) mod ncells
};

// The run of stencil range r for this block: its first particle ps and
// length len (0 when longer than cap or when the cell range wraps onto
// itself), its first cell lo and cell span.
struct StageRun {
  int ps, len, lo, span;
};
template <int D, int G>
__device__ __forceinline__ StageRun stage_run(const Grid& g, const int* __restrict__ cell,
                                              const int* __restrict__ cs, int r, int cap) {
  const int n = g.n, nc = g.ncells;
  const int p0 = blockIdx.x * (kBlock / G);
  const int p1 = min(p0 + kBlock / G, n);
  StageRun run{0, 0, 0, 0};
  if (p0 < n) {
    const int dy = r % 3 - 1, dz = (D == 3) ? r / 3 - 1 : 0;
    const int o = dy * g.nc[0] + dz * g.nc[0] * g.nc[1];
    const int cf = cell[p0], cl = cell[p1 - 1];
    run.lo = ((cf + o - 1) % nc + nc) % nc;
    const int hi = ((cl + o + 1) % nc + nc) % nc;
    run.span = hi - run.lo + (hi < run.lo ? nc : 0);
    if (run.span + 1 < nc) {
      run.ps = cs[run.lo];
      const int cnt = cs[hi + 1] - run.ps + (hi < run.lo ? n : 0);
      if (cnt <= cap) run.len = cnt;
    }
  }
  return run;
}

// Fills st for this block; every thread of the block calls it (it
// synchronises the block when CAP > 0).  src(j, v) reads particle j's NS values.
template <int D, int G, typename T, int NS, int CAP, typename Src>
__device__ __forceinline__ void stage_positions(const Grid& g, const int* __restrict__ cell,
                                                const int* __restrict__ cs,
                                                Stage<D, T, NS, CAP>& st, Src&& src) {
  if constexpr (CAP > 0) {
    constexpr int R = Stage<D, T, NS, CAP>::R;
    const int n = g.n;
    if (threadIdx.x < R) {
      const int r = threadIdx.x;
      const StageRun run = stage_run<D, G>(g, cell, cs, r, CAP);
      st.pstart[r] = run.ps;
      st.plen[r] = run.len;
      st.clo[r] = run.lo;
      st.cspan[r] = run.span;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int len = st.plen[r], ps = st.pstart[r];
      for (int t = threadIdx.x; t < len; t += kBlock) {
        int j = ps + t;
        j -= (j >= n) ? n : 0;
        T v[NS];
        src(j, v);
        typename Stage<D, T, NS, CAP>::Rec rc;
#pragma unroll
        for (int q = 0; q < Stage<D, T, NS, CAP>::W; ++q) rc.w[q] = q < NS ? v[q] : T(0);
        st.rec[r * CAP + t] = rc;
      }
    }
    __syncthreads();
  }
}

// kNotStaged if cell cc (reached with stencil range r, first particle b) is
// not staged, else delta such that particle j of cc sits in slot j + delta
// (delta = r CAP - first particle of the run, plus n past the end of the
// order: either sign).
constexpr int kNotStaged = -2147483647 - 1;

template <int D, typename T, int NS, int CAP>
__device__ __forceinline__ int staged_delta(const Grid& g, const Stage<D, T, NS, CAP>& st, int r,
                                            int cc, int b) {
  if constexpr (CAP == 0) {
    return kNotStaged;
  } else {
    int rel = cc - st.clo[r];
    rel += rel < 0 ? g.ncells : 0;
    if (st.plen[r] == 0 || rel > st.cspan[r]) return kNotStaged;
    int off = b - st.pstart[r];
    off += off < 0 ? g.n : 0;
    return r * CAP + off - b;
  }
}

// Stage of everything the force body reads of a neighbour in 2-D: for each
// stencil range of the block (the runs of stage_positions), offsets and
// velocity as one 4-vector and the density beside it.  A stored-list entry j
// of row r (its cell code's dy) is read from the stage when j lies in that
// row's run, from global memory otherwise (across the periodic seams, or a
// run longer than CAP): the values are the same either way.
template <typename T, int CAP>
struct BodyStage {
  static constexpr int R = 3;
  struct alignas(4 * sizeof(T)) V4 {
    T ox, oy, vx, vy;
  };
  V4 ov[R * CAP];
  T rho[R * CAP];
  int pstart[R];
  int plen[R];
};

// With runs (the same block's runs as an earlier sweep over the same state
// and grid stored them, found with the same cap), the runs are read from there
// instead of found again: one dependent round trip less.
template <int G, typename T, int CAP>
__device__ __forceinline__ void stage_bodies(const Grid& g, const int* __restrict__ cell,
                                             const int* __restrict__ cs,
                                             const T* __restrict__ off, const T* __restrict__ vel,
                                             const T* __restrict__ rho, BodyStage<T, CAP>& st,
                                             const int* __restrict__ runs = nullptr) {
  const int n = g.n;
  int rps[3], rlen[3];
  if (runs) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      // clamped, so runs of another state cost speed, never a wild read (a
      // slot o holds particle ps + o whatever ps and len are)
      rps[r] = min(max(runs[blockIdx.x * 6 + r], 0), n - 1);
      rlen[r] = min(max(runs[blockIdx.x * 6 + 3 + r], 0), min(CAP, n));
    }
    if (threadIdx.x < 3) {
      st.pstart[threadIdx.x] = rps[threadIdx.x];
      st.plen[threadIdx.x] = rlen[threadIdx.x];
    }
  } else {
    if (threadIdx.x < 3) {
      const StageRun run = stage_run<2, G>(g, cell, cs, threadIdx.x, CAP);
      st.pstart[threadIdx.x] = run.ps;
      st.plen[threadIdx.x] = run.len;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      rps[r] = st.pstart[r];
      rlen[r] = st.plen[r];
    }
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int len = rlen[r], ps = rps[r];
    for (int t = threadIdx.x; t < len; t += kBlock) {
      int j = ps + t;
      j -= (j >= n) ? n : 0;
      typename BodyStage<T, CAP>::V4 v;
      v.ox = off[j];
      v.oy = off[n + j];
      v.vx = vel[j];
      v.vy = vel[n + j];
      st.ov[r * CAP + t] = v;
      st.rho[r * CAP + t] = rho[j];
    }
  }
  __syncthreads();
}

// The plain candidate walk reading the candidates' test values from the
// position stage when every lane's cell of the wavefront is staged, through
// src otherwise: body(j, v, shift) with v the NS values of j (and the cell
// code, for a body that takes a fourth argument).  Same visiting order as
// for_each_candidate.
template <int D, int G, typename T, int NS, int SCAP, typename Src, typename Body>
__device__ __forceinline__ void for_each_candidate_staged(const Grid& g, const Coeffs<T>& k,
                                                          int cell, const int* __restrict__ cs,
                                                          int sub,
                                                          const Stage<D, T, NS, SCAP>& st,
                                                          Src&& src, Body&& body) {
  int c[3];
  decode_cell<D>(g, cell, c);
  constexpr int zlo = (D == 3) ? -1 : 0;
  constexpr int zhi = (D == 3) ? 1 : 0;
#pragma unroll
  for (int dz = zlo; dz <= zhi; ++dz) {
    const int z = (D == 3) ? wrap_index(c[2] + dz, g.nc[2]) : 0;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int y = wrap_index(c[1] + dy, g.nc[1]);
      const int row = g.nc[0] * (y + g.nc[1] * z);
      const int r = (dy + 1) + 3 * (dz - zlo);
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int cc = row + wrap_index(c[0] + dx, g.nc[0]);
        const int b = cs[cc];
        const int e = cs[cc + 1];
        const int delta = staged_delta<D>(g, st, r, cc, b);
        const T shift[3] = {T(dx) * k.L[0], T(dy) * k.L[1], T(dz) * k.L[2]};
        const unsigned code = cell_code<D>(dx, dy, dz);
        auto visit = [&](int j, const T* v) {
          if constexpr (std::is_invocable_v<Body&, int, const T*, const T*, unsigned>)
            body(j, v, shift, code);
          else
            body(j, v, shift);
        };
        if (__all(delta != kNotStaged)) {
          for (int j = b + sub; j < e; j += G) visit(j, st.rec[j + delta].w);
        } else {
          for (int j = b + sub; j < e; j += G) {
            T v[NS];
            src(j, v);
            visit(j, v);
          }
        }
      }
    }
  }
}

// The candidate walk for short pair bodies in the form that suits the
// configuration: from the position stage when there is one (2-D FP32),
// candidates in batches of candidate_batch() otherwise.  pair(j, v, shift,
// live) gets the NS test values v of j (offsets, then h with per-particle
// resolution) read by src(j, v); live is false for a batch's unused slots.
// A pair that takes a fifth argument also gets the candidate's cell code.
template <int D, int G, typename T, bool VAR, int NS, int SCAP, typename Src, typename Pair>
__device__ __forceinline__ void for_each_candidate_values(const Grid& g, const Coeffs<T>& k,
                                                          int cell, const int* __restrict__ cs,
                                                          int sub,
                                                          const Stage<D, T, NS, SCAP>& st,
                                                          Src&& src, Pair&& pair) {
  auto visit = [&](int j, const T* v, const T* sh, bool live, unsigned code) {
    if constexpr (std::is_invocable_v<Pair&, int, const T*, const T*, bool, unsigned>)
      pair(j, v, sh, live, code);
    else
      pair(j, v, sh, live);
  };
  if constexpr (SCAP > 0) {
    for_each_candidate_staged<D, G>(
        g, k, cell, cs, sub, st, src,
        [&](int j, const T* v, const T* sh, unsigned code) { visit(j, v, sh, true, code); });
  } else {
    struct Vals {
      T v[NS];
    };
    auto load = [&](int j) {
      Vals x;
      src(j, x.v);
      return x;
    };
    for_each_candidate_batched<D, G, candidate_batch<D, T, VAR>()>(
        g, k, cell, cs, sub, load, [&](const Vals& x, int j, const T* sh, bool live,
                                       unsigned code) { visit(j, x.v, sh, live, code); });
  }
}

// ---------------------------------------------------------------- compacted walk
// Neighbour walk in two phases for sweeps whose pair body is expensive.  The
// scan phase tests every candidate with test(j, v, shift), v the NS staged
// values of j (positions, and h with per-particle resolution; from the
// position stage or from src), and appends the hits to this thread's list in
// LDS; the body phase then runs body(j, shift) over the list alone, so the
// wavefront executes the body once per neighbour instead of once per
// candidate (outside the stage, each lane tests B candidates at a time, their
// loads issued together).  The list is flushed after each z-plane of cells
// (once in 2-D) and whenever it fills.  An entry is j in bits 0-27, dx + 1 in
// bits 28-29 and dy + 1 in bits 30-31.  The visiting order is that of
// for_each_candidate, so sums over the listed pairs are bit-identical to sums
// over a plain walk.
constexpr int kListBits = 28;
constexpr unsigned kListMask = (1u << kListBits) - 1u;

template <int CAP>
struct NeighbourList {
  unsigned slot[CAP][kBlock];   // [entry][thread]: one bank per thread
};

template <int D, int G, typename T, int NS, int B, int SCAP, int CAP, typename Src,
          typename Test, typename Body>
__device__ __forceinline__ void for_each_neighbour_listed(const Grid& g, const Coeffs<T>& k,
                                                          int cell, const int* __restrict__ cs,
                                                          int sub,
                                                          const Stage<D, T, NS, SCAP>& st,
                                                          NeighbourList<CAP>& nl, Src&& src,
                                                          Test&& test, Body&& body) {
  int c[3];
  decode_cell<D>(g, cell, c);
  const int tid = threadIdx.x;
  constexpr int zlo = (D == 3) ? -1 : 0;
  constexpr int zhi = (D == 3) ? 1 : 0;
  int cnt = 0;
#pragma unroll
  for (int dz = zlo; dz <= zhi; ++dz) {
    const int z = (D == 3) ? wrap_index(c[2] + dz, g.nc[2]) : 0;
    const T sz = T(dz) * k.L[2];
    auto flush = [&]() {
      for (int q = 0; q < cnt; ++q) {
        const unsigned e = nl.slot[q][tid];
        // (c - 1) L as c L - L: exact for c in {0, 1, 2}
        const T cx = T((e >> kListBits) & 3u), cy = T(e >> (kListBits + 2));
        const T shift[3] = {tfma(cx, k.L[0], -k.L[0]), tfma(cy, k.L[1], -k.L[1]), sz};
        body((int)(e & kListMask), shift);
      }
      cnt = 0;
    };
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int y = wrap_index(c[1] + dy, g.nc[1]);
      const int row = g.nc[0] * (y + g.nc[1] * z);
      const int r = (dy + 1) + 3 * (dz - zlo);
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int cc = row + wrap_index(c[0] + dx, g.nc[0]);
        const int b = cs[cc];
        const int e = cs[cc + 1];
        const int delta = staged_delta<D>(g, st, r, cc, b);
        const T shift[3] = {T(dx) * k.L[0], T(dy) * k.L[1], sz};
        const unsigned code = (unsigned)((dx + 1) | ((dy + 1) << 2)) << kListBits;
        // one source per wavefront and cell: the stage when every lane's cell
        // is staged, else global memory for all lanes
        if (__all(delta != kNotStaged)) {
          for (int j = b + sub; j < e; j += G) {
            const auto rc = st.rec[j + delta];
            if (test(j, rc.w, shift)) {
              nl.slot[cnt][tid] = (unsigned)j | code;
              if (++cnt == CAP) flush();
            }
          }
        } else {
          // B candidates per lane at a time, their loads issued together
          for (int j0 = b + sub; j0 < e; j0 += B * G) {
            T v[B][NS];
#pragma unroll
            for (int u = 0; u < B; ++u) src(j0 + u * G, v[u]);
#pragma unroll
            for (int u = 0; u < B; ++u) {
              const int j = j0 + u * G;
              const bool hit = test(j, v[u], shift);
              if ((j < e) & hit) {
                nl.slot[cnt][tid] = (unsigned)j | code;
                if (++cnt == CAP) flush();
              }
            }
          }
        }
      }
    }
    flush();
  }
}

// ---------------------------------------------------------------- stored neighbour lists
// Inside a multi-step run the density sweep records each lane's neighbours,
// in the lane's visiting order, for the force sweep that follows at the same
// positions, which then tests no candidates: entry q of lane L (the global
// thread index) sits at entry[q * stride + L] for q < cap (j and its cell
// code, as above), and count[L] is the lane's neighbour count — above cap
// when the list is incomplete, and that lane then walks its candidates
// itself.  Lane L serves the same particle and the same candidates in both
// sweeps, so sums over a stored list are bit-identical to sums over the walk.
// Capacities (entries per lane): about 1.6 times the mean neighbours per lane
// at h = 1.3 dx (20 per particle in 2-D, 80 in 3-D) plus a margin.
constexpr int list_cap(int dim, int G) {
  return dim == 3 ? (G == 2 ? 64 : (G == 4 ? 36 : 20)) : (G == 2 ? 20 : (G == 4 ? 12 : 8));
}

struct StoredList {
  unsigned* entry;   // null: no list
  int* count;
  int stride;        // lanes of the sweeps' grid (blocks * kBlock)
  // per block, the first particle and the length of its three stencil rows'
  // runs (2-D, as the position stage found them): six ints, or null
  int* runs = nullptr;
};

// What a pair body reads of a neighbour: offsets, velocity, density, and
// mass and h (per-particle resolution).
template <int D, typename T>
struct PairIn {
  T o[D], v[D], rho, m, h;
};

// Runs the pair body over lane L's stored list in batches of two: the two
// entries are read together, then fetch(e) for both entries (their
// loads issued together; past the list's end the last entry is fetched
// again and not used), then compute(values, shift) for each in order.  A
// lane whose list is incomplete walks its candidates instead, with
// test(j, v, shift) on the NS values v read by src(j, v) and fetch(j) (an
// index without cell code).  Same order as the walk that wrote the list.
template <int D, int G, typename T, int NS, typename Src, typename Test, typename Fetch,
          typename Compute>
__device__ __forceinline__ void for_each_neighbour_stored(const Grid& g, const Coeffs<T>& k,
                                                          int cell, const int* __restrict__ cs,
                                                          int sub, const StoredList& sl,
                                                          Src&& src, Test&& test, Fetch&& fetch,
                                                          Compute&& compute) {
  constexpr int CAP = list_cap(D, G);
  constexpr int JB = list_jbits<D>();
  const int L = blockIdx.x * kBlock + threadIdx.x;
  const int cnt = sl.count[L];
  if (cnt <= CAP) {
    constexpr int B = 2;
    for (int q0 = 0; q0 < cnt; q0 += B) {
      // rows q0 .. q0 + B - 1 (clamped to the list's rows: the same for every lane,
      // so the row address is scalar); entries past a lane's count are not used
      unsigned e[B];
#pragma unroll
      for (int u = 0; u < B; ++u) e[u] = (sl.entry + (size_t)min(q0 + u, CAP - 1) * sl.stride)[L];
      decltype(fetch(0u)) nb[B];
#pragma unroll
      for (int u = 0; u < B; ++u) nb[u] = fetch(e[u]);
#pragma unroll
      for (int u = 0; u < B; ++u) {
        if (q0 + u < cnt) {
          T shift[3];
          code_shift<D>(k, e[u] >> JB, shift);
          compute(nb[u], shift);
        }
      }
    }
  } else {
    for_each_candidate<D, G>(g, k, cell, cs, sub, [&](int j, const T* sh) {
      T v[NS];
      src(j, v);
      if (test(j, v, sh)) compute(fetch((unsigned)j), sh);   // no code, not staged
    });
  }
}

// body(j, shift) over lane L's stored list, two entries read at a time (the
// body reads what it needs of j itself); a lane whose list is incomplete
// walks its candidates with test(j, v, shift) on the NS values read by
// src(j, v).  Same order as the walk that wrote the list.
template <int D, int G, typename T, int NS, typename Src, typename Test, typename Body>
__device__ __forceinline__ void for_each_stored_entry(const Grid& g, const Coeffs<T>& k,
                                                      int cell, const int* __restrict__ cs,
                                                      int sub, const StoredList& sl, Src&& src,
                                                      Test&& test, Body&& body) {
  constexpr int CAP = list_cap(D, G);
  constexpr int JB = list_jbits<D>();
  constexpr unsigned JMASK = (1u << JB) - 1u;
  const int L = blockIdx.x * kBlock + threadIdx.x;
  const int cnt = sl.count[L];
  if (cnt <= CAP) {
    for (int q0 = 0; q0 < cnt; q0 += 2) {
      unsigned e[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) e[u] = (sl.entry + (size_t)min(q0 + u, CAP - 1) * sl.stride)[L];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        if (q0 + u < cnt) {
          T shift[3];
          code_shift<D>(k, e[u] >> JB, shift);
          body((int)(e[u] & JMASK), shift);
        }
      }
    }
  } else {
    for_each_candidate<D, G>(g, k, cell, cs, sub, [&](int j, const T* sh) {
      T v[NS];
      src(j, v);
      if (test(j, v, sh)) body(j, sh);
    });
  }
}

// ---------------------------------------------------------------- reductions
// Sum or maximum over the 64 lanes of a wavefront, in every lane: DPP moves
// combine pairs, quads, halves and whole rows of 16, then the four row
// results are read out and combined in the order 0, 16, 32, 48.  The order is
// fixed, so the result is bit-reproducible.  Maxima are taken over values
// >= 0 (a switched-off lane would read as 0).
template <bool MAX>
__device__ __forceinline__ double lane_combine(double a, double b) {
  return MAX ? (a > b ? a : b) : a + b;
}
template <bool MAX>
__device__ __forceinline__ double wave_reduce(double v) {
  v = lane_combine<MAX>(v, dpp_move<kDppQuadXor1>(v));
  v = lane_combine<MAX>(v, dpp_move<kDppQuadXor2>(v));
  v = lane_combine<MAX>(v, dpp_move<kDppRowHalfMirror>(v));
  v = lane_combine<MAX>(v, dpp_move<kDppRowMirror>(v));
  return lane_combine<MAX>(lane_combine<MAX>(read_lane<0>(v), read_lane<16>(v)),
                           lane_combine<MAX>(read_lane<32>(v), read_lane<48>(v)));
}
__device__ __forceinline__ double wave_sum(double v) { return wave_reduce<false>(v); }
__device__ __forceinline__ double wave_max(double v) { return wave_reduce<true>(v); }

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

// Block-wide sums / maxima of NV values per thread at once (one LDS pass);
// results valid in thread 0.  max_mask bit v selects a maximum for value v.
template <int NV>
__device__ __forceinline__ void block_reduce_multi(double* v, unsigned max_mask,
                                                   double (*lds)[kBlock / kWave]) {
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave;
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = ((max_mask >> q) & 1u) ? wave_max(v[q]) : wave_sum(v[q]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) lds[q][wave] = v[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double r = lds[q][0];
      for (int w = 1; w < kBlock / kWave; ++w)
        r = ((max_mask >> q) & 1u) ? (r > lds[q][w] ? r : lds[q][w]) : r + lds[q][w];
      v[q] = r;
    }
  }
}

// Diagnostic partials: one row per wavefront, stored column-major
// [kNumPartials][nrows] with nrows = (grid blocks) * (waves per block); every
// kernel that writes partials in a step runs on the same grid, so rows line
// up.  Each wavefront reduces its lanes with shuffles only (no block
// barrier) and its first lane writes the row.
constexpr int kWavesPerBlock = kBlock / kWave;

// Exact sum of an integer over the wavefront (same lane pattern as wave_reduce)
__device__ __forceinline__ int wave_sum_int(int v) {
  v += dpp_move<kDppQuadXor1>(v);
  v += dpp_move<kDppQuadXor2>(v);
  v += dpp_move<kDppRowHalfMirror>(v);
  v += dpp_move<kDppRowMirror>(v);
  return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) +
         __builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48);
}

// Bit q of max_mask: value q is reduced by maximum (else sum); of flag_mask:
// value q is 0 or 1 in every lane and is counted (ballot); of int_mask: value
// q is a small integer, summed as one.  Counts and integer sums are exact, so
// they equal the FP64 sums bit for bit.
template <int NV>
__device__ __forceinline__ void wave_partials(double* __restrict__ p, const int* cols,
                                              double* v, unsigned max_mask,
                                              unsigned flag_mask = 0u, unsigned int_mask = 0u) {
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    if ((flag_mask >> q) & 1u)
      v[q] = (double)__popcll(__ballot(v[q] != 0.0));
    else if ((int_mask >> q) & 1u)
      v[q] = (double)wave_sum_int((int)v[q]);
    else
      v[q] = ((max_mask >> q) & 1u) ? wave_max(v[q]) : wave_sum(v[q]);
  }
  if (threadIdx.x % kWave == 0) {
    const size_t nrows = (size_t)gridDim.x * kWavesPerBlock;
    const size_t row = (size_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < NV; ++q) p[cols[q] * nrows + row] = v[q];
  }
}

// Folds column `col` of the partials (nrows rows) into diag[col], in a fixed
// order (sum, or maximum for columns 4 and 8): deterministic.  One block per
// column; must run in a later launch than the writers.  Each thread keeps
// eight accumulators and issues its eight loads of a round together (the row
// index is clamped so every load is in bounds; rows past the end count as 0),
// so a round costs one memory latency.
template <bool MAX>
__device__ __forceinline__ double fold_rows(const double* __restrict__ c, int nrows) {
  constexpr int U = 8;
  double a[U];
#pragma unroll
  for (int u = 0; u < U; ++u) a[u] = 0.0;
  for (int r = threadIdx.x; r < nrows; r += U * kBlock) {
    double x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int rr = r + u * kBlock;
      x[u] = c[rr < nrows ? rr : nrows - 1];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) a[u] = lane_combine<MAX>(a[u], r + u * kBlock < nrows ? x[u] : 0.0);
  }
#pragma unroll
  for (int w = U / 2; w > 0; w /= 2) {
#pragma unroll
    for (int u = 0; u < w; ++u) a[u] = lane_combine<MAX>(a[u], a[u + w]);
  }
  return a[0];
}

__device__ __forceinline__ void fold_diag_column(const double* __restrict__ partials, int nrows,
                                                 int col, double* __restrict__ diag) {
  __shared__ double red[kBlock / kWave];
  const double* c = partials + (size_t)col * nrows;
  double v;
  if (col == 4 || col == 8)
    v = block_reduce<double, true>(fold_rows<true>(c, nrows), red);
  else
    v = block_reduce<double, false>(fold_rows<false>(c, nrows), red);
  if (threadIdx.x == 0) diag[col] = v;
}

}  // namespace sph
