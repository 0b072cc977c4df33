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
  const bool valid = i < n;
  int c = 0;
  if (valid) {
    c = src.cell[i];
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
  }
  const int sl = wave_claim_slot(valid, c, counts);
  if (valid) slot[i] = sl;
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

// ------------------------------------------------------------------ batched copies
// Up to kMaxCopies device-to-device copies of whole 4-byte words in one
// launch (blockIdx.y picks the copy): 16-byte moves where both ends are
// 16-byte aligned, 4-byte moves for the rest.  Sizes are multiples of 4.
__global__ __launch_bounds__(kBlock) void multi_copy_kernel(CopyBatch b) {
  const int c = blockIdx.y;
  if (c >= b.count) return;
  const char* __restrict__ src = b.src[c];
  char* __restrict__ dst = b.dst[c];
  const long words = b.bytes[c] / 4;
  const long stride = (long)gridDim.x * kBlock;
  long head = 0;
  if ((((unsigned long)src | (unsigned long)dst) & 15ul) == 0) {
    head = words / 4 * 4;
    const uint4* __restrict__ s4 = (const uint4*)src;
    uint4* __restrict__ d4 = (uint4*)dst;
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < head / 4; i += stride) d4[i] = s4[i];
  }
  const unsigned* __restrict__ s1 = (const unsigned*)src;
  unsigned* __restrict__ d1 = (unsigned*)dst;
  for (long i = head + (long)blockIdx.x * kBlock + threadIdx.x; i < words; i += stride) d1[i] = s1[i];
}

void launch_multi_copy(hipStream_t s, const CopyBatch& b) {
  if (b.count <= 0) return;
  long most = 0;
  for (int c = 0; c < b.count; ++c) most = b.bytes[c] > most ? b.bytes[c] : most;
  const long chunks = (most / 16 + kBlock - 1) / kBlock;
  const int bx = (int)(chunks < 1 ? 1 : (chunks > 1024 ? 1024 : chunks));
  hipLaunchKernelGGL(multi_copy_kernel, dim3(bx, b.count), dim3(kBlock), 0, s, b);
}

// ------------------------------------------------------------------ kick + drift + rebin
// v' = v + dt/2 a; o' = o + dt v' + dr, rebinned (drift_rebin); the moved
// particle goes to the staging buffers and, with counts given, claims a slot
// in its new cell (for the scan-and-scatter cell build).
template <int D, typename T, bool VAR>
__global__ __launch_bounds__(kBlock) void drift_kernel(Grid g, Coeffs<T> k, PArrays<T> p,
                                                       const T* __restrict__ dr, PArrays<T> stg,
                                                       int* __restrict__ counts,
                                                       int* __restrict__ slot,
                                                       unsigned* __restrict__ flags) {
  const int n = g.n;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool valid = i < n;
  int lin = 0;
  if (valid) {
    // wall particles keep their position and velocity
    const bool wall = wall_at(k, n, p.id, i);
    T o[3], vh[3], dri[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int d = 0; d < D; ++d) {
      vh[d] = wall ? p.vel[d * n + i] : tfma(k.half_dt, p.acc[d * n + i], p.vel[d * n + i]);
      o[d] = p.off[d * n + i];
      if (dr) dri[d] = dr[d * n + i];
    }
    unsigned f = 0;
    lin = wall ? p.cell[i] : drift_rebin<D>(g, k, p.cell[i], o, vh, dri, f);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      stg.off[d * n + i] = o[d];
      stg.vel[d * n + i] = vh[d];
    }
    stg.cell[i] = lin;
    stg.id[i] = p.id[i];
    if constexpr (VAR) {
      stg.mass[i] = p.mass[i];
      stg.h[i] = p.h[i];
    }
    if (f) atomicOr(flags, f);
  }
  if (counts) {
    const int sl = wave_claim_slot(valid, lin, counts);
    if (valid) slot[i] = sl;
  }
}

template <typename T>
void launch_drift(const Launch& l, const Grid& g, const Coeffs<T>& k, const PArrays<T>& p,
                  const T* dr, const PArrays<T>& stg, int* counts, int* slot, unsigned* flags) {
  if (g.n == 0) return;
#define SPH_DRIFT(D, V)                                                                        \
  hipLaunchKernelGGL((drift_kernel<D, T, V>), dim3(blocks_for(g.n)), dim3(kBlock), 0, l.stream, g, k, p, \
                     dr, stg, counts, slot, flags)
  if (l.dim == 2) { if (l.var) SPH_DRIFT(2, true); else SPH_DRIFT(2, false); }
  else { if (l.var) SPH_DRIFT(3, true); else SPH_DRIFT(3, false); }
#undef SPH_DRIFT
}

// ------------------------------------------------------------------ kick + diagnostics
// v = v + dt/2 a (when `write`), then per-block FP64 partials of the kinetic
// energy, momentum and max |v| of the resulting velocity, folded into diag
// by the last block.
template <int D, typename T>
__global__ __launch_bounds__(kBlock) void kick_kernel(Coeffs<T> k, int n, T* __restrict__ vel,
                                                      const T* __restrict__ acc,
                                                      const T* __restrict__ mass,
                                                      const int* __restrict__ id,
                                                      double* __restrict__ partials, int write,
                                                      int G, unsigned* __restrict__ flags) {
  // same particle-to-block mapping as the sweeps (G lanes per particle, the
  // first does the work), so per-block partials fold in the same order
  const int i = (blockIdx.x * kBlock + threadIdx.x) / G;
  double ke = 0.0, mom[3] = {0.0, 0.0, 0.0}, vmax = 0.0;
  if (i < n && threadIdx.x % G == 0 && !wall_at(k, n, id, i)) {
    const double m = mass ? (double)mass[i] : (double)k.mass;
    double v2 = 0.0;
    bool bad = false;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      T v = vel[d * n + i];
      if (write) {
        v = tfma(k.half_dt, acc[d * n + i], v);
        vel[d * n + i] = v;
      }
      bad |= !isfinite(v);
      v2 += (double)v * (double)v;
      mom[d] = m * (double)v;
    }
    ke = 0.5 * m * v2;
    vmax = sqrt(v2);
    if (bad && flags) atomicOr(flags, kFlagNonfinite);
  }
  if (partials) {
    const int cols[5] = {0, 1, 2, 3, 4};
    double v[5] = {ke, mom[0], mom[1], mom[2], vmax};
    wave_partials<5>(partials, cols, v, 1u << 4);
  }
}

template <typename T>
void launch_kick(const Launch& l, const Coeffs<T>& k, int n, T* vel, const T* acc,
                 const T* mass, const int* id, double* partials, bool write, unsigned* flags) {
  if (n == 0) return;
  if (l.dim == 2)
    hipLaunchKernelGGL((kick_kernel<2, T>), dim3(l.nblk), dim3(kBlock), 0, l.stream, k, n, vel,
                       acc, mass, id, partials, write ? 1 : 0, l.G, flags);
  else
    hipLaunchKernelGGL((kick_kernel<3, T>), dim3(l.nblk), dim3(kBlock), 0, l.stream, k, n, vel,
                       acc, mass, id, partials, write ? 1 : 0, l.G, flags);
}

__global__ __launch_bounds__(kBlock) void diag_fold_kernel(const double* __restrict__ partials,
                                                           int nrows, double* __restrict__ diag) {
  fold_diag_column(partials, nrows, blockIdx.x, diag);
}

void launch_diag_fold(hipStream_t s, DiagFold fold) {
  if (!fold.partials) return;
  hipLaunchKernelGGL(diag_fold_kernel, dim3(kNumPartials), dim3(kBlock), 0, s, fold.partials,
                     fold.nrows, fold.diag);
}

// blocks [0, nfold): one diagnostics column each; the others: the copy
__global__ __launch_bounds__(kBlock) void fold_copy_kernel(const double* __restrict__ partials,
                                                           int nrows, double* __restrict__ diag,
                                                           int nfold,
                                                           const unsigned* __restrict__ src,
                                                           unsigned* __restrict__ dst, long words) {
  if ((int)blockIdx.x < nfold) {
    fold_diag_column(partials, nrows, blockIdx.x, diag);
    return;
  }
  const long nb = (long)gridDim.x - nfold;
  for (long w = ((long)blockIdx.x - nfold) * kBlock + threadIdx.x; w < words; w += nb * kBlock)
    dst[w] = src[w];
}

void launch_fold_copy(hipStream_t s, DiagFold fold, const void* src, void* dst, size_t bytes) {
  const int nfold = fold.partials ? kNumPartials : 0;
  const long words = (long)(bytes / 4);
  const long nb = words > 0 ? blocks_for(words) : 0;
  const int ncopy = (int)(nb < 1024 ? nb : 1024);
  if (nfold + ncopy == 0) return;
  hipLaunchKernelGGL(fold_copy_kernel, dim3(nfold + ncopy), dim3(kBlock), 0, s, fold.partials,
                     fold.nrows, fold.diag, nfold, (const unsigned*)src, (unsigned*)dst, words);
}

__global__ __launch_bounds__(kBlock) void zero_double_kernel(double* __restrict__ p, long n) {
  long i = (long)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

void launch_zero_partials(hipStream_t s, int nblk, double* partials) {
  long n = (long)(nblk > 0 ? nblk : 1) * kWavesPerBlock * kNumPartials;
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
                               const int*, double*, bool, unsigned*);
SPH_INST(float)
SPH_INST(double)
#undef SPH_INST

}  // namespace sph
