// Cell-linked-list build: bin absolute positions into (cell, offset), then
// order particles by (cell, id).
//
// The order is a counting sort by cell (integer histogram with atomic slot
// claims, exclusive scan, scatter) followed by ranking inside each cell by
// id.  The slot claimed by the atomic is arbitrary, but the final order is
// not: a particle's destination is cell_start[cell] + |{ q in cell : id_q < id }|,
// a function of (cell, id) alone, so the result is bit-reproducible.
#include "sph_internal.hpp"

namespace sph {

// ------------------------------------------------------------------ binning
template <int D, typename T>
__global__ __launch_bounds__(kBlock) void bin_kernel(Grid g, Coeffs<T> k,
                                                     const double* __restrict__ pos,
                                                     int* __restrict__ cell, T* __restrict__ off,
                                                     unsigned* __restrict__ flags) {
  const int n = g.n;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int c[3] = {0, 0, 0};
  unsigned f = 0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    double x = pos[d * n + i];
    const double B = g.box[d];
    if (!isfinite(x)) {
      f |= kFlagNonfinite;
      x = 0.0;
    }
    if (!(x >= 0.0 && x < B)) {
      f |= kFlagOutOfBox;
      x -= B * floor(x / B);
      if (!(x < B)) x = 0.0;
    }
    const double L = g.L[d];
    int ci = (int)floor(x / L);
    ci = ci < 0 ? 0 : (ci >= g.nc[d] ? g.nc[d] - 1 : ci);
    double o = x - (double)ci * L;
    if (o < 0.0) {
      ci = wrap_index(ci - 1, g.nc[d]);
      o += L;
    }
    T ot = (T)o;
    if (ot >= k.L[d]) {           // rounds onto the face: start of the next cell
      ci = wrap_index(ci + 1, g.nc[d]);
      ot = T(0);
    }
    c[d] = ci;
    off[d * n + i] = ot;
  }
  int lin = c[0] + g.nc[0] * (c[1] + g.nc[1] * c[2]);
  cell[i] = lin;
  if (f) atomicOr(flags, f);
}

template <typename T>
void launch_bin(const Launch& l, const Grid& g, const Coeffs<T>& k, const double* pos,
                int* cell, T* off, unsigned* flags) {
  if (g.n == 0) return;
  if (l.dim == 2)
    hipLaunchKernelGGL((bin_kernel<2, T>), dim3(blocks_for(g.n)), dim3(kBlock), 0, l.stream, g, k, pos,
                       cell, off, flags);
  else
    hipLaunchKernelGGL((bin_kernel<3, T>), dim3(blocks_for(g.n)), dim3(kBlock), 0, l.stream, g, k, pos,
                       cell, off, flags);
}

// ------------------------------------------------------------------ fill
__global__ __launch_bounds__(kBlock) void fill_kernel(int* __restrict__ p, long n, int v) {
  long i = (long)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

void launch_fill(hipStream_t s, int* p, long n, int v) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3(blocks_for(n)), dim3(kBlock), 0, s, p, n, v);
}

// ------------------------------------------------------------------ scan
// Exclusive scan of the cell histogram into cell_start, leaving the
// histogram zeroed for the next build.
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

int scan_blocks(int ncells) { return (ncells + kScanTile - 1) / kScanTile; }

template <int BLOCK>
__device__ __forceinline__ int block_exclusive_scan(int v, int* lds, int* total) {
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave;
  int x = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) lds[wave] = x;
  __syncthreads();
  int base = 0, tot = 0;
  for (int w = 0; w < BLOCK / kWave; ++w) {
    if (w < wave) base += lds[w];
    tot += lds[w];
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

// Single pass with decoupled look-back: each block scans one tile of the
// histogram, publishes its tile total, then walks back over the tiles before
// it, adding their totals until it meets one that already carries its
// inclusive prefix.  Tiles are numbered in the order blocks start (an atomic
// ticket), so every tile a block waits on belongs to a block that is already
// running and publishes without waiting; the wait is bounded anyway (a block
// that gives up raises SPH_FLAG_INTERNAL instead of hanging).  Tile words
// carry the launch's epoch, so words left by earlier launches read as
// unpublished and nothing has to be re-armed between launches: no fences.
constexpr unsigned long long kTileAgg = 1ull << 62;
constexpr unsigned long long kTileInc = 2ull << 62;
constexpr unsigned long long kTileFlags = 3ull << 62;
constexpr long kSpinLimit = 1L << 22;

__device__ __forceinline__ unsigned long long tile_word(unsigned long long flag, unsigned epoch,
                                                        unsigned value) {
  return flag | ((unsigned long long)(epoch & 0x3fffffffu) << 32) | value;
}

__global__ __launch_bounds__(kBlock) void scan_lookback_kernel(
    int ncells, int ntiles, int* __restrict__ counts, int* __restrict__ cs,
    unsigned long long* __restrict__ tile_state, unsigned* __restrict__ tickets, unsigned epoch,
    unsigned* __restrict__ flags, DiagFold fold) {
  __shared__ int lds[kBlock / kWave];
  __shared__ int tile_s, prefix_s;
  if (fold.partials && (int)blockIdx.x >= ntiles) {
    // the extra blocks fold the previous step's diagnostics, one column each;
    // they take no ticket
    fold_diag_column(fold.partials, fold.nrows, blockIdx.x - ntiles, fold.diag);
    return;
  }
  if (threadIdx.x == 0)
    tile_s = (int)(atomicAdd(&tickets[0], 1u) - epoch * (unsigned)ntiles);
  __syncthreads();
  const int tile = tile_s;
  const int base = tile * kScanTile + threadIdx.x * kScanItems;
  int v[kScanItems];
  int s = 0;
#pragma unroll
  for (int t = 0; t < kScanItems; ++t) {
    v[t] = (base + t < ncells) ? counts[base + t] : 0;
    s += v[t];
  }
  int total;
  const int excl = block_exclusive_scan<kBlock>(s, lds, &total);
  if (threadIdx.x == 0) {
    const unsigned long long ep = (unsigned long long)(epoch & 0x3fffffffu) << 32;
    unsigned prefix = 0;
    if (tile == 0) {
      __hip_atomic_store(&tile_state[0], tile_word(kTileInc, epoch, (unsigned)total),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      __hip_atomic_store(&tile_state[tile], tile_word(kTileAgg, epoch, (unsigned)total),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      int p = tile - 1;
      long spins = 0;
      while (p >= 0) {
        const unsigned long long st =
            __hip_atomic_load(&tile_state[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long f = st & kTileFlags;
        if (f == 0 || (st & (0x3fffffffull << 32)) != ep) {
          if (++spins > kSpinLimit) {
            atomicOr(flags, kFlagInternal);
            break;
          }
          continue;
        }
        prefix += (unsigned)(st & 0xffffffffull);
        if (f == kTileInc) break;
        --p;
      }
      __hip_atomic_store(&tile_state[tile], tile_word(kTileInc, epoch, prefix + (unsigned)total),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    prefix_s = (int)prefix;
  }
  __syncthreads();
  int run = prefix_s + excl;
#pragma unroll
  for (int t = 0; t < kScanItems; ++t) {
    if (base + t < ncells) {
      cs[base + t] = run;
      counts[base + t] = 0;
    }
    run += v[t];
  }
  if (tile == ntiles - 1 && threadIdx.x == 0) cs[ncells] = prefix_s + total;
}

void launch_scan(hipStream_t s, int ncells, int* counts, ScanState st, unsigned epoch, int* cs,
                 unsigned* flags, DiagFold fold) {
  const int nt = scan_blocks(ncells);
  const int nb = nt + (fold.partials ? kNumPartials : 0);
  hipLaunchKernelGGL(scan_lookback_kernel, dim3(nb), dim3(kBlock), 0, s, ncells, nt, counts, cs,
                     st.tile_state, st.tickets, epoch, flags, fold);
}

// ------------------------------------------------------------------ scatter
// Each particle lands in slot `slot` of its new cell, together with its id
// and that cell's [start, end) so the ranking pass needs no further lookups.
__global__ __launch_bounds__(kBlock) void scatter_kernel(int n, const int* __restrict__ cell,
                                                         const int* __restrict__ id,
                                                         const int* __restrict__ slot,
                                                         const int* __restrict__ cs,
                                                         SortTmp tmp) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int c = cell[i];
  const int b = cs[c];
  const int e = cs[c + 1];
  const int pos = b + slot[i];
  tmp.src[pos] = i;
  tmp.id[pos] = id[i];
  tmp.range[pos] = make_int2(b, e);
}

void launch_scatter(hipStream_t s, int n, const int* cell, const int* id, const int* slot,
                    const int* cs, SortTmp tmp) {
  if (n == 0) return;
  hipLaunchKernelGGL(scatter_kernel, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, cell, id, slot,
                     cs, tmp);
}

// ------------------------------------------------------------------ rank + gather
// Slot p holds a particle of some cell; its final position is the cell start
// plus the number of cell members with a smaller id.  The gathered values are
// loaded first, so their latency overlaps the ranking, and the ranking reads
// the cell's ids eight at a time with the eight loads issued together (the
// index is clamped into the cell, which holds at least this particle; reads
// past its end are not counted): a few memory latencies per thread instead of
// one per cell member and one per array.
constexpr int kRankBatch = 8;

template <int D, typename T>
__global__ __launch_bounds__(kBlock) void rank_gather_kernel(int n, SortTmp tmp,
                                                             PArrays<T> stg, PArrays<T> dst,
                                                             int* __restrict__ perm) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= n) return;
  const int src = tmp.src[p];
  const int idk = tmp.id[p];
  const int2 be = tmp.range[p];
  const int cell = stg.cell[src];
  T off[D], vel[D], acc[D];
  T rho = T(0), mass = T(0), h = T(0);
#pragma unroll
  for (int d = 0; d < D; ++d) {
    off[d] = stg.off[d * n + src];
    vel[d] = dst.vel ? stg.vel[d * n + src] : T(0);
    acc[d] = dst.acc ? stg.acc[d * n + src] : T(0);
  }
  if (dst.rho) rho = stg.rho[src];
  if (dst.mass) mass = stg.mass[src];
  if (dst.h) h = stg.h[src];
  int rank = 0;
  for (int q = be.x; q < be.y; q += kRankBatch) {
    int ids[kRankBatch];
#pragma unroll
    for (int u = 0; u < kRankBatch; ++u) ids[u] = tmp.id[min(q + u, be.y - 1)];
#pragma unroll
    for (int u = 0; u < kRankBatch; ++u) rank += (q + u < be.y && ids[u] < idk) ? 1 : 0;
  }
  const int to = be.x + rank;
  if (perm) perm[to] = src;
  dst.cell[to] = cell;
  dst.id[to] = idk;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    dst.off[d * n + to] = off[d];
    if (dst.vel) dst.vel[d * n + to] = vel[d];
    if (dst.acc) dst.acc[d * n + to] = acc[d];
  }
  if (dst.rho) dst.rho[to] = rho;
  if (dst.mass) dst.mass[to] = mass;
  if (dst.h) dst.h[to] = h;
}

template <typename T>
void launch_rank_gather(const Launch& l, int n, SortTmp tmp, const PArrays<T>& stg,
                        const PArrays<T>& dst, int* perm) {
  if (n == 0) return;
  if (l.dim == 2)
    hipLaunchKernelGGL((rank_gather_kernel<2, T>), dim3(blocks_for(n)), dim3(kBlock), 0, l.stream,
                       n, tmp, stg, dst, perm);
  else
    hipLaunchKernelGGL((rank_gather_kernel<3, T>), dim3(blocks_for(n)), dim3(kBlock), 0, l.stream,
                       n, tmp, stg, dst, perm);
}

#define SPH_INST(T)                                                                          \
  template void launch_bin<T>(const Launch&, const Grid&, const Coeffs<T>&, const double*,   \
                              int*, T*, unsigned*);                                          \
  template void launch_rank_gather<T>(const Launch&, int, SortTmp, const PArrays<T>&,        \
                                      const PArrays<T>&, int*);
SPH_INST(float)
SPH_INST(double)
#undef SPH_INST

}  // namespace sph
