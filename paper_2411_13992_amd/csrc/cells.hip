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

// ------------------------------------------------------------------ rebuild
// One launch that puts particles back into (cell, id) order after a drift
// that moved each of them by at most one cell per axis (the drift flags and
// clamps anything else).  The previous order is sorted by the previous
// cells, with cell_start cs_old; the staging arrays hold every particle's new
// cell and values in that order.  Block b takes tile b: up to T consecutive
// cells of one x-row (tiles numbered in cell order).  The tile's particles were previous occupants
// of the cells within one cell of it — 3 row segments in 2-D, 9 in 3-D, each
// one or two runs of the previous order — so the block reads those runs'
// new cells, counts the tile's particles per cell in LDS, gets the number of
// particles in all earlier tiles by a decoupled look-back over the tiles'
// totals (the same scheme as scan_lookback_kernel), ranks each particle by id
// among its cell's particles and writes them (their densities too when dst.rho
// is given), its cells' starts and the permutation.  The order is a function of (cell, id) only.  A tile with more
// than kRebuildCap particles ranks them from global memory instead (slow,
// exact).  Extra blocks past the tiles fold diagnostics partials, as the
// scan's do.
constexpr int kRebuildCap = 2048;        // tile particles ranked in LDS
constexpr int kRebuildMaxCells = 512;    // cells per tile (host: T <= this)
constexpr int kRebuildBlock = 1024;     // threads per block
// Up to this many tiles every tile's block runs at once (one per CU) and the
// launch is one dependent chain: members' values are then loaded early.  With
// more tiles the registers that takes cost a block per CU (measured on a
// 1M-particle workload) and the plain path runs.
constexpr int kRebuildLatencyTiles = 256;

int rebuild_tile_cells(int dim, const int nc[3], long n, bool var) {
  const int ncells = nc[0] * nc[1] * (dim == 3 ? nc[2] : 1);
  const double occ = ncells > 0 ? (double)n / ncells : 0.0;
  // room for 1.5 times the mean occupancy per cell, 3 times with per-particle
  // resolution (cells sized by the largest h hold several times the mean
  // where h is smallest)
  const double room = var ? 3.0 : 1.5;
  int t = occ > 0.0 ? (int)(kRebuildCap / (room * occ)) : kRebuildMaxCells;
  t = t < 1 ? 1 : (t > kRebuildMaxCells ? kRebuildMaxCells : t);
  return t < nc[0] ? t : nc[0];
}

int rebuild_tiles(int dim, const int nc[3], long n, bool var) {
  const int t = rebuild_tile_cells(dim, nc, n, var);
  const int per_row = (nc[0] + t - 1) / t;
  return per_row * nc[1] * (dim == 3 ? nc[2] : 1);
}

// LAT: the latency regime (see kRebuildLatencyTiles).  The other 2-D
// instance keeps to 64 VGPRs (eight waves per SIMD), so two of its blocks
// share a CU (the 3-D one would spill: its nine rows' run bounds live in
// registers).
template <int D, typename T, bool LAT>
__global__ __launch_bounds__(kRebuildBlock, (LAT || D == 3) ? 4 : 8) void rebuild_kernel(Grid g, RebuildArgs a,
                                                                            PArrays<T> stg,
                                                                            PArrays<T> dst) {
  constexpr int NB = kRebuildBlock;
  constexpr int NR = D == 3 ? 9 : 3;             // rows of cells around the tile's row
  constexpr int NP = 2 * NR;                     // runs: one or two per row (x seam)
  __shared__ int s_off[kRebuildMaxCells + 1];   // counts, then exclusive offsets
  __shared__ int s_cur[kRebuildMaxCells];
  __shared__ int s_j[kRebuildCap];              // member: previous index
  __shared__ int s_c[kRebuildCap];              // member: cell within the tile
  __shared__ int s_id[kRebuildCap];             // member: particle id
  __shared__ int s_bucket[kRebuildCap];         // members grouped by cell
  __shared__ int s_bid[kRebuildCap];            // ids in grouped order
  __shared__ int s_order[kRebuildCap];          // previous index by destination
  __shared__ int s_ocell[kRebuildCap];          // new cell by destination
  __shared__ int s_pa[NP], s_pstart[NP + 1];
  __shared__ int s_nmem, s_prefix;
  __shared__ int s_red[NB / kWave];
  __shared__ double s_fold[kBlock / kWave];
  const int tid = threadIdx.x;
  const int lane = tid % kWave;
  if (a.fold.partials && (int)blockIdx.x >= a.ntiles) {
    // one diagnostics column, by the first kBlock threads in the order of
    // fold_diag_column (so the row equals a diag_fold_kernel fold bit for bit)
    const int col = blockIdx.x - a.ntiles;
    const bool mx = col == 4 || col == 8;
    const double* c = a.fold.partials + (size_t)col * a.fold.nrows;
    double v = 0.0;
    if (tid < kBlock)
      v = mx ? wave_max(fold_rows<true>(c, a.fold.nrows)) : wave_sum(fold_rows<false>(c, a.fold.nrows));
    if (tid < kBlock && lane == 0) s_fold[tid / kWave] = v;
    __syncthreads();
    if (tid == 0) {
      double r = s_fold[0];
      for (int w = 1; w < kBlock / kWave; ++w) r = mx ? (r > s_fold[w] ? r : s_fold[w]) : r + s_fold[w];
      a.fold.diag[col] = r;
    }
    return;
  }
  const int n = g.n;
  const int nx = g.nc[0], ny = g.nc[1], nz = D == 3 ? g.nc[2] : 1;
  // tile = block index: blocks start in index order on each XCD, so every
  // tile a block waits on belongs to a block that started before it and
  // publishes its total without waiting (and the wait is bounded anyway)
  const int tile = blockIdx.x;
  const int row = tile / a.tiles_per_row;
  const int x0 = (tile - row * a.tiles_per_row) * a.tile_cells;
  const int tc = min(a.tile_cells, nx - x0);
  const int tile0 = row * nx + x0;
  const int y = row % ny, z = row / ny;
  if (tid == 0) s_nmem = 0;
  // the runs of the previous order that hold the tile's particles: for each
  // row of cells next to the tile's, the cells [x0 - 1, x0 + tc] (the whole
  // row when that covers it), one or two runs across the x seam; clamped into
  // [0, n], so a cell_start that does not describe the previous order can
  // lose particles (flagged below) but not fault
  if (tid < NR) {
    const int dy = tid % 3 - 1, dz = D == 3 ? tid / 3 - 1 : 0;
    const int base = (wrap_index(y + dy, ny) + ny * wrap_index(z + dz, nz)) * nx;
    int pa0, pb0, pa1 = 0, pb1 = 0;
    if (tc + 2 >= nx) {
      pa0 = a.cs_old[base];
      pb0 = a.cs_old[base + nx];
    } else {
      const int xs = x0 - 1, xe = x0 + tc + 1;   // [xs, xe), may cross the x seam once
      if (xs < 0) {
        pa0 = a.cs_old[base + nx - 1];
        pb0 = a.cs_old[base + nx];
        pa1 = a.cs_old[base];
        pb1 = a.cs_old[base + xe];
      } else if (xe > nx) {
        pa0 = a.cs_old[base + xs];
        pb0 = a.cs_old[base + nx];
        pa1 = a.cs_old[base];
        pb1 = a.cs_old[base + xe - nx];
      } else {
        pa0 = a.cs_old[base + xs];
        pb0 = a.cs_old[base + xe];
      }
    }
    pa0 = min(max(pa0, 0), n);
    pb0 = min(max(pb0, pa0), n);
    pa1 = min(max(pa1, 0), n);
    pb1 = min(max(pb1, pa1), n);
    s_pa[2 * tid] = pa0;
    s_pa[2 * tid + 1] = pa1;
    s_pstart[2 * tid + 1] = pb0 - pa0;     // lengths for now
    s_pstart[2 * tid + 2] = pb1 - pa1;
  }
  for (int c = tid; c < tc; c += NB) s_off[c] = 0;
  __syncthreads();
  // run starts in the concatenated index range, held in registers: a
  // candidate's run is found by compares, not by LDS reads
  int pst[NP + 1], ppa[NP];
  pst[0] = 0;
#pragma unroll
  for (int r = 0; r < NP; ++r) {
    pst[r + 1] = pst[r] + s_pstart[r + 1];
    ppa[r] = s_pa[r];
  }
  const int total = pst[NP];
  // pass A: the tile's particles among the candidates, U per thread with
  // their loads issued together; the wavefront's members of a batch take
  // consecutive member slots (one LDS atomic per wavefront and batch).  When
  // every candidate fits one batch, each member's values are loaded here
  // too, into registers, and stored from here once its rank is known: the
  // loads overlap the count, the look-back and the ranking.  2-D only: the
  // 3-D stencil's nine rows of candidates seldom fit one batch.
  constexpr int U = 4;
  const bool early = D == 2 && LAT && total <= U * NB;
  constexpr int UE = D == 2 && LAT ? U : 1;      // early-path registers
  int mslot[U], cq_keep[UE], iq_keep[UE], qq_keep[UE];
  T mo[UE][D], mv[UE][D], mms[UE], mhs[UE], mrs[UE];
#pragma unroll
  for (int u = 0; u < U; ++u) mslot[u] = -1;     // no candidates: no members
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int b0 = 0; b0 < total; b0 += U * NB) {
    int cq[U], iq[U], qq[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int f = min(b0 + u * NB + tid, total - 1);
      int q = ppa[0] + f;
#pragma unroll
      for (int r = 1; r < NP; ++r) q = f >= pst[r] ? ppa[r] + (f - pst[r]) : q;
      qq[u] = q;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      cq[u] = stg.cell[qq[u]];
      iq[u] = stg.id[qq[u]];
    }
    unsigned long long mm[U];
    int wave_total = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int lc = cq[u] - tile0;
      const bool mem = b0 + u * NB + tid < total && lc >= 0 && lc < tc;
      mm[u] = __ballot(mem);
      wave_total += __popcll(mm[u]);
      if (mem) atomicAdd(&s_off[lc], 1);
    }
    int base = 0;
    if (lane == 0 && wave_total > 0) base = atomicAdd(&s_nmem, wave_total);
    base = __shfl(base, 0, kWave);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      mslot[u] = -1;
      if ((mm[u] >> lane) & 1ull) {
        const int m = base + __popcll(mm[u] & below);
        if (m < kRebuildCap) {
          s_j[m] = qq[u];
          s_c[m] = cq[u] - tile0;
          s_id[m] = iq[u];
          mslot[u] = m;
        }
      }
      base += __popcll(mm[u]);
    }
    if constexpr (UE == U) {
      if (early) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        cq_keep[u] = cq[u];
        iq_keep[u] = iq[u];
        qq_keep[u] = qq[u];
        if (mslot[u] < 0) continue;
        const int j = qq[u];
#pragma unroll
        for (int d = 0; d < D; ++d) {
          mo[u][d] = stg.off[d * n + j];
          mv[u][d] = dst.vel ? stg.vel[d * n + j] : T(0);
        }
        mms[u] = dst.mass ? stg.mass[j] : T(0);
        mhs[u] = dst.h ? stg.h[j] : T(0);
        mrs[u] = dst.rho ? stg.rho[j] : T(0);
      }
      }
    }
  }
  __syncthreads();
  const int nmem = s_nmem;
  // publish the tile's total at once, so later tiles can use it
  if (tid == 0)
    __hip_atomic_store(&a.st.tile_state[tile],
                       tile_word(tile == 0 ? kTileInc : kTileAgg, a.epoch, (unsigned)nmem),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // exclusive scan of the per-cell counts, one cell per thread
  {
    static_assert(kRebuildMaxCells <= NB, "one cell per thread");
    const int v = tid < tc ? s_off[tid] : 0;
    int tot;
    const int run = block_exclusive_scan<NB>(v, s_red, &tot);
    if (tid < tc) {
      s_off[tid] = run;
      s_cur[tid] = run;
    }
    if (tid == 0) s_off[tc] = tot;
  }
  __syncthreads();   // the offsets, for the grouping below
  // the particles of all earlier tiles: the first wavefront reads the tile
  // words of up to 256 earlier tiles at once, nearest first, and adds the
  // totals up to the nearest one that carries its inclusive prefix; tiles
  // before the first tile read as inclusive zeros.  Meanwhile the other
  // wavefronts group the members by cell (their ids beside them).
  if (tid >= kWave) {
    if (nmem <= kRebuildCap) {
      for (int m = tid - kWave; m < nmem; m += NB - kWave) {
        const int pos = atomicAdd(&s_cur[s_c[m]], 1);
        s_bucket[pos] = m;
        s_bid[pos] = s_id[m];
      }
    }
  } else {
    const unsigned ep = a.epoch & 0x3fffffffu;
    constexpr int NG = 4;           // groups of 64 tile words per round trip
    int prefix = 0;
    int p = tile - 1;
    long spins = 0;
    int ng = NG;                    // groups read: one while waiting on the nearest
    while (p >= 0) {
      unsigned long long w[NG];
#pragma unroll
      for (int u = 0; u < NG; ++u) {
        const int idx = p - lane - u * kWave;
        w[u] = u >= ng ? 0ull
               : idx >= 0 ? __hip_atomic_load(&a.st.tile_state[idx], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT)
                          : tile_word(kTileInc, a.epoch, 0u);
      }
      // groups nearest first: a complete group adds its totals; one holding
      // an inclusive prefix ends the look-back; one not ready ends the pass
      int v = 0, done = 0;
      bool found = false;
#pragma unroll
      for (int u = 0; u < NG; ++u) {
        if (found || done < u) continue;
        const unsigned long long f = w[u] & kTileFlags;
        const bool ready = f != 0 && (unsigned)((w[u] >> 32) & 0x3fffffffull) == ep;
        const unsigned long long incm = __ballot(ready && f == kTileInc);
        const unsigned long long notr = __ballot(!ready);
        const int lim = incm ? __ffsll((long long)incm) - 1 : kWave - 1;
        const unsigned long long need = lim == kWave - 1 ? ~0ull : ((2ull << lim) - 1);
        if (notr & need) continue;
        v += lane <= lim ? (int)(w[u] & 0xffffffffull) : 0;
        done = u + 1;
        found = incm != 0;
      }
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) v += __shfl_xor(v, o, kWave);
      prefix += v;
      if (found) break;
      if (done == 0) {
        if (++spins > kSpinLimit) {
          if (lane == 0) atomicOr(a.flags, kFlagInternal);
          break;
        }
        ng = 1;
        continue;
      }
      p -= done * kWave;
      ng = NG;
    }
    if (lane == 0) {
      if (tile > 0)
        __hip_atomic_store(&a.st.tile_state[tile],
                           tile_word(kTileInc, a.epoch, (unsigned)(prefix + nmem)),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_prefix = prefix;
    }
  }
  __syncthreads();
  const int prefix = s_prefix;
  auto put = [&](auto* ptr, auto v) { *ptr = v; };
  for (int c = tid; c < tc; c += NB) put(a.cs_new + (tile0 + c), prefix + s_off[c]);
  if (tile == a.ntiles - 1 && tid == 0) {
    a.cs_new[a.ncells] = prefix + nmem;
    if (prefix + nmem != n) atomicOr(a.flags, kFlagInternal);   // not a one-cell move
  }
  auto move = [&](int j, int to, int c) {
    if (to >= n) return;
    dst.cell[to] = c;
    dst.id[to] = stg.id[j];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      dst.off[d * n + to] = stg.off[d * n + j];
      if (dst.vel) dst.vel[d * n + to] = stg.vel[d * n + j];
    }
    if (dst.mass) dst.mass[to] = stg.mass[j];
    if (dst.h) dst.h[to] = stg.h[j];
    if (dst.rho) dst.rho[to] = stg.rho[j];
    if (a.perm) a.perm[to] = j;
  };
  if (nmem <= kRebuildCap) {
    // rank each member by id within its cell (grouped above), then move them
    // in destination order (consecutive threads, consecutive slots)
    for (int p = tid; p < nmem; p += NB) {
      const int m = s_bucket[p];
      const int lc = s_c[m], idm = s_bid[p];
      const int b = s_off[lc], e = s_off[lc + 1];
      // ties (equal ids, never in a valid state) by grouping position, so the
      // ranks are always a permutation of [b, e); eight ids read at a time
      int rank = 0;
      for (int r0 = b; r0 < e; r0 += 8) {
        int idr[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) idr[u] = s_bid[min(r0 + u, e - 1)];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int r = r0 + u;
          rank += (r < e && (idr[u] < idm || (idr[u] == idm && r < p))) ? 1 : 0;
        }
      }
      if (early) {
        s_order[m] = b + rank;          // member -> slot within the tile
      } else {
        s_order[b + rank] = s_j[m];
        s_ocell[b + rank] = tile0 + lc;
      }
    }
    __syncthreads();
    if constexpr (UE == U) {
      if (early) {
      // each member from the registers that pass A loaded it into
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (mslot[u] < 0) continue;
        const int to = prefix + s_order[mslot[u]];
        if (to >= n) continue;
        put(dst.cell + to, cq_keep[u]);
        put(dst.id + to, iq_keep[u]);
#pragma unroll
        for (int d = 0; d < D; ++d) {
          put(dst.off + (d * n + to), mo[u][d]);
          if (dst.vel) put(dst.vel + (d * n + to), mv[u][d]);
        }
        if (dst.mass) put(dst.mass + to, mms[u]);
        if (dst.h) put(dst.h + to, mhs[u]);
        if (dst.rho) put(dst.rho + to, mrs[u]);
        if (a.perm) put(a.perm + to, qq_keep[u]);
      }
      return;
      }
    }
    // two particles per thread at a time, every load issued before the stores
    for (int u0 = tid; u0 < nmem; u0 += 2 * NB) {
      int jj[2], cc[2], ii[2];
      T oo[2][D], vv[2][D], ms[2], hs[2], rs[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int uu = min(u0 + u * NB, nmem - 1);
        jj[u] = s_order[uu];
        cc[u] = s_ocell[uu];
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int j = jj[u];
        ii[u] = stg.id[j];
#pragma unroll
        for (int d = 0; d < D; ++d) {
          oo[u][d] = stg.off[d * n + j];
          vv[u][d] = dst.vel ? stg.vel[d * n + j] : T(0);
        }
        ms[u] = dst.mass ? stg.mass[j] : T(0);
        hs[u] = dst.h ? stg.h[j] : T(0);
        rs[u] = dst.rho ? stg.rho[j] : T(0);
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int to = prefix + u0 + u * NB;
        if (u0 + u * NB >= nmem || to >= n) continue;
        put(dst.cell + to, cc[u]);
        put(dst.id + to, ii[u]);
#pragma unroll
        for (int d = 0; d < D; ++d) {
          put(dst.off + (d * n + to), oo[u][d]);
          if (dst.vel) put(dst.vel + (d * n + to), vv[u][d]);
        }
        if (dst.mass) put(dst.mass + to, ms[u]);
        if (dst.h) put(dst.h + to, hs[u]);
        if (dst.rho) put(dst.rho + to, rs[u]);
        if (a.perm) put(a.perm + to, jj[u]);
      }
    }
  } else {
    // too many for LDS: rank each member by id among the particles of its
    // new cell, found in the previous occupants of the cells around it
    for (int f = tid; f < total; f += NB) {
      int q = ppa[0] + f;
#pragma unroll
      for (int r = 1; r < NP; ++r) q = f >= pst[r] ? ppa[r] + (f - pst[r]) : q;
      const int c = stg.cell[q];
      const int lc = c - tile0;
      if (lc < 0 || lc >= tc) continue;
      const int idq = stg.id[q];
      int cc[3];
      decode_cell<D>(g, c, cc);
      int rank = 0;
      for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            const int oc = wrap_index(cc[0] + dx, nx) +
                           nx * (wrap_index(cc[1] + dy, ny) + ny * wrap_index(cc[2] + dz, nz));
            const int rb = min(max(a.cs_old[oc], 0), n);
            const int re = min(max(a.cs_old[oc + 1], rb), n);
            for (int r = rb; r < re; ++r) {
              const int idr = stg.id[r];
              rank += (stg.cell[r] == c && (idr < idq || (idr == idq && r < q))) ? 1 : 0;
            }
          }
      move(q, prefix + s_off[lc] + rank, c);
    }
  }
}

template <typename T>
void launch_rebuild(const Launch& l, const Grid& g, const RebuildArgs& a, const PArrays<T>& stg,
                    const PArrays<T>& dst) {
  if (g.n == 0) return;
  const bool lat = a.ntiles <= kRebuildLatencyTiles;
  const int nb = a.ntiles + (a.fold.partials ? kNumPartials : 0);
#define SPH_REBUILD(D, LAT)                                                                   \
  hipLaunchKernelGGL((rebuild_kernel<D, T, LAT>), dim3(nb), dim3(kRebuildBlock), 0, l.stream, g, \
                     a, stg, dst)
  if (l.dim == 2) {
    if (lat) SPH_REBUILD(2, true);
    else SPH_REBUILD(2, false);
  } else {
    if (lat) SPH_REBUILD(3, true);
    else SPH_REBUILD(3, false);
  }
#undef SPH_REBUILD
}

#define SPH_INST(T)                                                                          \
  template void launch_rebuild<T>(const Launch&, const Grid&, const RebuildArgs&,            \
                                  const PArrays<T>&, const PArrays<T>&);                     \
  template void launch_bin<T>(const Launch&, const Grid&, const Coeffs<T>&, const double*,   \
                              int*, T*, unsigned*);                                          \
  template void launch_rank_gather<T>(const Launch&, int, SortTmp, const PArrays<T>&,        \
                                      const PArrays<T>&, int*);
SPH_INST(float)
SPH_INST(double)
#undef SPH_INST

}  // namespace sph
