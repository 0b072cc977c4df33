// Launchers shared between the libsph translation units (not part of the ABI).
#pragma once

#include "sph_dev.hpp"

namespace sph {

// Device flag bits (mirrors include/sph.h)
constexpr unsigned kFlagNonfinite = 1u;
constexpr unsigned kFlagCfl = 2u;
constexpr unsigned kFlagOutOfBox = 4u;
constexpr unsigned kFlagInternal = 8u;

struct Launch {
  int dim;
  bool var;            // per-particle mass and h present
  hipStream_t stream;
  int G;               // lanes per particle in the neighbour sweeps (1, 2 or 4)
  int nblk;            // blocks of the sweeps and of every kernel writing
                       // diagnostic partials: ceil(n * G / kBlock)
};

// Lanes per particle for the neighbour sweeps (2, 4 or 8).  A group of lanes
// shares one particle's candidate cells, which puts more wavefronts in flight
// and splits the serial candidate walk; the price is the group reduction and
// an epilogue run by one lane in G.  The largest G whose n * G lanes fit a
// budget (2^18 in 2-D, 2^19 in 3-D: the 3-D walk is ~8x longer), at least 2
// in 2-D and 4 in 3-D.  Measured on gfx950 (FP32 step, us): 2-D 2.5k
// particles 39.9 / 33.7 / 28.9 for G = 2 / 4 / 8, 40k 46.3 / 39.8 / 42.1,
// 160k 66.1 / 79.7 / 114.8; 3-D 4k 420 / 119 / 86, 33k 310 / 136 / 120,
// 262k 883 / 510 / 609.
inline int lanes_per_particle(int dim, long n) {
  const long budget = dim == 3 ? (1L << 19) : (1L << 18);
  const int gmin = dim == 3 ? 4 : 2;
  for (int g = 8; g > gmin; g /= 2)
    if (n * g <= budget) return g;
  return gmin;
}

inline int blocks_for(long n) { return (int)((n + kBlock - 1) / kBlock); }

// Particle arrays in the sweep precision T.
template <typename T>
struct PArrays {
  int* cell;
  int* id;
  T* off;
  T* vel;
  T* acc;
  T* rho;
  T* mass;   // null for uniform
  T* h;      // null for uniform
};

// Outputs of the fused force sweep inside a multi-step run: the next step's
// moved particles (staging, old order = this step's order), their cell slots,
// and the per-block diagnostic partials of this step (kinetic energy,
// momentum, max |v|) and of the next step (limiter counts, max |dr|/dt).
template <typename T>
struct FusedOut {
  int apply_next;      // correction applied at the next step
  PArrays<T> stg;
  int* counts;         // zeroed histogram for the next cell build (null: no slot claims)
  int* slot;
  double* part_cur;    // null: no diagnostics of this step
  double* part_next;   // null: none of the next step's correction
  T* g_next;           // null: no tape; else the next step's correction sum g [D][N]
  T* beta_next;        // and limiter value [N] (written when apply_next)
  // when set: the velocity after this step's second half kick into
  // kick_vel [D][N] (not the swept velocities: other blocks still read them)
  T* kick_vel = nullptr;
  // when set: clear[0, clear_n) zeroed on the side (the cell build's tile words)
  int* clear = nullptr;
  long clear_n = 0;
};

// ---- sweeps (sweeps.hip)
// with sl.entry set, also records every lane's neighbours for the force sweep
template <typename T>
void launch_density(const Launch& l, const Grid& g, const Coeffs<T>& k, const PArrays<T>& p,
                    const int* cs, T* rho_out, double* partials, int* counts, unsigned* flags,
                    const StoredList& sl = StoredList{});
// A correction sweep that also does the step's first half kick and drift
// (the drift sweep's arithmetic, with the correction just computed): every
// particle of src moved into stg; and clears clear[0, clear_n) on the side.
template <typename T>
struct TvDrift {
  PArrays<T> src;
  PArrays<T> stg;     // stg.off null: no drift
  unsigned* flags;
  int* clear;
  long clear_n;
};
template <typename T>
void launch_tv(const Launch& l, const Grid& g, const Coeffs<T>& k, const PArrays<T>& p,
               const int* cs, T* dr, T* beta, double* s_out, T* g_out, double* partials,
               const TvDrift<T>& td = TvDrift<T>{});
// with sl.entry set, over the stored lists of the density sweep just before
template <typename T>
void launch_forces(const Launch& l, const Grid& g, const Coeffs<T>& k, const PArrays<T>& p,
                   const int* cs, const T* vel, T* acc_out, unsigned* flags,
                   const StoredList& sl = StoredList{});
// with sl.entry set, over the stored lists of the density sweep just before
template <typename T>
void launch_forces_fused(const Launch& l, const Grid& g, const Coeffs<T>& k, const PArrays<T>& p,
                         const int* cs, const FusedOut<T>& fo, unsigned* flags,
                         const StoredList& sl = StoredList{});
// wall particles' density and mirror velocity from their fluid neighbours
// (p.rho, p.vel of walls written; wall_vel [D][n_wall] by id - nfluid); with
// wsum_out / wavg_out ([n_wall], [D][n_wall] by id - nfluid) also the kernel
// sum S_a and the averaged fluid velocity the adjoint needs
template <typename T>
void launch_wall_state(const Launch& l, const Grid& g, const Coeffs<T>& k, const PArrays<T>& p,
                       const int* cs, const T* wall_vel, int n_wall, T* wsum_out, T* wavg_out);

// ---- dual-criteria time stepping (dual.hip)
// One clock slot per acoustic substep of an advection step: the substep's
// start time and the largest speed at its start (bits of a non-negative
// double, gathered with integer atomic maxima).
struct DualSlot {
  double t;
  unsigned long long vmax_bits;
};
struct DualCoeffs {
  double cfl_ad, cfl_ac, u_ref, nu, h_min, c0;
  int K;        // substep launches per advection step (even, <= kMaxDualSubsteps)
  int cap;      // substeps allowed to run (K when not capped)
  int capped;   // 1: the caller capped the substeps (an uncovered step is not an error)
};
constexpr int kMaxDualSubsteps = 64;
template <typename T>
void launch_dual_start(hipStream_t s, int n, int dim, const T* vel, DualSlot* clk);
template <typename T>
void launch_dual_prologue(const Launch& l, const Grid& g, const Coeffs<T>& k, const DualCoeffs& q,
                          const PArrays<T>& p, const int* cs, T* visc, T* delta, T* drho,
                          const DualSlot* clk, DualSlot* clk_next, double* partials,
                          unsigned* flags);
template <typename T>
void launch_dual_pressure(const Launch& l, const Grid& g, const Coeffs<T>& k,
                          const DualCoeffs& q, int sk, const PArrays<T>& p, const int* cs,
                          const T* vel, const T* rho, const T* drho, const T* visc, T* vel_out,
                          T* delta, DualSlot* clk, unsigned* flags);
template <typename T>
void launch_dual_continuity(const Launch& l, const Grid& g, const Coeffs<T>& k,
                            const DualCoeffs& q, int sk, const PArrays<T>& p, const int* cs,
                            const T* vel, const T* rho, const T* drho, T* rho_out, T* drho_out,
                            DualSlot* clk, unsigned* flags);
template <typename T>
void launch_dual_move(const Launch& l, const Grid& g, const Coeffs<T>& k, const DualCoeffs& q,
                      const PArrays<T>& p, const T* delta, const PArrays<T>& stg, int* counts,
                      int* slot, const DualSlot* clk, DualSlot* clk_next, double* partials,
                      double* record, unsigned* flags);

// ---- cells (cells.hip)
template <typename T>
void launch_bin(const Launch& l, const Grid& g, const Coeffs<T>& k, const double* pos,
                int* cell, T* off, unsigned* flags);
void launch_fill(hipStream_t s, int* p, long n, int v);
// exclusive scan of counts[ncells] into cs[ncells + 1], leaving counts zeroed
// for the next histogram.  The look-back state (scan_blocks(ncells) tile words
// and a ticket counter) is zeroed once; scan number k (k = 0, 1, ...) after
// that zeroing passes epoch k.  With `fold` set, block 0 also folds a
// previous launch's diagnostic partials into a diagnostics row.
int scan_blocks(int ncells);
struct ScanState {
  unsigned long long* tile_state;
  unsigned* tickets;
};
struct DiagFold {
  const double* partials;   // null: nothing to fold
  int nrows;                // partial rows: blocks * waves per block
  double* diag;
};
void launch_scan(hipStream_t s, int ncells, int* counts, ScanState st, unsigned epoch, int* cs,
                 unsigned* flags, DiagFold fold);
void launch_diag_fold(hipStream_t s, DiagFold fold);
// The fold (when fold.partials is set) and a copy of `bytes` (a multiple of
// 4) from src to dst, in one launch.
void launch_fold_copy(hipStream_t s, DiagFold fold, const void* src, void* dst, size_t bytes);
// Sorting scratch: per destination slot, the source index, the particle id
// and the cell's [start, end).
struct SortTmp {
  int* src;
  int* id;
  int2* range;
};
void launch_scatter(hipStream_t s, int n, const int* cell, const int* id, const int* slot,
                    const int* cs, SortTmp tmp);
// Moves staged arrays (old order) into dst arrays (new order); null pointers skip.
template <typename T>
void launch_rank_gather(const Launch& l, int n, SortTmp tmp, const PArrays<T>& stg,
                        const PArrays<T>& dst, int* perm);

// One-launch cell build after a drift of at most one cell per axis (cells.hip:
// rebuild_kernel): from the staging arrays in the previous (cell, id) order
// with its cell starts cs_old into dst in the new order, cs_new, and perm
// (optional: perm[new index] = previous index).  Tiles of tile_cells cells of
// one x-row, ntiles of them (block b takes tile b), look-back words in
// st.tile_state tagged with epoch `epoch` (as launch_scan); fold as launch_scan.
struct RebuildArgs {
  int ncells, ntiles, tile_cells, tiles_per_row;
  const int* cs_old;
  int* cs_new;
  ScanState st;
  unsigned epoch;
  int* perm;
  unsigned* flags;
  DiagFold fold;
};
int rebuild_tile_cells(int dim, const int nc[3], long n, bool var);
int rebuild_tiles(int dim, const int nc[3], long n, bool var);
template <typename T>
void launch_rebuild(const Launch& l, const Grid& g, const RebuildArgs& a, const PArrays<T>& stg,
                    const PArrays<T>& dst);

// ---- integration (kdk.hip)
// Device-to-device copies of 4-byte words, up to kMaxCopies in one launch
// (tape records).
constexpr int kMaxCopies = 24;
struct CopyBatch {
  int count;
  const char* src[kMaxCopies];
  char* dst[kMaxCopies];
  long bytes[kMaxCopies];
  bool add(void* d, const void* s, size_t nbytes) {
    if (nbytes == 0) return true;
    if (count >= kMaxCopies || (nbytes & 3u)) return false;
    src[count] = (const char*)s;
    dst[count] = (char*)d;
    bytes[count] = (long)nbytes;
    ++count;
    return true;
  }
};
void launch_multi_copy(hipStream_t s, const CopyBatch& b);
template <typename T>
void launch_stage_copy(const Launch& l, int n, const PArrays<T>& src, const PArrays<T>& stg,
                       int* counts, int* slot);
template <typename T>
void launch_drift(const Launch& l, const Grid& g, const Coeffs<T>& k, const PArrays<T>& p,
                  const T* dr, const PArrays<T>& stg, int* counts, int* slot, unsigned* flags);
// v += dt/2 a (when `write`); with partials, writes this step's kinetic
// energy, momentum and max |v| partials (columns 0-4).  Wall particles (by
// id) are neither kicked nor counted.
template <typename T>
void launch_kick(const Launch& l, const Coeffs<T>& k, int n, T* vel, const T* acc,
                 const T* mass, const int* id, double* partials, bool write, unsigned* flags);
void launch_zero_partials(hipStream_t s, int nblk, double* partials);
template <typename T>
void launch_zero(hipStream_t s, T* p, long n);

// ---- adjoint (adjoint.hip)
// with sl.entry set, over stored lists recorded at the same state
template <typename T>
void launch_force_vjp(const Launch& l, const Grid& g, const Coeffs<T>& k, const PArrays<T>& p,
                      const int* cs, const T* vel, const T* a_bar, T* r_bar, T* v_bar, T* rho_bar,
                      const StoredList& sl = StoredList{});
template <typename T>
void launch_density_vjp(const Launch& l, const Grid& g, const Coeffs<T>& k, const PArrays<T>& p,
                        const int* cs, const T* rho_bar, T* r_bar, T* v_bar, T vcoef,
                        const StoredList& sl = StoredList{});
// What the correction's VJP also does for the reverse step, per particle in
// order n: the reverse of the first half kick (v_bar = vh_bar, a_bar =
// dt/2 vh_bar for fluid particles, 0 for walls told by id; skipped when v_bar
// is null), and, in one extra block, the fold of the xi partials of
// launch_unpermute_ghat into xi_bar (skipped when xi_bar is null).
template <typename T>
struct AdjFinish {
  const int* id;
  const T* vh_bar;
  T* v_bar;
  T* a_bar;
  const double* xi_partials;
  int xi_rows;
  double* xi_bar;
};
template <typename T>
void launch_tv_vjp(const Launch& l, const Grid& g, const Coeffs<T>& k, const PArrays<T>& p,
                   const int* cs, const T* ghat, const T* gsum, const T* beta, const T* r_in,
                   T* r_out, T* rho_out, const AdjFinish<T>& fin);
// r_n = r_bar and vh_n = v_bar taken back to order n through perm (new ->
// previous index), with the correction's ghat and its xi partials (one row
// per wavefront of a one-thread-per-particle grid)
template <typename T>
void launch_unpermute_ghat(const Launch& l, const Coeffs<T>& k, int n, const int* perm,
                           const T* r_bar, const T* v_bar, const T* gsum, const T* beta,
                           const T* rho, T* r_n, T* vh_n, T* ghat, double* partials);
template <typename T>
void launch_adj_kick(const Launch& l, const Coeffs<T>& k, int n, const int* id, const T* v_bar,
                     T* a_bar);
// reverse of the wall state: wall particles' velocity and density cotangents
// to their fluid neighbours (and position cotangents of both); wsum [N],
// wavg [D][N] and wall_cells [ncells] are scratch; the walls' v_bar and
// rho_bar are cleared
// wsum [n_wall] / wavg [D][n_wall] (by id - nfluid) hold the walls' kernel
// sums and averaged fluid velocities when sums_given (recorded by the forward
// wall state), else they are computed into them first
template <typename T>
void launch_wall_vjp(const Launch& l, const Grid& g, const Coeffs<T>& k, const PArrays<T>& p,
                     const int* cs, const T* vel, T* wsum, T* wavg, int n_wall, bool sums_given,
                     int* wall_cells, T* r_bar, T* v_bar, T* rho_bar,
                     const StoredList& sl = StoredList{});
// x[c][i] = 0 (c < ncomp) and, when given, y[i] = 0 for every wall particle i
// (told by id)
template <typename T>
void launch_zero_walls(const Launch& l, const Coeffs<T>& k, int n, const int* id, int ncomp,
                       T* x, T* y);

// Launches a sweep kernel template KERNEL<D, T, VAR, G> on a grid of
// n * G threads (G lanes per particle), dispatching on dimension, per-particle
// mass/h and G; needs `l` (Launch) and the type T in scope.
#define SPH_SWEEP_G(KERNEL, DD, VV, ...)                                                     \
  do {                                                                                        \
    if (l.G == 4)                                                                             \
      hipLaunchKernelGGL((KERNEL<DD, T, VV, 4>), grid_, block_, 0, l.stream, __VA_ARGS__);    \
    else if (l.G == 2)                                                                        \
      hipLaunchKernelGGL((KERNEL<DD, T, VV, 2>), grid_, block_, 0, l.stream, __VA_ARGS__);    \
    else                                                                                      \
      hipLaunchKernelGGL((KERNEL<DD, T, VV, 8>), grid_, block_, 0, l.stream, __VA_ARGS__);    \
  } while (0)
#define SPH_SWEEP(KERNEL, ARGS)                                                               \
  do {                                                                                        \
    const dim3 grid_(l.nblk), block_(kBlock);                                                 \
    if (l.dim == 2) {                                                                         \
      if (l.var) SPH_SWEEP_G(KERNEL, 2, true, ARGS);                                          \
      else SPH_SWEEP_G(KERNEL, 2, false, ARGS);                                               \
    } else {                                                                                  \
      if (l.var) SPH_SWEEP_G(KERNEL, 3, true, ARGS);                                          \
      else SPH_SWEEP_G(KERNEL, 3, false, ARGS);                                               \
    }                                                                                         \
  } while (0)
#define SPH_ARGS(...) __VA_ARGS__

}  // namespace sph
