// libsph C-ABI: argument checks, workspace and tape layout, and the order of
// kernel launches for each entry point.  Declarations and the contract of
// every function are in include/sph.h.
#include <cmath>
#include <cstring>
#include <mutex>

#include "sph.h"
#include "sph_internal.hpp"

namespace sph {
namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Sizes {
  int dim, n, ncells, nblk, nwall, G;
  size_t tsz;     // bytes per float element
  bool var;
};

// Workspace regions (byte offsets from the workspace base).
struct WsLayout {
  size_t flags, cellbuf, slot, tmp, tmp_id, tmp_range, perm;
  size_t stg_cell, stg_id, stg_off, stg_vel, stg_acc, stg_rho, stg_mass, stg_h;
  size_t dr, partials, partials2;
  size_t adj_r, adj_v, adj_rho, adj_g, adj_r2;
  size_t wall_cells;   // cells holding a wall particle (reverse of the wall state)
  size_t cs2;          // second cell_start of a run (the rebuild reads one, writes the other)
  size_t dual_clock;   // two clocks of the dual-criteria steps
  size_t base_total;   // every region above: the least a run can work with
  size_t nlist, ncount;   // stored neighbour lists of a run (0 bytes when not usable)
  size_t nruns;           // the density sweep's stage runs per block (2-D lists)
  size_t total;
};

// Whether the stored neighbour lists can index every particle (list_jbits),
// and their rows stay within 2^31 bytes.
bool lists_usable(const Sizes& s) {
  const long lanes = (long)(s.nblk > 0 ? s.nblk : 1) * kBlock;
  return (long)s.n < (1L << (s.dim == 3 ? 27 : 28)) &&
         lanes * list_cap(s.dim, s.G) * (long)sizeof(unsigned) < (1L << 31);
}

// One step's tape: the sorted state before the step (order n), the raw
// correction sum and limiter value at step n, the permutation from order
// n+1 to order n, and the sorted state after the forces (order n+1, with the
// half-step velocity).
struct TapeLayout {
  size_t pre_cell, pre_off, pre_rho, pre_mass, pre_h, pre_cs, g, beta, perm;
  size_t post_cell, post_off, post_vhalf, post_rho, post_mass, post_h, post_cs;
  size_t pre_id, post_id;   // particle ids (walled runs only: walls are told by id)
  size_t wsum, wavg;        // walls' kernel sums and averaged fluid velocity (walled runs)
  size_t total;
};

// One region holds everything the cell build and the diagnostics fold keep
// between launches, so a single fill zeroes it: counts[ncells], a spare word,
// the diagnostics ticket, two scan tickets, then 8-byte look-back tile states.
// The tile words serve the scan (scan_blocks tiles) or the one-launch rebuild
// (at most one tile per cell), never both in one run.
size_t cellbuf_head(int ncells) { return ((sizeof(int) * ((size_t)ncells + 4)) + 7) / 8 * 8; }
size_t cellbuf_bytes(int ncells) {
  const int words = scan_blocks(ncells) > ncells ? scan_blocks(ncells) : ncells;
  return cellbuf_head(ncells) + 8 * (size_t)words;
}

struct CellBuf {
  int* counts;
  unsigned* counter;
  ScanState scan;
  long fill_ints;
};

CellBuf cellbuf_of(char* ws, size_t off, int ncells) {
  CellBuf b;
  int* base = (int*)(ws + off);
  b.counts = base;
  b.counter = (unsigned*)(base + ncells + 1);
  b.scan.tickets = (unsigned*)(base + ncells + 2);
  b.scan.tile_state = (unsigned long long*)((char*)base + cellbuf_head(ncells));
  b.fill_ints = (long)(cellbuf_bytes(ncells) / sizeof(int));
  return b;
}

struct Cursor {
  size_t o = 0;
  size_t take(size_t bytes) {
    size_t r = o;
    o += align_up(bytes > 0 ? bytes : 1);
    return r;
  }
};

// lanes per particle of every sweep: params.lanes, or chosen by size (0)
int lanes_of(const sph_params* p) {
  return p->lanes != 0 ? p->lanes : lanes_per_particle(p->dim, (long)p->n);
}

Sizes sizes_of(const sph_params* p, bool var) {
  Sizes s;
  s.dim = p->dim;
  s.n = (int)p->n;
  s.ncells = p->ncell[0] * p->ncell[1] * (p->dim == 3 ? p->ncell[2] : 1);
  s.G = lanes_of(p);
  s.nblk = blocks_for((long)s.n * s.G);
  s.nwall = (int)p->n_wall;
  s.tsz = p->dtype == SPH_F64 ? 8 : 4;
  s.var = var;
  return s;
}

WsLayout ws_layout(const Sizes& s) {
  Cursor c;
  WsLayout w;
  const size_t n = (size_t)s.n, dn = (size_t)s.dim * n, t = s.tsz;
  w.flags = c.take(kAlign);
  // cell histogram, diagnostics ticket, scan tickets and look-back tile states
  w.cellbuf = c.take(cellbuf_bytes(s.ncells));
  w.slot = c.take(sizeof(int) * n);
  w.tmp = c.take(sizeof(int) * n);
  w.tmp_id = c.take(sizeof(int) * n);
  w.tmp_range = c.take(2 * sizeof(int) * n);
  w.perm = c.take(sizeof(int) * n);
  w.stg_cell = c.take(sizeof(int) * n);
  w.stg_id = c.take(sizeof(int) * n);
  w.stg_off = c.take(t * dn);
  w.stg_vel = c.take(t * dn);
  w.stg_acc = c.take(t * dn);
  w.stg_rho = c.take(t * n);
  w.stg_mass = c.take(t * n);
  w.stg_h = c.take(t * n);
  w.dr = c.take(t * dn);
  const size_t prow = (size_t)(s.nblk > 0 ? s.nblk : 1) * kWavesPerBlock;
  w.partials = c.take(sizeof(double) * kNumPartials * prow);
  w.partials2 = c.take(sizeof(double) * kNumPartials * prow);
  w.adj_r = c.take(t * dn);
  w.adj_v = c.take(t * dn);
  w.adj_rho = c.take(t * n);
  w.adj_g = c.take(t * dn);
  w.adj_r2 = c.take(t * dn);
  w.wall_cells = c.take(s.nwall > 0 ? sizeof(int) * (size_t)s.ncells : 0);
  w.dual_clock = c.take(2 * sizeof(DualSlot) * (kMaxDualSubsteps + 1));
  w.cs2 = c.take(sizeof(int) * ((size_t)s.ncells + 1));
  w.base_total = c.o;
  const size_t lanes = (size_t)(s.nblk > 0 ? s.nblk : 1) * kBlock;
  const bool lists = lists_usable(s);
  w.nlist = c.take(lists ? sizeof(unsigned) * lanes * list_cap(s.dim, s.G) : 0);
  w.ncount = c.take(lists ? sizeof(int) * lanes : 0);
  w.nruns = c.take(lists && s.dim == 2 ? sizeof(int) * 6 * (size_t)(s.nblk > 0 ? s.nblk : 1) : 0);
  w.total = c.o;
  return w;
}

// A caller's stored-list buffer (sph_list_size bytes): entries, counts, then
// (2-D) the density sweep's stage runs per block.
struct ListLayout {
  size_t entries, counts, runs, total;
};
ListLayout list_layout(const Sizes& s) {
  ListLayout ll{0, 0, 0, 0};
  if (!lists_usable(s)) return ll;
  Cursor c;
  const size_t lanes = (size_t)(s.nblk > 0 ? s.nblk : 1) * kBlock;
  ll.entries = c.take(sizeof(unsigned) * lanes * list_cap(s.dim, s.G));
  ll.counts = c.take(sizeof(int) * lanes);
  ll.runs = c.take(s.dim == 2 ? sizeof(int) * 6 * (size_t)(s.nblk > 0 ? s.nblk : 1) : 0);
  ll.total = c.o;
  return ll;
}

// The stored lists in a workspace (lists usable)
StoredList ws_lists(char* ws, const WsLayout& w, const Sizes& s) {
  return StoredList{(unsigned*)(ws + w.nlist), (int*)(ws + w.ncount), s.nblk * kBlock,
                    s.dim == 2 ? (int*)(ws + w.nruns) : nullptr};
}

TapeLayout tape_layout(const Sizes& s) {
  Cursor c;
  TapeLayout tl;
  const size_t n = (size_t)s.n, dn = (size_t)s.dim * n, t = s.tsz;
  const size_t cs = sizeof(int) * ((size_t)s.ncells + 1);
  tl.pre_cell = c.take(sizeof(int) * n);
  tl.pre_off = c.take(t * dn);
  tl.pre_rho = c.take(t * n);
  tl.pre_mass = c.take(s.var ? t * n : 0);
  tl.pre_h = c.take(s.var ? t * n : 0);
  tl.pre_cs = c.take(cs);
  tl.g = c.take(t * dn);
  tl.beta = c.take(t * n);
  tl.perm = c.take(sizeof(int) * n);
  tl.post_cell = c.take(sizeof(int) * n);
  tl.post_off = c.take(t * dn);
  tl.post_vhalf = c.take(t * dn);
  tl.post_rho = c.take(t * n);
  tl.post_mass = c.take(s.var ? t * n : 0);
  tl.post_h = c.take(s.var ? t * n : 0);
  tl.post_cs = c.take(cs);
  tl.pre_id = c.take(s.nwall > 0 ? sizeof(int) * n : 0);
  tl.post_id = c.take(s.nwall > 0 ? sizeof(int) * n : 0);
  tl.wsum = c.take(t * (size_t)s.nwall);
  tl.wavg = c.take(t * (size_t)s.dim * (size_t)s.nwall);
  tl.total = c.o;
  return tl;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

int32_t check_params(const sph_params* p) {
  if (!p) return SPH_E_ARG;
  if (p->dim != 2 && p->dim != 3) return SPH_E_UNSUPPORTED;
  if (p->dtype != SPH_F32 && p->dtype != SPH_F64) return SPH_E_UNSUPPORTED;
  if (p->n < 0) return SPH_E_ARG;
  // neighbour-list entries hold particle indices in 28 bits
  if (p->n >= (int64_t(1) << 28)) return SPH_E_UNSUPPORTED;
  if (p->tv_every < 0) return SPH_E_ARG;
  if (p->per_particle != 0 && p->per_particle != 1) return SPH_E_ARG;
  if (p->tv_mode != SPH_TV_LIMITED && p->tv_mode != SPH_TV_SCALED &&
      p->tv_mode != SPH_TV_BACKGROUND)
    return SPH_E_ARG;
  if (p->n_wall < 0 || p->n_wall > p->n) return SPH_E_ARG;
  // walls are built and tested for uniform resolution only
  if (p->n_wall > 0 && p->per_particle) return SPH_E_UNSUPPORTED;
  if (p->lanes != 0 && p->lanes != 2 && p->lanes != 4 && p->lanes != 8) return SPH_E_ARG;
  const double vals[] = {p->rho0, p->c0, p->h_min, p->h_max, p->kappa, p->mass};
  for (double v : vals)
    if (!std::isfinite(v)) return SPH_E_NONFINITE;
  const double maybe_zero[] = {p->eta, p->dt, p->xi, p->lim_c, p->lim_s0, p->riemann_eta,
                               p->band_tol};
  for (double v : maybe_zero)
    if (!std::isfinite(v)) return SPH_E_NONFINITE;
  if (!finite_pos(p->rho0) || !finite_pos(p->c0) || !finite_pos(p->h_min) ||
      !finite_pos(p->kappa) || !finite_pos(p->mass))
    return SPH_E_ARG;
  if (p->h_max < p->h_min || p->eta < 0.0 || p->dt < 0.0) return SPH_E_ARG;
  long ncells = 1;
  for (int k = 0; k < p->dim; ++k) {
    if (!finite_pos(p->box[k])) return SPH_E_ARG;
    if (p->ncell[k] < 3) return SPH_E_CELL_RANGE;
    const double L = p->box[k] / p->ncell[k];
    if (L < 2.0 * p->h_max * (1.0 - 1e-12)) return SPH_E_CELL_RANGE;
    ncells *= p->ncell[k];
  }
  // the cell scan handles up to 2048 * 2048 cells
  if (ncells > 2048L * 2048L) return SPH_E_UNSUPPORTED;
  return SPH_OK;
}

Grid grid_of(const sph_params* p) {
  Grid g;
  g.n = (int)p->n;
  for (int k = 0; k < 3; ++k) {
    const bool used = k < p->dim;
    g.nc[k] = used ? p->ncell[k] : 1;
    g.box[k] = used ? p->box[k] : 1.0;
    g.L[k] = used ? p->box[k] / p->ncell[k] : 1.0;
  }
  g.ncells = g.nc[0] * g.nc[1] * g.nc[2];
  return g;
}

template <typename T>
T round_down(double x) {
  T t = (T)x;
  if ((double)t > x) t = std::nextafter(t, T(0));
  return t;
}

template <typename T>
Coeffs<T> coeffs_of(const sph_params* p, const Grid& g) {
  Coeffs<T> k;
  for (int d = 0; d < 3; ++d) k.L[d] = round_down<T>(g.L[d]);
  const double h = p->h_min;
  const double alpha = p->dim == 2 ? 7.0 / (4.0 * kPi * h * h) : 21.0 / (16.0 * kPi * h * h * h);
  k.h = (T)h;
  k.inv_h = (T)(1.0 / h);
  k.sup2 = (T)(4.0 * h * h);
  k.alpha = (T)alpha;
  k.fcoef = (T)(-5.0 * alpha / (h * h));
  k.mass = (T)p->mass;
  k.rho0 = (T)p->rho0;
  k.c0 = (T)p->c0;
  k.c0sq = (T)(p->c0 * p->c0);
  k.inv_c0 = (T)(1.0 / p->c0);
  k.eta = (T)p->eta;
  k.riemann_eta = (T)p->riemann_eta;
  k.inv_kappa = (T)(1.0 / p->kappa);
  k.dt = (T)p->dt;
  k.half_dt = (T)(0.5 * p->dt);
  k.xi = p->xi;
  k.lim_c = p->lim_c;
  k.lim_s0 = p->lim_s0;
  k.hmin2 = h * h;
  k.band_tol = p->band_tol;
  k.inv_dt = p->dt > 0.0 ? 1.0 / p->dt : 0.0;
  k.tv_mode = p->tv_mode;
  k.bg = p->rho0 * p->c0 * p->c0 * p->dt * p->dt;
  k.nfluid = (int)(p->n - p->n_wall);
  return k;
}

template <typename T>
PArrays<T> arrays_of(const sph_particles* s) {
  PArrays<T> a;
  a.cell = s->cell;
  a.id = s->id;
  a.off = (T*)s->off;
  a.vel = (T*)s->vel;
  a.acc = (T*)s->acc;
  a.rho = (T*)s->rho;
  a.mass = (T*)s->mass;
  a.h = (T*)s->h;
  return a;
}

template <typename T>
PArrays<T> staging_of(char* ws, const WsLayout& w, bool var) {
  PArrays<T> a;
  a.cell = (int*)(ws + w.stg_cell);
  a.id = (int*)(ws + w.stg_id);
  a.off = (T*)(ws + w.stg_off);
  a.vel = (T*)(ws + w.stg_vel);
  a.acc = (T*)(ws + w.stg_acc);
  a.rho = (T*)(ws + w.stg_rho);
  a.mass = var ? (T*)(ws + w.stg_mass) : nullptr;
  a.h = var ? (T*)(ws + w.stg_h) : nullptr;
  return a;
}

int32_t hip_status() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPH_OK : SPH_E_HIP;
}

int32_t check_particles(const sph_params* p, const sph_particles* s, bool need_dyn) {
  if (!s) return SPH_E_ARG;
  if (p->n == 0) return SPH_OK;
  if (!s->cell || !s->id || !s->off) return SPH_E_ARG;
  if (need_dyn && (!s->vel || !s->acc || !s->rho)) return SPH_E_ARG;
  if (p->per_particle) {
    if (!s->mass || !s->h) return SPH_E_ARG;
  } else if (s->mass || s->h) {
    return SPH_E_ARG;
  }
  if ((p->n_wall > 0) != (s->wall_vel != nullptr)) return SPH_E_ARG;
  return SPH_OK;
}

bool is_var(const sph_params* p) { return p->per_particle == 1; }

Launch launch_of(const sph_params* p, bool var, void* stream) {
  Launch l;
  l.dim = p->dim;
  l.var = var;
  l.stream = (hipStream_t)stream;
  l.G = lanes_of(p);
  l.nblk = blocks_for(p->n * l.G);
  return l;
}

// a tape record that does not fit one copy batch (never with these layouts)
constexpr int32_t SPH_E_INTERNAL_COPY = SPH_E_HIP;

hipError_t copy_d2d(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
}

// ---------------------------------------------------------------- cell build
template <typename T>
int32_t build_cells_t(const sph_params* p, sph_particles* parts, int32_t* cs, int32_t* perm,
                      char* ws, hipStream_t stream) {
  const bool var = is_var(p);
  const Sizes sz = sizes_of(p, var);
  const WsLayout w = ws_layout(sz);
  Launch l = launch_of(p, var, stream);
  const CellBuf cb = cellbuf_of(ws, w.cellbuf, sz.ncells);
  int* counts = cb.counts;
  launch_fill(stream, counts, cb.fill_ints, 0);
  PArrays<T> src = arrays_of<T>(parts);
  PArrays<T> stg = staging_of<T>(ws, w, var);
  if (!src.vel) stg.vel = nullptr;
  if (!src.acc) stg.acc = nullptr;
  if (!src.rho) stg.rho = nullptr;
  launch_stage_copy<T>(l, sz.n, src, stg, counts, (int*)(ws + w.slot));
  launch_scan(stream, sz.ncells, counts, cb.scan, 0u, cs, (unsigned*)(ws + w.flags), DiagFold{});
  const SortTmp st{(int*)(ws + w.tmp), (int*)(ws + w.tmp_id), (int2*)(ws + w.tmp_range)};
  launch_scatter(stream, sz.n, stg.cell, stg.id, (int*)(ws + w.slot), cs, st);
  launch_rank_gather<T>(l, sz.n, st, stg, src, perm);
  return hip_status();
}

// ---------------------------------------------------------------- steps
// nsteps kick-drift-kick steps from step index step0.  The first step
// evaluates the correction with the standalone sweep and drifts with the
// standalone kernel; every later step takes both from the fused force sweep of
// the step before.  The last step finishes with the standalone kick.  Per step:
// the one-launch cell build (rebuild_kernel), density, forces (fused except
// the last).  The cell build reads the previous order's cell starts and
// writes the new ones into the other of two buffers (the caller's and the
// workspace's), arranged so that the last step writes the caller's.
// With tapes (nsteps consecutive tapes of tape_layout size), step s records
// its state before the step, its correction sum and limiter value (from the
// standalone sweep for the first step, from the fused force sweep of the
// step before for the others), the cell-build permutation and its state after
// the density sweep; the state after step s is the state before step s + 1.
// With `lists`, each step's density sweep records the neighbour lists its
// force sweep then reads (the workspace holds the list regions).
// With `resume`, the call continues a run: the workspace's staging already
// holds the first step's corrected, kicked and drifted state (every run's
// last force sweep leaves it there, with the next step's correction
// diagnostics and cleared tile words), so the first step starts with the
// cell build.  Partial rows alternate with the parity of the global step
// index, so those diagnostics are where the continuing call looks for them.
template <typename T>
int32_t run_steps_t(const sph_params* p, sph_particles* parts, int32_t* cs_caller, int64_t step0,
                    int64_t nsteps, char* ws, char* tapes, double* diag, hipStream_t stream,
                    bool lists, unsigned* flag_word = nullptr, bool resume = false) {
  const bool var = is_var(p);
  const Sizes sz = sizes_of(p, var);
  const WsLayout w = ws_layout(sz);
  const Grid g = grid_of(p);
  const Coeffs<T> k = coeffs_of<T>(p, g);
  const Launch l = launch_of(p, var, stream);
  unsigned* flags = flag_word ? flag_word : (unsigned*)(ws + w.flags);
  double* part[2] = {(double*)(ws + w.partials), (double*)(ws + w.partials2)};
  auto part_of = [&](int64_t s) { return part[(step0 + s) & 1]; };   // step s of this call
  PArrays<T> a = arrays_of<T>(parts);
  PArrays<T> stg = staging_of<T>(ws, w, var);
  const CellBuf cb = cellbuf_of(ws, w.cellbuf, sz.ncells);
  int* perm = (int*)(ws + w.perm);
  StoredList sl{};
  if (lists && lists_usable(sz)) sl = ws_lists(ws, w, sz);
  const size_t n = (size_t)sz.n, dn = (size_t)sz.dim * n, t = sz.tsz;
  const size_t csb = sizeof(int) * ((size_t)sz.ncells + 1);
  // the two cell_start buffers; step s reads csbuf[cur] and writes
  // csbuf[cur ^ 1].  With an odd number of steps the run starts from the
  // workspace copy, so the last step writes the caller's buffer.
  int* csbuf[2] = {cs_caller, (int*)(ws + w.cs2)};
  int cur = 0;
  if (nsteps & 1) {
    if (copy_d2d(csbuf[1], cs_caller, csb, stream) != hipSuccess) return SPH_E_HIP;
    cur = 1;
  }
  int* cs = csbuf[cur];
  auto applies = [&](int64_t s) { return p->tv_every > 0 && (s % p->tv_every) == 0; };
  const TapeLayout tl = tape_layout(sz);
  auto tape_of = [&](int64_t s) { return tapes + (size_t)s * tl.total; };
  // the sorted state (cell, offsets, density, mass, h, cell_start) into a
  // tape; the copies of one record go out in one launch
  auto record_state = [&](CopyBatch& b, char* tp, size_t o_cell, size_t o_off, size_t o_rho,
                          size_t o_mass, size_t o_h, size_t o_cs, size_t o_id) {
    bool ok = b.add(tp + o_cell, a.cell, sizeof(int) * n);
    if (p->n_wall > 0) ok = ok && b.add(tp + o_id, a.id, sizeof(int) * n);
    ok = ok && b.add(tp + o_off, a.off, t * dn);
    ok = ok && b.add(tp + o_rho, a.rho, t * n);
    if (var) {
      ok = ok && b.add(tp + o_mass, a.mass, t * n);
      ok = ok && b.add(tp + o_h, a.h, t * n);
    }
    return ok && b.add(tp + o_cs, cs, csb);
  };
  auto record_pre = [&](CopyBatch& b, char* tp) {
    return record_state(b, tp, tl.pre_cell, tl.pre_off, tl.pre_rho, tl.pre_mass, tl.pre_h,
                        tl.pre_cs, tl.pre_id);
  };
  auto record_post = [&](CopyBatch& b, char* tp) {
    bool ok = record_state(b, tp, tl.post_cell, tl.post_off, tl.post_rho, tl.post_mass,
                           tl.post_h, tl.post_cs, tl.post_id);
    ok = ok && b.add(tp + tl.perm, perm, sizeof(int) * n);
    return ok && b.add(tp + tl.post_vhalf, a.vel, t * dn);
  };
  if (tapes) {
    CopyBatch b{};
    if (!record_pre(b, tape_of(0))) return SPH_E_INTERNAL_COPY;
    launch_multi_copy(stream, b);
  }
  // first step: 1. correction at r^n (Eq. 14-16), 2. half kick + drift + rebin
  if (resume) {
    // done by the previous call's last force sweep
  } else if (applies(step0)) {
    // one sweep: the correction, then the kick and drift with it, and the
    // cell build's tile words cleared on the side (every diagnostics partial
    // of the first step is written by its sweeps: no clearing)
    const TvDrift<T> td{a, stg, flags, cb.counts, cb.fill_ints};
    launch_tv<T>(l, g, k, a, cs, (T*)(ws + w.dr), tapes ? (T*)(tapes + tl.beta) : nullptr,
                 nullptr, tapes ? (T*)(tapes + tl.g) : nullptr, diag ? part_of(0) : nullptr, td);
  } else {
    launch_fill(stream, cb.counts, cb.fill_ints, 0);
    if (diag) launch_zero_partials(stream, sz.nblk, part_of(0));
    if (tapes) {
      // no correction this step: record g = 0, beta = 0 (the reverse then adds nothing)
      launch_zero<T>(stream, (T*)(tapes + tl.g), (long)dn);
      launch_zero<T>(stream, (T*)(tapes + tl.beta), (long)n);
    }
    launch_drift<T>(l, g, k, a, nullptr, stg, nullptr, nullptr, flags);
  }

  PArrays<T> dst = a;
  dst.acc = nullptr;
  dst.rho = nullptr;
  RebuildArgs rb{};
  rb.ncells = sz.ncells;
  rb.tile_cells = rebuild_tile_cells(sz.dim, p->ncell, (long)n, var);
  rb.tiles_per_row = (p->ncell[0] + rb.tile_cells - 1) / rb.tile_cells;
  rb.ntiles = rebuild_tiles(sz.dim, p->ncell, (long)n, var);
  rb.st = cb.scan;
  rb.perm = tapes ? perm : nullptr;
  rb.flags = flags;
  for (int64_t s = 0; s < nsteps; ++s) {
    double* cur_part = diag ? part_of(s) : nullptr;
    double* nxt = diag ? part_of(s + 1) : nullptr;
    // 3. cell build, folding the previous step's diagnostics in its extra blocks
    rb.fold = DiagFold{};
    if (diag && s > 0)
      rb.fold = DiagFold{part_of(s - 1), sz.nblk * kWavesPerBlock,
                         diag + (size_t)SPH_NDIAG * (s - 1)};
    rb.cs_old = csbuf[cur];
    rb.cs_new = csbuf[cur ^ 1];
    rb.epoch = (unsigned)s;
    launch_rebuild<T>(l, g, rb, stg, dst);
    cur ^= 1;
    cs = csbuf[cur];
    // 4. density summation (Eq. 8), recording the neighbours for the fused
    // force sweep; wall particles from the fluid
    launch_density<T>(l, g, k, a, cs, a.rho, cur_part, nullptr, flags, sl);
    launch_wall_state<T>(l, g, k, a, cs, (const T*)parts->wall_vel, (int)p->n_wall,
                         tapes ? (T*)(tape_of(s) + tl.wsum) : nullptr,
                         tapes ? (T*)(tape_of(s) + tl.wavg) : nullptr);
    if (tapes) {
      // the state after this step (half-step velocity, new density, the
      // walls' state) is the state before the next
      CopyBatch b{};
      if (!record_post(b, tape_of(s))) return SPH_E_INTERNAL_COPY;
      if (s + 1 < nsteps && !record_pre(b, tape_of(s + 1))) return SPH_E_INTERNAL_COPY;
      launch_multi_copy(stream, b);
    }
    // 5-6. accelerations, 7. kick; the next step's correction and drift (the
    // last step's too: a later call may resume from them)
    const bool last = s + 1 == nsteps;
    FusedOut<T> fo{};
    fo.apply_next = applies(step0 + s + 1) ? 1 : 0;
    fo.stg = stg;
    fo.counts = nullptr;
    fo.slot = nullptr;
    fo.part_cur = cur_part;
    fo.part_next = last ? part_of(s + 1) : nxt;
    fo.g_next = nullptr;
    fo.beta_next = nullptr;
    if (tapes && !last) {
      char* tn = tape_of(s + 1);
      if (fo.apply_next) {
        fo.g_next = (T*)(tn + tl.g);
        fo.beta_next = (T*)(tn + tl.beta);
      } else {
        launch_zero<T>(stream, (T*)(tn + tl.g), (long)dn);
        launch_zero<T>(stream, (T*)(tn + tl.beta), (long)n);
      }
    }
    if (last) {
      // the state after the run: its velocity into scratch (the sweep still
      // reads the current one), copied back with the diagnostics fold; the
      // tile words cleared for a resuming call's first cell build
      fo.kick_vel = (T*)(ws + w.dr);
      fo.clear = cb.counts;
      fo.clear_n = cb.fill_ints;
    }
    launch_forces_fused<T>(l, g, k, a, cs, fo, flags, sl);
    if (last)
      launch_fold_copy(stream,
                       diag ? DiagFold{cur_part, sz.nblk * kWavesPerBlock,
                                       diag + (size_t)SPH_NDIAG * s}
                            : DiagFold{},
                       fo.kick_vel, a.vel, t * dn);
  }
  return hip_status();
}

// ---------------------------------------------------------------- dual-criteria steps
// nsteps advection steps of the dual-criteria scheme (dual.hip).  Per step:
// density summation, prologue sweep, K pressure + continuity substep
// sweeps, move, and the one-launch cell build (densities moved too).  The
// substeps reuse workspace regions the kick-drift-kick run and the adjoint
// use for other things: the correction buffer holds the displacement
// accumulator, the adjoint buffers the viscous acceleration, the second
// velocity and density buffers and both density-rate buffers.  Diagnostics
// partials alternate between the two partials buffers and are folded by the
// step's own cell build.
template <typename T>
int32_t dual_steps_t(const sph_params* p, const DualCoeffs& q, sph_particles* parts,
                     int32_t* cs_caller, int64_t nsteps, char* ws, double* diag, double* record,
                     hipStream_t stream) {
  const bool var = is_var(p);
  const Sizes sz = sizes_of(p, var);
  const WsLayout w = ws_layout(sz);
  const Grid g = grid_of(p);
  const Coeffs<T> k = coeffs_of<T>(p, g);
  const Launch l = launch_of(p, var, stream);
  unsigned* flags = (unsigned*)(ws + w.flags);
  double* part[2] = {(double*)(ws + w.partials), (double*)(ws + w.partials2)};
  PArrays<T> a = arrays_of<T>(parts);
  PArrays<T> stg = staging_of<T>(ws, w, var);
  const CellBuf cb = cellbuf_of(ws, w.cellbuf, sz.ncells);
  int* counts = cb.counts;
  const size_t n = (size_t)sz.n;
  // the two cell_start buffers, as in run_steps_t: step s reads csbuf[cur]
  // and its cell build writes csbuf[cur ^ 1]; an odd number of steps starts
  // from the workspace copy, so the last step writes the caller's buffer
  const size_t csb = sizeof(int) * ((size_t)sz.ncells + 1);
  int* csbuf[2] = {cs_caller, (int*)(ws + w.cs2)};
  int cur_cs = 0;
  if (nsteps & 1) {
    if (copy_d2d(csbuf[1], cs_caller, csb, stream) != hipSuccess) return SPH_E_HIP;
    cur_cs = 1;
  }
  T* delta = (T*)(ws + w.dr);
  T* visc = (T*)(ws + w.adj_r);
  T* vel_buf[2] = {a.vel, (T*)(ws + w.adj_v)};
  T* rho_buf[2] = {a.rho, (T*)(ws + w.adj_rho)};
  T* drho_buf[2] = {(T*)(ws + w.adj_g), (T*)(ws + w.adj_g) + n};
  DualSlot* clock[2] = {(DualSlot*)(ws + w.dual_clock),
                        (DualSlot*)(ws + w.dual_clock) + (kMaxDualSubsteps + 1)};
  launch_fill(stream, (int*)clock[0],
              (long)(2 * sizeof(DualSlot) * (kMaxDualSubsteps + 1) / sizeof(int)), 0);
  launch_fill(stream, counts, cb.fill_ints, 0);
  launch_dual_start<T>(stream, sz.n, sz.dim, a.vel, clock[0]);
  // the cell build moves the densities too (the run's result carries the
  // continuity equation's); the one-launch rebuild of the kick-drift-kick runs
  PArrays<T> dst = a;
  dst.acc = nullptr;
  RebuildArgs rb{};
  rb.ncells = sz.ncells;
  rb.tile_cells = rebuild_tile_cells(sz.dim, p->ncell, (long)n, var);
  rb.tiles_per_row = (p->ncell[0] + rb.tile_cells - 1) / rb.tile_cells;
  rb.ntiles = rebuild_tiles(sz.dim, p->ncell, (long)n, var);
  rb.st = cb.scan;
  rb.perm = nullptr;
  rb.flags = flags;
  for (int64_t s = 0; s < nsteps; ++s) {
    int* cs = csbuf[cur_cs];
    double* cur = diag ? part[s & 1] : nullptr;
    DualSlot* clk = clock[s & 1];
    DualSlot* nxt = clock[(s + 1) & 1];
    launch_density<T>(l, g, k, a, cs, a.rho, cur, nullptr, flags);
    launch_dual_prologue<T>(l, g, k, q, a, cs, visc, delta, drho_buf[0], clk, nxt, cur, flags);
    for (int sk = 0; sk < q.K; ++sk) {
      const int b = sk & 1;
      launch_dual_pressure<T>(l, g, k, q, sk, a, cs, vel_buf[b], rho_buf[b], drho_buf[b], visc,
                              vel_buf[b ^ 1], delta, clk, flags);
      launch_dual_continuity<T>(l, g, k, q, sk, a, cs, vel_buf[b ^ 1], rho_buf[b], drho_buf[b],
                                rho_buf[b ^ 1], drho_buf[b ^ 1], clk, flags);
    }
    launch_dual_move<T>(l, g, k, q, a, delta, stg, nullptr, nullptr, clk, nxt, cur,
                        record ? record + 3 * s : nullptr, flags);
    rb.fold = diag ? DiagFold{cur, sz.nblk * kWavesPerBlock, diag + (size_t)SPH_NDIAG * s}
                   : DiagFold{};
    rb.cs_old = csbuf[cur_cs];
    rb.cs_new = csbuf[cur_cs ^ 1];
    rb.epoch = (unsigned)s;
    launch_rebuild<T>(l, g, rb, stg, dst);
    cur_cs ^= 1;
  }
  return hip_status();
}

// ---------------------------------------------------------------- adjoint
template <typename T>
int32_t adjoint_step_t(const sph_params* p, const char* tape, sph_adjoint* adj, double* xi_bar,
                       char* ws, hipStream_t stream) {
  const bool var = is_var(p);
  const Sizes sz = sizes_of(p, var);
  const WsLayout w = ws_layout(sz);
  const TapeLayout tl = tape_layout(sz);
  const Grid g = grid_of(p);
  const Coeffs<T> k = coeffs_of<T>(p, g);
  const Launch l = launch_of(p, var, stream);
  T* r_bar = (T*)adj->r_bar;
  T* v_bar = (T*)adj->v_bar;
  T* a_bar = (T*)adj->a_bar;
  T* rho_bar = (T*)adj->rho_bar;
  // state after the step (order n+1) and before it (order n), as recorded
  PArrays<T> post{};
  post.cell = (int*)(tape + tl.post_cell);
  post.id = p->n_wall > 0 ? (int*)(tape + tl.post_id) : nullptr;
  post.off = (T*)(tape + tl.post_off);
  post.vel = (T*)(tape + tl.post_vhalf);
  post.rho = (T*)(tape + tl.post_rho);
  post.mass = var ? (T*)(tape + tl.post_mass) : nullptr;
  post.h = var ? (T*)(tape + tl.post_h) : nullptr;
  PArrays<T> pre{};
  pre.cell = (int*)(tape + tl.pre_cell);
  pre.id = p->n_wall > 0 ? (int*)(tape + tl.pre_id) : nullptr;
  pre.off = (T*)(tape + tl.pre_off);
  pre.rho = (T*)(tape + tl.pre_rho);
  pre.mass = var ? (T*)(tape + tl.pre_mass) : nullptr;
  pre.h = var ? (T*)(tape + tl.pre_h) : nullptr;
  const int* cs_post = (const int*)(tape + tl.post_cs);
  const int* cs_pre = (const int*)(tape + tl.pre_cs);
  T* r_n = (T*)(ws + w.adj_r);
  T* vh_n = (T*)(ws + w.adj_v);
  T* ghat = (T*)(ws + w.adj_g);
  double* partials = (double*)(ws + w.partials);

  // 7^T: v = v' + dt/2 a  =>  abar += dt/2 vbar, v'bar = vbar (fluid); the
  // walls' acceleration is not an output (always zero): no cotangent
  launch_adj_kick<T>(l, k, sz.n, post.id, v_bar, a_bar);
  // the neighbour lists of the state after the step, for the force, wall
  // and density VJPs (a density sweep recording them; its densities, equal
  // to the tape's, go to scratch).  In 3-D only: there a walk tests about
  // six candidates per neighbour; the 2-D walks test about three, from
  // positions staged in LDS, and cost less than the extra sweep.
  StoredList sl{};
  if (sz.dim == 3 && lists_usable(sz)) {
    sl = ws_lists(ws, w, sz);
    launch_density<T>(l, g, k, post, cs_post, (T*)(ws + w.stg_rho), nullptr, nullptr, nullptr,
                      sl);
  }
  // 6^T, 5^T: accelerations (r^{n+1}, v', rho^{n+1})
  launch_force_vjp<T>(l, g, k, post, cs_post, post.vel, a_bar, r_bar, v_bar, rho_bar, sl);
  // the walls' state from the fluid (r^{n+1}, rho^{n+1}, v'), reversed: the
  // walls' density and velocity cotangents go to their fluid neighbours
  if (p->n_wall > 0)
    launch_wall_vjp<T>(l, g, k, post, cs_post, post.vel, (T*)(tape + tl.wsum),
                       (T*)(tape + tl.wavg), (int)p->n_wall, true, (int*)(ws + w.wall_cells),
                       r_bar, v_bar, rho_bar, sl);
  // 4^T: density, then 2-3^T: r^{n+1} = r^n + dt v' + dr  =>  v'bar += dt rbar
  launch_density_vjp<T>(l, g, k, post, cs_post, rho_bar, r_bar, v_bar, k.dt, sl);
  // the cell build is a permutation: back to order n, with 1^T's first part
  // (ghat of the correction dr = T(r^n, rho^n; xi) and the xi partials)
  const int* perm = (const int*)(tape + tl.perm);
  launch_unpermute_ghat<T>(l, k, sz.n, perm, r_bar, v_bar, (const T*)(tape + tl.g),
                           (const T*)(tape + tl.beta), pre.rho, r_n, vh_n, ghat, partials);
  // 1^T's gather, then 2^T: v' = v^n + dt/2 a^n (fluid), and the xi fold
  AdjFinish<T> fin{pre.id, vh_n, v_bar, a_bar, partials, blocks_for(sz.n) * kWavesPerBlock,
                   xi_bar};
  launch_tv_vjp<T>(l, g, k, pre, cs_pre, ghat, (const T*)(tape + tl.g),
                   (const T*)(tape + tl.beta), r_n, r_bar, rho_bar, fin);
  return hip_status();
}

template <typename T>
int32_t adjoint_init_t(const sph_params* p, const sph_particles* parts, const int32_t* cs,
                       sph_adjoint* adj, char* ws, hipStream_t stream) {
  const bool var = is_var(p);
  const Sizes sz = sizes_of(p, var);
  const WsLayout w = ws_layout(sz);
  const Grid g = grid_of(p);
  const Coeffs<T> k = coeffs_of<T>(p, g);
  const Launch l = launch_of(p, var, stream);
  PArrays<T> a = arrays_of<T>(parts);
  T* r_bar = (T*)adj->r_bar;
  T* v_bar = (T*)adj->v_bar;
  T* a_bar = (T*)adj->a_bar;
  T* rho_bar = (T*)adj->rho_bar;
  if (p->n_wall > 0) launch_zero_walls<T>(l, k, sz.n, a.id, sz.dim, a_bar, (T*)nullptr);
  launch_force_vjp<T>(l, g, k, a, cs, a.vel, a_bar, r_bar, v_bar, rho_bar);
  // the walls' state from the fluid, reversed (their velocity and density
  // cotangents go to the fluid; walls' initial velocities are overwritten)
  if (p->n_wall > 0)
    launch_wall_vjp<T>(l, g, k, a, cs, a.vel, (T*)(ws + w.adj_rho), (T*)(ws + w.adj_r2),
                       (int)p->n_wall, false, (int*)(ws + w.wall_cells), r_bar, v_bar, rho_bar);
  launch_density_vjp<T>(l, g, k, a, cs, rho_bar, r_bar, nullptr, T(0));
  launch_zero<T>(stream, a_bar, (long)sz.dim * sz.n);
  launch_zero<T>(stream, rho_bar, (long)sz.n);
  return hip_status();
}

template <typename F>
int32_t dispatch(const sph_params* p, F&& f) {
  if (p->dtype == SPH_F64) return f(double(0));
  return f(float(0));
}

}  // namespace
}  // namespace sph

// ---------------------------------------------------------------- allocation-free runs
// Device scratch of sph_kdk_run_static: the workspace of a run, held by every
// device the library runs on until the process ends.  In host code `scratch`
// names a host-side stand-in, never a device address: its device address is
// looked up once per device (hipGetSymbolAddress, with that device current)
// and only that address is passed to kernels.
static __device__ __align__(256) char scratch[SPH_STATIC_SCRATCH_BYTES];

namespace sph {
namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mutex;
char* scratch_address[kMaxDevices] = {};

// Device address of the current device's scratch (looked up on its first use).
int32_t scratch_of_current_device(char** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return SPH_E_HIP;
  if (dev < 0 || dev >= kMaxDevices) return SPH_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (!scratch_address[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SPH_E_HIP;
    scratch_address[dev] = (char*)ptr;
  }
  *out = scratch_address[dev];
  return SPH_OK;
}
}  // namespace
}  // namespace sph

using namespace sph;

extern "C" {

int32_t sph_workspace_size(const sph_params* p, size_t* bytes) {
  int32_t st = check_params(p);
  if (st != SPH_OK) return st;
  if (!bytes) return SPH_E_ARG;
  // laid out for the variable-resolution case so one size fits both
  *bytes = ws_layout(sizes_of(p, true)).total;
  return SPH_OK;
}

int32_t sph_tape_size(const sph_params* p, size_t* bytes) {
  int32_t st = check_params(p);
  if (st != SPH_OK) return st;
  if (!bytes) return SPH_E_ARG;
  *bytes = tape_layout(sizes_of(p, is_var(p))).total;
  return SPH_OK;
}

int32_t sph_lattice_kappa(int32_t dim, double h_over_dx, double* kappa) {
  if ((dim != 2 && dim != 3) || !kappa || !(h_over_dx > 0.0) || !std::isfinite(h_over_dx))
    return SPH_E_ARG;
  // sum over integer lattice vectors k with |k| < 2 h/dx of W(|k|, h), self included
  const double h = h_over_dx;
  const double alpha = dim == 2 ? 7.0 / (4.0 * kPi * h * h) : 21.0 / (16.0 * kPi * h * h * h);
  const int reach = (int)std::ceil(2.0 * h);
  double sum = 0.0;
  for (int z = (dim == 3 ? -reach : 0); z <= (dim == 3 ? reach : 0); ++z)
    for (int y = -reach; y <= reach; ++y)
      for (int x = -reach; x <= reach; ++x) {
        const double q = std::sqrt((double)(x * x + y * y + z * z)) / h;
        if (q < 2.0) {
          const double t = 1.0 - 0.5 * q;
          sum += alpha * t * t * t * t * (1.0 + 2.0 * q);
        }
      }
  *kappa = sum;
  return SPH_OK;
}

int32_t sph_bin_positions(const sph_params* p, const double* pos, sph_particles* parts, void* ws,
                          size_t ws_bytes, void* stream) {
  int32_t st = check_params(p);
  if (st != SPH_OK) return st;
  if (!parts || !ws) return SPH_E_ARG;
  size_t need = 0;
  sph_workspace_size(p, &need);
  if (ws_bytes < need) return SPH_E_WORKSPACE;
  if (p->n == 0) return SPH_OK;
  if (!pos || !parts->cell || !parts->off) return SPH_E_ARG;
  const Grid g = grid_of(p);
  const Launch l = launch_of(p, is_var(p), stream);
  const WsLayout w = ws_layout(sizes_of(p, true));
  unsigned* flags = (unsigned*)((char*)ws + w.flags);
  return dispatch(p, [&](auto tag) {
    using T = decltype(tag);
    launch_bin<T>(l, g, coeffs_of<T>(p, g), pos, parts->cell, (T*)parts->off, flags);
    return hip_status();
  });
}

int32_t sph_build_cells(const sph_params* p, sph_particles* parts, int32_t* cell_start,
                        int32_t* perm, void* ws, size_t ws_bytes, void* stream) {
  int32_t st = check_params(p);
  if (st != SPH_OK) return st;
  st = check_particles(p, parts, false);
  if (st != SPH_OK) return st;
  if (!cell_start || !ws) return SPH_E_ARG;
  size_t need = 0;
  sph_workspace_size(p, &need);
  if (ws_bytes < need) return SPH_E_WORKSPACE;
  return dispatch(p, [&](auto tag) {
    using T = decltype(tag);
    return build_cells_t<T>(p, parts, cell_start, perm, (char*)ws, (hipStream_t)stream);
  });
}

int32_t sph_density(const sph_params* p, const sph_particles* parts, const int32_t* cell_start,
                    void* rho_out, void* stream) {
  int32_t st = check_params(p);
  if (st != SPH_OK) return st;
  st = check_particles(p, parts, false);
  if (st != SPH_OK) return st;
  if (p->n == 0) return SPH_OK;
  if (!cell_start || !rho_out) return SPH_E_ARG;
  const Grid g = grid_of(p);
  const Launch l = launch_of(p, is_var(p), stream);
  return dispatch(p, [&](auto tag) {
    using T = decltype(tag);
    launch_density<T>(l, g, coeffs_of<T>(p, g), arrays_of<T>(parts), cell_start, (T*)rho_out,
                      nullptr, nullptr, nullptr);
    return hip_status();
  });
}

int32_t sph_list_size(const sph_params* p, size_t* bytes) {
  int32_t st = check_params(p);
  if (st != SPH_OK) return st;
  if (!bytes) return SPH_E_ARG;
  *bytes = list_layout(sizes_of(p, is_var(p))).total;
  return SPH_OK;
}

static int32_t list_of(const sph_params* p, const void* lists, size_t list_bytes,
                       StoredList* out) {
  const Sizes sz = sizes_of(p, is_var(p));
  const ListLayout ll = list_layout(sz);
  if (ll.total == 0) return SPH_E_UNSUPPORTED;
  if (!lists) return SPH_E_ARG;
  if (list_bytes < ll.total) return SPH_E_WORKSPACE;
  char* b = (char*)const_cast<void*>(lists);
  *out = StoredList{(unsigned*)(b + ll.entries), (int*)(b + ll.counts), sz.nblk * kBlock,
                    sz.dim == 2 ? (int*)(b + ll.runs) : nullptr};
  return SPH_OK;
}

int32_t sph_density_lists(const sph_params* p, const sph_particles* parts,
                          const int32_t* cell_start, void* rho_out, void* lists,
                          size_t list_bytes, void* stream) {
  int32_t st = check_params(p);
  if (st != SPH_OK) return st;
  st = check_particles(p, parts, false);
  if (st != SPH_OK) return st;
  StoredList sl{};
  st = list_of(p, lists, list_bytes, &sl);
  if (st != SPH_OK) return st;
  if (p->n == 0) return SPH_OK;
  if (!cell_start || !rho_out) return SPH_E_ARG;
  const Grid g = grid_of(p);
  const Launch l = launch_of(p, is_var(p), stream);
  return dispatch(p, [&](auto tag) {
    using T = decltype(tag);
    launch_density<T>(l, g, coeffs_of<T>(p, g), arrays_of<T>(parts), cell_start, (T*)rho_out,
                      nullptr, nullptr, nullptr, sl);
    return hip_status();
  });
}

int32_t sph_forces_lists(const sph_params* p, const sph_particles* parts,
                         const int32_t* cell_start, const void* vel, void* acc_out,
                         const void* lists, size_t list_bytes, void* stream) {
  int32_t st = check_params(p);
  if (st != SPH_OK) return st;
  st = check_particles(p, parts, false);
  if (st != SPH_OK) return st;
  StoredList sl{};
  st = list_of(p, lists, list_bytes, &sl);
  if (st != SPH_OK) return st;
  if (p->n == 0) return SPH_OK;
  if (!cell_start || !vel || !acc_out || !parts->rho) return SPH_E_ARG;
  const Grid g = grid_of(p);
  const Launch l = launch_of(p, is_var(p), stream);
  return dispatch(p, [&](auto tag) {
    using T = decltype(tag);
    launch_forces<T>(l, g, coeffs_of<T>(p, g), arrays_of<T>(parts), cell_start, (const T*)vel,
                     (T*)acc_out, nullptr, sl);
    return hip_status();
  });
}

int32_t sph_neighbor_counts(const sph_params* p, const sph_particles* parts,
                            const int32_t* cell_start, int32_t* counts, void* stream) {
  int32_t st = check_params(p);
  if (st != SPH_OK) return st;
  st = check_particles(p, parts, false);
  if (st != SPH_OK) return st;
  if (p->n == 0) return SPH_OK;
  if (!cell_start || !counts || !parts->rho) return SPH_E_ARG;
  const Grid g = grid_of(p);
  const Launch l = launch_of(p, is_var(p), stream);
  // the density sweep counts its neighbours; it rewrites rho with the same values
  return dispatch(p, [&](auto tag) {
    using T = decltype(tag);
    PArrays<T> a = arrays_of<T>(parts);
    launch_density<T>(l, g, coeffs_of<T>(p, g), a, cell_start, a.rho, nullptr, counts, nullptr);
    return hip_status();
  });
}

int32_t sph_forces(const sph_params* p, const sph_particles* parts, const int32_t* cell_start,
                   const void* vel, void* acc_out, void* stream) {
  int32_t st = check_params(p);
  if (st != SPH_OK) return st;
  st = check_particles(p, parts, false);
  if (st != SPH_OK) return st;
  if (p->n == 0) return SPH_OK;
  if (!cell_start || !vel || !acc_out || !parts->rho) return SPH_E_ARG;
  const Grid g = grid_of(p);
  const Launch l = launch_of(p, is_var(p), stream);
  return dispatch(p, [&](auto tag) {
    using T = decltype(tag);
    launch_forces<T>(l, g, coeffs_of<T>(p, g), arrays_of<T>(parts), cell_start, (const T*)vel,
                     (T*)acc_out, nullptr);
    return hip_status();
  });
}

int32_t sph_wall_state(const sph_params* p, sph_particles* parts, const int32_t* cell_start,
                       void* stream) {
  int32_t st = check_params(p);
  if (st != SPH_OK) return st;
  st = check_particles(p, parts, true);
  if (st != SPH_OK) return st;
  if (p->n == 0 || p->n_wall == 0) return SPH_OK;
  if (!cell_start) return SPH_E_ARG;
  const Grid g = grid_of(p);
  const Launch l = launch_of(p, is_var(p), stream);
  return dispatch(p, [&](auto tag) {
    using T = decltype(tag);
    launch_wall_state<T>(l, g, coeffs_of<T>(p, g), arrays_of<T>(parts), cell_start,
                         (const T*)parts->wall_vel, (int)p->n_wall, (T*)nullptr, (T*)nullptr);
    return hip_status();
  });
}

int32_t sph_tv_correction(const sph_params* p, const sph_particles* parts,
                          const int32_t* cell_start, void* dr_out, void* beta_out, double* s_out,
                          void* g_out, void* stream) {
  int32_t st = check_params(p);
  if (st != SPH_OK) return st;
  st = check_particles(p, parts, false);
  if (st != SPH_OK) return st;
  if (p->n == 0) return SPH_OK;
  if (!cell_start || !dr_out || !parts->rho) return SPH_E_ARG;
  const Grid g = grid_of(p);
  const Launch l = launch_of(p, is_var(p), stream);
  return dispatch(p, [&](auto tag) {
    using T = decltype(tag);
    launch_tv<T>(l, g, coeffs_of<T>(p, g), arrays_of<T>(parts), cell_start, (T*)dr_out,
                 (T*)beta_out, s_out, (T*)g_out, nullptr);
    return hip_status();
  });
}

static int32_t kdk_common(const sph_params* p, sph_particles* parts, int32_t* cell_start,
                          int64_t step_index, int64_t nsteps, void* ws, size_t ws_bytes,
                          void* tape, double* diag, void* stream, bool resume = false) {
  int32_t st = check_params(p);
  if (st != SPH_OK) return st;
  st = check_particles(p, parts, true);
  if (st != SPH_OK) return st;
  if (!cell_start || !ws || step_index < 0 || nsteps < 0) return SPH_E_ARG;
  size_t need = 0;
  sph_workspace_size(p, &need);
  if (ws_bytes < need) return SPH_E_WORKSPACE;
  if (nsteps == 0) return SPH_OK;
  if (p->n == 0) {
    if (diag) launch_zero<double>((hipStream_t)stream, diag, (long)SPH_NDIAG * nsteps);
    return hip_status();
  }
  return dispatch(p, [&](auto tag) {
    using T = decltype(tag);
    return run_steps_t<T>(p, parts, cell_start, step_index, nsteps, (char*)ws, (char*)tape, diag,
                          (hipStream_t)stream, true, nullptr, resume);
  });
}

int32_t sph_kdk_step(const sph_params* p, sph_particles* parts, int32_t* cell_start,
                     int64_t step_index, void* ws, size_t ws_bytes, void* tape, double* diag,
                     void* stream) {
  return kdk_common(p, parts, cell_start, step_index, 1, ws, ws_bytes, tape, diag, stream);
}

int32_t sph_kdk_run(const sph_params* p, sph_particles* parts, int32_t* cell_start,
                    int64_t step_index, int64_t nsteps, void* ws, size_t ws_bytes, void* tapes,
                    double* diag, void* stream) {
  return kdk_common(p, parts, cell_start, step_index, nsteps, ws, ws_bytes, tapes, diag, stream);
}

int32_t sph_kdk_run_resume(const sph_params* p, sph_particles* parts, int32_t* cell_start,
                           int64_t step_index, int64_t nsteps, void* ws, size_t ws_bytes,
                           double* diag, void* stream) {
  return kdk_common(p, parts, cell_start, step_index, nsteps, ws, ws_bytes, nullptr, diag, stream,
                    true);
}

int32_t sph_kdk_run_static(const sph_params* p, sph_particles* parts, int32_t* cell_start,
                           int64_t step_index, int64_t nsteps, void* tapes, double* diag,
                           uint32_t* flags, void* stream) {
  int32_t st = check_params(p);
  if (st != SPH_OK) return st;
  st = check_particles(p, parts, true);
  if (st != SPH_OK) return st;
  if (!cell_start || step_index < 0 || nsteps < 0) return SPH_E_ARG;
  // the run needs the workspace without its stored neighbour lists, and
  // records lists when they fit too
  const WsLayout wl = ws_layout(sizes_of(p, true));
  if (wl.base_total > (size_t)SPH_STATIC_SCRATCH_BYTES) return SPH_E_TOO_LARGE;
  const bool lists = wl.total <= (size_t)SPH_STATIC_SCRATCH_BYTES;
  if (nsteps == 0) return SPH_OK;
  hipStream_t s = (hipStream_t)stream;
  if (p->n == 0) {
    if (diag) launch_zero<double>(s, diag, (long)SPH_NDIAG * nsteps);
    return hip_status();
  }
  char* ws = nullptr;
  st = scratch_of_current_device(&ws);
  if (st != SPH_OK) return st;
  // the scratch keeps the previous call's contents: its own flag word is
  // cleared here (the run itself clears its histogram, scan state and
  // diagnostics partials before use, as it does in a caller's workspace)
  unsigned* flag_word = (unsigned*)flags;
  if (!flag_word) {
    flag_word = (unsigned*)ws;
    launch_fill(s, (int*)flag_word, 1, 0);
  }
  return dispatch(p, [&](auto tag) {
    using T = decltype(tag);
    return run_steps_t<T>(p, parts, cell_start, step_index, nsteps, ws, (char*)tapes, diag, s,
                          lists, flag_word);
  });
}

int32_t sph_dual_run(const sph_params* p, const sph_dual_params* q, sph_particles* parts,
                     int32_t* cell_start, int64_t nsteps, void* ws, size_t ws_bytes, double* diag,
                     double* steps, void* stream) {
  int32_t st = check_params(p);
  if (st != SPH_OK) return st;
  st = check_particles(p, parts, true);
  if (st != SPH_OK) return st;
  if (!q || !cell_start || !ws || nsteps < 0) return SPH_E_ARG;
  if (p->n_wall > 0 || p->tv_mode == SPH_TV_BACKGROUND) return SPH_E_UNSUPPORTED;
  const double vals[] = {q->cfl_ad, q->cfl_ac, q->u_ref, q->nu};
  for (double v : vals)
    if (!std::isfinite(v)) return SPH_E_NONFINITE;
  if (q->cfl_ad <= 0.0 || q->cfl_ac <= 0.0 || q->u_ref <= 0.0 || q->nu < 0.0) return SPH_E_ARG;
  if (q->max_substeps < 0 || q->max_substeps > kMaxDualSubsteps) return SPH_E_ARG;
  DualCoeffs dq;
  dq.cfl_ad = q->cfl_ad;
  dq.cfl_ac = q->cfl_ac;
  dq.u_ref = q->u_ref;
  dq.nu = q->nu;
  dq.h_min = p->h_min;
  dq.c0 = p->c0;
  dq.capped = q->max_substeps > 0 ? 1 : 0;
  if (dq.capped) {
    dq.cap = q->max_substeps;
  } else {
    // the substeps of Eq. 11 needed to cover Eq. 9-10 while the largest
    // speed stays below twice max(|v|_max at the step's start, U_ref)
    const double bound = std::ceil(q->cfl_ad / q->cfl_ac * (2.0 + p->c0 / q->u_ref)) + 1.0;
    if (!(bound <= kMaxDualSubsteps)) return SPH_E_UNSUPPORTED;
    dq.cap = (int)bound;
  }
  dq.K = dq.cap + (dq.cap & 1);    // even: the substeps end in the state's own buffers
  if (dq.K > kMaxDualSubsteps) return SPH_E_UNSUPPORTED;
  size_t need = 0;
  sph_workspace_size(p, &need);
  if (ws_bytes < need) return SPH_E_WORKSPACE;
  if (nsteps == 0) return SPH_OK;
  hipStream_t s = (hipStream_t)stream;
  if (p->n == 0) {
    if (diag) launch_zero<double>(s, diag, (long)SPH_NDIAG * nsteps);
    if (steps) launch_zero<double>(s, steps, 3L * nsteps);
    return hip_status();
  }
  return dispatch(p, [&](auto tag) {
    using T = decltype(tag);
    return dual_steps_t<T>(p, dq, parts, cell_start, nsteps, (char*)ws, diag, steps, s);
  });
}

int32_t sph_diagnostics(const sph_params* p, const sph_particles* parts, const int32_t* cell_start,
                        void* ws, size_t ws_bytes, double* diag, void* stream) {
  int32_t st = check_params(p);
  if (st != SPH_OK) return st;
  st = check_particles(p, parts, true);
  if (st != SPH_OK) return st;
  if (!ws || !diag) return SPH_E_ARG;
  size_t need = 0;
  sph_workspace_size(p, &need);
  if (ws_bytes < need) return SPH_E_WORKSPACE;
  const bool var = is_var(p);
  const Sizes sz = sizes_of(p, var);
  const WsLayout w = ws_layout(sz);
  hipStream_t s = (hipStream_t)stream;
  if (p->n == 0) {
    launch_zero<double>(s, diag, SPH_NDIAG);
    return hip_status();
  }
  if (!cell_start) return SPH_E_ARG;
  double* partials = (double*)((char*)ws + w.partials);
  launch_zero_partials(s, sz.nblk, partials);
  const Grid g = grid_of(p);
  const Launch l = launch_of(p, var, stream);
  st = dispatch(p, [&](auto tag) {
    using T = decltype(tag);
    const Coeffs<T> k = coeffs_of<T>(p, g);
    PArrays<T> a = arrays_of<T>(parts);
    // pair count from a density sweep into the staging buffer (state untouched)
    launch_density<T>(l, g, k, a, cell_start, (T*)((char*)ws + w.stg_rho), partials, nullptr,
                      nullptr);
    launch_kick<T>(l, k, sz.n, a.vel, a.acc, a.mass, a.id, partials, false, nullptr);
    launch_diag_fold(s, DiagFold{partials, sz.nblk * kWavesPerBlock, diag});
    return SPH_OK;
  });
  if (st != SPH_OK) return st;
  return hip_status();
}

int32_t sph_adjoint_step(const sph_params* p, const void* tape, sph_adjoint* adj, double* xi_bar,
                         void* ws, size_t ws_bytes, void* stream) {
  int32_t st = check_params(p);
  if (st != SPH_OK) return st;
  if (!tape || !adj || !ws) return SPH_E_ARG;
  size_t need = 0;
  sph_workspace_size(p, &need);
  if (ws_bytes < need) return SPH_E_WORKSPACE;
  if (p->n == 0) return SPH_OK;
  if (!adj->r_bar || !adj->v_bar || !adj->a_bar || !adj->rho_bar) return SPH_E_ARG;
  return dispatch(p, [&](auto tag) {
    using T = decltype(tag);
    return adjoint_step_t<T>(p, (const char*)tape, adj, xi_bar, (char*)ws, (hipStream_t)stream);
  });
}

int32_t sph_adjoint_init(const sph_params* p, const sph_particles* parts, const int32_t* cell_start,
                         sph_adjoint* adj, void* ws, size_t ws_bytes, void* stream) {
  int32_t st = check_params(p);
  if (st != SPH_OK) return st;
  st = check_particles(p, parts, true);
  if (st != SPH_OK) return st;
  if (!adj || !ws) return SPH_E_ARG;
  size_t need = 0;
  sph_workspace_size(p, &need);
  if (ws_bytes < need) return SPH_E_WORKSPACE;
  if (p->n == 0) return SPH_OK;
  if (!cell_start || !adj->r_bar || !adj->v_bar || !adj->a_bar || !adj->rho_bar) return SPH_E_ARG;
  return dispatch(p, [&](auto tag) {
    using T = decltype(tag);
    return adjoint_init_t<T>(p, parts, cell_start, adj, (char*)ws, (hipStream_t)stream);
  });
}

int32_t sph_get_flags(void* ws, void* stream, uint32_t* host_flags) {
  if (!ws || !host_flags) return SPH_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (hipStreamSynchronize(s) != hipSuccess) return SPH_E_HIP;
  if (hipMemcpy(host_flags, ws, sizeof(uint32_t), hipMemcpyDeviceToHost) != hipSuccess)
    return SPH_E_HIP;
  launch_fill(s, (int*)ws, 1, 0);
  if (hipStreamSynchronize(s) != hipSuccess) return SPH_E_HIP;
  return hip_status();
}

int32_t sph_clear_flags(void* ws, void* stream) {
  if (!ws) return SPH_E_ARG;
  launch_fill((hipStream_t)stream, (int*)ws, 1, 0);
  return hip_status();
}

const char* sph_status_string(int32_t status) {
  switch (status) {
    case SPH_OK: return "ok";
    case SPH_E_ARG: return "invalid argument";
    case SPH_E_HIP: return "HIP runtime error";
    case SPH_E_WORKSPACE: return "workspace or tape too small";
    case SPH_E_CELL_RANGE: return "cell grid too fine for the kernel support (need >= 3 cells of edge >= 2 h_max per axis)";
    case SPH_E_NONFINITE: return "non-finite parameter";
    case SPH_E_UNSUPPORTED: return "unsupported dimension, dtype or size";
    case SPH_E_TOO_LARGE:
      return "problem needs more workspace than the static scratch of sph_kdk_run_static holds";
    default: return "unknown status";
  }
}

}  // extern "C"
