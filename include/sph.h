/*
 * libsph: C-ABI for the data-parallel hot path of one transport-velocity
 * weakly-compressible SPH step on a gfx950 GPU (method of Wang, Haidn & Hu,
 * arXiv 2411.13992).
 *
 * One step n -> n+1 (kick-drift-kick with fixed dt):
 *   1. transport correction at r^n:  g_i = sum_j V_j grad_i W_ij, V_j = m_j/rho_j,
 *      s_i = h_min^2 |g_i|^2, beta_i = min(C s_i, 1) if s_i > s0 else 0,
 *      dr_i = xi beta_i h_min^2 g_i                              (Sec. 3, Eq. 14-16)
 *   2. half kick v' = v + dt/2 a; drift r += dt v' + dr; rebin to cells
 *   3. cell build: particles sorted by (cell, id)
 *   4. density summation rho_i = sum_{j incl. i} m_j W_ij / kappa      (Eq. 8)
 *   5. EOS p = c0^2 (rho - rho0)                                        (Eq. 2)
 *   6. accelerations: Riemann pressure term with the limited linear
 *      solver and the viscous shear term                       (Eq. 3b, 5-7)
 *   7. half kick v = v' + dt/2 a
 *
 * Kernel: Wendland C2 with support 2h, h = 1.3 dp (Sec. 4).  The kernel
 * gradient is taken with respect to r_i; the Riemann axis points from i to j;
 * pairs of different smoothing length use h_ij = (h_i + h_j)/2; neighbours are
 * j != i with r_ij < 2 h_ij.
 *
 * Conventions for every entry point:
 *  - returns SPH_OK (0) or a negative SPH_E_* status; no exception crosses
 *    the boundary; sph_status_string() names the status;
 *  - every array pointer is a DEVICE pointer owned by the caller; the library
 *    allocates no device memory and keeps no state between calls; scratch
 *    memory is the caller's workspace of sph_workspace_size() bytes (the one
 *    exception, sph_kdk_run_static, takes it from a static device array);
 *  - every call is asynchronous on `stream` (a hipStream_t, NULL = the null
 *    stream) and never synchronises, except sph_get_flags();
 *  - argument errors are detected on the host and returned at once, before
 *    anything is enqueued; errors found on the device (non-finite values, a
 *    particle that moved more than one cell in a step, a position outside the
 *    box) set bits in a flag word held in the workspace (sph_get_flags);
 *  - vector fields are structure-of-arrays [D][N] (component-major,
 *    contiguous); all floating-point arrays have the element type named by
 *    params.dtype (float for SPH_F32, double for SPH_F64) unless stated;
 *  - positions are stored as a linear cell index (x fastest) plus cell-local
 *    offsets in [0, L_k), L_k = box[k] / ncell[k] >= 2 h_max;
 *  - particle ids are preserved through every reordering, so a caller maps
 *    results back to its own order through `id`.
 */
#ifndef SPH_H
#define SPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SPH_OK             0
#define SPH_E_ARG         -1  /* invalid argument (null pointer, size, shape) */
#define SPH_E_HIP         -2  /* a HIP runtime call failed                    */
#define SPH_E_WORKSPACE   -3  /* workspace or tape smaller than required      */
#define SPH_E_CELL_RANGE  -4  /* cell grid does not satisfy L_k >= 2 h_max, or
                                 fewer than 3 cells on an axis                */
#define SPH_E_NONFINITE   -5  /* non-finite parameter                         */
#define SPH_E_UNSUPPORTED -6  /* dimension or dtype not supported             */
#define SPH_E_TOO_LARGE   -7  /* the run needs more workspace than the static
                                 scratch of sph_kdk_run_static holds          */

/* Size of the device scratch array behind sph_kdk_run_static (64 MiB per
 * device): enough for about 570,000 particles in 2-D FP32, 340,000 in 2-D
 * FP64 and 430,000 in 3-D FP32 (sph_workspace_size bytes per run). */
#define SPH_STATIC_SCRATCH_BYTES (64u << 20)

/* device flag bits (sph_get_flags) */
#define SPH_FLAG_NONFINITE  1u  /* a velocity, acceleration or density is NaN/Inf */
#define SPH_FLAG_CFL        2u  /* a particle moved more than one cell in a step  */
#define SPH_FLAG_OUT_OF_BOX 4u  /* an input position lies outside [0, box)        */
#define SPH_FLAG_INTERNAL   8u  /* a bounded internal wait gave up (results of the
                                   call are invalid; should not happen)         */

/* dtype */
#define SPH_F32 0
#define SPH_F64 1

/* transport-velocity formulation (params.tv_mode); g_i = sum_j V_j grad_i W_ij,
 * V_j = m_j / rho_j, s_i = h_min^2 |g_i|^2 */
#define SPH_TV_LIMITED    0  /* Eq. 15-16: dr = xi beta h_min^2 g, beta the limiter   */
#define SPH_TV_SCALED     1  /* Eq. 14 without limiter: dr = xi h_min^2 g (beta = 1)   */
#define SPH_TV_BACKGROUND 2  /* Eq. 12 with background pressure p0 = rho0 c0^2 in the
                                kick-drift-kick drift: the transport acceleration
                                a_t = -2 (p0 / rho_i) g_i acts as dr = a_t dt^2 / 2,
                                i.e. dr = -(rho0 c0^2 dt^2 / rho_i) g (beta = 1)       */

/* Run parameters.  Symbols follow the paper: rho0 reference density, c0
 * artificial sound speed (Eq. 2), eta dynamic viscosity (Eq. 7), xi the
 * correction coefficient (-0.2, Eq. 14/16), lim_c and lim_s0 the limiter slope
 * (1e3) and threshold (5e-4) of Eq. 15, riemann_eta the dissipation limiter
 * constant (3, Eq. 6). */
typedef struct {
    int32_t dim;          /* 2 or 3                                              */
    int32_t dtype;        /* SPH_F32 or SPH_F64: storage and sweep precision     */
    int64_t n;            /* number of particles, 0 <= n < 2^28                  */
    int32_t ncell[3];     /* cells per axis (>= 3); unused axes ignored          */
    int32_t tv_every;     /* apply the correction on steps with index % k == 0;
                             0 disables it                                       */
    int32_t per_particle; /* 1: particles carry their own mass and h arrays
                             (variable resolution); 0: uniform mass and h_min    */
    int32_t tv_mode;      /* SPH_TV_LIMITED (default), SPH_TV_SCALED or
                             SPH_TV_BACKGROUND; other values: SPH_E_ARG          */
    double box[3];        /* periodic box edges                                  */
    double rho0, c0, eta;
    double h_min, h_max;  /* smallest / largest smoothing length                 */
    double mass;          /* particle mass when particles.mass == NULL           */
    double kappa;         /* perfect-lattice kernel sum times dx^D, the reference
                             sum of Eq. 8 (sph_lattice_kappa)                     */
    double dt, xi, lim_c, lim_s0, riemann_eta;
    double band_tol;      /* relative half-width of the limiter band counted in
                             the diagnostics: |s - s0| <= band_tol * s0          */
    int64_t n_wall;       /* 0 <= n_wall <= n: particles with id >= n - n_wall
                             are wall particles (see sph_wall_state); with
                             per_particle = 1: SPH_E_UNSUPPORTED                 */
    int32_t lanes;        /* lanes per particle in the neighbour sweeps: 2, 4 or
                             8, or 0 to let the library choose by size (more
                             lanes for small n); other values: SPH_E_ARG.  The
                             choice changes only the summation order (results
                             within rounding, not bit-identical across lanes)  */
} sph_params;

/* Particle arrays, all device pointers of length N (or [D][N]). */
typedef struct {
    int32_t *cell;  /* linear cell index, x fastest                          */
    int32_t *id;    /* original particle id                                  */
    void *off;      /* [D][N] cell-local offsets, 0 <= off_k < L_k           */
    void *vel;      /* [D][N] velocity                                       */
    void *acc;      /* [D][N] acceleration                                   */
    void *rho;      /* [N] density                                           */
    void *mass;     /* [N] per-particle mass (params.per_particle = 1), else
                       NULL and params.mass applies to all                   */
    void *h;        /* [N] per-particle smoothing length (per_particle = 1),
                       else NULL and h_min applies to all                    */
    void *wall_vel; /* [D][n_wall] prescribed velocity of wall particle
                       id = n - n_wall + w at column w (params.n_wall > 0),
                       else NULL; never reordered                            */
} sph_particles;

/* Cotangents (adjoint variables) of a state, device arrays in the particle
 * order of the state they belong to. */
typedef struct {
    void *r_bar;    /* [D][N] cotangent of positions     */
    void *v_bar;    /* [D][N] cotangent of velocities    */
    void *a_bar;    /* [D][N] cotangent of accelerations */
    void *rho_bar;  /* [N]    cotangent of densities     */
} sph_adjoint;

/* Number of diagnostics written by sph_kdk_step / sph_diagnostics. */
#define SPH_NDIAG 9
/* Over the fluid particles (all particles without walls):
 * diag[0] kinetic energy 1/2 sum m |v|^2, diag[1..3] momentum sum m v,
 * diag[4] max |v|, diag[5] ordered neighbour pairs at r^{n+1} (every
 * particle's),
 * diag[6] particles with beta > 0 at step n, diag[7] particles in the
 * limiter band, diag[8] max |dr| / dt (the transport-velocity magnitude of
 * Sec. 3's overcorrection discussion).  All reductions are FP64 and
 * deterministic (fixed-order two-pass, no floating-point atomics). */

/* ---- sizes and constants (host only, synchronous) ------------------------ */

/* Bytes of workspace the step and sweep calls need for these parameters. */
int32_t sph_workspace_size(const sph_params *p, size_t *bytes);

/* Bytes of one step's tape (the recorded intermediates the adjoint needs). */
int32_t sph_tape_size(const sph_params *p, size_t *bytes);

/* kappa_D: sum of W(|k| dx, h) dx^D over a perfect lattice, self included,
 * at h = h_over_dx * dx (dimensionless).  Eq. 8's reference sum; with it a
 * perfect lattice has rho = rho0 exactly. */
int32_t sph_lattice_kappa(int32_t dim, double h_over_dx, double *kappa);

/* ---- hot path (asynchronous on `stream`) --------------------------------- */

/* Bin absolute FP64 positions pos[D][N] (device, inside [0, box)) into
 * particles.cell and particles.off.  Positions outside the box are wrapped
 * and flagged SPH_FLAG_OUT_OF_BOX.  Does not sort. */
int32_t sph_bin_positions(const sph_params *p, const double *pos, sph_particles *parts,
                          void *ws, size_t ws_bytes, void *stream);

/* Cell-linked-list build: sort every particle array in place into
 * (cell, id) order and write cell_start[ncells + 1] (CSR offsets: the
 * particles of cell c are cell_start[c] .. cell_start[c+1]-1).  perm
 * (optional, [N] int32) receives, for each new position, the particle's
 * previous position.  Neighbour search itself is not in the paper; this is
 * the data structure every sweep below iterates (3^D cells per particle). */
int32_t sph_build_cells(const sph_params *p, sph_particles *parts, int32_t *cell_start,
                        int32_t *perm, void *ws, size_t ws_bytes, void *stream);

/* Density summation, Eq. 8: rho_out[i] = sum_{j in N(i) + i} m_j W_ij / kappa.
 * Requires the particles sorted and cell_start built.  FP32 sums are
 * Kahan-compensated. */
int32_t sph_density(const sph_params *p, const sph_particles *parts,
                    const int32_t *cell_start, void *rho_out, void *stream);

/* Accelerations, Eq. 3b with the limited linear Riemann solver (Eq. 5-6),
 * the EOS of Eq. 2 and the viscous term of Eq. 7, from positions, the given
 * velocity vel[D][N] and parts->rho.  acc_out[D][N].  Coincident particles
 * contribute no pressure term (their Riemann axis is undefined). */
int32_t sph_forces(const sph_params *p, const sph_particles *parts,
                   const int32_t *cell_start, const void *vel, void *acc_out, void *stream);

/* Bytes of the stored neighbour lists of sph_density_lists and
 * sph_forces_lists for these parameters; 0 when the lists cannot index this
 * many particles (2^28 in 2-D, 2^27 in 3-D) or would pass 2^31 bytes, and
 * the two calls then return SPH_E_UNSUPPORTED. */
int32_t sph_list_size(const sph_params *p, size_t *bytes);

/* sph_density (Eq. 8) that also records every particle's neighbours, in the
 * sweep's own visiting order, into lists (device, caller-owned, list_bytes
 * >= sph_list_size; an opaque layout) for sph_forces_lists at the same
 * positions.  rho_out equals sph_density's bit for bit.  The kick-drift-kick
 * runs do the same inside every step. */
int32_t sph_density_lists(const sph_params *p, const sph_particles *parts,
                          const int32_t *cell_start, void *rho_out, void *lists,
                          size_t list_bytes, void *stream);

/* sph_forces (Eq. 2, 3b, 5-7) over the lists sph_density_lists recorded for
 * the same sorted positions, cell_start and params: the sweep tests no
 * candidates.  acc_out equals sph_forces' bit for bit.  Lists of another
 * state give wrong accelerations (they are not checked). */
int32_t sph_forces_lists(const sph_params *p, const sph_particles *parts,
                         const int32_t *cell_start, const void *vel, void *acc_out,
                         const void *lists, size_t list_bytes, void *stream);

/* Wall particles (the lid-driven cavity of Sec. 4.2; the paper names no wall
 * treatment, this is the library's): params.n_wall > 0 marks the particles
 * with id >= n - n_wall as walls.  They stay where they are, take part in
 * every sum of the fluid particles as ordinary neighbours, and get no
 * correction, kick or drift; their acceleration is zero and the diagnostics
 * cover the fluid only.  sph_wall_state sets, for every wall particle a, from
 * its fluid neighbours f (kernel-weighted averages):
 *   p_a = sum_f p_f W_af / sum_f W_af,  rho_a = rho0 + p_a / c0^2,
 *   vel_a = 2 u_a - sum_f v_f W_af / sum_f W_af   (no-slip mirror),
 * with u_a = parts->wall_vel (p_a = 0, vel_a = u_a without fluid
 * neighbours).  It writes parts->rho and parts->vel of wall particles only
 * and reads those of fluid particles.  sph_kdk_step / sph_kdk_run call it
 * after each density summation; a caller evaluating sph_forces by hand calls
 * it between sph_density and sph_forces.  The box stays periodic: walls at
 * least 2 h_max thick keep the fluid from reaching across its seam.  Walled
 * runs are differentiable: their tapes also record the particle ids and each
 * wall's kernel sum and averaged fluid velocity, and the
 * adjoint entry points reverse the wall state too (the walls' density and
 * velocity cotangents go to their fluid neighbours, and to both sides'
 * positions); the walls' acceleration is not an output (its cotangent is
 * ignored) and their velocity before a step does not reach its outputs (its
 * cotangent comes back zero). */
int32_t sph_wall_state(const sph_params *p, sph_particles *parts, const int32_t *cell_start,
                       void *stream);

/* Transport-velocity correction in the formulation params.tv_mode (Eq. 14-16,
 * or Eq. 12 for SPH_TV_BACKGROUND), from positions and parts->rho:
 * dr_out[D][N]; beta_out [N] (optional) the limiter value (1 for the unlimited
 * formulations); s_out [N] FP64 (optional) h_min^2 |g|^2 (the limiter test is
 * made in FP64); g_out [D][N] (optional) the raw sum g.  */
int32_t sph_tv_correction(const sph_params *p, const sph_particles *parts,
                          const int32_t *cell_start, void *dr_out, void *beta_out,
                          double *s_out, void *g_out, void *stream);

/* One kick-drift-kick step n -> n+1 (steps 1-7 above) on a state that is
 * sorted with cell_start built and holds rho^n and a^n.  On return the
 * particle arrays hold step n+1 in (cell, id) order and cell_start matches.
 * step_index = n decides whether the correction applies (tv_every).  tape
 * (optional, sph_tape_size bytes) records what sph_adjoint_step needs.  diag
 * (optional, device, SPH_NDIAG doubles) receives the diagnostics. */
int32_t sph_kdk_step(const sph_params *p, sph_particles *parts, int32_t *cell_start,
                     int64_t step_index, void *ws, size_t ws_bytes, void *tape,
                     double *diag, void *stream);

/* nsteps consecutive kick-drift-kick steps from step index step_index, with
 * the same arithmetic as nsteps calls of sph_kdk_step (bit-identical
 * results), but fused across steps: the force sweep of step n also evaluates
 * the correction sum of step n+1 at the same positions and densities (the
 * pairs, kernel values and volumes of Eq. 14 are those of the force sum),
 * then applies the second half kick of step n and the first half kick,
 * correction and drift of step n+1.  tapes (optional, device, nsteps *
 * sph_tape_size bytes) receive one tape per step, byte-identical to those of
 * nsteps sph_kdk_step calls.  diag (optional, device) receives nsteps rows of
 * SPH_NDIAG doubles, one per step. */
int32_t sph_kdk_run(const sph_params *p, sph_particles *parts, int32_t *cell_start,
                    int64_t step_index, int64_t nsteps, void *ws, size_t ws_bytes,
                    void *tapes, double *diag, void *stream);

/* sph_kdk_run continuing a run: every sph_kdk_run or sph_kdk_step ends with
 * the force sweep that (as inside a run) also evaluates the next step's
 * correction and applies its first half kick and drift, into the workspace;
 * this call starts from there instead of evaluating the correction sweep of
 * its first step again.  Results are bit-identical to an uninterrupted run of
 * the same steps.  The caller guarantees that nothing has changed the
 * particle arrays, cell_start, the params or the workspace since the
 * previous sph_kdk_run / sph_kdk_step / sph_kdk_run_resume on this workspace
 * (that call ended at step step_index); this is not checked, and anything
 * else gives wrong results.  No tapes (use sph_kdk_run to record).  Same
 * arguments and errors as sph_kdk_run otherwise. */
int32_t sph_kdk_run_resume(const sph_params *p, sph_particles *parts, int32_t *cell_start,
                           int64_t step_index, int64_t nsteps, void *ws, size_t ws_bytes,
                           double *diag, void *stream);

/* sph_kdk_run without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the same kernels and arithmetic
 * (bit-identical results), with the run's scratch taken from a static device
 * array of SPH_STATIC_SCRATCH_BYTES that the library holds on every device it
 * runs on until the process ends.  The call allocates nothing; the caller
 * still owns and passes every input and output.  Runs whose
 * sph_workspace_size exceeds SPH_STATIC_SCRATCH_BYTES return SPH_E_TOO_LARGE
 * before anything is enqueued.  The array belongs to the device current at
 * the call (which must be the stream's device) and is shared by every call
 * on that device: calls that overlap on one device (concurrent streams or
 * host threads) race and must be serialised by the caller.
 * flags (optional, device, one uint32_t owned by the caller) is the device
 * flag word of the run: bits are ORed in, never cleared, and read and clear
 * with sph_get_flags(flags, stream, &host) / sph_clear_flags(flags, stream);
 * with flags == NULL the run's flags are not reported. */
int32_t sph_kdk_run_static(const sph_params *p, sph_particles *parts, int32_t *cell_start,
                           int64_t step_index, int64_t nsteps, void *tapes, double *diag,
                           uint32_t *flags, void *stream);

/* Dual-criteria time stepping (Sec. 2.4): CFL numbers of the advection and
 * acoustic criteria (Eq. 9 and 11: 0.25 and 0.6), the reference speed U_ref
 * and the kinematic viscosity nu of Eq. 10, and an optional cap on the
 * acoustic substeps of one advection step. */
typedef struct {
    double cfl_ad, cfl_ac;
    double u_ref;           /* > 0                                              */
    double nu;              /* eta / rho0, >= 0                                 */
    int32_t max_substeps;   /* 0: as many as the advection step needs (up to a
                               bound, see sph_dual_run); 1..64: end each
                               advection step after this many substeps even if
                               they do not cover it                            */
} sph_dual_params;

/* nsteps advection steps of the dual-criteria scheme (Sec. 2.3-2.4, Sec. 3)
 * on a sorted state with cell_start built (rho and acc on entry are not
 * used).  Each advection step:
 *   1. dt_ad = CFL_ad h_min / max(|v|_max, nu / h_min, U_ref)   (Eq. 9-10)
 *   2. the topology (cells, cell-local offsets and hence the neighbour pairs
 *      and their kernel values) of the step's start is kept through the step
 *   3. density by summation (Eq. 8)
 *   4. viscous acceleration (Eq. 7), held for the step
 *   5. the correction of Eq. 16 (SPH_TV_LIMITED) or Eq. 14 (SPH_TV_SCALED)
 *      at the step's start, added once to the displacement
 *   6. acoustic substeps of dt = min(CFL_ac h_min / (|v|_max + c0), dt_ad - t)
 *      (Eq. 11) until dt_ad is covered, each
 *        rho' = rho + dt/2 drho/dt,  v+ = v + dt (a^p + a^visc) with the
 *        Riemann pressure term of Eq. 3b, 5-6 at (rho', v),
 *        displacement += dt (v + v+)/2,
 *        drho/dt of Eq. 3a with U* of Eq. 5 at (rho', v+),
 *        rho+ = rho' + dt/2 drho/dt
 *      (the first substep's drho/dt is evaluated at the step's start)
 *   7. positions += displacement, rebinning, cell build.
 * The step sizes are computed on the device (FP64 maxima of |v|), so a run
 * never synchronises; the substeps are launched a fixed number of times per
 * step (the even number above max_substeps, or above the bound
 * ceil(CFL_ad / CFL_ac (2 + c0 / U_ref)) + 1, which covers every step whose
 * largest speed stays below twice max(|v|_max at its start, U_ref)); a
 * launch past the covering substeps does nothing.  A step the automatic
 * bound does not cover sets SPH_FLAG_CFL.  params.dt and tv_every are not
 * used; xi = 0 turns the correction off.  On return the particle arrays hold
 * the state after the last step in (cell, id) order: rho the density of the
 * last substep (not re-summed), acc overwritten.  diag (optional, device)
 * receives one row of SPH_NDIAG per step (KE, momentum, max|v| after it; the
 * pairs of its topology; limiter counts and max |dr| / dt_ad of its
 * correction); steps (optional, device, 3 doubles per step) dt_ad, the
 * substeps taken and the time they covered.  Walls and SPH_TV_BACKGROUND:
 * SPH_E_UNSUPPORTED. */
int32_t sph_dual_run(const sph_params *p, const sph_dual_params *q, sph_particles *parts,
                     int32_t *cell_start, int64_t nsteps, void *ws, size_t ws_bytes,
                     double *diag, double *steps, void *stream);

/* Diagnostics of the current state alone (KE, momentum, max|v|, pairs);
 * entries 6-8 are zero. */
int32_t sph_diagnostics(const sph_params *p, const sph_particles *parts,
                        const int32_t *cell_start, void *ws, size_t ws_bytes,
                        double *diag, void *stream);

/* Reverse of one sph_kdk_step recorded in `tape`.  On entry adj holds the
 * cotangents of step n+1 in step n+1's order; on return those of step n in
 * step n's order.  xi_bar (device, one double) is incremented by the
 * derivative with respect to xi (which SPH_TV_BACKGROUND does not use: no
 * contribution there).  The neighbour sets are taken as fixed (the
 * C2 kernel's value and first two derivatives vanish at the support edge);
 * the limiter jump at s0 has zero derivative. */
int32_t sph_adjoint_step(const sph_params *p, const void *tape, sph_adjoint *adj,
                         double *xi_bar, void *ws, size_t ws_bytes, void *stream);

/* Reverse of the initial evaluation rho^0 = R(r^0), a^0 = A(r^0, v^0, rho^0)
 * on the sorted initial state: adds A^T a_bar to (r_bar, v_bar, rho_bar) and
 * then R^T rho_bar to r_bar.  a_bar and rho_bar are consumed. */
int32_t sph_adjoint_init(const sph_params *p, const sph_particles *parts,
                         const int32_t *cell_start, sph_adjoint *adj, void *ws,
                         size_t ws_bytes, void *stream);

/* Per-particle neighbour counts |N(i)| (int32 [N]) of the current sorted
 * state. */
int32_t sph_neighbor_counts(const sph_params *p, const sph_particles *parts,
                            const int32_t *cell_start, int32_t *counts, void *stream);

/* ---- errors --------------------------------------------------------------- */

/* Synchronise `stream`, then read (and clear) the device flag word: the
 * first word of a workspace, or the flag word a caller passed to
 * sph_kdk_run_static. */
int32_t sph_get_flags(void *ws, void *stream, uint32_t *host_flags);

/* Clear the device flag word (asynchronous). */
int32_t sph_clear_flags(void *ws, void *stream);

const char *sph_status_string(int32_t status);

#ifdef __cplusplus
}
#endif

#endif /* SPH_H */
