/*
 * Plain FP64 CPU oracle for one transport-velocity WCSPH step
 * (Wang, Haidn & Hu, "The efficient implementation of transport velocity
 * formulation", arXiv 2411.13992).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library links, includes or
 * calls this file; it exists so that tests and the benchmark's CPU baseline
 * can check the GPU path against a slow, obviously correct statement of the
 * method.  It works on absolute FP64 positions in a periodic box, keeps
 * explicit neighbour lists, and takes every sum in plain index order.
 *
 * Layout: vector fields are structure-of-arrays, x[k*n + i] is component k of
 * particle i.  Every particle carries its own mass m_i and smoothing length h_i.
 *
 * Readings of the paper (where it is silent or ambiguous):
 *  - kernel: Wendland C2 with support radius 2h (Sec. 4 names "the Wendland
 *    kernel" with h = 1.3 dp but prints no form);
 *  - kernel gradient: grad_i W_ij = W'(r) (r_i - r_j)/r, the gradient with
 *    respect to r_i (the sign that makes Eq. 3b repulsive for positive P*);
 *  - Riemann axis: unit vector from i towards j, so U_l - U_r > 0 means the
 *    pair approaches (Eq. 4-6);
 *  - pair smoothing length h_ij = (h_i + h_j)/2; neighbours are j != i with
 *    r_ij < 2 h_ij (strict);
 *  - density (Eq. 8): rho_i = sum_{j incl. i} m_j W_ij / kappa_D, with kappa_D
 *    the perfect-lattice kernel sum times dx^D at h = 1.3 dx, so a perfect
 *    lattice has rho = rho0 exactly;
 *  - transport correction (Eq. 14-16): V_j = m_j / rho_j, h = h_min;
 *  - original correction in kick-drift-kick (Eq. 12 with p0 = rho0 c0^2): the
 *    extra transport acceleration a_t = -2 sum_j m_j p0/(rho_i rho_j) grad_i W_ij
 *    acts over the drift as dr = a_t dt^2 / 2 (the same half-acceleration-
 *    times-step-squared step that turns Eq. 12 into Eq. 14), so
 *    dr_i = -(p0 dt^2 / rho_i) g_i with g_i = sum_j V_j grad_i W_ij;
 *  - time integration: kick-drift-kick with fixed dt; the correction is added to
 *    the drift; forces use the half-step velocity;
 *  - walls (the lid-driven cavity of Sec. 4.2; the paper names no wall
 *    treatment): fixed wall particles on the fluid lattice, several layers
 *    thick, taking part in every sum of the fluid particles as ordinary
 *    neighbours.  Before each force evaluation every wall particle a gets a
 *    pressure and a velocity from its fluid neighbours f by kernel-weighted
 *    (Shepard) averages, p_a = sum p_f W_af / sum W_af, rho_a = rho0 + p_a/c0^2
 *    (EOS inverted), and the no-slip mirror v_a = 2 u_a - sum v_f W_af / sum
 *    W_af with u_a the prescribed wall velocity (p_a = 0, v_a = u_a without
 *    fluid neighbours).  Wall particles are not corrected, kicked or moved;
 *    the diagnostics cover the fluid only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_PI 3.14159265358979323846

typedef struct {
    double rho0;        /* reference density                          */
    double c0;          /* artificial sound speed (Eq. 2)             */
    double eta;         /* dynamic viscosity (Eq. 7)                  */
    double dt;          /* fixed time step                            */
    double xi;          /* correction coefficient, -0.2 (Eq. 14, 16)  */
    double lim_c;       /* limiter slope C = 1e3 (Eq. 15)             */
    double lim_s0;      /* limiter threshold 5e-4 (Eq. 15)            */
    double riemann_eta; /* Riemann dissipation limiter eta = 3 (Eq. 6)*/
    double h_min;       /* smallest smoothing length (Eq. 15-16)      */
    double kappa;       /* lattice kernel sum times dx^D              */
    double band_tol;    /* relative half-width of the limiter band    */
    int32_t tv_every;   /* apply the correction every k-th step       */
    int32_t use_grid;   /* 1: bucket neighbour search, 0: brute force */
    int32_t tv_mode;    /* ORACLE_TV_* below                          */
    int64_t n_wall;     /* the last n_wall particles are walls        */
    const double *wall_vel; /* [D][n_wall] prescribed wall velocity   */
} oracle_params;

/* Transport-velocity formulations */
#define ORACLE_TV_LIMITED 0    /* h-scaled with the limiter, Eq. (16)          */
#define ORACLE_TV_SCALED 1     /* h-scaled without limiter, Eq. (14)           */
#define ORACLE_TV_BACKGROUND 2 /* background pressure rho0 c0^2 in KDK, Eq. (12) */

/* ------------------------------------------------------------------ */
/* threads                                                             */
/* ------------------------------------------------------------------ */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Wendland C2 kernel, support 2h                                      */
/* ------------------------------------------------------------------ */
static double wendland_alpha(int dim, double h)
{
    if (dim == 2) return 7.0 / (4.0 * ORACLE_PI * h * h);
    return 21.0 / (16.0 * ORACLE_PI * h * h * h);
}

/* W(r, h) = alpha_D (1 - q/2)^4 (1 + 2q) for q = r/h < 2, else 0 */
double oracle_kernel_w(int dim, double r, double h)
{
    double q = r / h;
    if (q >= 2.0) return 0.0;
    double t = 1.0 - 0.5 * q;
    return wendland_alpha(dim, h) * t * t * t * t * (1.0 + 2.0 * q);
}

/* F(r, h) = W'(r) / r = -5 alpha_D (1 - q/2)^3 / h^2, finite at r = 0 */
double oracle_kernel_f(int dim, double r, double h)
{
    double q = r / h;
    if (q >= 2.0) return 0.0;
    double t = 1.0 - 0.5 * q;
    return -5.0 * wendland_alpha(dim, h) * t * t * t / (h * h);
}

/* Kernel sum over a perfect lattice of spacing 1 including the particle
 * itself, at h = h_over_dx: sum_k W(|k|, h_over_dx).  Multiplying by dx^D is
 * implicit (W scales as 1/h^D), so this is the dimensionless constant kappa_D. */
double oracle_lattice_kappa(int dim, double h_over_dx)
{
    int reach = (int)ceil(2.0 * h_over_dx) + 1;
    double sum = 0.0;
    for (int a = -reach; a <= reach; ++a)
        for (int b = -reach; b <= reach; ++b) {
            if (dim == 2) {
                sum += oracle_kernel_w(2, sqrt((double)(a * a + b * b)), h_over_dx);
            } else {
                for (int c = -reach; c <= reach; ++c)
                    sum += oracle_kernel_w(3, sqrt((double)(a * a + b * b + c * c)), h_over_dx);
            }
        }
    return sum;
}

/* ------------------------------------------------------------------ */
/* geometry                                                            */
/* ------------------------------------------------------------------ */
/* minimum-image component of r_i - r_j in a periodic box of edge b */
static double min_image(double d, double b)
{
    return d - b * round(d / b);
}

/* r_ij = r_i - r_j (minimum image), returns |r_ij| */
static double displacement(int dim, int64_t n, const double *pos, const double *box,
                           int64_t i, int64_t j, double *rij)
{
    double r2 = 0.0;
    for (int k = 0; k < dim; ++k) {
        rij[k] = min_image(pos[k * n + i] - pos[k * n + j], box[k]);
        r2 += rij[k] * rij[k];
    }
    return sqrt(r2);
}

static int is_neighbour(int dim, int64_t n, const double *pos, const double *h,
                        const double *box, int64_t i, int64_t j)
{
    double rij[3];
    if (i == j) return 0;
    double r = displacement(dim, n, pos, box, i, j, rij);
    double hij = 0.5 * (h[i] + h[j]);
    return r < 2.0 * hij;
}

/* ------------------------------------------------------------------ */
/* neighbour sets N(i) = { j != i : r_ij < 2 h_ij }, as CSR lists in   */
/* ascending j.  With list == NULL only start[] (n+1) is filled.       */
/* ------------------------------------------------------------------ */
int64_t oracle_neighbors_brute(int dim, int64_t n, const double *pos, const double *h,
                               const double *box, int64_t *start, int32_t *list)
{
    if (list == NULL) {
        start[0] = 0;
        for (int64_t i = 0; i < n; ++i) {
            int64_t c = 0;
            for (int64_t j = 0; j < n; ++j) c += is_neighbour(dim, n, pos, h, box, i, j);
            start[i + 1] = start[i] + c;
        }
        return start[n];
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        int64_t w = start[i];
        for (int64_t j = 0; j < n; ++j)
            if (is_neighbour(dim, n, pos, h, box, i, j)) list[w++] = (int32_t)j;
    }
    return start[n];
}

/* Bucket search: the same set as the brute-force definition, found by binning
 * particles into cells of edge >= 2 h_max and testing the 3^D surrounding
 * cells.  Falls back to brute force when a box axis holds fewer than 3 cells. */
typedef struct {
    int nc[3];
    int64_t ncells;
    int64_t *cstart;   /* ncells + 1 */
    int64_t *members;  /* n, particle ids grouped by cell, ascending within cell */
    int64_t *cellof;   /* n */
} bucket_grid;

static int build_grid(int dim, int64_t n, const double *pos, const double *h,
                      const double *box, bucket_grid *g)
{
    double hmax = 0.0;
    for (int64_t i = 0; i < n; ++i) if (h[i] > hmax) hmax = h[i];
    g->ncells = 1;
    for (int k = 0; k < 3; ++k) g->nc[k] = 1;
    for (int k = 0; k < dim; ++k) {
        g->nc[k] = (int)floor(box[k] / (2.0 * hmax));
        if (g->nc[k] < 3) return 0;
        g->ncells *= g->nc[k];
    }
    g->cstart = (int64_t *)calloc((size_t)g->ncells + 1, sizeof(int64_t));
    g->members = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    g->cellof = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        int64_t lin = 0, stride = 1;
        for (int k = 0; k < dim; ++k) {
            double lc = box[k] / g->nc[k];
            int64_t c = (int64_t)floor(pos[k * n + i] / lc);
            if (c < 0) c = 0;
            if (c >= g->nc[k]) c = g->nc[k] - 1;
            lin += c * stride;
            stride *= g->nc[k];
        }
        g->cellof[i] = lin;
        g->cstart[lin + 1]++;
    }
    for (int64_t c = 0; c < g->ncells; ++c) g->cstart[c + 1] += g->cstart[c];
    int64_t *fill = (int64_t *)malloc((size_t)g->ncells * sizeof(int64_t));
    memcpy(fill, g->cstart, (size_t)g->ncells * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) g->members[fill[g->cellof[i]]++] = i;
    free(fill);
    return 1;
}

static void free_grid(bucket_grid *g)
{
    free(g->cstart);
    free(g->members);
    free(g->cellof);
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* candidates of i: members of the 3^D cells around i's cell */
static int64_t grid_scan(int dim, int64_t n, const double *pos, const double *h,
                         const double *box, const bucket_grid *g, int64_t i, int32_t *out)
{
    int64_t c = g->cellof[i];
    int ci[3] = {0, 0, 0};
    int64_t rem = c;
    for (int k = 0; k < dim; ++k) { ci[k] = (int)(rem % g->nc[k]); rem /= g->nc[k]; }
    int64_t cnt = 0;
    int span2 = dim >= 3 ? 1 : 0;
    for (int dz = -span2; dz <= span2; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int cx = (ci[0] + dx + g->nc[0]) % g->nc[0];
                int cy = (ci[1] + dy + g->nc[1]) % g->nc[1];
                int cz = dim >= 3 ? (ci[2] + dz + g->nc[2]) % g->nc[2] : 0;
                int64_t lin = cx + (int64_t)g->nc[0] * (cy + (int64_t)g->nc[1] * cz);
                for (int64_t m = g->cstart[lin]; m < g->cstart[lin + 1]; ++m) {
                    int64_t j = g->members[m];
                    if (is_neighbour(dim, n, pos, h, box, i, j)) {
                        if (out) out[cnt] = (int32_t)j;
                        cnt++;
                    }
                }
            }
    if (out) qsort(out, (size_t)cnt, sizeof(int32_t), cmp_i32);
    return cnt;
}

int64_t oracle_neighbors_grid(int dim, int64_t n, const double *pos, const double *h,
                              const double *box, int64_t *start, int32_t *list)
{
    bucket_grid g;
    if (!build_grid(dim, n, pos, h, box, &g)) {
        /* build_grid allocates nothing when it declines */
        return oracle_neighbors_brute(dim, n, pos, h, box, start, list);
    }
    if (list == NULL) {
        int64_t *cnt = (int64_t *)malloc((size_t)n * sizeof(int64_t));
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) cnt[i] = grid_scan(dim, n, pos, h, box, &g, i, NULL);
        start[0] = 0;
        for (int64_t i = 0; i < n; ++i) start[i + 1] = start[i] + cnt[i];
        free(cnt);
    } else {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) grid_scan(dim, n, pos, h, box, &g, i, list + start[i]);
    }
    free_grid(&g);
    return start[n];
}

/* ------------------------------------------------------------------ */
/* Density summation, Eq. (8): rho_i = sum_{j in N(i) + i} m_j W_ij / kappa */
/* ------------------------------------------------------------------ */
void oracle_density(int dim, int64_t n, const double *pos, const double *mass,
                    const double *h, const double *box, const int64_t *start,
                    const int32_t *list, double kappa, double *rho)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double sum = mass[i] * oracle_kernel_w(dim, 0.0, h[i]);
        for (int64_t e = start[i]; e < start[i + 1]; ++e) {
            int64_t j = list[e];
            double rij[3];
            double r = displacement(dim, n, pos, box, i, j, rij);
            sum += mass[j] * oracle_kernel_w(dim, r, 0.5 * (h[i] + h[j]));
        }
        rho[i] = sum / kappa;
    }
}

/* ------------------------------------------------------------------ */
/* Transport-velocity correction, Eq. (12), (14)-(16)                  */
/*   g_i    = sum_j V_j grad_i W_ij,  V_j = m_j / rho_j                 */
/*   s_i    = h_min^2 |g_i|^2                                          */
/* limited (Eq. 15-16):                                                */
/*   beta_i = min(C s_i, 1) if s_i > s0 else 0                         */
/*   dr_i   = xi beta_i h_min^2 g_i                                    */
/* scaled, no limiter (Eq. 14): beta_i = 1, dr_i = xi h_min^2 g_i       */
/* background pressure in KDK (Eq. 12): beta_i = 1,                     */
/*   dr_i   = -(bg / rho_i) g_i,  bg = p0 dt^2 = rho0 c0^2 dt^2         */
/* gscale_i = sum_j |V_j grad_i W_ij| (the summation-error scale)      */
/* ------------------------------------------------------------------ */
void oracle_tv(int dim, int64_t n, const double *pos, const double *mass,
               const double *rho, const double *h, const double *box,
               const int64_t *start, const int32_t *list, double h_min, double xi,
               double lim_c, double lim_s0, int tv_mode, double bg, double *g, double *s,
               double *beta, double *dr, double *gscale)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double gi[3] = {0.0, 0.0, 0.0};
        double scale = 0.0;
        for (int64_t e = start[i]; e < start[i + 1]; ++e) {
            int64_t j = list[e];
            double rij[3];
            double r = displacement(dim, n, pos, box, i, j, rij);
            double f = oracle_kernel_f(dim, r, 0.5 * (h[i] + h[j]));
            double vj = mass[j] / rho[j];
            double mag = 0.0;
            for (int k = 0; k < dim; ++k) {
                double t = vj * f * rij[k];
                gi[k] += t;
                mag += t * t;
            }
            scale += sqrt(mag);
        }
        double g2 = 0.0;
        for (int k = 0; k < dim; ++k) g2 += gi[k] * gi[k];
        double si = h_min * h_min * g2;
        double bi, coef;
        if (tv_mode == ORACLE_TV_LIMITED) {
            bi = 0.0;
            if (si > lim_s0) bi = fmin(lim_c * si, 1.0);
            coef = xi * bi * h_min * h_min;
        } else if (tv_mode == ORACLE_TV_SCALED) {
            bi = 1.0;
            coef = xi * h_min * h_min;
        } else {
            bi = 1.0;
            coef = -bg / rho[i];
        }
        for (int k = 0; k < dim; ++k) {
            if (g) g[k * n + i] = gi[k];
            if (dr) dr[k * n + i] = coef * gi[k];
        }
        if (s) s[i] = si;
        if (beta) beta[i] = bi;
        if (gscale) gscale[i] = scale;
    }
}

/* ------------------------------------------------------------------ */
/* Pressure + viscous accelerations, Eq. (2), (3b), (5)-(7)           */
/*   p = c0^2 (rho - rho0)                                              */
/*   e_ij = (r_j - r_i)/r, U_l = v_i.e, U_r = v_j.e                     */
/*   beta^R = min(eta_R max((U_l - U_r)/c0, 0), 1)                      */
/*   Pstar = (p_i + p_j)/2 + beta^R rhobar c0 (U_l - U_r) / 2          */
/*   a_i = sum_j -2 m_j Pstar (rho_i rho_j)^-1 grad_i W_ij              */
/*              + 2 m_j eta (rho_i rho_j)^-1 (v_i - v_j) F_ij           */
/* ascale_i = sum_j |term_ij|                                          */
/* ------------------------------------------------------------------ */
void oracle_forces(int dim, int64_t n, const double *pos, const double *vel,
                   const double *mass, const double *rho, const double *h,
                   const double *box, const int64_t *start, const int32_t *list,
                   double rho0, double c0, double eta, double riemann_eta,
                   double *acc, double *ascale)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double ai[3] = {0.0, 0.0, 0.0};
        double scale = 0.0;
        double pi_ = c0 * c0 * (rho[i] - rho0);
        for (int64_t e = start[i]; e < start[i + 1]; ++e) {
            int64_t j = list[e];
            double rij[3];
            double r = displacement(dim, n, pos, box, i, j, rij);
            double f = oracle_kernel_f(dim, r, 0.5 * (h[i] + h[j]));
            double pj = c0 * c0 * (rho[j] - rho0);
            double du = 0.0; /* U_l - U_r */
            if (r > 0.0) {
                for (int k = 0; k < dim; ++k) {
                    double ek = -rij[k] / r;
                    du += (vel[k * n + i] - vel[k * n + j]) * ek;
                }
            }
            double beta_r = fmin(riemann_eta * fmax(du / c0, 0.0), 1.0);
            double rhobar = 0.5 * (rho[i] + rho[j]);
            double pstar = 0.5 * (pi_ + pj) + 0.5 * beta_r * rhobar * c0 * du;
            double coef = 2.0 * mass[j] / (rho[i] * rho[j]);
            double mag = 0.0;
            for (int k = 0; k < dim; ++k) {
                double t = -coef * pstar * f * rij[k]
                           + coef * eta * (vel[k * n + i] - vel[k * n + j]) * f;
                ai[k] += t;
                mag += t * t;
            }
            scale += sqrt(mag);
        }
        for (int k = 0; k < dim; ++k) acc[k * n + i] = ai[k];
        if (ascale) ascale[i] = scale;
    }
}

/* ------------------------------------------------------------------ */
/* Wall particles a = n - n_wall .. n-1 from their fluid neighbours:  */
/*   S = sum_f W_af, p_a = sum_f p_f W_af / S, vbar = sum_f v_f W_af / S */
/*   rho_a = rho0 + p_a / c0^2,  v_a = 2 u_a - vbar                    */
/* (p_a = 0 and vbar = u_a when S = 0).  Writes rho and vel of walls. */
/* ------------------------------------------------------------------ */
void oracle_wall_bc(int dim, int64_t n, int64_t n_wall, const double *pos, const double *h,
                    const double *box, const int64_t *start, const int32_t *list,
                    double rho0, double c0, const double *wall_vel, double *rho, double *vel)
{
    int64_t nf = n - n_wall;
#pragma omp parallel for schedule(static)
    for (int64_t a = nf; a < n; ++a) {
        double S = 0.0, P = 0.0, V[3] = {0.0, 0.0, 0.0};
        for (int64_t e = start[a]; e < start[a + 1]; ++e) {
            int64_t f = list[e];
            if (f >= nf) continue;
            double raf[3];
            double r = displacement(dim, n, pos, box, a, f, raf);
            double w = oracle_kernel_w(dim, r, 0.5 * (h[a] + h[f]));
            S += w;
            P += c0 * c0 * (rho[f] - rho0) * w;
            for (int k = 0; k < dim; ++k) V[k] += vel[k * n + f] * w;
        }
        double pa = S > 0.0 ? P / S : 0.0;
        rho[a] = rho0 + pa / (c0 * c0);
        for (int k = 0; k < dim; ++k) {
            double ua = wall_vel[k * n_wall + (a - nf)];
            vel[k * n + a] = 2.0 * ua - (S > 0.0 ? V[k] / S : ua);
        }
    }
}

/* ------------------------------------------------------------------ */
/* neighbour list helper for the step: malloc'd CSR                   */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t *start;
    int32_t *list;
    int64_t npairs;
} nbr_lists;

static void make_lists(int dim, int64_t n, const double *pos, const double *h,
                       const double *box, int use_grid, nbr_lists *nl)
{
    nl->start = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    if (use_grid) nl->npairs = oracle_neighbors_grid(dim, n, pos, h, box, nl->start, NULL);
    else nl->npairs = oracle_neighbors_brute(dim, n, pos, h, box, nl->start, NULL);
    nl->list = (int32_t *)malloc((size_t)(nl->npairs > 0 ? nl->npairs : 1) * sizeof(int32_t));
    if (use_grid) oracle_neighbors_grid(dim, n, pos, h, box, nl->start, nl->list);
    else oracle_neighbors_brute(dim, n, pos, h, box, nl->start, nl->list);
}

static void free_lists(nbr_lists *nl)
{
    free(nl->start);
    free(nl->list);
}

/* zero the [D][N] field f on the wall particles */
static void zero_walls(int dim, int64_t n, int64_t n_wall, double *f)
{
    if (!f) return;
    for (int k = 0; k < dim; ++k)
        for (int64_t a = n - n_wall; a < n; ++a) f[k * n + a] = 0.0;
}

/* ------------------------------------------------------------------ */
/* initial state: rho^0 by summation, a^0 from the initial velocity    */
/* (walls: their state from the fluid before the forces)              */
/* ------------------------------------------------------------------ */
void oracle_init(int dim, int64_t n, const double *pos, double *vel,
                 const double *mass, const double *h, const double *box,
                 const oracle_params *p, double *rho, double *acc)
{
    nbr_lists nl;
    make_lists(dim, n, pos, h, box, p->use_grid, &nl);
    oracle_density(dim, n, pos, mass, h, box, nl.start, nl.list, p->kappa, rho);
    if (p->n_wall > 0)
        oracle_wall_bc(dim, n, p->n_wall, pos, h, box, nl.start, nl.list, p->rho0, p->c0,
                       p->wall_vel, rho, (double *)vel);
    oracle_forces(dim, n, pos, vel, mass, rho, h, box, nl.start, nl.list,
                  p->rho0, p->c0, p->eta, p->riemann_eta, acc, NULL);
    zero_walls(dim, n, p->n_wall, acc);
    free_lists(&nl);
}

/* Diagnostics of a state (fluid particles), plain sequential FP64 sums:
 * diag[0] KE = 1/2 sum m |v|^2, diag[1..3] momentum, diag[4] max|v|,
 * diag[5] ordered neighbour pairs, diag[6] count(beta > 0),
 * diag[7] count of limiter-band particles, diag[8] max |dr| / dt. */
#define ORACLE_NDIAG 9

static void diagnostics(int dim, int64_t n, const double *vel, const double *mass,
                        int64_t npairs, const double *beta, const double *s,
                        const double *dr, const oracle_params *p, double *diag)
{
    double ke = 0.0, mom[3] = {0.0, 0.0, 0.0}, vmax = 0.0, drmax = 0.0;
    int64_t nbeta = 0, nband = 0;
    for (int64_t i = 0; i < n - p->n_wall; ++i) {
        double v2 = 0.0;
        for (int k = 0; k < dim; ++k) {
            double v = vel[k * n + i];
            v2 += v * v;
            mom[k] += mass[i] * v;
        }
        ke += 0.5 * mass[i] * v2;
        if (sqrt(v2) > vmax) vmax = sqrt(v2);
        if (beta && beta[i] > 0.0) nbeta++;
        if (s && fabs(s[i] - p->lim_s0) <= p->band_tol * p->lim_s0) nband++;
        if (dr) {
            double d2 = 0.0;
            for (int k = 0; k < dim; ++k) d2 += dr[k * n + i] * dr[k * n + i];
            if (sqrt(d2) > drmax) drmax = sqrt(d2);
        }
    }
    diag[0] = ke;
    diag[1] = mom[0];
    diag[2] = mom[1];
    diag[3] = mom[2];
    diag[4] = vmax;
    diag[5] = (double)npairs;
    diag[6] = (double)nbeta;
    diag[7] = (double)nband;
    diag[8] = drmax / p->dt;
}

/* ------------------------------------------------------------------ */
/* One kick-drift-kick step n -> n+1 with the transport correction.    */
/* pos, vel, acc, rho hold step n on entry and step n+1 on return.     */
/* Optional outputs (NULL to skip) are the correction at step n:       */
/* dr [D][N], beta [N], s [N], g [D][N].                               */
/* ------------------------------------------------------------------ */
void oracle_kdk_step(int dim, int64_t n, double *pos, double *vel, double *acc,
                     double *rho, const double *mass, const double *h, const double *box,
                     const oracle_params *p, int64_t step_index, double *dr_out,
                     double *beta_out, double *s_out, double *g_out, double *diag)
{
    size_t dn = (size_t)dim * (size_t)n;
    double *dr = (double *)calloc(dn, sizeof(double));
    double *beta = (double *)calloc((size_t)n, sizeof(double));
    double *s = (double *)calloc((size_t)n, sizeof(double));
    double *g = (double *)calloc(dn, sizeof(double));
    nbr_lists nl;

    int64_t nf = n - p->n_wall;

    /* 1. transport correction at r^n with rho^n (none for walls) */
    make_lists(dim, n, pos, h, box, p->use_grid, &nl);
    if (p->tv_every > 0 && step_index % p->tv_every == 0)
        oracle_tv(dim, n, pos, mass, rho, h, box, nl.start, nl.list, p->h_min, p->xi,
                  p->lim_c, p->lim_s0, p->tv_mode, p->rho0 * p->c0 * p->c0 * p->dt * p->dt,
                  g, s, beta, dr, NULL);
    free_lists(&nl);
    zero_walls(dim, n, p->n_wall, dr);
    zero_walls(dim, n, p->n_wall, g);
    zero_walls(1, n, p->n_wall, beta);
    zero_walls(1, n, p->n_wall, s);

    /* 2. half kick, 3. drift with the correction, wrapped into the box
     * (fluid only: walls keep position and velocity) */
    for (int64_t i = 0; i < nf; ++i)
        for (int k = 0; k < dim; ++k) {
            size_t a = (size_t)k * n + i;
            vel[a] = vel[a] + 0.5 * p->dt * acc[a];
            double x = pos[a] + p->dt * vel[a] + dr[a];
            x = x - box[k] * floor(x / box[k]);
            if (x >= box[k]) x -= box[k];
            pos[a] = x;
        }

    /* 4. density at r^{n+1}; walls from the fluid (density, half-step
     * velocity); 5-6. forces with the half-step velocity */
    make_lists(dim, n, pos, h, box, p->use_grid, &nl);
    oracle_density(dim, n, pos, mass, h, box, nl.start, nl.list, p->kappa, rho);
    if (p->n_wall > 0)
        oracle_wall_bc(dim, n, p->n_wall, pos, h, box, nl.start, nl.list, p->rho0, p->c0,
                       p->wall_vel, rho, vel);
    oracle_forces(dim, n, pos, vel, mass, rho, h, box, nl.start, nl.list,
                  p->rho0, p->c0, p->eta, p->riemann_eta, acc, NULL);
    zero_walls(dim, n, p->n_wall, acc);

    /* 7. second half kick (fluid) */
    for (int k = 0; k < dim; ++k)
        for (int64_t i = 0; i < nf; ++i) {
            size_t a = (size_t)k * n + i;
            vel[a] = vel[a] + 0.5 * p->dt * acc[a];
        }

    /* 8. diagnostics of the new state (pairs at r^{n+1}, correction at r^n) */
    if (diag) diagnostics(dim, n, vel, mass, nl.npairs, beta, s, dr, p, diag);
    free_lists(&nl);

    if (dr_out) memcpy(dr_out, dr, dn * sizeof(double));
    if (beta_out) memcpy(beta_out, beta, (size_t)n * sizeof(double));
    if (s_out) memcpy(s_out, s, (size_t)n * sizeof(double));
    if (g_out) memcpy(g_out, g, dn * sizeof(double));
    free(dr);
    free(beta);
    free(s);
    free(g);
}

/* nsteps consecutive steps starting at step index step0; diag may be NULL or
 * hold nsteps * 9 doubles */
void oracle_run(int dim, int64_t n, double *pos, double *vel, double *acc, double *rho,
                const double *mass, const double *h, const double *box,
                const oracle_params *p, int64_t step0, int64_t nsteps, double *diag)
{
    for (int64_t s = 0; s < nsteps; ++s)
        oracle_kdk_step(dim, n, pos, vel, acc, rho, mass, h, box, p, step0 + s,
                        NULL, NULL, NULL, NULL, diag ? diag + ORACLE_NDIAG * s : NULL);
}

/* ================================================================== */
/* Dual-criteria time stepping (Sec. 2.4, Eq. 9-11) with the          */
/* continuity equation (Eq. 3a) and the Riemann solver (Eq. 5-6).     */
/*                                                                    */
/* One advection step of size dt_ad:                                  */
/*  1. dt_ad = CFL_ad h_min / |v|_ad, |v|_ad = max(|v|_max,           */
/*     max(nu / h_min, U_ref))                           (Eq. 9-10)   */
/*  2. topology at the current positions r0: the neighbour sets and   */
/*     the pair geometry (r_ij, F_ij = W'(r_ij)/r_ij) are fixed for   */
/*     the whole advection step (the advection criterion updates the  */
/*     topology, the acoustic one pressure and density)               */
/*  3. density reinitialised by summation                  (Eq. 8)    */
/*  4. viscous acceleration (Eq. 7), held over the step               */
/*  5. transport-velocity correction at r0 (Eq. 14 or 16), applied    */
/*     once to the positions                                          */
/*  6. acoustic substeps until the step is covered, each of size      */
/*     dt = min(CFL_ac h_min / (|v|_max + c0), dt_ad - t)  (Eq. 11)   */
/*     in a Verlet (half density, full velocity, half density) form:  */
/*       rho' = rho + dt/2 drho/dt                                    */
/*       v^+  = v + dt (a^p(rho', v) + a^visc)        (Eq. 3b, 5-6)   */
/*       r   += dt (v + v^+) / 2                                      */
/*       drho/dt = continuity at (rho', v^+)          (Eq. 3a, 5)     */
/*       rho^+ = rho' + dt/2 drho/dt                                  */
/*     with drho/dt before the first substep evaluated at the          */
/*     reinitialised density and the step's initial velocity.         */
/* Continuity with U* of Eq. 5 (e_ij from i to j, U_l - U_r > 0 when   */
/* approaching):                                                      */
/*   drho_i/dt = 2 rho_i sum_j V_j (U*_ij - v_i.e_ij) W'_ij           */
/*             = rho_i sum_j V_j F_ij [ v_ij.r_ij                     */
/*                                      + (p_i - p_j) r_ij / (rhobar c0) ] */
/* ================================================================== */
typedef struct {
    double cfl_ad;          /* 0.25 (Eq. 9)                                   */
    double cfl_ac;          /* 0.6 (Eq. 11)                                   */
    double u_ref;           /* reference speed U_ref (Eq. 10)                 */
    double nu;              /* kinematic viscosity eta / rho0 (Eq. 10)        */
    int32_t max_substeps;   /* > 0: end the advection step after this many
                               substeps even if dt_ad is not covered          */
    int32_t refresh_geometry; /* 1: pair geometry follows the particles through
                               the substeps (neighbour sets still fixed)      */
} oracle_dual_params;

/* Eq. 9-10 */
double oracle_dt_advection(double vmax, double h_min, const oracle_dual_params *q)
{
    double vad = fmax(vmax, fmax(q->nu / h_min, q->u_ref));
    return q->cfl_ad * h_min / vad;
}

/* Eq. 11 */
double oracle_dt_acoustic(double vmax, double h_min, double c0, const oracle_dual_params *q)
{
    return q->cfl_ac * h_min / (vmax + c0);
}

/* pair geometry of CSR neighbour lists at fixed positions */
typedef struct {
    double *rij;   /* [3][P]  r_i - r_j (minimum image)           */
    double *r;     /* [P]     |r_ij|                              */
    double *f;     /* [P]     F = W'(r)/r with h_ij               */
} pair_geometry;

static void make_geometry(int dim, int64_t n, const double *pos, const double *h,
                          const double *box, const int64_t *start, const int32_t *list,
                          pair_geometry *pg)
{
    int64_t np = start[n];
    size_t m = (size_t)(np > 0 ? np : 1);
    pg->rij = (double *)malloc(3 * m * sizeof(double));
    pg->r = (double *)malloc(m * sizeof(double));
    pg->f = (double *)malloc(m * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = start[i]; e < start[i + 1]; ++e) {
            int64_t j = list[e];
            double d[3] = {0.0, 0.0, 0.0};
            double r = displacement(dim, n, pos, box, i, j, d);
            for (int k = 0; k < 3; ++k) pg->rij[(size_t)k * m + e] = d[k];
            pg->r[e] = r;
            pg->f[e] = oracle_kernel_f(dim, r, 0.5 * (h[i] + h[j]));
        }
}

static void free_geometry(pair_geometry *pg)
{
    free(pg->rij);
    free(pg->r);
    free(pg->f);
}

#define GEO_R(pg, np, k, e) ((pg)->rij[(size_t)(k) * (size_t)((np) > 0 ? (np) : 1) + (e)])

/* drho/dt of Eq. 3a with U* of Eq. 5 on fixed pair geometry */
static void continuity_geo(int dim, int64_t n, const int64_t *start, const int32_t *list,
                           const pair_geometry *pg, const double *vel, const double *mass,
                           const double *rho, double rho0, double c0, double *drho)
{
    int64_t np = start[n];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double sum = 0.0;
        double pi_ = c0 * c0 * (rho[i] - rho0);
        for (int64_t e = start[i]; e < start[i + 1]; ++e) {
            int64_t j = list[e];
            double vr = 0.0;
            for (int k = 0; k < dim; ++k)
                vr += (vel[k * n + i] - vel[k * n + j]) * GEO_R(pg, np, k, e);
            double pj = c0 * c0 * (rho[j] - rho0);
            double rhobar = 0.5 * (rho[i] + rho[j]);
            double term = vr + (pi_ - pj) * pg->r[e] / (rhobar * c0);
            sum += mass[j] / rho[j] * pg->f[e] * term;
        }
        drho[i] = rho[i] * sum;
    }
}

/* pressure acceleration of Eq. 3b with P* of Eq. 5-6 on fixed geometry */
static void pressure_geo(int dim, int64_t n, const int64_t *start, const int32_t *list,
                         const pair_geometry *pg, const double *vel, const double *mass,
                         const double *rho, double rho0, double c0, double riemann_eta,
                         double *acc)
{
    int64_t np = start[n];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double ai[3] = {0.0, 0.0, 0.0};
        double pi_ = c0 * c0 * (rho[i] - rho0);
        for (int64_t e = start[i]; e < start[i + 1]; ++e) {
            int64_t j = list[e];
            double r = pg->r[e];
            double du = 0.0;
            if (r > 0.0)
                for (int k = 0; k < dim; ++k)
                    du += (vel[k * n + i] - vel[k * n + j]) * (-GEO_R(pg, np, k, e) / r);
            double beta_r = fmin(riemann_eta * fmax(du / c0, 0.0), 1.0);
            double pj = c0 * c0 * (rho[j] - rho0);
            double rhobar = 0.5 * (rho[i] + rho[j]);
            double pstar = 0.5 * (pi_ + pj) + 0.5 * beta_r * rhobar * c0 * du;
            double coef = 2.0 * mass[j] / (rho[i] * rho[j]);
            for (int k = 0; k < dim; ++k) ai[k] += -coef * pstar * pg->f[e] * GEO_R(pg, np, k, e);
        }
        for (int k = 0; k < dim; ++k) acc[k * n + i] = ai[k];
    }
}

/* viscous acceleration of Eq. 7 on fixed geometry */
static void viscous_geo(int dim, int64_t n, const int64_t *start, const int32_t *list,
                        const pair_geometry *pg, const double *vel, const double *mass,
                        const double *rho, double eta, double *acc)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double ai[3] = {0.0, 0.0, 0.0};
        for (int64_t e = start[i]; e < start[i + 1]; ++e) {
            int64_t j = list[e];
            double coef = 2.0 * mass[j] * eta / (rho[i] * rho[j]) * pg->f[e];
            for (int k = 0; k < dim; ++k) ai[k] += coef * (vel[k * n + i] - vel[k * n + j]);
        }
        for (int k = 0; k < dim; ++k) acc[k * n + i] = ai[k];
    }
}

/* Eq. 3a with U* of Eq. 5 at the given positions (for checks) */
void oracle_continuity(int dim, int64_t n, const double *pos, const double *vel,
                       const double *mass, const double *rho, const double *h,
                       const double *box, const int64_t *start, const int32_t *list,
                       double rho0, double c0, double *drho)
{
    pair_geometry pg;
    make_geometry(dim, n, pos, h, box, start, list, &pg);
    continuity_geo(dim, n, start, list, &pg, vel, mass, rho, rho0, c0, drho);
    free_geometry(&pg);
}

static double max_speed(int dim, int64_t n, const double *vel)
{
    double vmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double v2 = 0.0;
        for (int k = 0; k < dim; ++k) v2 += vel[k * n + i] * vel[k * n + i];
        if (sqrt(v2) > vmax) vmax = sqrt(v2);
    }
    return vmax;
}

static void wrap_positions(int dim, int64_t n, double *pos, const double *box)
{
    for (int k = 0; k < dim; ++k)
        for (int64_t i = 0; i < n; ++i) {
            size_t a = (size_t)k * n + i;
            double x = pos[a] - box[k] * floor(pos[a] / box[k]);
            if (x >= box[k]) x -= box[k];
            pos[a] = x;
        }
}

/* One advection step (steps 1-6 above) of a wall-free state.  pos and vel
 * hold the state on entry and after the step on return; rho receives the
 * density after the last substep.  info (optional, 3 doubles): dt_ad, the
 * number of substeps, the time advanced.  dt_sub (optional, max_substeps or
 * 64 doubles): the substep sizes.  dr_out / beta_out / s_out (optional): the
 * correction at r0.  diag (optional): the 9 diagnostics of the new state (KE,
 * momentum, max|v|, the pairs of the step's topology, the limiter counts and
 * max |dr| / dt_ad).  Returns the number of substeps. */
int64_t oracle_dual_step(int dim, int64_t n, double *pos, double *vel, double *rho,
                         const double *mass, const double *h, const double *box,
                         const oracle_params *p, const oracle_dual_params *q, double *info,
                         double *dt_sub, double *dr_out, double *beta_out, double *s_out,
                         double *diag)
{
    size_t dn = (size_t)dim * (size_t)n;
    double *visc = (double *)calloc(dn > 0 ? dn : 1, sizeof(double));
    double *ap = (double *)calloc(dn > 0 ? dn : 1, sizeof(double));
    double *vnew = (double *)calloc(dn > 0 ? dn : 1, sizeof(double));
    double *dr = (double *)calloc(dn > 0 ? dn : 1, sizeof(double));
    double *g = (double *)calloc(dn > 0 ? dn : 1, sizeof(double));
    double *beta = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *s = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *drho = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *rhoh = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));

    /* 1. advection step size */
    double dt_ad = oracle_dt_advection(max_speed(dim, n, vel), p->h_min, q);

    /* 2. topology at r0, 3. density by summation */
    nbr_lists nl;
    make_lists(dim, n, pos, h, box, p->use_grid, &nl);
    pair_geometry pg;
    make_geometry(dim, n, pos, h, box, nl.start, nl.list, &pg);
    oracle_density(dim, n, pos, mass, h, box, nl.start, nl.list, p->kappa, rho);

    /* 4. viscous acceleration, held */
    viscous_geo(dim, n, nl.start, nl.list, &pg, vel, mass, rho, p->eta, visc);

    /* 5. correction at r0 (limited Eq. 16 or unlimited Eq. 14), applied once */
    oracle_tv(dim, n, pos, mass, rho, h, box, nl.start, nl.list, p->h_min, p->xi, p->lim_c,
              p->lim_s0, p->tv_mode, 0.0, g, s, beta, dr, NULL);
    for (size_t a = 0; a < dn; ++a) pos[a] += dr[a];
    wrap_positions(dim, n, pos, box);

    /* 6. acoustic substeps */
    continuity_geo(dim, n, nl.start, nl.list, &pg, vel, mass, rho, p->rho0, p->c0, drho);
    double t = 0.0;
    int64_t nsub = 0;
    while (t < dt_ad && (q->max_substeps <= 0 || nsub < q->max_substeps)) {
        double dt = fmin(oracle_dt_acoustic(max_speed(dim, n, vel), p->h_min, p->c0, q),
                         dt_ad - t);
        if (dt_sub && nsub < (q->max_substeps > 0 ? q->max_substeps : 64)) dt_sub[nsub] = dt;
        for (int64_t i = 0; i < n; ++i) rhoh[i] = rho[i] + 0.5 * dt * drho[i];
        if (q->refresh_geometry) {
            /* pressure at r + dt/2 v */
            double *ph = (double *)malloc((dn > 0 ? dn : 1) * sizeof(double));
            for (size_t a = 0; a < dn; ++a) ph[a] = pos[a] + 0.5 * dt * vel[a];
            free_geometry(&pg);
            make_geometry(dim, n, ph, h, box, nl.start, nl.list, &pg);
            free(ph);
        }
        pressure_geo(dim, n, nl.start, nl.list, &pg, vel, mass, rhoh, p->rho0, p->c0,
                     p->riemann_eta, ap);
        for (size_t a = 0; a < dn; ++a) {
            vnew[a] = vel[a] + dt * (ap[a] + visc[a]);
            pos[a] += 0.5 * dt * (vel[a] + vnew[a]);
        }
        memcpy(vel, vnew, dn * sizeof(double));
        if (q->refresh_geometry) {
            free_geometry(&pg);
            make_geometry(dim, n, pos, h, box, nl.start, nl.list, &pg);
        }
        continuity_geo(dim, n, nl.start, nl.list, &pg, vel, mass, rhoh, p->rho0, p->c0, drho);
        for (int64_t i = 0; i < n; ++i) rho[i] = rhoh[i] + 0.5 * dt * drho[i];
        t += dt;
        nsub++;
    }
    wrap_positions(dim, n, pos, box);

    if (info) {
        info[0] = dt_ad;
        info[1] = (double)nsub;
        info[2] = t;
    }
    if (diag) {
        oracle_params pd = *p;
        pd.dt = dt_ad;        /* transport speed |dr| / dt_ad */
        pd.n_wall = 0;
        diagnostics(dim, n, vel, mass, nl.npairs, beta, s, dr, &pd, diag);
    }
    if (dr_out) memcpy(dr_out, dr, dn * sizeof(double));
    if (beta_out) memcpy(beta_out, beta, (size_t)n * sizeof(double));
    if (s_out) memcpy(s_out, s, (size_t)n * sizeof(double));
    free_geometry(&pg);
    free_lists(&nl);
    free(visc);
    free(ap);
    free(vnew);
    free(dr);
    free(g);
    free(beta);
    free(s);
    free(drho);
    free(rhoh);
    return nsub;
}
