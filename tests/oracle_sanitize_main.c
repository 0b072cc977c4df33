/*
 * Host-only driver for a sanitizer build of the FP64 oracle (test
 * infrastructure).  tests/test_oracle_sanitize.py compiles this file, which
 * includes the oracle's single source, with -fsanitize=address,undefined and
 * runs it: every code path of the oracle is exercised on small inputs
 * (kernel and lattice sums, brute-force and bucket neighbour search in 2-D
 * and 3-D, the sweeps, the Taylor-Green step with each correction
 * formulation and tv_every > 1, and a walled box), with a few sanity checks
 * so that a silent wrong answer also fails.  Exit status 0 means clean.
 */
#include <stdio.h>

#include "../oracle/sph_oracle.c"

static int failures = 0;

#define CHECK(cond, what)                                   \
    do {                                                    \
        if (!(cond)) {                                      \
            fprintf(stderr, "check failed: %s\n", what);    \
            failures++;                                     \
        }                                                   \
    } while (0)

/* cell-centred n^dim lattice of spacing 1/n in [0,1)^dim, x fastest, with a
 * deterministic jitter of amplitude amp * dx (a fixed integer hash) */
static void lattice(int dim, int n, double amp, double *pos)
{
    int64_t np = dim == 2 ? (int64_t)n * n : (int64_t)n * n * n;
    double dx = 1.0 / n;
    for (int64_t id = 0; id < np; ++id) {
        int64_t rem = id;
        for (int k = 0; k < dim; ++k) {
            int64_t ik = rem % n;
            rem /= n;
            uint32_t hsh = (uint32_t)(id * 2654435761u + (uint32_t)k * 40503u);
            hsh ^= hsh >> 13;
            hsh *= 0x5bd1e995u;
            hsh ^= hsh >> 15;
            double u = (double)(hsh & 0xffffff) / (double)0x1000000 * 2.0 - 1.0;
            double x = (ik + 0.5) * dx + amp * dx * u;
            if (x < 0.0) x += 1.0;
            if (x >= 1.0) x -= 1.0;
            pos[k * np + id] = x;
        }
    }
}

static void search_case(int dim, int n, double amp)
{
    int64_t np = dim == 2 ? (int64_t)n * n : (int64_t)n * n * n;
    double *pos = malloc(sizeof(double) * dim * np);
    double *h = malloc(sizeof(double) * np);
    double box[3] = {1.0, 1.0, 1.0};
    lattice(dim, n, amp, pos);
    for (int64_t i = 0; i < np; ++i) h[i] = 1.3 / n * (1.0 - 0.2 * (double)(i % 3) / 3.0);
    int64_t *s1 = malloc(sizeof(int64_t) * (np + 1));
    int64_t *s2 = malloc(sizeof(int64_t) * (np + 1));
    int64_t p1 = oracle_neighbors_brute(dim, np, pos, h, box, s1, NULL);
    int64_t p2 = oracle_neighbors_grid(dim, np, pos, h, box, s2, NULL);
    CHECK(p1 == p2 && p1 > 0, "pair counts of brute and bucket search");
    int32_t *l1 = malloc(sizeof(int32_t) * (p1 > 0 ? p1 : 1));
    int32_t *l2 = malloc(sizeof(int32_t) * (p2 > 0 ? p2 : 1));
    oracle_neighbors_brute(dim, np, pos, h, box, s1, l1);
    oracle_neighbors_grid(dim, np, pos, h, box, s2, l2);
    int same = 1;
    for (int64_t i = 0; i <= np; ++i) same &= s1[i] == s2[i];
    for (int64_t e = 0; e < p1 && same; ++e) same &= l1[e] == l2[e];
    CHECK(same, "neighbour lists of brute and bucket search");
    free(pos); free(h); free(s1); free(s2); free(l1); free(l2);
}

static void tg_case(int n, double amp, int tv_mode, int tv_every, int nsteps)
{
    int64_t np = (int64_t)n * n;
    double dx = 1.0 / n;
    double *pos = malloc(sizeof(double) * 2 * np), *vel = malloc(sizeof(double) * 2 * np);
    double *acc = malloc(sizeof(double) * 2 * np), *rho = malloc(sizeof(double) * np);
    double *m = malloc(sizeof(double) * np), *h = malloc(sizeof(double) * np);
    double *diag = malloc(sizeof(double) * ORACLE_NDIAG * nsteps);
    double box[3] = {1.0, 1.0, 1.0};
    lattice(2, n, amp, pos);
    for (int64_t i = 0; i < np; ++i) {
        double x = pos[i], y = pos[np + i];
        vel[i] = -cos(2 * ORACLE_PI * x) * sin(2 * ORACLE_PI * y);
        vel[np + i] = sin(2 * ORACLE_PI * x) * cos(2 * ORACLE_PI * y);
        m[i] = dx * dx;
        h[i] = 1.3 * dx;
    }
    oracle_params p = {0};
    p.rho0 = 1.0; p.c0 = 10.0; p.eta = 0.01;
    p.dt = 0.6 * 1.3 * dx / 11.0; p.xi = -0.2; p.lim_c = 1e3; p.lim_s0 = 5e-4;
    p.riemann_eta = 3.0; p.h_min = 1.3 * dx; p.kappa = oracle_lattice_kappa(2, 1.3);
    p.band_tol = 1e-5; p.tv_every = tv_every; p.use_grid = 1; p.tv_mode = tv_mode;
    oracle_init(2, np, pos, vel, m, h, box, &p, rho, acc);
    double px0 = 0.0;
    for (int64_t i = 0; i < np; ++i) px0 += m[i] * vel[i];
    double *dr = malloc(sizeof(double) * 2 * np), *beta = malloc(sizeof(double) * np);
    double *s = malloc(sizeof(double) * np), *g = malloc(sizeof(double) * 2 * np);
    oracle_kdk_step(2, np, pos, vel, acc, rho, m, h, box, &p, 0, dr, beta, s, g, diag);
    oracle_run(2, np, pos, vel, acc, rho, m, h, box, &p, 1, nsteps - 1, diag + ORACLE_NDIAG);
    int finite = 1;
    for (int64_t i = 0; i < 2 * np; ++i) finite &= isfinite(pos[i]) && isfinite(vel[i]);
    CHECK(finite, "finite Taylor-Green state");
    CHECK(fabs(diag[ORACLE_NDIAG * (nsteps - 1) + 1] - px0) < 1e-14, "momentum is conserved");
    CHECK(diag[0] > 0.2 && diag[0] < 0.26, "kinetic energy after one step");
    free(pos); free(vel); free(acc); free(rho); free(m); free(h); free(diag);
    free(dr); free(beta); free(s); free(g);
}

/* fluid on an n x n lattice inside three wall layers (a small cavity whose
 * top layers move), all in one periodic box */
static void wall_case(int n, int nsteps)
{
    int layers = 3, side = n + 2 * layers;
    int64_t np = (int64_t)side * side, nw = np - (int64_t)n * n;
    double dx = 1.0 / n, edge = side * dx;
    double *pos = malloc(sizeof(double) * 2 * np), *vel = calloc(2 * np, sizeof(double));
    double *acc = malloc(sizeof(double) * 2 * np), *rho = malloc(sizeof(double) * np);
    double *m = malloc(sizeof(double) * np), *h = malloc(sizeof(double) * np);
    double *wv = calloc(2 * nw, sizeof(double));
    double box[3] = {edge, edge, edge};
    int64_t f = 0, w = (int64_t)n * n;
    for (int iy = 0; iy < side; ++iy)
        for (int ix = 0; ix < side; ++ix) {
            int fluid = ix >= layers && ix < layers + n && iy >= layers && iy < layers + n;
            int64_t id = fluid ? f++ : w++;
            pos[id] = (ix + 0.5) * dx;
            pos[np + id] = (iy + 0.5) * dx;
            m[id] = dx * dx;
            h[id] = 1.3 * dx;
            if (!fluid && iy >= layers + n) {
                wv[id - (int64_t)n * n] = 1.0;
                vel[id] = 1.0;
            }
        }
    oracle_params p = {0};
    p.rho0 = 1.0; p.c0 = 10.0; p.eta = 0.01;
    p.dt = 0.6 * 1.3 * dx / 11.0; p.xi = -0.2; p.lim_c = 1e3; p.lim_s0 = 5e-4;
    p.riemann_eta = 3.0; p.h_min = 1.3 * dx; p.kappa = oracle_lattice_kappa(2, 1.3);
    p.band_tol = 1e-5; p.tv_every = 1; p.use_grid = 1; p.n_wall = nw; p.wall_vel = wv;
    oracle_init(2, np, pos, vel, m, h, box, &p, rho, acc);
    oracle_run(2, np, pos, vel, acc, rho, m, h, box, &p, 0, nsteps, NULL);
    double umax = 0.0;
    for (int64_t i = 0; i < (int64_t)n * n; ++i) umax = fmax(umax, fabs(vel[i]));
    CHECK(umax > 0.0 && umax < 1.0, "lid drives the fluid below lid speed");
    free(pos); free(vel); free(acc); free(rho); free(m); free(h); free(wv);
}

int main(void)
{
    CHECK(fabs(oracle_lattice_kappa(2, 1.3) - 1.010473152107) < 1e-11, "kappa_2");
    CHECK(oracle_kernel_w(2, 2.0, 1.0) == 0.0, "kernel support");
    search_case(2, 12, 0.3);
    search_case(2, 5, 0.2);   /* fewer than 3 cells: brute-force fallback */
    search_case(3, 7, 0.2);
    tg_case(20, 0.05, ORACLE_TV_LIMITED, 1, 4);
    tg_case(16, 0.1, ORACLE_TV_SCALED, 3, 4);
    tg_case(16, 0.1, ORACLE_TV_BACKGROUND, 1, 3);
    wall_case(12, 3);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle sanitizer run clean\n");
    return 0;
}
