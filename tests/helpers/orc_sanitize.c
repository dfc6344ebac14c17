/*
 * orc_sanitize.c -- host-only driver that runs every exported oracle function on small
 * meshes, built together with the oracle under AddressSanitizer and UndefinedBehavior-
 * Sanitizer by tests/test_oracle_sanitize.py (gcc, no GPU code).  It checks memory
 * safety and undefined behaviour of the oracle, not its values (the pins do that): the
 * program exits with 0 when every call returned its success code and every result is
 * finite, and the sanitizers abort it on the first finding.
 *
 * Inputs are deterministic: a positive density with small high-order modes and a small
 * momentum, built from a fixed linear congruential sequence.
 */
#include "../../oracle/orc.c"

#include <stdio.h>

static uint64_t lcg_state = 12345u;

static double draw(void)
{
    lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg_state >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

static int failures = 0;

#define CHECK(cond, what)                                               \
    do {                                                                \
        if (!(cond)) {                                                  \
            fprintf(stderr, "check failed: %s (%s:%d)\n", what, __FILE__, __LINE__); \
            ++failures;                                                 \
        }                                                               \
    } while (0)

static int all_finite(const double *a, long n)
{
    for (long i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

/* density mean 1 with high modes of amplitude 0.02, momentum modes of amplitude 0.1 */
static double *make_state(const orc_cfg *cfg)
{
    int nb = orc_nbasis(cfg->k);
    long nc = ncell_of(cfg);
    double *u = malloc(sizeof(double) * NV * nb * nc);
    for (int v = 0; v < NV; ++v)
        for (int l = 0; l < nb; ++l)
            for (long c = 0; c < nc; ++c) {
                double a = v == 0 ? (l == 0 ? 1.0 + 0.2 * draw() : 0.02 * draw()) : 0.1 * draw();
                u[((long)v * nb + l) * nc + c] = a;
            }
    return u;
}

static void run_mesh(int nx, int ny, int nz, int k)
{
    orc_cfg cfg = {nx, ny, nz, k, 1.0 / nx, 1.0, 0.3, 2.0, 0.2, 1e-3, 0, 0.0, 0.1};
    int nb = orc_nbasis(k);
    long nc = ncell_of(&cfg);
    long n = (long)NV * nb * nc;
    double *u = make_state(&cfg);
    double *out = malloc(sizeof(double) * n);
    double *vh = malloc(sizeof(double) * 3 * nb * nc);
    double *nu = malloc(sizeof(double) * nc);
    int *fb = malloc(sizeof(int) * nc);
    for (long c = 0; c < nc; ++c) {
        nu[c] = 1e-3 * (0.5 + draw());
        fb[c] = (c % 3) == 0;
    }
    /* a driving table on the integer shell and one general wavevector */
    double modes[2 * 9] = {1, 0, 0, 0.3, -0.1, 0.2, 0.05, -0.4, 0.1,
                           1.5, -0.5, 2.0, 0.1, 0.2, -0.3, 0.4, 0.0, 0.2};
    const int flagsets[] = {ORC_POS_LIMITER,
                            ORC_AV | ORC_POS_LIMITER,
                            ORC_AV | ORC_PRIM_PROJ | ORC_POS_LIMITER | ORC_FORCING | ORC_FORCE_MEANFREE,
                            ORC_AV | ORC_PRIM_PROJ | ORC_POS_LIMITER | ORC_HLLC | ORC_RK_BY_ORDER,
                            ORC_AV | ORC_PRIM_PROJ | ORC_POS_LIMITER | ORC_LEARNED};
    for (unsigned f = 0; f < sizeof(flagsets) / sizeof(flagsets[0]); ++f) {
        cfg.flags = flagsets[f];
        cfg.rho_floor_rel = (f & 1) ? 0.1 : 0.0;
        const int learned = cfg.flags & ORC_LEARNED;
        double dt = learned ? orc_dt_max_learned(&cfg, u, nu, fb) : orc_dt_max(&cfg, u);
        CHECK(dt > 0.0 && isfinite(dt), "time step");
        CHECK(orc_project_primitive(&cfg, u, vh) == ORC_OK && all_finite(vh, 3L * nb * nc), "projection");
        CHECK(orc_rhs(&cfg, u, out, dt, modes, 2, learned ? nu : NULL, learned ? fb : NULL) == ORC_OK &&
                  all_finite(out, n), "rhs");
        double abar[3];
        CHECK(orc_forcing_mean(&cfg, u, modes, 2, abar) == ORC_OK && all_finite(abar, 3), "forcing mean");
        long cells[4] = {0, nc - 1, nc / 2, 0};
        double *oc = malloc(sizeof(double) * 4 * NV * nb);
        CHECK(orc_rhs_cells(&cfg, u, dt, modes, 2, abar, learned ? nu : NULL, learned ? fb : NULL, 4, cells, oc) ==
                  ORC_OK && all_finite(oc, 4L * NV * nb), "rhs cells");
        free(oc);
        double *w = malloc(sizeof(double) * n);
        memcpy(w, u, sizeof(double) * n);
        int st = orc_rk_step(&cfg, w, dt, modes, 2, learned ? nu : NULL, learned ? fb : NULL);
        CHECK(st == ORC_OK && all_finite(w, n), "rk step");
        double *theta = malloc(sizeof(double) * nc);
        CHECK(orc_limit(&cfg, w, theta) >= 0 && all_finite(theta, nc), "limiter");
        free(theta);
        double sums[4];
        CHECK(orc_conserved_sums(&cfg, w, sums) == ORC_OK && all_finite(sums, 4), "sums");
        free(w);
    }
    CHECK(orc_rk_stages(&cfg) >= 2, "stages");
    CHECK(isfinite(orc_rk_linear(&cfg, -1.0, 0.1, 1.0)), "linear scheme");
    if (k == 2) {
        double *x = malloc(sizeof(double) * 20 * nc);
        CHECK(orc_sensor_features(&cfg, u, x) == ORC_OK && all_finite(x, 20 * nc), "features");
        free(x);
    }
    CHECK(orc_sensor_labels(&cfg, u, nu) == ORC_OK && all_finite(nu, nc), "labels");
    /* projection of sampled fields and errors with a (k+3)-point rule */
    int nq = k + 3;
    long np = (long)nq * nq * nq;
    double *pts = malloc(sizeof(double) * nc * np * 3);
    double *vals = malloc(sizeof(double) * NV * nc * np);
    double *wp = malloc(sizeof(double) * n);
    CHECK(orc_points(&cfg, nq, pts) == ORC_OK, "points");
    for (long i = 0; i < NV * nc * np; ++i) vals[i] = 1.0 + 0.1 * sin(6.283185307179586 * pts[(i % (nc * np)) * 3]);
    CHECK(orc_project_values(&cfg, nq, NV, vals, wp) == ORC_OK && all_finite(wp, n), "project values");
    CHECK(orc_eval_points(&cfg, nq, NV, wp, vals) == ORC_OK && all_finite(vals, NV * nc * np), "eval points");
    double l1[NV];
    CHECK(orc_l1_error(&cfg, nq, NV, wp, vals, l1) == ORC_OK && all_finite(l1, NV), "l1 error");
    free(pts);
    free(vals);
    free(wp);
    /* flow statistics */
    double lb[4], s2[4];
    CHECK(orc_sf_bins(&cfg, 4, lb) == ORC_OK, "bins");
    CHECK(orc_structure_function(&cfg, u, 4, 0, 4, lb, 50, 7u, s2) == ORC_OK && all_finite(s2, 4), "structure function");
    int p = k + 1;
    double *grid = malloc(sizeof(double) * 3 * nc * p * p * p);
    CHECK(orc_velocity_grid(&cfg, u, p, grid) == ORC_OK && all_finite(grid, 3L * nc * p * p * p), "velocity grid");
    free(grid);
    free(u);
    free(out);
    free(vh);
    free(nu);
    free(fb);
}

int main(void)
{
    for (int n = 1; n <= 6; ++n) {
        double x[6], w[6], v, d;
        orc_gauss(n, x, w);
        orc_leg(n, x[0], &v, &d);
        CHECK(all_finite(x, n) && all_finite(w, n), "gauss rule");
    }
    for (int k = 1; k <= 3; ++k) {
        double xi[3] = {0.1, -0.3, 0.7}, phi, dphi[3];
        for (int l = 0; l < orc_nbasis(k); ++l) orc_basis_eval(k, l, xi, &phi, dphi);
        run_mesh(5, 4, 3, k);
        run_mesh(3, 1, 2, k);
    }
    double uL[4] = {1.0, 0.3, -0.2, 0.1}, uR[4] = {0.8, -0.1, 0.2, 0.0}, F[4];
    for (int d = 0; d < 3; ++d) {
        orc_rusanov(d, 1.0, uL, uR, F);
        orc_hllc(d, 1.0, uL, uR, F);
    }
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle sanitizer run: ok\n");
    return 0;
}
