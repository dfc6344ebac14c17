/*
 * orc.c -- plain FP64 CPU oracle for the modal Discontinuous Galerkin right-hand
 * side and SSP-RK3 step of 3D isothermal Euler on a periodic Cartesian mesh
 * (Cernetic, Springel, Guillet & Pakmor 2024, "Supersonic turbulence simulations
 * with GPU-based high-order Discontinuous Galerkin hydrodynamics").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct reference
 * that the GPU library is checked against.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it; the product path never
 * does.  It shares no code, header or table with the GPU library.
 *
 * Everything is double precision, written as plain loops over cells, points and
 * modes (OpenMP only over independent cells).  Each function names the passage
 * of the paper it follows.  Where the paper is silent the reading used is stated
 * at the function.
 *
 * Conventions (own reading where the paper defers to its companion paper):
 *   - basis: phi_(a,b,c)(xi) = Lt_a(xi1) Lt_b(xi2) Lt_c(xi3), Lt_n = sqrt(2n+1) P_n,
 *     total degree a+b+c <= k (Sec. 2.1 and the footnote of Sec. 3.2; Sec. 7 b_k);
 *     modes ordered by n=a+b+c ascending, then a descending, then b descending.
 *   - reference coordinate xi = 2(x - x_K)/h in [-1,1]^3; (1/|K|) Int phi_l phi_m = delta.
 *   - k+1 Gauss-Legendre points per dimension for volume and faces (Sec. 7 v_k, s_k).
 *   - state u = (rho, m_x, m_y, m_z), isothermal pressure p = cs^2 rho.
 *   - storage u[var][mode][cell], cell = i + nx*(j + ny*l).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>

#define ORC_AV            1
#define ORC_PRIM_PROJ     2
#define ORC_FORCING       4
#define ORC_POS_LIMITER   8
#define ORC_LEARNED      16
#define ORC_FORCE_MEANFREE 32
#define ORC_HLLC         64
#define ORC_RK_BY_ORDER  128

#define ORC_OK      0
#define ORC_RETRY   1
#define ORC_EINVAL -1

#define NV 4
#define KMAX 3
#define NBMAX 20
#define NQ1MAX (KMAX + 3)

typedef struct {
    int nx, ny, nz, k;
    double h, cs, cfl, alpha, beta, rho_floor;
    int flags;
    double rho_floor_rel;
    double cfl_visc;
} orc_cfg;

/* ---------------------------------------------------------------- 1D pieces */

/* Legendre P_n and P_n' by the three-term (Bonnet) recurrence. */
static void legendre(int n, double x, double *p, double *dp)
{
    double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
    if (n == 0) { *p = 1.0; *dp = 0.0; return; }
    for (int j = 1; j < n; ++j) {
        double p2 = ((2.0 * j + 1.0) * x * p1 - j * p0) / (j + 1.0);
        double d2 = d0 + (2.0 * j + 1.0) * p1;   /* P'_{j+1} = P'_{j-1} + (2j+1) P_j */
        p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    }
    *p = p1; *dp = d1;
}

/* Orthonormal 1D Legendre function Lt_n = sqrt(2n+1) P_n and its derivative
 * (normalisation (1/2) Int_{-1}^{1} Lt_m Lt_n = delta_mn, Sec. 2.2). */
void orc_leg(int n, double x, double *val, double *der)
{
    double p, dp;
    legendre(n, x, &p, &dp);
    double s = sqrt(2.0 * n + 1.0);
    *val = s * p;
    *der = s * dp;
}

/* n-point Gauss-Legendre nodes (ascending) and weights (sum 2) by Newton
 * iteration on P_n (Sec. 2.2, Gaussian quadrature). */
void orc_gauss(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre(n, z, &p, &dp);
            double dz = p / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        double p, dp;
        legendre(n, z, &p, &dp);
        x[n - 1 - i] = z;
        w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* ------------------------------------------------------------------- basis */

int orc_nbasis(int k) { return (k + 1) * (k + 2) * (k + 3) / 6; }

/* Exponents (a,b,c) of every mode in the graded order. */
int orc_basis_exps(int k, int *exps)
{
    int m = 0;
    for (int n = 0; n <= k; ++n)
        for (int a = n; a >= 0; --a)
            for (int b = n - a; b >= 0; --b) {
                exps[3 * m + 0] = a;
                exps[3 * m + 1] = b;
                exps[3 * m + 2] = n - a - b;
                ++m;
            }
    return m;
}

/* phi_l(xi) and its three reference-coordinate derivatives. */
void orc_basis_eval(int k, int l, const double xi[3], double *phi, double dphi[3])
{
    int exps[3 * NBMAX];
    orc_basis_exps(k, exps);
    double v[3], d[3];
    for (int a = 0; a < 3; ++a) orc_leg(exps[3 * l + a], xi[a], &v[a], &d[a]);
    *phi = v[0] * v[1] * v[2];
    if (dphi) {
        dphi[0] = d[0] * v[1] * v[2];
        dphi[1] = v[0] * d[1] * v[2];
        dphi[2] = v[0] * v[1] * d[2];
    }
}

/* --------------------------------------------------------------- helpers */

typedef struct {
    int k, nb, n1, nq, nf;          /* degree, modes, 1D points, volume points, face points */
    double g[KMAX + 1], w[KMAX + 1];
    /* volume points */
    double vxi[(KMAX + 1) * (KMAX + 1) * (KMAX + 1)][3];
    double vw[(KMAX + 1) * (KMAX + 1) * (KMAX + 1)];
    double vphi[(KMAX + 1) * (KMAX + 1) * (KMAX + 1)][NBMAX];
    double vdphi[(KMAX + 1) * (KMAX + 1) * (KMAX + 1)][3][NBMAX];
    /* face points: [dir][side][r], side 0 = low (xi_d = -1), side 1 = high (xi_d = +1) */
    double fxi[3][2][(KMAX + 1) * (KMAX + 1)][3];
    double fw[(KMAX + 1) * (KMAX + 1)];
    double fphi[3][2][(KMAX + 1) * (KMAX + 1)][NBMAX];
} tabs_t;

static void make_tabs(int k, tabs_t *T)
{
    T->k = k;
    T->nb = orc_nbasis(k);
    T->n1 = k + 1;
    T->nq = T->n1 * T->n1 * T->n1;
    T->nf = T->n1 * T->n1;
    orc_gauss(T->n1, T->g, T->w);
    for (int qz = 0; qz < T->n1; ++qz)
        for (int qy = 0; qy < T->n1; ++qy)
            for (int qx = 0; qx < T->n1; ++qx) {
                int q = qx + T->n1 * (qy + T->n1 * qz);
                T->vxi[q][0] = T->g[qx];
                T->vxi[q][1] = T->g[qy];
                T->vxi[q][2] = T->g[qz];
                T->vw[q] = T->w[qx] * T->w[qy] * T->w[qz];
                for (int l = 0; l < T->nb; ++l) {
                    double d[3];
                    orc_basis_eval(k, l, T->vxi[q], &T->vphi[q][l], d);
                    T->vdphi[q][0][l] = d[0];
                    T->vdphi[q][1][l] = d[1];
                    T->vdphi[q][2][l] = d[2];
                }
            }
    for (int r2 = 0; r2 < T->n1; ++r2)
        for (int r1 = 0; r1 < T->n1; ++r1)
            T->fw[r1 + T->n1 * r2] = T->w[r1] * T->w[r2];
    for (int d = 0; d < 3; ++d) {
        int t1 = (d == 0) ? 1 : 0;
        int t2 = (d == 2) ? 1 : 2;
        for (int s = 0; s < 2; ++s)
            for (int r2 = 0; r2 < T->n1; ++r2)
                for (int r1 = 0; r1 < T->n1; ++r1) {
                    int r = r1 + T->n1 * r2;
                    double *xi = T->fxi[d][s][r];
                    xi[d] = s ? 1.0 : -1.0;
                    xi[t1] = T->g[r1];
                    xi[t2] = T->g[r2];
                    for (int l = 0; l < T->nb; ++l)
                        orc_basis_eval(k, l, xi, &T->fphi[d][s][r][l], NULL);
                }
    }
}

static inline long ncell_of(const orc_cfg *c) { return (long)c->nx * c->ny * c->nz; }

static inline long cell_id(const orc_cfg *c, int i, int j, int l)
{
    return (long)i + (long)c->nx * ((long)j + (long)c->ny * l);
}

static inline void cell_ijk(const orc_cfg *c, long id, int *i, int *j, int *l)
{
    *i = (int)(id % c->nx);
    *j = (int)((id / c->nx) % c->ny);
    *l = (int)(id / ((long)c->nx * c->ny));
}

/* neighbour of a cell across direction d, side s (0 = low, 1 = high), periodic */
static long neighbour(const orc_cfg *c, long id, int d, int s)
{
    int ijk[3];
    cell_ijk(c, id, &ijk[0], &ijk[1], &ijk[2]);
    int n[3] = {c->nx, c->ny, c->nz};
    ijk[d] += s ? 1 : -1;
    if (ijk[d] < 0) ijk[d] += n[d];
    if (ijk[d] >= n[d]) ijk[d] -= n[d];
    return cell_id(c, ijk[0], ijk[1], ijk[2]);
}

static inline double U(const double *u, int nb, long nc, int v, int l, long c)
{
    return u[((long)v * nb + l) * nc + c];
}

/* expansion value of variable v of cell c at a point whose basis values are phi[] */
static double expand(const double *u, int nb, long nc, int v, long c, const double *phi)
{
    double s = 0.0;
    for (int l = 0; l < nb; ++l) s += U(u, nb, nc, v, l, c) * phi[l];
    return s;
}

/* physical position of reference point xi in cell c (unit-spaced cells of size h,
 * the box is [0, nx h) x [0, ny h) x [0, nz h)) */
static void position(const orc_cfg *c, long id, const double xi[3], double x[3])
{
    int ijk[3];
    cell_ijk(c, id, &ijk[0], &ijk[1], &ijk[2]);
    for (int a = 0; a < 3; ++a) x[a] = (ijk[a] + 0.5 + 0.5 * xi[a]) * c->h;
}

/* Driving acceleration a(x) = sum_m Re[ ahat_m exp(2 pi i n_m . x) ] (Sec. 4.2).
 * modes[m] = (n_x, n_y, n_z, Re ax, Im ax, Re ay, Im ay, Re az, Im az). */
static void accel(const double *modes, int nm, const double x[3], double a[3])
{
    a[0] = a[1] = a[2] = 0.0;
    for (int m = 0; m < nm; ++m) {
        const double *e = modes + 9 * m;
        double ph = 2.0 * M_PI * (e[0] * x[0] + e[1] * x[1] + e[2] * x[2]);
        double cp = cos(ph), sp = sin(ph);
        for (int d = 0; d < 3; ++d) a[d] += e[3 + 2 * d] * cp - e[4 + 2 * d] * sp;
    }
}

void orc_accel(const double *modes, int nm, const double *x, double *a) { accel(modes, nm, x, a); }

/* ---------------------------------------------------- primitive projection */

/* Projection of the velocity onto the basis (Sec. 3.2, eq. weights_equation):
 * v_q = m_q / rho_q at the interior Gauss points, Vhat_{d,l} = (1/8) sum_q w_q phi_l(q) v_{d,q}.
 * vh[d*nb + l]. */
static void project_cell(const tabs_t *T, const double *u, long nc, long c, double *vh)
{
    int nb = T->nb;
    for (int i = 0; i < 3 * nb; ++i) vh[i] = 0.0;
    for (int q = 0; q < T->nq; ++q) {
        double rho = expand(u, nb, nc, 0, c, T->vphi[q]);
        for (int d = 0; d < 3; ++d) {
            double v = expand(u, nb, nc, 1 + d, c, T->vphi[q]) / rho;
            for (int l = 0; l < nb; ++l) vh[d * nb + l] += 0.125 * T->vw[q] * T->vphi[q][l] * v;
        }
    }
}

int orc_project_primitive(const orc_cfg *cfg, const double *u, double *vhat)
{
    if (cfg->k < 1 || cfg->k > KMAX) return ORC_EINVAL;
    tabs_t *T = malloc(sizeof(tabs_t));
    make_tabs(cfg->k, T);
    long nc = ncell_of(cfg);
    int nb = T->nb;
    #pragma omp parallel for schedule(static)
    for (long c = 0; c < nc; ++c) {
        double vh[3 * NBMAX];
        project_cell(T, u, nc, c, vh);
        for (int d = 0; d < 3; ++d)
            for (int l = 0; l < nb; ++l) vhat[((long)d * nb + l) * nc + c] = vh[d * nb + l];
    }
    free(T);
    return ORC_OK;
}

/* ------------------------------------------------------------------ physics */

/* isothermal flux in direction d for state (rho, m) with pressure p (Sec. 2, flux
 * matrix without the energy row): F_d = (m_d, m_d m / rho + p e_d) */
static void flux(int d, double rho, const double m[3], double p, double F[NV])
{
    F[0] = m[d];
    for (int j = 0; j < 3; ++j) F[1 + j] = m[d] * m[j] / rho;
    F[1 + d] += p;
}

/* Rusanov (local Lax-Friedrichs) flux across a face with normal +e_d between the
 * low-side state L and the high-side state R: half the sum of the two physical
 * fluxes minus half the largest signal speed times the jump.  Speed = largest
 * |v_d| of the two sides plus cs.  (The paper uses HLLC, available below as the
 * alternative; Rusanov is the default interface solver, Sec. 2.2 numerical flux.) */
void orc_rusanov(int d, double cs, const double uL[NV], const double uR[NV], double Fh[NV])
{
    double FL[NV], FR[NV];
    double mL[3] = {uL[1], uL[2], uL[3]}, mR[3] = {uR[1], uR[2], uR[3]};
    flux(d, uL[0], mL, cs * cs * uL[0], FL);
    flux(d, uR[0], mR, cs * cs * uR[0], FR);
    double vL = fabs(uL[1 + d] / uL[0]), vR = fabs(uR[1 + d] / uR[0]);
    double lam = (vL > vR ? vL : vR) + cs;
    for (int v = 0; v < NV; ++v) Fh[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * lam * (uR[v] - uL[v]);
}

/* HLLC-type flux for the isothermal equations (the paper uses Toro's HLLC for the
 * adiabatic equations, Sec. 2.2; isothermal gas has no contact in the normal subsystem, so
 * the contact-resolving part concerns the shear waves): wave speeds S_L = min(v_L, v_R) - cs
 * and S_R = max(v_L, v_R) + cs (v: normal velocity); density and normal momentum take the
 * HLL flux (F_L if S_L >= 0, F_R if S_R <= 0, else (S_R F_L - S_L F_R + S_L S_R (u_R - u_L))
 * / (S_R - S_L)); each tangential momentum is carried by that mass flux with the tangential
 * velocity of the upwind side (left if the mass flux is >= 0). */
void orc_hllc(int d, double cs, const double uL[NV], const double uR[NV], double Fh[NV])
{
    double FL[NV], FR[NV];
    double mL[3] = {uL[1], uL[2], uL[3]}, mR[3] = {uR[1], uR[2], uR[3]};
    flux(d, uL[0], mL, cs * cs * uL[0], FL);
    flux(d, uR[0], mR, cs * cs * uR[0], FR);
    double vL = uL[1 + d] / uL[0], vR = uR[1 + d] / uR[0];
    double SL = (vL < vR ? vL : vR) - cs;
    double SR = (vL > vR ? vL : vR) + cs;
    int comp[2] = {0, 1 + d};                  /* density, normal momentum */
    for (int i = 0; i < 2; ++i) {
        int v = comp[i];
        if (SL >= 0.0) Fh[v] = FL[v];
        else if (SR <= 0.0) Fh[v] = FR[v];
        else Fh[v] = (SR * FL[v] - SL * FR[v] + SL * SR * (uR[v] - uL[v])) / (SR - SL);
    }
    for (int t = 0; t < 3; ++t) {
        if (t == d) continue;
        double vt = Fh[0] >= 0.0 ? uL[1 + t] / uL[0] : uR[1 + t] / uR[0];
        Fh[1 + t] = Fh[0] * vt;
    }
}

/* von Neumann-Richtmyer viscous pressure (Sec. 3.1): for a compressing point
 * (div v < 0), Pi = alpha rho (h/p)^2 |div v|^2 + beta rho cs (h/p) |div v|, capped at
 * Pi_max = (1/2) rho (h/p)^2 |div v| / dt with p = k+1 the spatial order.  dt <= 0
 * means no cap. */
double orc_vnr_pi(const orc_cfg *cfg, double rho, double divv, double dt)
{
    if (!(divv < 0.0)) return 0.0;
    double s = -divv;
    double hp = cfg->h / (cfg->k + 1);
    double pi = cfg->alpha * rho * hp * hp * s * s + cfg->beta * rho * cfg->cs * hp * s;
    if (dt > 0.0) {
        double pmax = 0.5 * rho * hp * hp * s / dt;
        if (pi > pmax) pi = pmax;
    }
    return pi;
}

/* Learned-sensor viscous pressure at a point: the network gives the cell a bulk
 * viscosity nu (the vNR form is Pi = rho nu_vnr s with nu_vnr = alpha (h/p)^2 s +
 * beta cs (h/p)); the learned form is Pi = rho nu s at compressed points (s = -div v > 0),
 * none at expanding points, with the cap Pi_max of Sec. 3.1 (none for dt <= 0). */
static double learned_pi(const orc_cfg *cfg, double rho, double nu, double divv, double dt)
{
    double s = -divv;
    if (!(s > 0.0) || !(nu > 0.0)) return 0.0;
    double pi = rho * nu * s;
    double hp = cfg->h / (cfg->k + 1);
    if (dt > 0.0) {
        double pmax = 0.5 * rho * hp * hp * s / dt;
        if (pi > pmax) pi = pmax;
    }
    return pi;
}

/* face trace (rho, m) of cell c at a face point with basis values phi (Sec. 3.2):
 * rho from the density expansion; with primitive projection the velocity comes
 * from the projected polynomial vh and m = rho v, otherwise m from its own expansion */
static void trace(const orc_cfg *cfg, const tabs_t *T, const double *u, long nc, long c,
                  const double *vh, const double *phi, double out[NV])
{
    int nb = T->nb;
    double rho = expand(u, nb, nc, 0, c, phi);
    out[0] = rho;
    for (int d = 0; d < 3; ++d) {
        if (cfg->flags & ORC_PRIM_PROJ) {
            double v = 0.0;
            for (int l = 0; l < nb; ++l) v += vh[d * nb + l] * phi[l];
            out[1 + d] = rho * v;
        } else {
            out[1 + d] = expand(u, nb, nc, 1 + d, c, phi);
        }
    }
}


/* ------------------------------------------------------------- the RHS */

typedef struct {
    const orc_cfg *cfg;
    const tabs_t *T;
    const double *u;
    const double *vhat;     /* [3][nb][nc], or NULL: computed per cell on demand */
    double dt;
    const double *modes;
    int nmodes;
    const double *abar;     /* mass-weighted mean acceleration to remove, or NULL */
    const double *nu;       /* learned-sensor viscosity per cell (learned mode) */
    const int *fallback;    /* per-cell: 1 = use the plain sensor (learned mode) */
} rhs_ctx;

static void get_vhat(const rhs_ctx *R, long c, double *vh)
{
    long nc = ncell_of(R->cfg);
    int nb = R->T->nb;
    if (R->vhat) {
        for (int d = 0; d < 3; ++d)
            for (int l = 0; l < nb; ++l) vh[d * nb + l] = R->vhat[((long)d * nb + l) * nc + c];
    } else {
        project_cell(R->T, R->u, nc, c, vh);
    }
}

/* Time derivative of the weights of one cell (Sec. 2.2, eq. weight_evolution):
 * |K| dw_l/dt = Int_K grad(phi_l) . F dx - Oint_dK phi_l F*(u+, u-) . n dS
 * With x = x_K + (h/2) xi, |K| = h^3, dx = (h/2)^3 dxi, dS = (h/2)^2 dxi_face and
 * grad = (2/h) grad_xi this is
 *   dw_l/dt = (1/(4h)) sum_q w_q sum_d dphi_l/dxi_d F_d(q)
 *           - (1/(4h)) sum_faces sum_r w_r phi_l(r) (n . e_d) F*_d(r)
 * plus the forcing source (1/8) sum_q w_q phi_l(q) rho_q (a(x_q) - abar) in the
 * momentum rows (Sec. 4.2) and the artificial pressure Pi in the volume flux only
 * (Sec. 3.1). out[v*nb + l]. */
static void rhs_cell(const rhs_ctx *R, long c, double *out)
{
    const orc_cfg *cfg = R->cfg;
    const tabs_t *T = R->T;
    const double *u = R->u;
    int nb = T->nb;
    long nc = ncell_of(cfg);
    double inv4h = 1.0 / (4.0 * cfg->h);
    double vh[3 * NBMAX];
    get_vhat(R, c, vh);
    for (int i = 0; i < NV * nb; ++i) out[i] = 0.0;

    int learned = (cfg->flags & ORC_LEARNED) && R->nu && !(R->fallback && R->fallback[c]);

    /* volume integral */
    for (int q = 0; q < T->nq; ++q) {
        double rho = expand(u, nb, nc, 0, c, T->vphi[q]);
        double m[3];
        for (int d = 0; d < 3; ++d) m[d] = expand(u, nb, nc, 1 + d, c, T->vphi[q]);
        double pi = 0.0;
        if (cfg->flags & ORC_AV) {
            double divv = 0.0;
            for (int d = 0; d < 3; ++d)
                for (int l = 0; l < nb; ++l) divv += vh[d * nb + l] * T->vdphi[q][d][l];
            divv *= 2.0 / cfg->h;
            pi = learned ? learned_pi(cfg, rho, R->nu[c], divv, R->dt) : orc_vnr_pi(cfg, rho, divv, R->dt);
        }
        double p = cfg->cs * cfg->cs * rho + pi;
        for (int d = 0; d < 3; ++d) {
            double F[NV];
            flux(d, rho, m, p, F);
            for (int v = 0; v < NV; ++v)
                for (int l = 0; l < nb; ++l)
                    out[v * nb + l] += inv4h * T->vw[q] * T->vdphi[q][d][l] * F[v];
        }
        if ((cfg->flags & ORC_FORCING) && R->modes && R->nmodes > 0) {
            double x[3], a[3];
            position(cfg, c, T->vxi[q], x);
            accel(R->modes, R->nmodes, x, a);
            for (int d = 0; d < 3; ++d) {
                double ad = a[d] - (R->abar ? R->abar[d] : 0.0);
                for (int l = 0; l < nb; ++l)
                    out[(1 + d) * nb + l] += 0.125 * T->vw[q] * T->vphi[q][l] * rho * ad;
            }
        }
    }

    /* surface integral: for each face, Rusanov flux between the low-side and
     * high-side traces, lifted with the outward normal sign */
    for (int d = 0; d < 3; ++d)
        for (int s = 0; s < 2; ++s) {
            long nbc = neighbour(cfg, c, d, s);
            double vhn[3 * NBMAX];
            get_vhat(R, nbc, vhn);
            double sign = s ? 1.0 : -1.0;
            for (int r = 0; r < T->nf; ++r) {
                double uin[NV], uout[NV], Fh[NV];
                trace(cfg, T, u, nc, c, vh, T->fphi[d][s][r], uin);
                trace(cfg, T, u, nc, nbc, vhn, T->fphi[d][1 - s][r], uout);
                void (*riemann)(int, double, const double *, const double *, double *) =
                    (cfg->flags & ORC_HLLC) ? orc_hllc : orc_rusanov;
                if (s) riemann(d, cfg->cs, uin, uout, Fh);
                else   riemann(d, cfg->cs, uout, uin, Fh);
                for (int v = 0; v < NV; ++v)
                    for (int l = 0; l < nb; ++l)
                        out[v * nb + l] -= inv4h * T->fw[r] * T->fphi[d][s][r][l] * sign * Fh[v];
            }
        }
}

/* Mass-weighted mean of the driving acceleration over the box, abar = Int rho a / Int rho,
 * evaluated with the same interior quadrature as the source term.  Removing it from
 * the source keeps the total momentum exactly conserved (the paper is silent on this;
 * reading stated in the design notes). */
int orc_forcing_mean(const orc_cfg *cfg, const double *u, const double *modes, int nmodes,
                     double abar[3])
{
    if (cfg->k < 1 || cfg->k > KMAX) return ORC_EINVAL;
    tabs_t *T = malloc(sizeof(tabs_t));
    make_tabs(cfg->k, T);
    long nc = ncell_of(cfg);
    int nb = T->nb;
    double *part = malloc(sizeof(double) * 4 * nc);
    #pragma omp parallel for schedule(static)
    for (long c = 0; c < nc; ++c) {
        double s[4] = {0, 0, 0, 0};
        for (int q = 0; q < T->nq; ++q) {
            double rho = expand(u, nb, nc, 0, c, T->vphi[q]);
            double x[3], a[3];
            position(cfg, c, T->vxi[q], x);
            accel(modes, nmodes, x, a);
            for (int d = 0; d < 3; ++d) s[d] += 0.125 * T->vw[q] * rho * a[d];
            s[3] += 0.125 * T->vw[q] * rho;
        }
        for (int i = 0; i < 4; ++i) part[4 * c + i] = s[i];
    }
    double tot[4] = {0, 0, 0, 0};
    for (long c = 0; c < nc; ++c)
        for (int i = 0; i < 4; ++i) tot[i] += part[4 * c + i];
    for (int d = 0; d < 3; ++d) abar[d] = tot[d] / tot[3];
    free(part);
    free(T);
    return ORC_OK;
}

static int check_cfg(const orc_cfg *cfg)
{
    if (!cfg || cfg->k < 1 || cfg->k > KMAX || cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 1 ||
        !(cfg->h > 0.0))
        return ORC_EINVAL;
    return ORC_OK;
}

/* Full right-hand side dudt[var][mode][cell].  nu/fallback only matter with the
 * learned-sensor flag (may be NULL otherwise). */
int orc_rhs(const orc_cfg *cfg, const double *u, double *dudt, double dt,
            const double *modes, int nmodes, const double *nu, const int *fallback)
{
    if (check_cfg(cfg)) return ORC_EINVAL;
    tabs_t *T = malloc(sizeof(tabs_t));
    make_tabs(cfg->k, T);
    long nc = ncell_of(cfg);
    int nb = T->nb;
    double *vhat = malloc(sizeof(double) * 3 * nb * nc);
    orc_project_primitive(cfg, u, vhat);
    double abar[3] = {0, 0, 0};
    int use_mean = (cfg->flags & ORC_FORCING) && (cfg->flags & ORC_FORCE_MEANFREE) && modes && nmodes > 0;
    if (use_mean) orc_forcing_mean(cfg, u, modes, nmodes, abar);
    rhs_ctx R = {cfg, T, u, vhat, dt, modes, nmodes, use_mean ? abar : NULL, nu, fallback};
    #pragma omp parallel for schedule(dynamic, 64)
    for (long c = 0; c < nc; ++c) {
        double out[NV * NBMAX];
        rhs_cell(&R, c, out);
        for (int v = 0; v < NV; ++v)
            for (int l = 0; l < nb; ++l) dudt[((long)v * nb + l) * nc + c] = out[v * nb + l];
    }
    free(vhat);
    free(T);
    return ORC_OK;
}

/* RHS of a sample of cells only (for checks at sizes where the full oracle is too
 * slow).  abar is the mean acceleration to remove (from orc_forcing_mean) or NULL.
 * out[s][var][mode]. */
int orc_rhs_cells(const orc_cfg *cfg, const double *u, double dt, const double *modes, int nmodes,
                  const double *abar, const double *nu, const int *fallback,
                  long ns, const long *cells, double *out)
{
    if (check_cfg(cfg)) return ORC_EINVAL;
    tabs_t *T = malloc(sizeof(tabs_t));
    make_tabs(cfg->k, T);
    int nb = T->nb;
    int use_mean = (cfg->flags & ORC_FORCING) && (cfg->flags & ORC_FORCE_MEANFREE) && modes && nmodes > 0;
    rhs_ctx R = {cfg, T, u, NULL, dt, modes, nmodes, use_mean ? abar : NULL, nu, fallback};
    #pragma omp parallel for schedule(dynamic, 4)
    for (long s = 0; s < ns; ++s) rhs_cell(&R, cells[s], out + (long)s * NV * nb);
    free(T);
    return ORC_OK;
}

/* ------------------------------------------------------------ time step */

/* Time step.  Advective part (Sec. 7: dt proportional to h/(k+1)); reading:
 * dt_adv = cfl h / ((k+1) max_{K,q} sum_d (|m_d/rho| + cs)) over the interior Gauss points.
 * Viscous part (reading; the paper only caps Pi so that one step cannot reverse the
 * compression, Sec. 3.1): with artificial viscosity on, the viscous pressure acts as a
 * bulk viscosity nu = Pi / (rho |div v|) = alpha (h/p)^2 |div v| + beta cs (h/p) at
 * compressing points (div v of the projected velocity, p = k+1), and the explicit
 * stability bound dt_visc = cfl_visc (h/p)^2 / max nu applies; dt = min(dt_adv, dt_visc).
 * cfl_visc <= 0 or AV off: advective part only.  With the learned sensor (nu != NULL and
 * the LEARNED flag) a cell whose fallback flag is 0 contributes its prescribed bulk
 * viscosity nu[c] instead of the maximum over its points. */
static double dt_max_impl(const orc_cfg *cfg, const double *u, const double *nuc, const int *fallback)
{
    if (check_cfg(cfg)) return -1.0;
    tabs_t *T = malloc(sizeof(tabs_t));
    make_tabs(cfg->k, T);
    long nc = ncell_of(cfg);
    int nb = T->nb;
    double hp = cfg->h / (cfg->k + 1);
    int visc = (cfg->flags & ORC_AV) && cfg->cfl_visc > 0.0;
    int learned = (cfg->flags & ORC_LEARNED) && nuc != NULL;
    double *smax = malloc(sizeof(double) * nc);
    double *numax = malloc(sizeof(double) * nc);
    #pragma omp parallel for schedule(static)
    for (long c = 0; c < nc; ++c) {
        double sm = 0.0, nm = 0.0;
        double vh[3 * NBMAX];
        if (visc) project_cell(T, u, nc, c, vh);
        for (int q = 0; q < T->nq; ++q) {
            double rho = expand(u, nb, nc, 0, c, T->vphi[q]);
            double s = 0.0;
            for (int d = 0; d < 3; ++d) s += fabs(expand(u, nb, nc, 1 + d, c, T->vphi[q]) / rho) + cfg->cs;
            if (s > sm) sm = s;
            if (visc && !(learned && !(fallback && fallback[c]))) {
                double divv = 0.0;
                for (int d = 0; d < 3; ++d)
                    for (int l = 0; l < nb; ++l) divv += vh[d * nb + l] * T->vdphi[q][d][l];
                divv *= 2.0 / cfg->h;
                if (divv < 0.0) {
                    double nu = cfg->alpha * hp * hp * (-divv) + cfg->beta * cfg->cs * hp;
                    if (nu > nm) nm = nu;
                }
            }
        }
        if (visc && learned && !(fallback && fallback[c])) nm = nuc[c] > 0.0 ? nuc[c] : 0.0;
        smax[c] = sm;
        numax[c] = nm;
    }
    double m = 0.0, nmax = 0.0;
    for (long c = 0; c < nc; ++c) {
        if (smax[c] > m) m = smax[c];
        if (numax[c] > nmax) nmax = numax[c];
    }
    free(smax);
    free(numax);
    free(T);
    double dt = cfg->cfl * cfg->h / ((cfg->k + 1) * m);
    if (visc && nmax > 0.0) {
        double dv = cfg->cfl_visc * hp * hp / nmax;
        if (dv < dt) dt = dv;
    }
    return dt;
}

double orc_dt_max(const orc_cfg *cfg, const double *u) { return dt_max_impl(cfg, u, NULL, NULL); }

double orc_dt_max_learned(const orc_cfg *cfg, const double *u, const double *nu, const int *fallback)
{
    return dt_max_impl(cfg, u, nu, fallback);
}

/* ----------------------------------------------------- positivity limiter */

/* Positivity limiter of one cell (Sec. 3.1, last paragraph; floor 1e-3 from the
 * density-PDF figure): rho_min over all volume and face Gauss points; if below the
 * target while the mean is above the floor, scale every high-order weight of all four
 * variables by theta = (mean - target)/(mean - rho_min).  Reading (the paper does not
 * state the value the scaling aims at): target = max(floor, rho_floor_rel * mean), so a
 * limited cell keeps no near-vacuum interior point where m/rho would be unbounded.  A mean
 * at or below the floor cannot be fixed by scaling: return 1 (the step must be retried
 * with a smaller dt).  Returns 0 otherwise; *theta_out gets the factor used (1 = none). */
static int limit_cell(const orc_cfg *cfg, const tabs_t *T, double *u, long nc, long c, double *theta_out)
{
    int nb = T->nb;
    double mean = U(u, nb, nc, 0, 0, c);
    double rmin = INFINITY;
    for (int q = 0; q < T->nq; ++q) {
        double r = expand(u, nb, nc, 0, c, T->vphi[q]);
        if (r < rmin) rmin = r;
    }
    for (int d = 0; d < 3; ++d)
        for (int s = 0; s < 2; ++s)
            for (int r = 0; r < T->nf; ++r) {
                double v = expand(u, nb, nc, 0, c, T->fphi[d][s][r]);
                if (v < rmin) rmin = v;
            }
    if (theta_out) *theta_out = 1.0;
    if (!(mean > cfg->rho_floor)) return 1;
    double target = cfg->rho_floor;
    if (cfg->rho_floor_rel * mean > target) target = cfg->rho_floor_rel * mean;
    if (rmin < target) {
        double theta = (mean - target) / (mean - rmin);
        for (int v = 0; v < NV; ++v)
            for (int l = 1; l < nb; ++l) u[((long)v * nb + l) * nc + c] *= theta;
        if (theta_out) *theta_out = theta;
    }
    return 0;
}

/* Limit every cell in place; returns the number of cells whose mean is at or below
 * the floor (non-zero means retry).  theta (may be NULL) gets the per-cell factor. */
long orc_limit(const orc_cfg *cfg, double *u, double *theta)
{
    if (check_cfg(cfg)) return -1;
    tabs_t *T = malloc(sizeof(tabs_t));
    make_tabs(cfg->k, T);
    long nc = ncell_of(cfg);
    long nfail = 0;
    #pragma omp parallel for schedule(static) reduction(+:nfail)
    for (long c = 0; c < nc; ++c) {
        double th;
        nfail += limit_cell(cfg, T, u, nc, c, &th);
        if (theta) theta[c] = th;
    }
    free(T);
    return nfail;
}

/* ------------------------------------------------------- SSP Runge-Kutta */

/* Explicit strong-stability-preserving Runge-Kutta schemes in Shu-Osher form:
 *   u(0) = u^n,  u(i) = sum_{j<i} ( alpha_ij u(j) + beta_ij dt L(u(j)) ),  u^{n+1} = u(S).
 * Sec. 7 counts k+1 right-hand-side evaluations per step for degree k (Sec. 2.2: the
 * time integrator matches the spatial order).  Without ORC_RK_BY_ORDER every degree uses
 * the three-stage third-order scheme (Shu & Osher); with it, degree 1 uses the two-stage
 * second-order scheme (Heun), degree 2 the three-stage one and degree 3 the five-stage
 * fourth-order scheme of Spiteri & Ruuth (2002). */
#define RK_SMAX 5
typedef struct {
    int stages;
    double alpha[RK_SMAX][RK_SMAX];   /* alpha[i-1][j]: weight of u(j) in u(i) */
    double beta[RK_SMAX][RK_SMAX];    /* beta[i-1][j]:  weight of dt L(u(j)) in u(i) */
} rk_scheme;

static const rk_scheme RK2 = {2, {{1.0}, {0.5, 0.5}}, {{1.0}, {0.0, 0.5}}};
static const rk_scheme RK3 = {3, {{1.0}, {0.75, 0.25}, {1.0 / 3.0, 0.0, 2.0 / 3.0}},
                              {{1.0}, {0.0, 0.25}, {0.0, 0.0, 2.0 / 3.0}}};
static const rk_scheme RK54 = {5,
    {{1.0},
     {0.444370493651235, 0.555629506348765},
     {0.620101851488403, 0.0, 0.379898148511597},
     {0.178079954393132, 0.0, 0.0, 0.821920045606868},
     {0.0, 0.0, 0.517231671970585, 0.096059710526147, 0.386708617503269}},
    {{0.391752226571890},
     {0.0, 0.368410593050371},
     {0.0, 0.0, 0.251891774271694},
     {0.0, 0.0, 0.0, 0.544974750228521},
     {0.0, 0.0, 0.0, 0.063692468666290, 0.226007483236906}}};

static const rk_scheme *scheme_of(const orc_cfg *cfg)
{
    if (!(cfg->flags & ORC_RK_BY_ORDER)) return &RK3;
    return cfg->k == 1 ? &RK2 : (cfg->k == 2 ? &RK3 : &RK54);
}

/* stage i (1-based) of a scheme: out = sum_{j<i} alpha_ij X[j] + beta_ij dt LX[j] */
static void stage_combination(const rk_scheme *R, int i, long n, double dt, double *const *X,
                              double *const *LX, double *out)
{
    #pragma omp parallel for schedule(static)
    for (long e = 0; e < n; ++e) {
        double acc = 0.0;
        for (int j = 0; j < i; ++j) acc += R->alpha[i - 1][j] * X[j][e] + R->beta[i - 1][j] * dt * LX[j][e];
        out[e] = acc;
    }
}

/* The scheme of a configuration on the scalar linear test equation du/dt = lambda u,
 * with the same stage arithmetic as orc_rk_step (used to pin the coefficients). */
double orc_rk_linear(const orc_cfg *cfg, double lambda, double dt, double u0)
{
    const rk_scheme *R = scheme_of(cfg);
    double xs[RK_SMAX + 1], ls[RK_SMAX + 1];
    double *X[RK_SMAX + 1], *LX[RK_SMAX + 1];
    for (int j = 0; j <= RK_SMAX; ++j) { X[j] = &xs[j]; LX[j] = &ls[j]; }
    xs[0] = u0;
    for (int i = 1; i <= R->stages; ++i) {
        ls[i - 1] = lambda * xs[i - 1];
        stage_combination(R, i, 1, dt, X, LX, &xs[i]);
    }
    return xs[R->stages];
}

/* Number of right-hand-side evaluations per step of a configuration. */
int orc_rk_stages(const orc_cfg *cfg) { return scheme_of(cfg)->stages; }

/* One Runge-Kutta step in place with the positivity limiter after every stage
 * (Sec. 3.1: positivity checked in all intermediate Runge-Kutta steps; dt too large
 * when a flat cell cannot be fixed).  Returns ORC_RETRY with u restored to u^n when
 * any cell mean fell to or below the floor. */
int orc_rk_step(const orc_cfg *cfg, double *u, double dt, const double *modes, int nmodes,
                const double *nu, const int *fallback)
{
    if (check_cfg(cfg)) return ORC_EINVAL;
    const rk_scheme *R = scheme_of(cfg);
    int nb = orc_nbasis(cfg->k);
    long n = (long)NV * nb * ncell_of(cfg);
    double *X[RK_SMAX + 1], *LX[RK_SMAX];
    for (int j = 0; j <= R->stages; ++j) X[j] = malloc(sizeof(double) * n);
    for (int j = 0; j < R->stages; ++j) LX[j] = malloc(sizeof(double) * n);
    memcpy(X[0], u, sizeof(double) * n);
    int status = ORC_OK;
    for (int i = 1; i <= R->stages; ++i) {
        orc_rhs(cfg, X[i - 1], LX[i - 1], dt, modes, nmodes, nu, fallback);
        stage_combination(R, i, n, dt, X, LX, X[i]);
        if (cfg->flags & ORC_POS_LIMITER) {
            if (orc_limit(cfg, X[i], NULL) > 0) { status = ORC_RETRY; break; }
        }
    }
    if (status == ORC_OK) memcpy(u, X[R->stages], sizeof(double) * n);
    for (int j = 0; j <= R->stages; ++j) free(X[j]);
    for (int j = 0; j < R->stages; ++j) free(LX[j]);
    return status;
}

/* ------------------------------------------------------ global diagnostics */

/* Conserved totals (mass, momentum): w_0 is the cell mean (orthonormality,
 * Sec. 2.2), so M = h^3 sum_K W_rho,0 and P_d = h^3 sum_K W_m_d,0. */
int orc_conserved_sums(const orc_cfg *cfg, const double *u, double out[4])
{
    if (check_cfg(cfg)) return ORC_EINVAL;
    int nb = orc_nbasis(cfg->k);
    long nc = ncell_of(cfg);
    double h3 = cfg->h * cfg->h * cfg->h;
    for (int v = 0; v < NV; ++v) {
        double s = 0.0;
        for (long c = 0; c < nc; ++c) s += U(u, nb, nc, v, 0, c);
        out[v] = h3 * s;
    }
    return ORC_OK;
}

/* ---------------------------------------------- projection of given fields */

/* Physical coordinates of an nq^3 Gauss-Legendre rule in every cell (for projecting
 * initial conditions and measuring errors): xyz[cell][q][3], q = qx + nq (qy + nq qz). */
int orc_points(const orc_cfg *cfg, int nq, double *xyz)
{
    if (check_cfg(cfg) || nq < 1 || nq > 8) return ORC_EINVAL;
    double g[8], w[8];
    orc_gauss(nq, g, w);
    long nc = ncell_of(cfg);
    long np = (long)nq * nq * nq;
    for (long c = 0; c < nc; ++c)
        for (int qz = 0; qz < nq; ++qz)
            for (int qy = 0; qy < nq; ++qy)
                for (int qx = 0; qx < nq; ++qx) {
                    long q = qx + nq * (qy + (long)nq * qz);
                    double xi[3] = {g[qx], g[qy], g[qz]}, x[3];
                    position(cfg, c, xi, x);
                    for (int a = 0; a < 3; ++a) xyz[(c * np + q) * 3 + a] = x[a];
                }
    return ORC_OK;
}

/* Projection of sampled fields onto the basis (Sec. 3.2, eq. weights_equation,
 * w_l = (1/|K|) Int f phi_l dV with an nq-point rule): vals[var][cell][q] -> w[var][mode][cell]. */
int orc_project_values(const orc_cfg *cfg, int nq, int nvar, const double *vals, double *w)
{
    if (check_cfg(cfg) || nq < 1 || nq > 8) return ORC_EINVAL;
    double g[8], gw[8];
    orc_gauss(nq, g, gw);
    int nb = orc_nbasis(cfg->k);
    long nc = ncell_of(cfg);
    long np = (long)nq * nq * nq;
    #pragma omp parallel for schedule(static)
    for (long c = 0; c < nc; ++c) {
        double acc[NV * 2 * NBMAX];
        for (int i = 0; i < nvar * nb; ++i) acc[i] = 0.0;
        for (int qz = 0; qz < nq; ++qz)
            for (int qy = 0; qy < nq; ++qy)
                for (int qx = 0; qx < nq; ++qx) {
                    long q = qx + nq * (qy + (long)nq * qz);
                    double xi[3] = {g[qx], g[qy], g[qz]};
                    double wq = gw[qx] * gw[qy] * gw[qz];
                    for (int l = 0; l < nb; ++l) {
                        double phi;
                        orc_basis_eval(cfg->k, l, xi, &phi, NULL);
                        for (int v = 0; v < nvar; ++v)
                            acc[v * nb + l] += 0.125 * wq * phi * vals[((long)v * nc + c) * np + q];
                    }
                }
        for (int v = 0; v < nvar; ++v)
            for (int l = 0; l < nb; ++l) w[((long)v * nb + l) * nc + c] = acc[v * nb + l];
    }
    return ORC_OK;
}

/* Values of the expansions at an nq^3 Gauss-Legendre rule: out[var][cell][q]. */
int orc_eval_points(const orc_cfg *cfg, int nq, int nvar, const double *w, double *out)
{
    if (check_cfg(cfg) || nq < 1 || nq > 8) return ORC_EINVAL;
    double g[8], gw[8];
    orc_gauss(nq, g, gw);
    int nb = orc_nbasis(cfg->k);
    long nc = ncell_of(cfg);
    long np = (long)nq * nq * nq;
    #pragma omp parallel for schedule(static)
    for (long c = 0; c < nc; ++c)
        for (int qz = 0; qz < nq; ++qz)
            for (int qy = 0; qy < nq; ++qy)
                for (int qx = 0; qx < nq; ++qx) {
                    long q = qx + nq * (qy + (long)nq * qz);
                    double xi[3] = {g[qx], g[qy], g[qz]};
                    double phi[NBMAX];
                    for (int l = 0; l < nb; ++l) orc_basis_eval(cfg->k, l, xi, &phi[l], NULL);
                    for (int v = 0; v < nvar; ++v)
                        out[((long)v * nc + c) * np + q] = expand(w, nb, nc, v, c, phi);
                }
    return ORC_OK;
}

/* L1 error norm of eq. l1_norm (Sec. 2.2) averaged over all cells, per variable,
 * with an nq-point rule: exact[var][cell][q] are the exact values at orc_points. */
int orc_l1_error(const orc_cfg *cfg, int nq, int nvar, const double *w, const double *exact, double *l1)
{
    if (check_cfg(cfg) || nq < 1 || nq > 8) return ORC_EINVAL;
    double g[8], gw[8];
    orc_gauss(nq, g, gw);
    int nb = orc_nbasis(cfg->k);
    long nc = ncell_of(cfg);
    long np = (long)nq * nq * nq;
    for (int v = 0; v < nvar; ++v) l1[v] = 0.0;
    for (long c = 0; c < nc; ++c)
        for (int qz = 0; qz < nq; ++qz)
            for (int qy = 0; qy < nq; ++qy)
                for (int qx = 0; qx < nq; ++qx) {
                    long q = qx + nq * (qy + (long)nq * qz);
                    double xi[3] = {g[qx], g[qy], g[qz]};
                    double wq = 0.125 * gw[qx] * gw[qy] * gw[qz];
                    double phi[NBMAX];
                    for (int l = 0; l < nb; ++l) orc_basis_eval(cfg->k, l, xi, &phi[l], NULL);
                    for (int v = 0; v < nvar; ++v)
                        l1[v] += wq * fabs(exact[((long)v * nc + c) * np + q] - expand(w, nb, nc, v, c, phi));
                }
    for (int v = 0; v < nvar; ++v) l1[v] /= (double)nc;
    return ORC_OK;
}

/* -------------------------------------------------- learned-sensor pieces */

/* Per-cell input features of the learned sensor (degree 2 only, 20 values):
 *   [0..5]   density shape W_rho,l / W_rho,0 for the modes (100),(010),(001),(200),(020),(002)
 *   [6]      log10 W_rho,0
 *   [7..15]  cell-mean velocity gradient G_de = (2 sqrt(3)/h) Vhat_d,(unit e), scaled by (h/p)/cs
 *   [16..18] slopes D_i of the divergence of vhat across the cell (div = D0 + sum D_i xi_i,
 *            physical units), scaled by (h/p)/cs
 *   [19]     |mean velocity| / cs with mean velocity = Vhat_d,0
 * x[cell][20]. */
int orc_sensor_features(const orc_cfg *cfg, const double *u, double *x)
{
    if (check_cfg(cfg) || cfg->k != 2) return ORC_EINVAL;
    tabs_t *T = malloc(sizeof(tabs_t));
    make_tabs(cfg->k, T);
    long nc = ncell_of(cfg);
    int nb = T->nb;
    double hp = cfg->h / (cfg->k + 1);
    #pragma omp parallel for schedule(static)
    for (long c = 0; c < nc; ++c) {
        double vh[3 * NBMAX];
        project_cell(T, u, nc, c, vh);
        double r0 = U(u, nb, nc, 0, 0, c);
        double *xc = x + c * 20;
        /* density: linear modes (100),(010),(001) and axis quadratics (200),(020),(002) */
        static const int dmode[6] = {1, 2, 3, 4, 7, 9};
        for (int i = 0; i < 6; ++i) xc[i] = U(u, nb, nc, 0, dmode[i], c) / r0;
        xc[6] = log10(r0);
        /* cell-mean velocity gradient from the linear modes of vhat: d/dxi Lt_1 = sqrt(3) */
        for (int d = 0; d < 3; ++d)
            for (int e = 0; e < 3; ++e)
                xc[7 + 3 * d + e] = (hp / cfg->cs) * (2.0 * sqrt(3.0) / cfg->h) * vh[d * nb + 1 + e];
        /* slopes of the divergence of vhat across the cell: div vhat is linear in xi at
         * degree 2, div = D0 + sum_i D_i xi_i, and D_i = 3 * (1/8) int div xi_i (exact with
         * the (k+1)-point rule) */
        double slope[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < T->nq; ++q) {
            double divv = 0.0;
            for (int d = 0; d < 3; ++d)
                for (int l = 0; l < nb; ++l) divv += vh[d * nb + l] * T->vdphi[q][d][l];
            for (int i = 0; i < 3; ++i) slope[i] += 3.0 * 0.125 * T->vw[q] * divv * T->vxi[q][i];
        }
        for (int i = 0; i < 3; ++i) xc[16 + i] = (hp / cfg->cs) * (2.0 / cfg->h) * slope[i];
        double vm = sqrt(vh[0] * vh[0] + vh[nb] * vh[nb] + vh[2 * nb] * vh[2 * nb]);
        xc[19] = vm / cfg->cs;
    }
    free(T);
    return ORC_OK;
}

/* Plain-sensor label of a cell: the vNR bulk viscosity nu(s) = alpha (h/p)^2 s + beta cs
 * (h/p) (Pi = rho nu s without the Pi_max cap) averaged over the compressed interior
 * points (s = -div v > 0) with weights omega_q s_q, so that rho nu_K s reproduces the
 * cell's quadrature sum of the vNR pressure where rho is uniform:
 *   nu_K = sum omega s nu(s) / sum omega s;  0 when no point is compressed. */
int orc_sensor_labels(const orc_cfg *cfg, const double *u, double *nu)
{
    if (check_cfg(cfg)) return ORC_EINVAL;
    tabs_t *T = malloc(sizeof(tabs_t));
    make_tabs(cfg->k, T);
    long nc = ncell_of(cfg);
    int nb = T->nb;
    double hp = cfg->h / (cfg->k + 1);
    #pragma omp parallel for schedule(static)
    for (long c = 0; c < nc; ++c) {
        double vh[3 * NBMAX];
        project_cell(T, u, nc, c, vh);
        double num = 0.0, den = 0.0;
        for (int q = 0; q < T->nq; ++q) {
            double divv = 0.0;
            for (int d = 0; d < 3; ++d)
                for (int l = 0; l < nb; ++l) divv += vh[d * nb + l] * T->vdphi[q][d][l];
            divv *= 2.0 / cfg->h;
            if (divv < 0.0) {
                double sq = -divv;
                double nuq = cfg->alpha * hp * hp * sq + cfg->beta * cfg->cs * hp;
                num += T->vw[q] * sq * nuq;
                den += T->vw[q] * sq;
            }
        }
        nu[c] = den > 0.0 ? num / den : 0.0;
    }
    free(T);
    return ORC_OK;
}

/* ------------------------------------------------------------ flow statistics
 * Velocity structure function and the velocity grid for power spectra (Sec. 4.3, the
 * definition of the scale-dependent velocity v(l), and the subsection on measuring
 * structure functions and power spectra).
 *
 * Random numbers: the counter-based SplitMix64 generator (Steele, Lea & Flood 2014):
 * draw i of stream `seed` is the SplitMix64 output for the state seed + (i+1) gamma,
 * gamma = 0x9E3779B97F4A7C15, and a uniform double in [0,1) is its top 53 bits times
 * 2^-53.  Pair j of bin b owns the draws 256 (b npairs + j) + t, t < 256.
 *
 * Readings (the paper gives the recipe in words):
 *   - bins: nbins log-spaced bins between the resolution limit h/(k+1) and half the
 *     shortest box side; the distance of bin b is the geometric centre
 *     lmin (lmax/lmin)^((b + 1/2)/nbins);
 *   - first point uniform in the box (draws t = 0, 1, 2); direction uniform on the unit
 *     sphere by rejection from the cube [-1,1]^3 (attempt a uses draws 3 + 3a + 0..2,
 *     accepted when 1e-12 < r^2 <= 1, at most 84 attempts, else +z); second point
 *     x + l n (one fused multiply-add per axis), wrapped into the periodic box;
 *   - velocity v = m / max(rho, rho_floor) from the expansions of the cell that holds the
 *     point (positivity is only enforced at the Gauss points), cell index floor(x/h)
 *     clamped to the mesh;
 *   - S2(l) = mean over the pairs of |v(x) - v(x + l n)|^2; v(l) = sqrt(S2 / 2).
 */
uint64_t orc_splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double uniform01(uint64_t seed, uint64_t i)
{
    return (double)(orc_splitmix64(seed, i) >> 11) * 0x1.0p-53;
}

static void box_of(const orc_cfg *cfg, double L[3])
{
    L[0] = cfg->nx * cfg->h;
    L[1] = cfg->ny * cfg->h;
    L[2] = cfg->nz * cfg->h;
}

int orc_sf_bins(const orc_cfg *cfg, int nbins, double *l)
{
    if (check_cfg(cfg) || nbins < 1) return ORC_EINVAL;
    double L[3];
    box_of(cfg, L);
    double lmax = 0.5 * fmin(L[0], fmin(L[1], L[2]));
    double lmin = cfg->h / (cfg->k + 1);
    for (int b = 0; b < nbins; ++b) l[b] = lmin * pow(lmax / lmin, (b + 0.5) / nbins);
    return ORC_OK;
}

/* the two points of pair `pair` at distance l */
void orc_sf_pair(const orc_cfg *cfg, uint64_t seed, uint64_t pair, double l, double x1[3], double x2[3])
{
    double L[3];
    box_of(cfg, L);
    const uint64_t base = pair * 256u;
    for (int a = 0; a < 3; ++a) x1[a] = uniform01(seed, base + a) * L[a];
    double n[3] = {0.0, 0.0, 1.0};
    for (int t = 0; t < 84; ++t) {
        double c[3];
        for (int a = 0; a < 3; ++a) c[a] = 2.0 * uniform01(seed, base + 3 + 3 * t + a) - 1.0;
        double r2 = fma(c[2], c[2], fma(c[1], c[1], c[0] * c[0]));
        if (r2 > 1e-12 && r2 <= 1.0) {
            double r = sqrt(r2);
            for (int a = 0; a < 3; ++a) n[a] = c[a] / r;
            break;
        }
    }
    for (int a = 0; a < 3; ++a) {
        double y = fma(l, n[a], x1[a]);
        if (y >= L[a]) y -= L[a];
        else if (y < 0.0) y += L[a];
        x2[a] = y;
    }
}

/* v = m / max(rho, floor) at a point of the box */
void orc_velocity_at(const orc_cfg *cfg, const double *u, const double x[3], double v[3])
{
    int n[3] = {cfg->nx, cfg->ny, cfg->nz}, ijk[3];
    double xi[3];
    for (int a = 0; a < 3; ++a) {
        double s = x[a] / cfg->h;
        int i = (int)floor(s);
        if (i < 0) i = 0;
        if (i > n[a] - 1) i = n[a] - 1;
        ijk[a] = i;
        xi[a] = 2.0 * (s - i) - 1.0;
    }
    long c = cell_id(cfg, ijk[0], ijk[1], ijk[2]);
    int nb = orc_nbasis(cfg->k);
    long nc = ncell_of(cfg);
    double phi[NBMAX];
    for (int l = 0; l < nb; ++l) orc_basis_eval(cfg->k, l, xi, &phi[l], NULL);
    double rho = fmax(expand(u, nb, nc, 0, c, phi), cfg->rho_floor);
    for (int d = 0; d < 3; ++d) v[d] = expand(u, nb, nc, 1 + d, c, phi) / rho;
}

/* S2 of the bins b0 .. b0+nsel-1 of an nbins-bin measurement with npairs pairs per bin
 * (the pairs of a bin do not depend on the other bins, so bins can be computed alone). */
int orc_structure_function(const orc_cfg *cfg, const double *u, int nbins, int b0, int nsel, const double *l,
                           long npairs, uint64_t seed, double *s2)
{
    if (check_cfg(cfg) || nbins < 1 || b0 < 0 || nsel < 0 || b0 + nsel > nbins || npairs < 1) return ORC_EINVAL;
    #pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < nsel; ++i) {
        int b = b0 + i;
        double sum = 0.0;
        for (long j = 0; j < npairs; ++j) {
            double x1[3], x2[3], v1[3], v2[3];
            orc_sf_pair(cfg, seed, (uint64_t)b * (uint64_t)npairs + (uint64_t)j, l[b], x1, x2);
            orc_velocity_at(cfg, u, x1, v1);
            orc_velocity_at(cfg, u, x2, v2);
            for (int d = 0; d < 3; ++d) sum += (v1[d] - v2[d]) * (v1[d] - v2[d]);
        }
        s2[i] = sum / (double)npairs;
    }
    return ORC_OK;
}

/* Velocity on the uniform grid of p points per cell per dimension (cell-centred
 * sub-points xi_s = -1 + (2s+1)/p; the N p grid of the paper's spectra):
 * grid[d][z][y][x], x fastest, (nz p) x (ny p) x (nx p) points. */
int orc_velocity_grid(const orc_cfg *cfg, const double *u, int p, double *grid)
{
    if (check_cfg(cfg) || p < 1) return ORC_EINVAL;
    long X = (long)cfg->nx * p, Y = (long)cfg->ny * p, Z = (long)cfg->nz * p;
    long npts = X * Y * Z;
    int nb = orc_nbasis(cfg->k);
    long nc = ncell_of(cfg);
    #pragma omp parallel for schedule(static)
    for (long gz = 0; gz < Z; ++gz)
        for (long gy = 0; gy < Y; ++gy)
            for (long gx = 0; gx < X; ++gx) {
                long g[3] = {gx, gy, gz};
                int ijk[3];
                double xi[3];
                for (int a = 0; a < 3; ++a) {
                    ijk[a] = (int)(g[a] / p);
                    xi[a] = -1.0 + (2.0 * (double)(g[a] % p) + 1.0) / p;
                }
                long c = cell_id(cfg, ijk[0], ijk[1], ijk[2]);
                double phi[NBMAX];
                for (int l = 0; l < nb; ++l) orc_basis_eval(cfg->k, l, xi, &phi[l], NULL);
                double rho = fmax(expand(u, nb, nc, 0, c, phi), cfg->rho_floor);
                long o = gx + X * (gy + Y * gz);
                for (int d = 0; d < 3; ++d) grid[d * npts + o] = expand(u, nb, nc, 1 + d, c, phi) / rho;
            }
    return ORC_OK;
}
