/*
 * dg.h -- C ABI of libdg: the modal Discontinuous Galerkin right-hand side and
 * SSP-RK3 stage update for 3D isothermal Euler on a periodic Cartesian mesh, on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Cernetic, Springel, Guillet & Pakmor (2024), "Supersonic turbulence
 * simulations with GPU-based high-order Discontinuous Galerkin hydrodynamics",
 * Sec. 2 (modal Legendre basis, Gauss quadrature, weak form), Sec. 3.1 (von
 * Neumann-Richtmyer artificial viscosity, positivity), Sec. 3.2 (primitive
 * projection), Sec. 4.2 (solenoidal Ornstein-Uhlenbeck driving), Sec. 7 (cost,
 * time step scaling).
 *
 * Conventions used by every entry point:
 *   - cells: nx * ny * nz cubes of edge h, periodic; cell = i + nx*(j + ny*l).
 *   - basis: phi_(a,b,c)(xi) = Lt_a(xi_1) Lt_b(xi_2) Lt_c(xi_3), Lt_n = sqrt(2n+1) P_n,
 *     a+b+c <= k, nb = (k+1)(k+2)(k+3)/6 modes ordered by total degree ascending, then a
 *     descending, then b descending; xi = 2(x - x_K)/h; (1/|K|) Int phi_l phi_m = delta_lm,
 *     so mode 0 is the cell mean.
 *   - state u: the weights, stored [var][mode][cell] (var = rho, m_x, m_y, m_z), contiguous,
 *     element type double (DG_FP64) or float (DG_FP32), in DEVICE memory owned by the caller.
 *   - projected velocity vhat: [dir][mode][cell], same element type.
 *   - every device array an entry point is handed (state, output, workspace, scratch) must
 *     lie inside one allocation the HIP runtime tracks (hipMalloc, hipMallocManaged,
 *     hipHostMalloc, pools and mapped ranges), aligned to its element size: a null pointer,
 *     a pointer the runtime cannot place in an allocation, or an array that would run past
 *     the end of its allocation is rejected with DG_EINVAL before anything is launched.
 *   - every call is asynchronous on the stream given in the configuration unless it says
 *     it synchronises.  Calls on one context must not overlap in time (one stream).
 *   - return value: DG_OK (0); DG_RETRY (1, recoverable); negative on error, with a
 *     message from dg_last_error.  No C++ exception crosses the ABI.
 */
#ifndef DG_H
#define DG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum dg_status {
    DG_OK = 0,
    DG_RETRY = 1,          /* positivity failure: retry the step with a smaller dt (Sec. 3.1) */
    DG_EINVAL = -1,        /* null / misaligned / unallocated pointer, array past its allocation's end,
                              bad size or parameter */
    DG_EUNSUPPORTED = -2,  /* degree outside 1..3, feature not available for this degree */
    DG_EHIP = -3,          /* a HIP runtime call failed (text in dg_last_error) */
    DG_ENOMEM = -4,        /* workspace missing or too small */
    DG_ESTATE = -5         /* call order violated (e.g. learned sensor without weights) */
};

enum dg_precision { DG_FP64 = 0, DG_FP32 = 1 };

enum dg_flags {
    DG_AV = 1,                 /* von Neumann-Richtmyer viscous pressure in the volume flux (Sec. 3.1) */
    DG_PRIM_PROJ = 2,          /* face velocities from the projected velocity polynomial (Sec. 3.2) */
    DG_FORCING = 4,            /* driving acceleration source rho a in the momentum rows (Sec. 4.2) */
    DG_POS_LIMITER = 8,        /* positivity limiter after every stage (Sec. 3.1) */
    DG_LEARNED_SENSOR = 16,    /* viscosity from the learned per-cell sensor (not in the paper) */
    DG_FORCE_MEANFREE = 32,    /* remove the mass-weighted mean acceleration (exact momentum conservation) */
    DG_HLLC = 64,              /* HLLC-type interface flux instead of Rusanov: the isothermal counterpart of
                                  the HLLC solver of Sec. 2.2 (HLL for density and normal momentum,
                                  tangential momentum carried by the mass flux, upwinded) */
    DG_RK_BY_ORDER = 128,      /* SSP Runge-Kutta scheme by degree (Sec. 7: k+1 stages per step): two stages
                                  (second order) at degree 1, three at degree 2, five stages of fourth order
                                  at degree 3; without it every degree uses three stages (third order) */
    DG_VOLUME_MFMA = 256,      /* FP32 at degree 2 only (DG_EUNSUPPORTED otherwise): the volume integral's
                                  evaluation at the points and its flux and driving contractions (Sec. 2.2,
                                  Sec. 7: the dominant dense products) on the matrix cores instead of the
                                  vector units; same results within the FP32 tolerance; tables off the
                                  driving shell keep the vector form */
    DG_SEPARATE_STAGE = 512,   /* every Runge-Kutta stage of a step as its own kernel after the stored
                                  right-hand side */
    DG_SPLIT_STAGE = 1024      /* the stages without a side combination split between the right-hand-side
                                  kernel, which forms the stage's combination instead of storing the
                                  right-hand side, and a kernel that limits and projects it (the last
                                  stage: the stage kernel, which writes the caller's array from the
                                  combination unless a cell failed).  The same results as DG_SEPARATE_STAGE (bit for bit, or to rounding
                                  with mean-free driving on the driving shell, whose mean the split path
                                  sums in modal form).  With neither flag the split is used where it
                                  measured faster (meshes of at least 2^21 cells); the two-lane FP64
                                  degree-3 kernel and DG_VOLUME_MFMA never split.  Both flags together:
                                  DG_EINVAL */
};

typedef struct dg_config {
    int nx, ny, nz;        /* cells per dimension, each >= 1 */
    int degree;            /* polynomial degree k in {1, 2, 3} (spatial order k+1) */
    int precision;         /* DG_FP64 or DG_FP32 (bulk arithmetic; reductions are FP64 always) */
    int flags;             /* OR of dg_flags */
    double h;              /* cell edge; <= 0 selects 1/nx (unit box along x) */
    double cs;             /* isothermal sound speed (pressure = cs^2 rho) */
    double cfl;            /* Courant factor of dg_dt_max */
    double alpha_visc;     /* quadratic vNR coefficient (paper default 2) */
    double beta_visc;      /* linear (bulk) coefficient (paper default 0.2) */
    double rho_floor;      /* positivity floor of the density (1e-3) */
    double rho_floor_rel;  /* the limiter lifts the minimum point density to max(rho_floor,
                              rho_floor_rel * cell mean) (0.1; 0 = absolute floor only) */
    double cfl_visc;       /* viscous stability factor of dg_dt_max (0.1; <= 0 disables) */
    void *stream;          /* hipStream_t for every launch; NULL = default stream */
} dg_config;

typedef struct dg_ctx dg_ctx;

/* Fill a configuration with the defaults: k = 2, FP64, AV | PRIM_PROJ | POS_LIMITER,
 * h = 1/nx, cs = 1, cfl = 0.3, alpha = 2, beta = 0.2 (Sec. 3.1), floor 1e-3, relative
 * floor 0.1, viscous factor 0.1. */
void dg_config_default(dg_config *cfg, int nx, int ny, int nz);

/* Create a context: checks the configuration, builds the basis / quadrature tables on
 * the host in FP64 and uploads them (small, owned by the context).  *out = NULL on error.
 * Errors: DG_EINVAL (null, bad sizes), DG_EUNSUPPORTED (degree), DG_EHIP. */
int dg_init(const dg_config *cfg, dg_ctx **out);

/* Release the context and its small device tables (not the caller's workspace). */
void dg_free(dg_ctx *ctx);

/* Text of the last error on this context (static storage inside the context). */
const char *dg_last_error(const dg_ctx *ctx);

/* Wall-clock bound, in seconds, of the host wait inside dg_rk_step_next and
 * dg_rk_step_next_ahead for the step's published status (default 300).  When the bound is
 * exceeded the call returns DG_EHIP while the step's kernels may still be running on the
 * stream: the caller must synchronise the stream before using or discarding the state.
 * The step, once finished, leaves the state it would have left.  Errors: DG_EINVAL
 * (seconds not positive; +infinity waits without a bound). */
int dg_set_wait_limit(dg_ctx *ctx, double seconds);

/* Bytes of device scratch the caller must provide (traces, projected velocity, Runge-Kutta
 * temporaries, driving field at the quadrature points, reduction partials, flags). */
size_t dg_workspace_bytes(const dg_ctx *ctx);

/* Hand a device workspace of at least dg_workspace_bytes() bytes, 256-byte aligned, to
 * the context.  The caller owns it and must keep it alive.  Errors: DG_EINVAL, DG_ENOMEM. */
int dg_set_workspace(dg_ctx *ctx, void *ws, size_t bytes);

/* Driving modes (Sec. 4.2): modes_host[nmodes][9] = (n_x, n_y, n_z, Re a_x, Im a_x,
 * Re a_y, Im a_y, Re a_z, Im a_z), host memory, FP64; the acceleration is
 * a(x) = sum_m Re[a_m exp(2 pi i n_m . x)] with x in box units (cell centres at (i+1/2)h).
 * The table is copied; the field at the quadrature points is rebuilt before the next
 * right-hand side.  nmodes in 0..64.  Errors: DG_EINVAL. */
int dg_set_forcing(dg_ctx *ctx, const double *modes_host, int nmodes);

/* Right-hand side dudt = d(weights)/dt of the weak form (Sec. 2.2, weight evolution):
 * volume flux quadrature with the viscous pressure at interior points, Rusanov fluxes at
 * the face points, surface lift, driving source.  u and dudt: [4][nb][ncell] device
 * arrays; dudt is fully overwritten.  dt is the step size used by the Pi_max cap
 * (Sec. 3.1); dt <= 0 disables the cap.  With DG_LEARNED_SENSOR the per-cell viscosity
 * nu stored by dg_sensor_infer / dg_sensor_set_nu (DG_ESTATE if none) is the bulk
 * viscosity of cells whose fallback flag is 0: Pi = min(rho nu s, Pi_max) at compressed
 * points (s = -div vhat > 0), none at expanding points.
 * Errors: DG_EINVAL, DG_ENOMEM (no workspace), DG_ESTATE. */
int dg_rhs(dg_ctx *ctx, const void *u, void *dudt, double dt);

/* One SSP Runge-Kutta step in place (Shu-Osher form; three stages of third order, or the
 * scheme chosen by DG_RK_BY_ORDER; with DG_LEARNED_SENSOR
 * the stored per-cell viscosity serves the three stages: call dg_sensor_infer on u^n
 * first, DG_ESTATE if none is stored), positivity limiter
 * after every stage when DG_POS_LIMITER is set (Sec. 3.1: all high-order weights of a cell
 * scaled by one factor so that the density at every volume and face Gauss point is at
 * least max(rho_floor, rho_floor_rel * cell mean)).  Synchronises the stream once to read
 * the 4-byte status into *status_host (may be NULL).  Returns DG_RETRY, with u left at its
 * value at entry, when a cell mean fell to or below the floor, i.e. the caller must retry
 * with a smaller dt (Sec. 3.1): only the last stage writes u, its failure is decided before
 * it writes, and once any stage has failed it writes nothing. */
int dg_rk_step(dg_ctx *ctx, void *u, double dt, int *status_host);

/* The same step, also returning the time step of the new state: on DG_OK,
 * *dt_next_host equals dg_dt_max of u^(n+1) (same definition and FP64 reduction, computed
 * inside the last stage), and the projection of u^(n+1) is kept in the workspace.
 * reuse = 1 states that u has not been modified since the previous dg_rk_step_next call
 * on this context returned DG_OK for the same array; the step then starts from the kept
 * projection.  The library additionally checks the array pointer and that no other
 * state-changing call (dg_rhs, dg_rk_step, dg_limit, dg_set_workspace) came in between,
 * and recomputes the projection otherwise; it cannot see writes made outside libdg.
 * One wait per call: the step's last kernel stores the status and dt_next into pinned host
 * memory and the call returns once they are visible, when every other kernel of the step has
 * completed.  With
 * DG_LEARNED_SENSOR the stages use the stored viscosity (of u^n), and after the last stage
 * the network runs on u^(n+1) (as dg_sensor_infer would): its viscosity is stored for the
 * next step and enters *dt_next_host, which then equals dg_sensor_infer followed by
 * dg_dt_max of u^(n+1).  On DG_RETRY u is u^n and the stored viscosity is that of u^n.
 * A judge call between steps changes the fallback flags: take dg_dt_max afterwards instead
 * of the returned value.  DG_ESTATE when no viscosity is stored yet. */
int dg_rk_step_next(dg_ctx *ctx, void *u, double dt, int reuse, int *status_host, double *dt_next_host);

/* dg_rk_step_next that also launches the next step's first stage ahead of the caller: when
 * the step succeeds and *dt_next_host < horizon, the right-hand side, mean acceleration and
 * stage kernel of the first stage of the next step (from u^(n+1), with *dt_next_host) are
 * queued before the call returns.  They write only workspace buffers.  The next
 * dg_rk_step_next or dg_rk_step_next_ahead call on the same array with dt equal to that
 * time step and reuse = 1 continues from them instead of launching them again, so the GPU
 * is not idle while the caller prepares the call.  Any other outcome discards them:
 *   - a different array or time step, or reuse = 0;
 *   - a state-changing call in between (dg_rhs, dg_rk_step, dg_limit, dg_set_workspace);
 *   - dg_set_forcing, dg_forcing_ou_advance or dg_forcing_ou_set;
 *   - any dg_sensor_set_params, dg_sensor_infer, dg_sensor_judge or dg_sensor_set_nu.
 * The results are the same either way.  horizon <= 0 never launches ahead; a driver passes the
 * time left before its next driving update, so that no launched stage is discarded for one.
 * Errors as dg_rk_step_next; DG_EINVAL for a NaN horizon. */
int dg_rk_step_next_ahead(dg_ctx *ctx, void *u, double dt, int reuse, double horizon, int *status_host,
                          double *dt_next_host);

/* 1 when the steps of this context split their stages between the right-hand-side kernel
 * (which forms the stage's combination) and a limit-and-project kernel, the last stage's
 * stage kernel writing the caller's array from the combination (DG_SPLIT_STAGE, or the
 * default choice for the mesh and precision; the SSP-RK
 * combination of Sec. 2.2 / 7 with the limiter of Sec. 3.1 either way), else 0; DG_EINVAL
 * for a null context.  No device call. */
int dg_split_stages(const dg_ctx *ctx);

/* Time step dt = min(dt_adv, dt_visc), reduced in FP64 over all cells and interior points:
 * dt_adv = cfl h / ((k+1) max sum_d (|m_d/rho| + cs)) (Sec. 7: dt proportional to h/(k+1));
 * with DG_AV and cfl_visc > 0, dt_visc = cfl_visc (h/p)^2 / max nu, the explicit stability
 * bound of the viscous pressure read as a bulk viscosity nu = alpha (h/p)^2 |div v| +
 * beta cs (h/p) at compressing points (Sec. 3.1; p = k+1); with DG_LEARNED_SENSOR a cell
 * whose fallback flag is 0 contributes its stored viscosity instead (DG_ESTATE if none is
 * stored).  on_host = 1: *dt_out is host memory and the call synchronises; on_host = 0:
 * *dt_out is device memory (8 bytes). */
int dg_dt_max(dg_ctx *ctx, const void *u, double *dt_out, int on_host);

/* dg_dt_max for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same time step, bit for bit,
 * without a workspace.  Its per-block maxima and the reduced value live in a static device
 * array of the library (1 MiB + 256 bytes per GPU, held until the process ends), so the call
 * allocates nothing and needs no dg_set_workspace.  Limit: at most 16,777,216 cells (65,536
 * blocks of 256 cells), DG_EINVAL beyond.  The array is shared by every context on a GPU
 * and keeps the last call's contents (nothing in it needs clearing): calls that overlap in
 * time on one GPU race, so issue them on one stream or serialise them.  The device current
 * at the call must be the context's.  on_host = 1: *dt_out is host memory and the call
 * synchronises; on_host = 0: *dt_out is device memory (8 bytes).  Errors: DG_EINVAL (null or
 * misaligned pointer, mesh too large, other device current), DG_EUNSUPPORTED (learned
 * sensor, whose viscosity lives in the workspace), DG_EHIP. */
int dg_dt_max_noalloc(dg_ctx *ctx, const void *u, double *dt_out, int on_host);

/* Projected velocity (Sec. 3.2, eq. weights_equation with the interior rule):
 * vhat_{d,l} = (1/8) sum_q w_q phi_l(q) m_d(q)/rho(q); vhat is [3][nb][ncell] device. */
int dg_project_primitive(dg_ctx *ctx, const void *u, void *vhat);

/* Apply the positivity limiter once (e.g. to initial conditions); synchronises;
 * *nfail_host = number of cells whose mean is at or below the floor. */
int dg_limit(dg_ctx *ctx, void *u, long *nfail_host);

/* Conserved totals (mass, momentum x/y/z) = h^3 sum_cells W_v,0 (Sec. 2.2: the basis is
 * orthonormal with phi_0 = 1, so the weight W_v,0 is the cell average of variable v and
 * |K| W_v,0 its content; the weak form conserves these totals), FP64 fixed-order
 * reduction; u is [4][nb][ncell] device memory; out_host[4] host memory; synchronises.
 * Errors: DG_EINVAL (null or misaligned pointer), DG_ENOMEM (no workspace). */
int dg_conserved_sums(dg_ctx *ctx, const void *u, double *out_host);

/* Instrumentation: launches issued by dg_rhs / dg_rk_step / dg_rk_step_next are bracketed
 * by HIP events on the context stream (without the system-scope fence) and the elapsed
 * times are accumulated (counters cleared).  Each event leaves the GPU idle for a few
 * microseconds, so enable = 1 brackets only the right-hand-side kernel of every dg_rhs and
 * of the first stage of every step (with split stages, DG_SPLIT_STAGE, that kernel also
 * forms the stage's combination); enable = 3 brackets only the right-hand side of the last
 * stage of every step (always stored for a stage kernel); enable = 2 brackets every
 * right-hand-side and stage launch (a split stage's limit-and-project kernel counts as a
 * stage launch); enable = 0 stops.  dg_profile_read synchronises and writes out_host[4] =
 * {RHS-kernel milliseconds, RHS launches, stage-kernel milliseconds, stage launches}. */
int dg_profile(dg_ctx *ctx, int enable);
int dg_profile_read(dg_ctx *ctx, double *out_host);

/* Ornstein-Uhlenbeck driving on the shell 1 <= |n| <= 2 (Sec. 4.2), host-side FP64:
 * dg_forcing_ou_init sets the correlation time t_c and the stationary standard deviation
 * sigma and zeroes the mode state; dg_forcing_ou_advance applies one update
 * x <- f x + sigma sqrt(1-f^2) z with f = exp(-dt_drive/t_c), z = the caller's standard
 * normal draws (z_host[dg_forcing_ou_ndraws()]), projects each mode onto the plane
 * perpendicular to n (solenoidal) and installs the table as by dg_set_forcing. */
int dg_forcing_ou_ndraws(void);
int dg_forcing_ou_init(dg_ctx *ctx, double t_c, double sigma);
int dg_forcing_ou_advance(dg_ctx *ctx, const double *z_host, double dt_drive);
/* The OU state itself (before the solenoidal projection), dg_forcing_ou_ndraws() doubles
 * of host memory: get copies it out; set replaces it (after dg_forcing_ou_init) and
 * installs its table, so a run can be resumed or copied with identical driving. */
int dg_forcing_ou_get(const dg_ctx *ctx, double *x_host);
int dg_forcing_ou_set(dg_ctx *ctx, const double *x_host);

/* Copy of the current mode table (nmodes_max rows of 9 doubles); returns nmodes. */
int dg_forcing_get(const dg_ctx *ctx, double *modes_host, int nmodes_max);

/* ---------------------------------------------------------------------------------
 * Learned shock sensor (not in the paper; stands in for the compression sensor of
 * Sec. 3.1).  Network Linear(20,64)-GELU-Linear(64,64)-GELU-Linear(64,1), bf16 weights
 * and activations on the matrix cores with FP32 accumulation.  Parameters are an FP32
 * device array of DG_MLP_NPARAM values: W1[64][20], b1[64], W2[64][64], b2[64], W3[1][64],
 * b3[1] (y = W x + b per layer).  The output t gives nu = 1e-3 (exp(t) - 1), clipped >= 0.
 * Degree 2 only (DG_EUNSUPPORTED otherwise).
 * ------------------------------------------------------------------------------- */
#define DG_MLP_NIN 20
#define DG_MLP_NHID 64
#define DG_MLP_NPARAM (64 * 20 + 64 + 64 * 64 + 64 + 64 + 1)

/* Per-cell features x[ncell][20] (float, device): density shape W_rho,l/W_rho,0 for the
 * modes (100),(010),(001),(200),(020),(002); log10 W_rho,0; cell-mean velocity gradient
 * (from the linear modes of vhat) times (h/(k+1))/cs; the three slopes of div vhat across
 * the cell (div vhat is linear at degree 2) times (h/(k+1))/cs; |mean velocity|/cs. */
int dg_sensor_features(dg_ctx *ctx, const void *u, float *x_dev);

/* Plain-sensor labels nu[ncell] (double, device): the vNR bulk viscosity
 * nu(s) = alpha (h/p)^2 s + beta cs (h/p) averaged over the compressed interior points
 * (s = -div vhat > 0) with weights omega_q s_q, 0 if none is compressed. */
int dg_sensor_labels(dg_ctx *ctx, const void *u, double *nu_dev);

/* Training targets t[ncell] (float, device): t = log(1 + nu/1e-3) of the plain-sensor
 * labels above, the network's output space.  Degree 2 only. */
int dg_sensor_targets(dg_ctx *ctx, const void *u, float *t_dev);

/* Install network parameters (FP32 device array, DG_MLP_NPARAM values, copied). */
int dg_sensor_set_params(dg_ctx *ctx, const float *params_dev);

/* Run features + network on u; the per-cell viscosity used by DG_LEARNED_SENSOR is
 * stored in the workspace. */
int dg_sensor_infer(dg_ctx *ctx, const void *u);

/* Judge: recompute the plain labels of u and mark for fallback (plain sensor) every
 * cell with |nu_learned - nu_plain| / (nu_plain + 1e-3) > tau; synchronises and returns
 * the number of marked cells in *nfallback_host (may be NULL). */
int dg_sensor_judge(dg_ctx *ctx, const void *u, double tau, long *nfallback_host);

/* Overwrite the stored per-cell viscosity (same element type as the state, device) and
 * fallback flags (int32 device, 1 = plain sensor); either pointer may be NULL to keep. */
int dg_sensor_set_nu(dg_ctx *ctx, const void *nu_dev, const int32_t *fallback_dev);

/* Network forward pass for n rows: x[n][20] float -> y[n] float (device). */
int dg_mlp_forward(dg_ctx *ctx, const float *params_dev, const float *x_dev, int n, float *y_dev);

/* Mean-squared-error loss and its gradient with respect to the parameters for n rows:
 * grad_dev[DG_MLP_NPARAM] float (overwritten), loss_dev[1] float (device). */
int dg_mlp_grad(dg_ctx *ctx, const float *params_dev, const float *x_dev, const float *t_dev,
                int n, float *grad_dev, float *loss_dev);

/* Adam update (Kingma & Ba) of the FP32 parameters in place; m_dev and v_dev are the
 * moment buffers (DG_MLP_NPARAM floats each, zero before step 1); step counts from 1. */
int dg_mlp_adam(dg_ctx *ctx, float *params_dev, const float *grad_dev, float *m_dev,
                float *v_dev, int step, float lr);

/* ---------------------------------------------------------------- flow statistics
 * Sec. 4.3 (the scale-dependent velocity v(l) and the subsection on measuring structure
 * functions and power spectra).  The velocity is v = m / max(rho, rho_floor) evaluated from
 * the expansions of the cell that holds a point (positivity is only enforced at the Gauss
 * points).  Both calls take a caller scratch buffer in DEVICE memory (256-byte aligned, at
 * least dg_stats_scratch_bytes bytes, contents not preserved), leave the state untouched,
 * and synchronise. */

/* The separations of an nbins-bin structure function: logarithmic bins between the
 * resolution limit h/(k+1) and half the shortest box side, each bin represented by its
 * geometric centre, l_b = lmin (lmax/lmin)^((b + 1/2)/nbins).  l_host[nbins] host memory. */
int dg_sf_bins(const dg_ctx *ctx, int nbins, double *l_host);

/* Scratch bytes for dg_structure_function with nbins bins (0: not needed) and for
 * dg_velocity_spectrum with p samples per cell (0: not needed); the larger of the two.
 * Structure function: 4 nb ncell doubles of cell records plus 65 nbins doubles.  Spectrum:
 * the velocity grid (3 X Y Z doubles), its half spectrum (3 (X/2+1) Y Z complex doubles)
 * and 1024 per-block shell histograms. */
size_t dg_stats_scratch_bytes(const dg_ctx *ctx, int nbins, int p);

/* Second-order velocity structure function S2(l_b) = mean over npairs random pairs of
 * |v(x) - v(x + l_b n)|^2 for every bin of dg_sf_bins (the paper's v(l) = sqrt(S2/2);
 * typically 100 bins of 1e5 pairs).  Pair j of bin b: first point uniform in the periodic
 * box, direction uniform on the unit sphere (rejection from the cube), second point wrapped
 * into the box; the random numbers are draws 256 (b npairs + j) + t of the counter-based
 * SplitMix64 stream `seed` (Steele, Lea & Flood 2014), so the pairs of a bin do not
 * depend on the other bins or on the launch shape.  FP64 evaluation and sums for either
 * state precision; deterministic.  s2_host[nbins] host memory.
 * Errors: DG_EINVAL (null/misaligned pointer, nbins outside 1..65535, npairs < 1),
 * DG_ENOMEM (scratch too small). */
int dg_structure_function(dg_ctx *ctx, const void *u, int nbins, long long npairs, unsigned long long seed,
                          void *scratch, size_t scratch_bytes, double *s2_host);

/* Number of integer shells K = 0 .. Kmax of the p-sample grid, Kmax = round(|(X/2, Y/2,
 * Z/2)|) with X = nx p etc. (integer division); negative on bad arguments. */
int dg_spectrum_nshell(const dg_ctx *ctx, int p);

/* Velocity power spectrum on the grid of p cell-centred points per cell per dimension
 * (sub-points xi_s = -1 + (2s+1)/p): e_host[K] = sum over wave vectors kappa (box units)
 * with round(|kappa|) = K of 1/2 |v_hat(kappa)|^2, v_hat = the discrete Fourier transform
 * divided by the number of grid points, so that sum_K e_host[K] = 1/2 <|v|^2> over the grid.
 * FP64 grid and FFT (hipFFT, double precision real-to-complex).  e_host has
 * dg_spectrum_nshell(p) entries (host memory).
 * Errors: DG_EINVAL (bad pointer, p < 1, fewer than 2 grid points along an axis),
 * DG_EUNSUPPORTED (more than 4096 shells), DG_ENOMEM (scratch too small), DG_EHIP. */
int dg_velocity_spectrum(dg_ctx *ctx, const void *u, int p, void *scratch, size_t scratch_bytes, double *e_host);

#ifdef __cplusplus
}
#endif

#endif /* DG_H */
