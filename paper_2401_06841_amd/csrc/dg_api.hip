// dg_api.hip -- host side of libdg: configuration checks, quadrature tables, workspace
// layout, kernel launches and the C ABI declared in include/dg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "dg.h"
#include "dg_ctx.hpp"
#include "dg_kernels.hpp"

using namespace dg;

// ------------------------------------------------------------ static scratch
// Device memory of dg_dt_max_noalloc, for callers that cannot allocate: the per-block
// time-step maxima (two doubles per block) and the reduced time step.  Every GPU the
// library runs on holds its own copy for the life of the process.  In host code the array's
// name is not a device address: its address on each device is looked up once, at the first
// dg_init with that device current, and only that address is handed to kernels.
constexpr int NOALLOC_MAX_BLOCKS = 65536;                        // 16,777,216 cells
constexpr int NOALLOC_DT_SLOT = 2 * NOALLOC_MAX_BLOCKS;
static __device__ __align__(256) double scratch[NOALLOC_DT_SLOT + 32];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex noalloc_mu;
double *noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// address of this device's copy of the scratch array (looked up once per device)
int noalloc_setup(dg_ctx *c, int dev)
{
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return DG_OK;      // the entry point reports it
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (noalloc_ptr[dev]) return DG_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return dg_fail(c, DG_EHIP, "hipGetSymbolAddress of the static scratch failed: %s", hipGetErrorString(e));
    noalloc_ptr[dev] = (double *)ptr;
    return DG_OK;
}
}  // namespace

// ------------------------------------------------------------------ errors
int dg_fail(dg_ctx *ctx, int code, const char *fmt, ...)
{
    if (ctx) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(ctx->err, sizeof(ctx->err), fmt, ap);
        va_end(ap);
    }
    return code;
}

// ------------------------------------------------------------------ tables
// Host-side FP64 construction of the basis / quadrature tables.
namespace {

// Legendre P_n and P_n' (recurrences (j+1)P_{j+1} = (2j+1)x P_j - j P_{j-1} and
// P'_{j+1} = (j+1) P_j + x P'_j)
void legendre_host(int n, double x, double &p, double &dp)
{
    double pm = 1.0, pc = x, dm = 0.0, dc = 1.0;
    if (n == 0) { p = 1.0; dp = 0.0; return; }
    for (int j = 1; j < n; ++j) {
        const double pn = ((2 * j + 1) * x * pc - j * pm) / (j + 1);
        const double dn = (j + 1) * pc + x * dc;
        pm = pc; pc = pn; dm = dc; dc = dn;
    }
    (void)dm;
    p = pc;
    dp = dc;
}

double lt(int n, double x)
{
    double p, dp;
    legendre_host(n, x, p, dp);
    return std::sqrt(2.0 * n + 1.0) * p;
}

double dlt(int n, double x)
{
    double p, dp;
    legendre_host(n, x, p, dp);
    return std::sqrt(2.0 * n + 1.0) * dp;
}

// Gauss-Legendre rule with n <= 4 points from the closed-form nodes; weights
// 2 / ((1 - x^2) P_n'(x)^2)
void gauss_host(int n, double *x, double *w)
{
    switch (n) {
    case 1: x[0] = 0.0; break;
    case 2: x[0] = -1.0 / std::sqrt(3.0); x[1] = -x[0]; break;
    case 3: x[0] = -std::sqrt(0.6); x[1] = 0.0; x[2] = -x[0]; break;
    case 4: {
        const double a = std::sqrt(3.0 / 7.0 + 2.0 / 7.0 * std::sqrt(1.2));
        const double b = std::sqrt(3.0 / 7.0 - 2.0 / 7.0 * std::sqrt(1.2));
        x[0] = -a; x[1] = -b; x[2] = b; x[3] = a;
        break;
    }
    default: break;
    }
    for (int i = 0; i < n; ++i) {
        double p, dp;
        legendre_host(n, x[i], p, dp);
        w[i] = 2.0 / ((1.0 - x[i] * x[i]) * dp * dp);
    }
}

template <int K>
void build_tables(std::vector<double> &t)
{
    using S = Shape<K>;
    using TL = TabLayout<K>;
    constexpr Modes<K> M = make_modes<K>();
    t.assign(TL::SIZE, 0.0);
    double g[K + 1], w[K + 1];
    gauss_host(K + 1, g, w);
    for (int qz = 0; qz < S::N1; ++qz)
        for (int qy = 0; qy < S::N1; ++qy)
            for (int qx = 0; qx < S::N1; ++qx) {
                const int q = qx + S::N1 * (qy + S::N1 * qz);
                const double xi[3] = {g[qx], g[qy], g[qz]};
                t[TL::VW + q] = w[qx] * w[qy] * w[qz];
                for (int a = 0; a < 3; ++a) t[TL::VXI + 3 * q + a] = xi[a];
                for (int l = 0; l < S::NB; ++l) {
                    const int *e = M.e[l];
                    t[TL::VPHI + q * S::NB + l] = lt(e[0], xi[0]) * lt(e[1], xi[1]) * lt(e[2], xi[2]);
                    for (int d = 0; d < 3; ++d) {
                        if (M.dj[d][l] < 0) continue;
                        double v = 1.0;
                        for (int a = 0; a < 3; ++a) v *= (a == d) ? dlt(e[a], xi[a]) : lt(e[a], xi[a]);
                        t[TL::VDPHI + (q * 3 + d) * S::ND + M.dj[d][l]] = v;
                    }
                }
            }
    for (int r2 = 0; r2 < S::N1; ++r2)
        for (int r1 = 0; r1 < S::N1; ++r1) {
            const int r = r1 + S::N1 * r2;
            t[TL::FW + r] = w[r1] * w[r2];
            for (int j = 0; j < S::NB2; ++j)
                t[TL::F2 + r * S::NB2 + j] = lt(M.p2[j][0], g[r1]) * lt(M.p2[j][1], g[r2]);
        }
    for (int n = 0; n <= K; ++n) {
        t[TL::LEND + 2 * n + 0] = lt(n, -1.0);
        t[TL::LEND + 2 * n + 1] = lt(n, 1.0);
    }
    for (int p = 0; p <= K; ++p)
        for (int a = 0; a <= K; ++a) t[TL::WLT + p * (K + 1) + a] = w[p] * lt(a, g[p]);
    // basis values on the faces: the face point r = r1 + (k+1) r2 has the tangential
    // coordinates (g[r1], g[r2]) along the axes tan1(d) < tan2(d), and xi_d = -1 or +1
    for (int d = 0; d < 3; ++d)
        for (int s = 0; s < 2; ++s)
            for (int r2 = 0; r2 < S::N1; ++r2)
                for (int r1 = 0; r1 < S::N1; ++r1) {
                    const int r = r1 + S::N1 * r2;
                    double xi[3];
                    xi[d] = s ? 1.0 : -1.0;
                    xi[tan1(d)] = g[r1];
                    xi[tan2(d)] = g[r2];
                    for (int l = 0; l < S::NB; ++l) {
                        const int *e = M.e[l];
                        t[TL::PLIFT + ((d * 2 + s) * S::NF + r) * S::NB + l] =
                            lt(e[0], xi[0]) * lt(e[1], xi[1]) * lt(e[2], xi[2]);
                    }
                }
}

// A-operand tables of the matrix-core volume integral at degree 2 (MfmaTab) from the host
// tables t: lane = 16 g + j; padded points take point 0's values for evaluations and zero
// weights for the contractions; padded modes are zero.
void build_mfma_tables(const std::vector<double> &t, std::vector<float> &mt)
{
    using S = Shape<2>;
    using TL = TabLayout<2>;
    constexpr Modes<2> M = make_modes<2>();
    mt.assign(MfmaTab::SIZE, 0.0f);
    auto phi = [&](int q, int l) { return t[TL::VPHI + q * S::NB + l]; };
    auto dphi = [&](int q, int d, int l) {
        return M.dj[d][l] < 0 ? 0.0 : t[TL::VDPHI + (q * 3 + d) * S::ND + M.dj[d][l]];
    };
    for (int lane = 0; lane < 64; ++lane) {
        const int g = lane / 16, j = lane % 16;
        for (int P = 0; P < 2; ++P) {
            const int qa = 16 * P + j, qae = qa < S::NQ ? qa : 0;
            for (int st = 0; st < 3; ++st) {
                const int mode = 4 * st + g;
                mt[MfmaTab::EV + (P * 3 + st) * 64 + lane] = mode < S::NB ? (float)phi(qae, mode) : 0.0f;
            }
            mt[MfmaTab::DV + P * 64 + lane] = (float)phi(qae, g);
            for (int r = 0; r < 4; ++r) {
                const int q = 16 * P + 4 * g + r;
                const bool ok = q < S::NQ && j < S::NB;
                const double w = q < S::NQ ? t[TL::VW + q] : 0.0;
                for (int d = 0; d < 3; ++d)
                    mt[MfmaTab::CT + ((d * 2 + P) * 4 + r) * 64 + lane] = ok ? (float)(w * dphi(q, d, j)) : 0.0f;
                mt[MfmaTab::FT + (P * 4 + r) * 64 + lane] = ok ? (float)(w * phi(q, j)) : 0.0f;
                mt[MfmaTab::WQ + (P * 4 + r) * 64 + lane] = (float)w;
            }
        }
    }
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

// ------------------------------------------------------------------ layout
static void layout(dg_ctx *c, size_t *total)
{
    const size_t es = c->es;
    const size_t nc = (size_t)c->nc;
    const size_t state = align_up(4 * (size_t)c->nb * nc * es);
    const size_t vh = align_up(3 * (size_t)c->nb * nc * es);
    size_t o = 0;
    c->off.stA = o; o += state;
    c->off.stB = o; o += state;
    // a third stage buffer for the five-stage scheme (degree 3 with DG_RK_BY_ORDER)
    c->off.stC = o; o += ((c->cfg.flags & DG_RK_BY_ORDER) && c->k == 3) ? state : 0;
    c->off.L = o; o += state;
    // with the two-lane right-hand side (FP64, degree 3) each projection buffer is preceded by
    // a copy of the density weights, so that density and projected velocity form one
    // [4][nb][nc] array (vh_rho_of)
    const size_t rho_blk = (c->es == 8 && c->k == 3) ? align_up((size_t)c->nb * nc * es) : 0;
    c->off.vh0 = o + rho_blk; o = c->off.vh0 + vh;
    c->off.vh1 = o + rho_blk; o = c->off.vh1 + vh;
    // driving field in pencil form: header, (k+1)^2 entries of 16 values per y-z pencil, and
    // the x phases (PencilLayout)
    c->off.ftab = o;
    {
        const int nx = c->cfg.nx, ny = c->cfg.ny, nz = c->cfg.nz;
        const size_t reals = c->k == 1 ? PencilLayout<1>::size(nx, ny, nz)
                             : c->k == 2 ? PencilLayout<2>::size(nx, ny, nz) : PencilLayout<3>::size(nx, ny, nz);
        o += (c->cfg.flags & DG_FORCING) ? align_up(reals * es) : 0;
    }
    const bool learned = c->cfg.flags & DG_LEARNED_SENSOR;
    c->off.nu = o; o += align_up(nc * es);
    c->off.fb = o; o += align_up(nc * 4);
    c->off.feat = o; o += learned ? align_up(nc * DG_MLP_NIN * 4) : 0;
    c->off.lab = o; o += learned ? align_up(nc * 8) : 0;
    c->off.mlp = o; o += align_up((size_t)MLP_PART_ROWS * (DG_MLP_NPARAM + 1) * 4);   // per-wave network gradients
    // per-block partials: the FP64 degree-3 right-hand side runs two lanes per cell (twice
    // the blocks)
    c->off.part = o; o += align_up((size_t)c->nblk * 2 * 4 * 8);
    // the step's last stage: per-block time-step maxima (apart from the right-hand side's
    // partials, which the same stage reads)
    c->off.spart = o; o += align_up((size_t)c->nblk * 2 * 8);
    // mean-acceleration partials of a stage's input formed before its right-hand side (split
    // stages), apart from the right-hand side's own
    c->off.dpart = o; o += align_up((size_t)c->nblk * 4 * 8);
    c->off.scal = o; o += align_up(64 * 8);
    c->off.iflags = o; o += align_up(64 * 4);
    *total = o;
}

void dg_config_default(dg_config *cfg, int nx, int ny, int nz)
{
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->nx = nx; cfg->ny = ny; cfg->nz = nz;
    cfg->degree = 2;
    cfg->precision = DG_FP64;
    cfg->flags = DG_AV | DG_PRIM_PROJ | DG_POS_LIMITER;
    cfg->h = nx > 0 ? 1.0 / nx : 0.0;
    cfg->cs = 1.0;
    cfg->cfl = 0.3;
    cfg->alpha_visc = 2.0;
    cfg->beta_visc = 0.2;
    cfg->rho_floor = 1e-3;
    cfg->rho_floor_rel = 0.1;
    cfg->cfl_visc = 0.1;
    cfg->stream = nullptr;
}

int dg_init(const dg_config *cfg, dg_ctx **out)
{
    if (!out) return DG_EINVAL;
    *out = nullptr;
    if (!cfg) return DG_EINVAL;
    if (cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 1) return DG_EINVAL;
    if ((long long)cfg->nx * cfg->ny * cfg->nz > (1LL << 30)) return DG_EINVAL;
    if (cfg->degree < 1 || cfg->degree > 3) return DG_EUNSUPPORTED;
    if (cfg->precision != DG_FP64 && cfg->precision != DG_FP32) return DG_EINVAL;
    if (!(cfg->cs > 0.0) || !(cfg->cfl > 0.0) || cfg->alpha_visc < 0.0 || cfg->beta_visc < 0.0 ||
        !(cfg->rho_floor >= 0.0) || !(cfg->rho_floor_rel >= 0.0) || !(cfg->rho_floor_rel < 1.0))
        return DG_EINVAL;
    const int known = DG_AV | DG_PRIM_PROJ | DG_FORCING | DG_POS_LIMITER | DG_LEARNED_SENSOR | DG_FORCE_MEANFREE |
                      DG_HLLC | DG_RK_BY_ORDER | DG_VOLUME_MFMA | DG_SEPARATE_STAGE | DG_SPLIT_STAGE;
    if (cfg->flags & ~known) return DG_EINVAL;
    if ((cfg->flags & DG_VOLUME_MFMA) && !(cfg->precision == DG_FP32 && cfg->degree == 2)) return DG_EUNSUPPORTED;
    if ((cfg->flags & DG_SEPARATE_STAGE) && (cfg->flags & DG_SPLIT_STAGE)) return DG_EINVAL;
    if ((cfg->flags & DG_LEARNED_SENSOR) && cfg->degree != 2) return DG_EUNSUPPORTED;
    {
        // each [var] block of nb mode planes is addressed through one buffer descriptor
        const long long ncl = (long long)cfg->nx * cfg->ny * cfg->nz;
        const int kk = cfg->degree, nbk = (kk + 1) * (kk + 2) * (kk + 3) / 6;
        const long long es = cfg->precision == DG_FP64 ? 8 : 4;
        if ((long long)nbk * ncl * es >= (1LL << 32)) return DG_EINVAL;
    }
    dg_ctx *c = new (std::nothrow) dg_ctx();
    if (!c) return DG_ENOMEM;
    c->cfg = *cfg;
    if (!(c->cfg.h > 0.0)) c->cfg.h = 1.0 / cfg->nx;
    c->k = cfg->degree;
    c->nb = (c->k + 1) * (c->k + 2) * (c->k + 3) / 6;
    c->nq = (c->k + 1) * (c->k + 1) * (c->k + 1);
    c->nc = cfg->nx * cfg->ny * cfg->nz;
    c->es = cfg->precision == DG_FP64 ? 8 : 4;
    c->nblk = (c->nc + BLOCK - 1) / BLOCK;
    c->stream = (hipStream_t)cfg->stream;
    {
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
            c->ncu = ncu;
        c->device = dev;
        if (noalloc_setup(c, dev) != DG_OK) {
            delete c;
            return DG_EHIP;
        }
    }
    layout(c, &c->ws_need);

    std::vector<double> t;
    switch (c->k) {
    case 1: build_tables<1>(t); break;
    case 2: build_tables<2>(t); break;
    default: build_tables<3>(t); break;
    }
    int rc = DG_OK;
    hipError_t e = hipMalloc(&c->tab, t.size() * c->es);
    if (e != hipSuccess) { delete c; return DG_EHIP; }
    if (c->es == 8) {
        e = hipMemcpy(c->tab, t.data(), t.size() * 8, hipMemcpyHostToDevice);
    } else {
        std::vector<float> tf(t.begin(), t.end());
        e = hipMemcpy(c->tab, tf.data(), tf.size() * 4, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMalloc((void **)&c->modes_dev, 64 * 9 * sizeof(double));
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&c->modes_stage, dg_ctx::MODE_SLOTS * 64 * 9 * sizeof(double), hipHostMallocDefault);
    // coherent: the step's last kernel stores its published values straight to host memory
    if (e == hipSuccess) e = hipHostMalloc((void **)&c->pinned, 256, hipHostMallocCoherent);
    if (e == hipSuccess) std::memset(c->pinned, 0, 256);
    if (e == hipSuccess) e = hipMalloc((void **)&c->mlp_bf16, 8 * DG_MLP_NPARAM);
    if (e == hipSuccess && (c->cfg.flags & DG_VOLUME_MFMA)) {
        std::vector<float> mt;
        build_mfma_tables(t, mt);
        e = hipMalloc((void **)&c->mfma_tab, mt.size() * sizeof(float));
        if (e == hipSuccess) e = hipMemcpy(c->mfma_tab, mt.data(), mt.size() * sizeof(float), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) rc = DG_EHIP;
    if (rc != DG_OK) { dg_free(c); return rc; }
    *out = c;
    return DG_OK;
}

void dg_free(dg_ctx *c)
{
    if (!c) return;
    for (int i = 0; i < 2 * dg_ctx::NEV; ++i)
        for (int j = 0; j < 2; ++j)
            if (c->ev[i][j]) (void)hipEventDestroy(c->ev[i][j]);
    if (c->tab) (void)hipFree(c->tab);
    if (c->modes_dev) (void)hipFree(c->modes_dev);
    if (c->pinned) (void)hipHostFree(c->pinned);
    for (int i = 0; i < dg_ctx::MODE_SLOTS; ++i)
        if (c->modes_ev[i]) (void)hipEventDestroy(c->modes_ev[i]);
    if (c->modes_stage) (void)hipHostFree(c->modes_stage);
    if (c->mlp_bf16) (void)hipFree(c->mlp_bf16);
    if (c->mfma_tab) (void)hipFree(c->mfma_tab);
    stats_release(c);
    delete c;
}

const char *dg_last_error(const dg_ctx *c) { return c ? c->err : "null context"; }

int dg_set_wait_limit(dg_ctx *c, double seconds)
{
    if (!c) return DG_EINVAL;
    if (!(seconds > 0.0)) return dg_fail(c, DG_EINVAL, "wait limit must be positive (got %g)", seconds);
    c->wait_limit_s = seconds;
    return DG_OK;
}

size_t dg_workspace_bytes(const dg_ctx *c) { return c ? c->ws_need : 0; }

int dg_set_workspace(dg_ctx *c, void *ws, size_t bytes)
{
    if (!c) return DG_EINVAL;
    if (!ws) return dg_fail(c, DG_EINVAL, "workspace pointer is null");
    if ((uintptr_t)ws & 255) return dg_fail(c, DG_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < c->ws_need)
        return dg_fail(c, DG_ENOMEM, "workspace too small: %zu < %zu bytes", bytes, c->ws_need);
    if (int rc = dg_check_array(c, ws, c->ws_need, 256, "workspace")) return rc;
    c->ws = (char *)ws;
    c->gen++;
    c->forcing_dirty = c->nmodes > 0;
    c->have_nu = false;
    if (c->cfg.flags & DG_LEARNED_SENSOR) return sensor_reset_flags(c);
    return DG_OK;
}

static int need_ws(dg_ctx *c)
{
    if (!c->ws) return dg_fail(c, DG_ENOMEM, "no workspace set (dg_set_workspace)");
    return DG_OK;
}

int dg_check_array(dg_ctx *c, const void *p, size_t bytes, size_t align, const char *name)
{
    if (!p) return dg_fail(c, DG_EINVAL, "%s is null", name);
    if ((uintptr_t)p & (align - 1)) return dg_fail(c, DG_EINVAL, "%s is misaligned", name);
    // the extent of the allocation that holds p (the lookup's error is cleared: it is
    // reported here, not by a later call)
    void *base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, const_cast<void *>(p)) != hipSuccess || !base) {
        (void)hipGetLastError();
        return dg_fail(c, DG_EINVAL, "%s (%p) is not inside an allocation of the HIP runtime", name, p);
    }
    const uintptr_t off = (uintptr_t)p - (uintptr_t)base;
    if ((uintptr_t)p < (uintptr_t)base || off > size || bytes > size - off)
        return dg_fail(c, DG_EINVAL, "%s: %zu bytes at offset %zu of an allocation of %zu bytes overrun it", name,
                       bytes, (size_t)off, size);
    return DG_OK;
}

static int check_ptr(dg_ctx *c, const void *p, const char *name, int nvar = 4)
{
    return dg_check_array(c, p, dg_state_bytes(c, nvar), c->es, name);
}

int dg_set_forcing(dg_ctx *c, const double *modes_host, int nmodes)
{
    if (!c) return DG_EINVAL;
    if (nmodes < 0 || nmodes > 64 || (nmodes > 0 && !modes_host))
        return dg_fail(c, DG_EINVAL, "bad forcing table (nmodes=%d)", nmodes);
    std::memcpy(c->modes_host, modes_host, sizeof(double) * 9 * nmodes);
    c->nmodes = nmodes;
    c->spec_valid = false;          // a launched next stage used the previous field
    // pencil form of the driving field: every n_x an integer in [-2, 2]
    bool sep = true;
    for (int m = 0; m < nmodes; ++m) {
        const double n = modes_host[9 * m];
        sep = sep && n == std::nearbyint(n) && std::fabs(n) <= 2.0;
    }
    c->modes_sep = sep;
    // asynchronous upload from a ring of pinned slots: a slot is rewritten only after the
    // copy that last read it has completed
    const int slot = c->modes_slot;
    c->modes_slot = (slot + 1) % dg_ctx::MODE_SLOTS;
    if (c->modes_ev[slot]) HIPCHK(c, hipEventSynchronize(c->modes_ev[slot]));
    else HIPCHK(c, hipEventCreateWithFlags(&c->modes_ev[slot], hipEventDisableTiming));
    double *stage = c->modes_stage + (size_t)slot * 64 * 9;
    std::memcpy(stage, c->modes_host, sizeof(double) * 9 * nmodes);
    if (nmodes > 0) {
        HIPCHK(c, hipMemcpyAsync(c->modes_dev, stage, sizeof(double) * 9 * nmodes, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipEventRecord(c->modes_ev[slot], c->stream));
    }
    c->forcing_dirty = true;
    return DG_OK;
}

int dg_forcing_get(const dg_ctx *c, double *modes_host, int nmodes_max)
{
    if (!c || !modes_host) return DG_EINVAL;
    const int n = c->nmodes < nmodes_max ? c->nmodes : nmodes_max;
    std::memcpy(modes_host, c->modes_host, sizeof(double) * 9 * n);
    return c->nmodes;
}

// ------------------------------------------------------------------ timing
static int prof_drain(dg_ctx *c)
{
    for (int i = 0; i < c->nev; ++i) {
        float ms = 0.0f;
        HIPCHK(c, hipEventSynchronize(c->ev[i][1]));
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev[i][0], c->ev[i][1]));
        c->prof_ms[c->ev_kind[i]] += ms;
        c->prof_n[c->ev_kind[i]] += 1;
    }
    c->nev = 0;
    return DG_OK;
}

// bracket one launch with events when profiling: call with stop = 0 before, 1 after
// Each event costs the GPU a few microseconds of idle time (measured: about 2 us per
// event without the system-scope fence, 3 to 6 us with it), so level 1 brackets only the
// right-hand side of a step's first stage (the three right-hand sides of a step are the same
// kernel on the same mesh) and level 2 every right-hand-side and stage launch.
static int prof_mark(dg_ctx *c, int kind, int stop)
{
    if (!c->prof) return DG_OK;
    if (c->prof == 1 && (kind != 0 || !c->prof_first)) return DG_OK;
    if (c->prof == 3 && (kind != 0 || !c->prof_last)) return DG_OK;
    if (!stop && c->nev >= 2 * dg_ctx::NEV) {
        int rc = prof_drain(c);
        if (rc) return rc;
    }
    const int i = c->nev;
    HIPCHK(c, hipEventRecord(c->ev[i][stop], c->stream));
    if (stop) {
        c->ev_kind[i] = kind;
        c->nev++;
    }
    return DG_OK;
}

int dg_profile(dg_ctx *c, int enable)
{
    if (!c) return DG_EINVAL;
    if (enable) {
        for (int i = 0; i < 2 * dg_ctx::NEV; ++i)
            for (int j = 0; j < 2; ++j)
                if (!c->ev[i][j]) HIPCHK(c, hipEventCreateWithFlags(&c->ev[i][j], hipEventDisableSystemFence));
        c->nev = 0;
        c->prof_ms[0] = c->prof_ms[1] = 0.0;
        c->prof_n[0] = c->prof_n[1] = 0;
    }
    c->prof = enable < 0 ? 0 : (enable > 3 ? 3 : enable);
    return DG_OK;
}

int dg_profile_read(dg_ctx *c, double *out)
{
    if (!c || !out) return DG_EINVAL;
    int rc = prof_drain(c);
    if (rc) return rc;
    out[0] = c->prof_ms[0];
    out[1] = (double)c->prof_n[0];
    out[2] = c->prof_ms[1];
    out[3] = (double)c->prof_n[1];
    return DG_OK;
}

// ------------------------------------------------------------------ launches
// the pencil table of the driving field (tables whose n_x are integers in [-2, 2]); other
// tables are evaluated mode by mode inside the right-hand-side kernel and need no table
template <typename T, int K>
static int launch_forcing_table(dg_ctx *c)
{
    if (!c->modes_sep) return DG_OK;
    const Mesh g{c->cfg.nx, c->cfg.ny, c->cfg.nz, c->nc};
    const long long nt = std::max((long long)c->cfg.ny * c->cfg.nz * (K + 1) * (K + 1), (long long)c->cfg.nx);
    const int nb = (int)((nt + BLOCK - 1) / BLOCK);
    hipLaunchKernelGGL((k_forcing_pencils<T, K>), dim3(nb), dim3(BLOCK), 0, c->stream, c->wp(c->off.ftab),
                       c->modes_dev, c->nmodes, c->tab, g, c->cfg.h);
    LAUNCHCHK(c);
    // the pencils' moments from the values just written (stream order)
    const long long nm = (long long)c->cfg.ny * c->cfg.nz * PencilLayout<K>::NB2 * 3;
    hipLaunchKernelGGL((k_forcing_moments<T, K>), dim3((int)((nm + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, c->stream,
                       c->wp(c->off.ftab), c->tab, g);
    LAUNCHCHK(c);
    return DG_OK;
}

static ProjArgs proj_args(const dg_ctx *c)
{
    ProjArgs pa;
    pa.cs = c->cfg.cs;
    pa.h = c->cfg.h;
    pa.alpha = c->cfg.alpha_visc;
    pa.beta = c->cfg.beta_visc;
    pa.visc = (c->cfg.flags & DG_AV) && c->cfg.cfl_visc > 0.0;
    const bool learned = (c->cfg.flags & DG_LEARNED_SENSOR) && (c->cfg.flags & DG_AV) && c->have_nu;
    // learned_bounds_later: the learned cells' viscosities are reduced by the network's
    // forward pass instead (the fused step's last stage, before the network has run)
    pa.nu = learned && !c->learned_bounds_later ? c->wp(c->off.nu) : nullptr;
    pa.fb = learned ? (const int *)c->wp(c->off.fb) : nullptr;
    return pa;
}

// the density copy in front of a workspace projection buffer (two-lane configuration), or
// NULL for any other buffer or configuration
static void *vh_rho_of(const dg_ctx *c, const void *vh)
{
    if (!(c->es == 8 && c->k == 3) || !vh) return nullptr;
    if (vh != c->wp(c->off.vh0) && vh != c->wp(c->off.vh1)) return nullptr;
    return (char *)const_cast<void *>(vh) - (size_t)c->nb * c->nc * c->es;
}

template <typename T, int K>
static int launch_project(dg_ctx *c, const void *u, void *vh, double *part, int *fail)
{
    const Mesh g{c->cfg.nx, c->cfg.ny, c->cfg.nz, c->nc};
    const ProjArgs pa = proj_args(c);
    hipLaunchKernelGGL((k_project<T, K>), dim3(c->nblk), dim3(BLOCK), 0, c->stream, u, vh, c->tab, g, pa,
                       part, fail, vh_rho_of(c, vh));
    LAUNCHCHK(c);
    return DG_OK;
}

// The FP64 right-hand side at degree 3 runs two lanes per cell (k_rhs_pair): one lane per
// cell fits only one wave per SIMD there, two lanes fit two (measured 15 % faster at 64^3).
// At degrees 1 and 2 the one-lane kernel is faster (the pair costs twice the loads and a
// lane swap per point value, 194 -> 265 us at 64^3 degree 2).
template <typename T, int K>
constexpr bool rhs_pair() { return sizeof(T) == 8 && K == 3; }


// failure prediction of a last stage (RhsArgs::pred_fail): its u^n operand and coefficients
struct StagePred {
    const void *un;
    const double *coef;
};

// planes per tile of the right-hand-side kernels' block order (plane_tiled); measured on
// driven states, alternated on one MI355X: 256^3 degree 2 FP64 step 50.9 ms with the plain
// j-fastest order, 48.7 / 48.4 / 48.3 ms with tiles of 4 / 8 / 16 planes; 128^3 degree 3
// FP64 34.6 -> 33.1 / 32.5 / 32.6 ms; 64^3 unchanged up to 8 and slower at 16
constexpr int RHS_ZTILE = 8;

// st: the split stage whose combination the right-hand-side kernel forms, or NULL:
// the right-hand side is stored into out
template <typename T, int K>
static int launch_rhs(dg_ctx *c, const void *u, const void *vh, void *out, double dt, int *fail_reset = nullptr,
                      const StagePred *pred = nullptr, const double *dt_dev = nullptr, const StageArgs *st = nullptr)
{
    if ((c->cfg.flags & DG_FORCING) && c->forcing_dirty) {
        int rc = launch_forcing_table<T, K>(c);
        if (rc) return rc;
        c->forcing_dirty = false;
    }
    RhsArgs a;
    a.u = u;
    a.vh = vh;
    a.vh_rho = nullptr;
    a.pair_vstride = 0;
    a.out = out;
    a.tab = c->tab;
    a.ftab = c->wp(c->off.ftab);
    a.modes = c->modes_dev;
    a.nmodes = c->nmodes;
    a.nu = c->wp(c->off.nu);
    a.fb = (const int *)c->wp(c->off.fb);
    a.part = (double *)c->wp(c->off.part);
    a.fail_reset = fail_reset;
    a.pred_fail = pred ? c->fail() : nullptr;
    a.pred_un = pred ? pred->un : nullptr;
    a.pred_ca = pred ? pred->coef[0] : 0.0;
    a.pred_cb = pred ? pred->coef[1] : 0.0;
    a.pred_cc = pred ? pred->coef[2] : 0.0;
    a.rho_floor = c->cfg.rho_floor;
    a.g = Mesh{c->cfg.nx, c->cfg.ny, c->cfg.nz, c->nc};
    a.flags = c->cfg.flags;
    if (c->nmodes == 0) a.flags &= ~DG_FORCING;
    a.h = c->cfg.h;
    a.cs = c->cfg.cs;
    a.alpha = c->cfg.alpha_visc;
    a.beta = c->cfg.beta_visc;
    a.dt = dt;
    a.dt_dev = dt_dev;
    int rc = prof_mark(c, 0, 0);
    if (rc) return rc;
    // tables off the pencil form: the kernel's direct (mode by mode) driving field
    const bool direct = (a.flags & DG_FORCING) && !c->modes_sep;
    a.mfma = c->mfma_tab;
    const StageArgs st0{};
    if (st) a.part = nullptr;   // a split stage's kernel reads the partials of its input
    // sweep order: tiles of planes when whole blocks make up a plane
    {
        const int cpb = rhs_pair<T, K>() ? BLOCK / 2 : BLOCK;
        const long long plane = (long long)c->cfg.nx * c->cfg.ny;
        a.bpp = plane % cpb == 0 ? (int)(plane / cpb) : 0;
        a.zt = RHS_ZTILE;
    }
    if constexpr (rhs_pair<T, K>()) {
        c->rhs_nblk = (c->nc + BLOCK / 2 - 1) / (BLOCK / 2);
        // each lane loads only its own variables when two variable blocks and a cell offset fit
        // a 32-bit buffer offset, and (projected traces) the density copy is in front of vh
        const size_t vb = (size_t)c->nb * c->nc * 8;
        const bool prim = c->cfg.flags & DG_PRIM_PROJ;
        a.vh_rho = vh_rho_of(c, vh);
        const bool lsel = 2 * vb + (size_t)c->nc * 8 < ((size_t)1 << 32) && (!prim || a.vh_rho);
        a.pair_vstride = lsel ? (unsigned)(2 * vb) : 0u;
        if (lsel) {
            if (direct) hipLaunchKernelGGL((k_rhs_pair<K, true, true>), dim3(c->rhs_nblk), dim3(BLOCK), 0, c->stream, a);
            else hipLaunchKernelGGL((k_rhs_pair<K, false, true>), dim3(c->rhs_nblk), dim3(BLOCK), 0, c->stream, a);
        } else {
            if (direct) hipLaunchKernelGGL((k_rhs_pair<K, true, false>), dim3(c->rhs_nblk), dim3(BLOCK), 0, c->stream, a);
            else hipLaunchKernelGGL((k_rhs_pair<K, false, false>), dim3(c->rhs_nblk), dim3(BLOCK), 0, c->stream, a);
        }
    } else {
        c->rhs_nblk = c->nblk;
        bool done = false;
        if (st) {
            // u^n enters the combination when its coefficient is not zero
            const dim3 gr(c->nblk), bl(BLOCK);
            if (st->ca != 0.0) {
                if (direct) hipLaunchKernelGGL((k_rhs<T, K, true, false, 2>), gr, bl, 0, c->stream, a, *st);
                else hipLaunchKernelGGL((k_rhs<T, K, false, false, 2>), gr, bl, 0, c->stream, a, *st);
            } else {
                if (direct) hipLaunchKernelGGL((k_rhs<T, K, true, false, 1>), gr, bl, 0, c->stream, a, *st);
                else hipLaunchKernelGGL((k_rhs<T, K, false, false, 1>), gr, bl, 0, c->stream, a, *st);
            }
            done = true;
        }
        if constexpr (sizeof(T) == 4 && K == 2) {
            // volume integral on the matrix cores (tables in the pencil form or no driving)
            if (!done && (c->cfg.flags & DG_VOLUME_MFMA) && !direct) {
                hipLaunchKernelGGL((k_rhs<T, K, false, true>), dim3(c->nblk), dim3(BLOCK), 0, c->stream, a, st0);
                done = true;
            }
        }
        if (!done) {
            if (direct) hipLaunchKernelGGL((k_rhs<T, K, true>), dim3(c->nblk), dim3(BLOCK), 0, c->stream, a, st0);
            else hipLaunchKernelGGL((k_rhs<T, K, false>), dim3(c->nblk), dim3(BLOCK), 0, c->stream, a, st0);
        }
    }
    LAUNCHCHK(c);
    return prof_mark(c, 0, 1);
}

// the largest count of right-hand-side blocks whose partials a stage block reduces itself
constexpr int ABAR_IN_STAGE_BLOCKS = 1024;

static bool use_meanfree(const dg_ctx *c)
{
    return (c->cfg.flags & DG_FORCING) && (c->cfg.flags & DG_FORCE_MEANFREE) && c->nmodes > 0;
}

// the removed mean acceleration from per-block partials: by default the right-hand side's
static int launch_abar(dg_ctx *c, const double *part = nullptr, int np = 0)
{
    if (!part) {
        part = (const double *)c->wp(c->off.part);
        np = c->rhs_nblk;
    }
    hipLaunchKernelGGL(k_final, dim3(1), dim3(BLOCK), 0, c->stream, part, np, 1, 1.0, 0.0, c->abar(),
                       (const int *)nullptr, (volatile long long *)nullptr, 0LL, (const double *)nullptr, 0);
    LAUNCHCHK(c);
    return DG_OK;
}

// the arguments of one stage (k_stage, or the split stage of k_rhs: L is then not read, and
// with mean-free driving the partials or the mean are those of ui)
static StageArgs stage_args(dg_ctx *c, const void *ui, const void *un, const void *L, void *out, void *vh_out,
                            bool skip_if_failed, const double (&coef)[3], double dt, long long *nlim, double *part,
                            void *w, const double (&wcoef)[3], const double *dt_dev, bool split = false)
{
    StageArgs a;
    a.ui = ui;
    a.un = un;
    a.L = L;
    a.out = out;
    a.vh_out = vh_out;
    a.rho_out = vh_rho_of(c, vh_out);
    a.skip_flag = skip_if_failed ? c->fail() : nullptr;
    a.tab = c->tab;
    // abar_in_stage: every block reduces the right-hand side's partials to the removed mean
    // acceleration itself (no separate reduction kernel)
    // (a stage whose combination the right-hand-side kernel forms reads the partials of its
    // input from the region k_drive_parts and k_limit_project write)
    const bool mf = (L || split) && use_meanfree(c);
    a.abar = mf && !c->abar_in_stage ? c->abar() : nullptr;
    a.abar_part = mf && c->abar_in_stage ? (const double *)c->wp(split ? c->off.dpart : c->off.part) : nullptr;
    a.abar_np = split ? c->nblk : c->rhs_nblk;
    a.fail = c->fail();
    a.nlim = nlim;
    a.part = part;
    a.pa = proj_args(c);
    a.g = Mesh{c->cfg.nx, c->cfg.ny, c->cfg.nz, c->nc};
    a.flags = c->cfg.flags;
    a.ca = coef[0];
    a.cb = coef[1];
    a.cc = coef[2];
    a.w_src = w;
    a.w_out = w;
    a.wa = wcoef[0];
    a.wb = wcoef[1];
    a.wc = wcoef[2];
    a.dt = dt;
    a.dt_dev = dt_dev;
    a.rho_floor = c->cfg.rho_floor;
    a.rho_floor_rel = c->cfg.rho_floor_rel;
    a.drive_part = nullptr;
    a.fail_on_mean = 0;
    a.ftab = c->wp(c->off.ftab);
    a.modes = c->modes_dev;
    a.nmodes = c->nmodes;
    return a;
}

template <typename T, int K>
static int launch_stage(dg_ctx *c, const void *ui, const void *un, const void *L, void *out, void *vh_out,
                        bool skip_if_failed, const double (&coef)[3], double dt, long long *nlim, double *part = nullptr,
                        void *w = nullptr, const double (&wcoef)[3] = {0.0, 0.0, 0.0},
                        const double *dt_dev = nullptr)
{
    const StageArgs a = stage_args(c, ui, un, L, out, vh_out, skip_if_failed, coef, dt, nlim, part, w, wcoef, dt_dev);
    int rc = prof_mark(c, 1, 0);
    if (rc) return rc;
    // u^n enters when its coefficient is not zero; the side combination when it has an output
    const bool unv = a.L && a.ca != 0.0, side = a.L && a.w_out;
    if (side) {
        if (unv) hipLaunchKernelGGL((k_stage<T, K, true, true>), dim3(c->nblk), dim3(BLOCK), 0, c->stream, a);
        else hipLaunchKernelGGL((k_stage<T, K, false, true>), dim3(c->nblk), dim3(BLOCK), 0, c->stream, a);
    } else {
        if (unv) hipLaunchKernelGGL((k_stage<T, K, true, false>), dim3(c->nblk), dim3(BLOCK), 0, c->stream, a);
        else hipLaunchKernelGGL((k_stage<T, K, false, false>), dim3(c->nblk), dim3(BLOCK), 0, c->stream, a);
    }
    LAUNCHCHK(c);
    return prof_mark(c, 1, 1);
}

template <typename T, int K>
static int do_rhs(dg_ctx *c, const void *u, void *dudt, double dt)
{
    int rc = launch_project<T, K>(c, u, c->wp(c->off.vh0), nullptr, nullptr);
    if (rc) return rc;
    c->prof_first = true;
    rc = launch_rhs<T, K>(c, u, c->wp(c->off.vh0), dudt, dt);
    if (rc) return rc;
    if (use_meanfree(c)) {
        rc = launch_abar(c);
        if (rc) return rc;
        hipLaunchKernelGGL((k_meanfree<T, K>), dim3(c->nblk), dim3(BLOCK), 0, c->stream, u, dudt, c->abar(), c->nc);
        LAUNCHCHK(c);
    }
    return DG_OK;
}

// seq > 0: also publish the time step and the failure flag to the host (dg_ctx::PUB);
// vmax: np2 further partial maxima of the viscosity (the learned cells'), or NULL
template <typename T, int K>
static int launch_dt_final(dg_ctx *c, const double *src, double *dst, long long seq = 0, const double *vmax = nullptr,
                           int np2 = 0)
{
    const double hp = c->cfg.h / (K + 1);
    volatile long long *pub = seq > 0 ? (volatile long long *)(c->pinned + dg_ctx::PUB) : nullptr;
    hipLaunchKernelGGL(k_final, dim3(1), dim3(BLOCK), 0, c->stream, src, c->nblk, 2,
                       c->cfg.cfl * c->cfg.h / (K + 1), c->cfg.cfl_visc > 0.0 ? c->cfg.cfl_visc * hp * hp : 0.0,
                       dst, (const int *)(pub ? c->fail() : nullptr), pub, seq, vmax, np2);
    LAUNCHCHK(c);
    return DG_OK;
}

// Wait until the kernel launched by launch_dt_final(c, c->scal() + 8, seq) has published:
// spin on the sequence number in pinned memory (far lower latency than a copy back and a
// stream synchronisation), bounded by the stream's own completion and by the context's
// wall-clock limit.  Should the stream complete without the number showing, the values are
// copied back from the device slots k_final filled (time step and the step's own failure
// flag: the live flag may already have been cleared by a stage queued behind it).
static int wait_published(dg_ctx *c, long long seq, double *dt, int *fail_flag)
{
    volatile long long *pub = (volatile long long *)(c->pinned + dg_ctx::PUB);
    const auto t0 = std::chrono::steady_clock::now();
    for (unsigned it = 1;; ++it) {
        if (pub[0] == seq) break;
        if ((it & 63) == 0) {
            const hipError_t q = hipStreamQuery(c->stream);
            if (q == hipSuccess) {
                if (pub[0] == seq) break;
                double vals[2];
                HIPCHK(c, hipMemcpy(vals, c->scal() + 8, sizeof(vals), hipMemcpyDeviceToHost));
                long long bits;
                std::memcpy(&bits, &vals[0], sizeof(bits));
                pub[1] = bits;
                pub[2] = (long long)vals[1];
                break;
            }
            if (q != hipErrorNotReady)
                return dg_fail(c, DG_EHIP, "stream query while waiting for the step failed: %s", hipGetErrorString(q));
            const double waited = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (waited > c->wait_limit_s)
                return dg_fail(c, DG_EHIP,
                               "the step did not complete within %.3g s (the stream is still running: synchronise it "
                               "before using the state)", c->wait_limit_s);
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    const long long bits = pub[1];
    std::memcpy(dt, &bits, sizeof(double));
    *fail_flag = (int)pub[2];
    return DG_OK;
}

// SSP Runge-Kutta schemes in the compact Shu-Osher form the stage kernel evaluates:
// stage s reads buffer `in` (u^(s)) and buffer `un` (u^n or an earlier side combination)
// and writes out = a un + b in + c dt R(in); a stage may also write the side combination
// w = wa w + wb in + wc dt R(in) into buffer `w` in place.  Buffers: 0 = the state array
// (u^n until the last stage writes u^(n+1)), 1..3 = workspace stage buffers.
struct StageSpec {
    int in, un, out;
    double coef[3];
    int w;
    double wcoef[3];
};
struct Scheme {
    int stages;
    StageSpec s[5];
};
// two stages, second order (Heun)
static const Scheme SSPRK2 = {2, {{0, 0, 1, {0.0, 1.0, 1.0}, 0, {}}, {1, 0, 0, {0.5, 0.5, 0.5}, 0, {}}}};
// three stages, third order (Shu & Osher)
static const Scheme SSPRK3 = {3,
                              {{0, 0, 1, {0.0, 1.0, 1.0}, 0, {}},
                               {1, 0, 2, {0.75, 0.25, 0.25}, 0, {}},
                               {2, 0, 0, {1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0}, 0, {}}}};
// five stages, fourth order (Spiteri & Ruuth 2002); its last stage combines u^(2), u^(3),
// L(u^(3)), u^(4), L(u^(4)): the first three are folded into a side combination by the
// fourth stage, written over u^(2)
static const Scheme SSPRK54 = {
    5,
    {{0, 0, 1, {0.0, 1.0, 0.391752226571890}, 0, {}},
     {1, 0, 2, {0.444370493651235, 0.555629506348765, 0.368410593050371}, 0, {}},
     {2, 0, 1, {0.620101851488403, 0.379898148511597, 0.251891774271694}, 0, {}},
     {1, 0, 3, {0.178079954393132, 0.821920045606868, 0.544974750228521}, 2,
      {0.517231671970585, 0.096059710526147, 0.063692468666290}},
     {3, 2, 0, {1.0, 0.386708617503269, 0.226007483236906}, 0, {}}}};

static const Scheme &scheme_of(const dg_ctx *c)
{
    if (!(c->cfg.flags & DG_RK_BY_ORDER)) return SSPRK3;
    return c->k == 1 ? SSPRK2 : (c->k == 2 ? SSPRK3 : SSPRK54);
}

// Whether a stage is split between its right-hand-side kernel, which forms the stage's
// combination (k_rhs with COMB), and k_limit_project, which limits and projects it, instead of
// storing the right-hand side for a stage kernel: the one-lane kernel with the vector volume
// integral, a stage without a side combination that writes a workspace buffer other than its
// input, and not turned off by DG_SEPARATE_STAGE.  The last stage writes the caller's array,
// which must keep u^n when the step fails: split, it stores its combination into a free
// workspace buffer (raising the failure flag from the combination's mean density) and k_stage
// writes the caller's array from there unless a cell failed.  Split and separate stages give
// the same bits (to rounding with mean-free driving on the driving shell).
// The split pays where the mesh takes many rounds of blocks: measured on one MI355X (split
// against separate, alternated in one call, degree 2, driven, mean-free): 256^3 FP64 42.7 vs
// 43.8 ms per step, 256^3 FP32 21.5 vs 22.2 ms, 128^3 FP64 5.43 vs 5.52 ms, 128^3 FP32 2.76 vs
// 2.79 ms; slower at 64^3 FP64 (0.81-0.82 vs 0.78 ms).
constexpr long long SPLIT_MIN_CELLS = 1LL << 21;

// (The split last stage: 256^3 FP64 39.19 against 39.83 ms per step, FP32 20.22 against 20.71
// ms, 128^3 FP32 2.57 against 2.60 ms, alternated in one call; before the combination's loads
// and k_stage's were batched it measured 44.2 against 44.1 ms.)
// a workspace stage buffer that stage g neither reads nor writes (a split last stage stores its
// combination there), or 0
static int free_stage_buffer(const dg_ctx *c, const StageSpec &g)
{
    const int n = ((c->cfg.flags & DG_RK_BY_ORDER) && c->k == 3) ? 3 : 2;
    for (int b = 1; b <= n; ++b)
        if (b != g.in && b != g.un && b != g.w) return b;
    return 0;
}

template <typename T, int K>
static bool split_stage(const dg_ctx *c, const StageSpec &g, bool last)
{
    if (rhs_pair<T, K>() || g.w || g.out == g.in) return false;
    if (last ? free_stage_buffer(c, g) == 0 : g.out == 0) return false;
    if (c->cfg.flags & (DG_SEPARATE_STAGE | DG_VOLUME_MFMA)) return false;
    if (c->cfg.flags & DG_SPLIT_STAGE) return true;
    return (long long)c->nc >= SPLIT_MIN_CELLS;
}

// whether stage s is split and leaves the partials of its result for stage s + 1
// (k_limit_project): the next stage is split too and reads that result, and the driving table
// is in the pencil form
template <typename T, int K>
static bool next_split_partials(const dg_ctx *c, const Scheme &S, int s)
{
    return s + 1 < S.stages && S.s[s + 1].in == S.s[s].out && c->modes_sep &&
           split_stage<T, K>(c, S.s[s], s == S.stages - 1) && split_stage<T, K>(c, S.s[s + 1], s + 1 == S.stages - 1);
}

// the mean-acceleration partials of u alone (k_drive_parts) into the split stages' region
template <typename T, int K>
static int launch_drive_parts(dg_ctx *c, const void *u, int *fail_reset)
{
    if ((c->cfg.flags & DG_FORCING) && c->forcing_dirty) {
        int rc = launch_forcing_table<T, K>(c);
        if (rc) return rc;
        c->forcing_dirty = false;
    }
    RhsArgs a{};
    a.u = u;
    a.tab = c->tab;
    a.ftab = c->wp(c->off.ftab);
    a.modes = c->modes_dev;
    a.nmodes = c->nmodes;
    a.part = (double *)c->wp(c->off.dpart);
    a.fail_reset = fail_reset;
    a.g = Mesh{c->cfg.nx, c->cfg.ny, c->cfg.nz, c->nc};
    a.h = c->cfg.h;
    if (!c->modes_sep) hipLaunchKernelGGL((k_drive_parts<T, K, true>), dim3(c->nblk), dim3(BLOCK), 0, c->stream, a);
    else hipLaunchKernelGGL((k_drive_parts<T, K, false>), dim3(c->nblk), dim3(BLOCK), 0, c->stream, a);
    LAUNCHCHK(c);
    return DG_OK;
}

// Stage s of the scheme: right-hand side, mean acceleration, stage kernel.  reset_fail:
// this right-hand side clears the failure flag (a first stage starting from a kept
// projection); want_next: the step also returns the next time step (the last stage keeps the
// projection of the new state and reduces its time-step maxima).
template <typename T, int K>
static int launch_step_stage(dg_ctx *c, void *u, int s, double dt, bool reset_fail, bool want_next,
                             const double *dt_dev = nullptr)
{
    const Scheme &S = scheme_of(c);
    void *vh[2] = {c->wp(c->off.vh0), c->wp(c->off.vh1)};
    void *buf[4] = {u, c->wp(c->off.stA), c->wp(c->off.stB), c->wp(c->off.stC)};
    const StageSpec &g = S.s[s];
    const bool last = s == S.stages - 1;
    if constexpr (!rhs_pair<T, K>()) if (split_stage<T, K>(c, g, last)) {
        int rc = DG_OK;
        int *reset = reset_fail ? c->fail() : nullptr;
        const bool mf = use_meanfree(c);
        const bool in_stage = c->nblk <= ABAR_IN_STAGE_BLOCKS;
        // the mean acceleration of the input: its partials come from the previous split stage's
        // k_limit_project, else from k_drive_parts; more blocks than a block reduces itself go
        // through one reduction kernel
        const bool prev_split = s > 0 && next_split_partials<T, K>(c, S, s - 1);
        if (mf && !prev_split) {
            if ((rc = launch_drive_parts<T, K>(c, buf[g.in], reset))) return rc;
            reset = nullptr;
        }
        if (reset) {
            hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(1), 0, c->stream, reset);
            LAUNCHCHK(c);
        }
        if (mf && !in_stage && (rc = launch_abar(c, (const double *)c->wp(c->off.dpart), c->nblk))) return rc;
        c->abar_in_stage = in_stage;
        const int outb = last ? free_stage_buffer(c, g) : g.out;
        StageArgs st = stage_args(c, buf[g.in], buf[g.un], nullptr, buf[outb], vh[(s + 1) & 1], false, g.coef, dt,
                                  nullptr, nullptr, nullptr, g.wcoef, dt_dev, true);
        st.fail_on_mean = last;
        c->abar_in_stage = false;
        c->prof_first = s == 0;
        c->prof_last = last;
        if ((rc = launch_rhs<T, K>(c, buf[g.in], vh[s & 1], nullptr, dt, nullptr, nullptr, dt_dev, &st))) return rc;
        c->prof_last = false;
        if (last) {
            // the caller's array from the combination, unless a cell failed (the stage kernel's
            // limiter, projection and time-step maxima)
            void *vnext = want_next ? vh[0] : nullptr;
            double *part = want_next ? (double *)c->wp(c->off.spart) : nullptr;
            c->learned_bounds_later = want_next && (c->cfg.flags & DG_LEARNED_SENSOR);
            rc = launch_stage<T, K>(c, buf[outb], buf[outb], nullptr, buf[g.out], vnext, true, g.coef, dt, nullptr,
                                    part, nullptr, g.wcoef, dt_dev);
            c->learned_bounds_later = false;
            return rc;
        }
        // the next stage's partials, when it is split too and reads this stage's result (tables
        // in the pencil form: the mode-by-mode field costs too many registers there, and the
        // next stage runs k_drive_parts)
        st.drive_part = mf && next_split_partials<T, K>(c, S, s) ? (double *)c->wp(c->off.dpart) : nullptr;
        if ((rc = prof_mark(c, 1, 0))) return rc;
        if (st.drive_part)
            hipLaunchKernelGGL((k_limit_project<T, K, true>), dim3(c->nblk), dim3(BLOCK), 0, c->stream, st);
        else
            hipLaunchKernelGGL((k_limit_project<T, K, false>), dim3(c->nblk), dim3(BLOCK), 0, c->stream, st);
        LAUNCHCHK(c);
        return prof_mark(c, 1, 1);
    }
    // learned sensor: the network's viscosity of the new state serves its time step (and the
    // next step's stages).  The last stage reduces the signal speeds and the fallback cells'
    // viscosities; the network's forward pass on the new state reduces the learned cells'.
    const bool learned_next = want_next && (c->cfg.flags & DG_LEARNED_SENSOR);
    c->prof_first = s == 0;
    c->prof_last = last;
    // the last stage writes the caller's array: its failure is decided by its right-hand
    // side, so that on failure the stage kernel leaves u^n in place (no copy to restore)
    const StagePred pred{buf[g.un], g.coef};
    int rc = launch_rhs<T, K>(c, buf[g.in], vh[s & 1], c->wp(c->off.L), dt, reset_fail ? c->fail() : nullptr,
                              last ? &pred : nullptr, dt_dev);
    if (rc) return rc;
    // mean-free driving: with few right-hand-side blocks every stage block reduces their
    // partials itself (at most 32 KB of reads per block, no reduction kernel); with more, one
    // k_final reduces them once, as the repeated reads would grow with the square of the mesh
    const bool in_stage = c->rhs_nblk <= ABAR_IN_STAGE_BLOCKS;
    if (use_meanfree(c) && !in_stage) {
        rc = launch_abar(c);
        if (rc) return rc;
    }
    void *vnext = !last ? vh[(s + 1) & 1] : (want_next ? vh[0] : nullptr);
    double *part = (last && want_next) ? (double *)c->wp(c->off.spart) : nullptr;
    c->learned_bounds_later = learned_next && last;
    c->abar_in_stage = in_stage;
    c->prof_last = false;
    rc = launch_stage<T, K>(c, buf[g.in], buf[g.un], c->wp(c->off.L), buf[g.out], vnext, last, g.coef, dt, nullptr,
                            part, g.w ? buf[g.w] : nullptr, g.wcoef, dt_dev);
    c->learned_bounds_later = false;
    c->abar_in_stage = false;
    return rc;
}

// One Runge-Kutta step.  reuse: start from the projection kept by the previous step of
// this context (when it is still valid); dt_next: also compute the time step of the new
// state in the last stage (its projection is then kept in vh0).  horizon: when the next
// step is expected to go on without a driving update (1.25 dt < horizon), the first stage of
// the next step is queued right behind this step's last kernel, reading the new time step
// from device memory, so that the GPU does not wait for the host; it is kept (spec_valid)
// when this step succeeds with *dt_next < horizon, and a following step of the same array
// with that time step and a valid kept projection continues from it.  Calls that change what
// that stage computes drop it.
template <typename T, int K>
static int do_step(dg_ctx *c, void *u, double dt, int *status_host, bool reuse, double *dt_next, double horizon)
{
    const Scheme &S = scheme_of(c);
    const bool cached = reuse && c->vh_cache_u == u && c->vh_cache_gen == c->gen;
    const bool resume = cached && c->spec_valid && c->spec_u == u && c->spec_dt == dt;
    const bool ahead = dt_next && 1.25 * dt < horizon;
    c->spec_valid = false;
    c->gen++;
    c->vh_cache_u = nullptr;
    int rc = DG_OK;
    if (!cached) {
        rc = launch_project<T, K>(c, u, c->wp(c->off.vh0), nullptr, c->fail());
        if (rc) return rc;
    }
    for (int s = resume ? 1 : 0; s < S.stages; ++s) {
        rc = launch_step_stage<T, K>(c, u, s, dt, s == 0 && cached, dt_next != nullptr);
        if (rc) return rc;
    }
    int st_flag = 0;
    double dt_pub = 0.0;
    if (dt_next) {
        const double *vmax = nullptr;
        int nvmax = 0;
        if (c->cfg.flags & DG_LEARNED_SENSOR) {
            // the last stage left the projection of u^(n+1) in vh0 (unless the step failed)
            if ((rc = sensor_infer_impl(c, u, &nvmax, c->wp(c->off.vh0)))) return rc;
            if (proj_args(c).visc) vmax = (const double *)c->wp(c->off.mlp);
        }
        const long long seq = ++c->pub_seq;
        rc = launch_dt_final<T, K>(c, (const double *)c->wp(c->off.spart), c->scal() + 8, seq, vmax, nvmax);
        if (rc) return rc;
        if (ahead) {
            // from u^(n+1) with the time step k_final has just stored; written only into
            // workspace buffers, and discarded if this step fails
            rc = launch_step_stage<T, K>(c, u, 0, 0.0, true, true, c->scal() + 8);
            if (rc) return rc;
        }
        rc = wait_published(c, seq, &dt_pub, &st_flag);
        if (rc) return rc;
    } else {
        HIPCHK(c, hipMemcpyAsync(c->pinned, c->fail(), sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        st_flag = ((volatile int *)c->pinned)[0];
    }
    if (status_host) *status_host = st_flag ? DG_RETRY : DG_OK;
    // on failure the last stage wrote nothing: u is still u^n, and the network viscosity
    // inferred after the stages is that of u^n
    if (st_flag) return DG_RETRY;
    if (dt_next) {
        *dt_next = dt_pub;
        c->vh_cache_u = u;
        c->vh_cache_gen = c->gen;
        if (ahead && dt_pub < horizon) {
            c->spec_valid = true;
            c->spec_u = u;
            c->spec_dt = dt_pub;
        }
    }
    return DG_OK;
}

template <typename T, int K>
static int split_stages_impl(const dg_ctx *c)
{
    const Scheme &S = scheme_of(c);
    for (int s = 0; s < S.stages; ++s)
        if (split_stage<T, K>(c, S.s[s], s == S.stages - 1)) return 1;
    return 0;
}

#define DISPATCH(c, FN, ...)                                                        \
    ((c)->es == 8 ? ((c)->k == 1   ? FN<double, 1>(__VA_ARGS__)                     \
                     : (c)->k == 2 ? FN<double, 2>(__VA_ARGS__)                     \
                                   : FN<double, 3>(__VA_ARGS__))                    \
                  : ((c)->k == 1   ? FN<float, 1>(__VA_ARGS__)                      \
                     : (c)->k == 2 ? FN<float, 2>(__VA_ARGS__)                      \
                                   : FN<float, 3>(__VA_ARGS__)))

static int learned_ready(dg_ctx *c)
{
    if ((c->cfg.flags & DG_LEARNED_SENSOR) && !c->have_nu)
        return dg_fail(c, DG_ESTATE, "learned sensor enabled but no viscosity stored (dg_sensor_infer or dg_sensor_set_nu)");
    return DG_OK;
}

int dg_rhs(dg_ctx *c, const void *u, void *dudt, double dt)
{
    if (!c) return DG_EINVAL;
    int rc;
    if ((rc = need_ws(c)) || (rc = check_ptr(c, u, "u")) || (rc = check_ptr(c, dudt, "dudt"))) return rc;
    if ((rc = learned_ready(c))) return rc;
    c->gen++;
    return DISPATCH(c, do_rhs, c, u, dudt, dt);
}

int dg_rk_step(dg_ctx *c, void *u, double dt, int *status_host)
{
    if (!c) return DG_EINVAL;
    int rc;
    if ((rc = need_ws(c)) || (rc = check_ptr(c, u, "u"))) return rc;
    if (!(dt > 0.0) || !std::isfinite(dt)) return dg_fail(c, DG_EINVAL, "dt must be positive and finite");
    if ((rc = learned_ready(c))) return rc;
    return DISPATCH(c, do_step, c, u, dt, status_host, false, (double *)nullptr, -1.0);
}

int dg_rk_step_next(dg_ctx *c, void *u, double dt, int reuse, int *status_host, double *dt_next_host)
{
    if (!c) return DG_EINVAL;
    int rc;
    if ((rc = need_ws(c)) || (rc = check_ptr(c, u, "u"))) return rc;
    if (!(dt > 0.0) || !std::isfinite(dt)) return dg_fail(c, DG_EINVAL, "dt must be positive and finite");
    if (!dt_next_host) return dg_fail(c, DG_EINVAL, "dt_next_host is null");
    if ((rc = learned_ready(c))) return rc;
    return DISPATCH(c, do_step, c, u, dt, status_host, reuse != 0, dt_next_host, -1.0);
}

int dg_rk_step_next_ahead(dg_ctx *c, void *u, double dt, int reuse, double horizon, int *status_host,
                          double *dt_next_host)
{
    if (!c) return DG_EINVAL;
    int rc;
    if ((rc = need_ws(c)) || (rc = check_ptr(c, u, "u"))) return rc;
    if (!(dt > 0.0) || !std::isfinite(dt)) return dg_fail(c, DG_EINVAL, "dt must be positive and finite");
    if (!dt_next_host) return dg_fail(c, DG_EINVAL, "dt_next_host is null");
    if (std::isnan(horizon)) return dg_fail(c, DG_EINVAL, "horizon is NaN");
    if ((rc = learned_ready(c))) return rc;
    return DISPATCH(c, do_step, c, u, dt, status_host, reuse != 0, dt_next_host, horizon);
}

int dg_split_stages(const dg_ctx *c)
{
    if (!c) return DG_EINVAL;
    return DISPATCH(c, split_stages_impl, c);
}

template <typename T, int K>
static int do_dt(dg_ctx *c, const void *u, double *dt_out, int on_host)
{
    double *part = (double *)c->wp(c->off.part);
    int rc = launch_project<T, K>(c, u, nullptr, part, nullptr);
    if (rc) return rc;
    double *dst = on_host ? c->scal() + 8 : dt_out;
    rc = launch_dt_final<T, K>(c, part, dst);
    if (rc) return rc;
    if (on_host) {
        HIPCHK(c, hipMemcpyAsync(c->pinned, dst, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        *dt_out = ((volatile double *)c->pinned)[0];
    }
    return DG_OK;
}

int dg_dt_max(dg_ctx *c, const void *u, double *dt_out, int on_host)
{
    if (!c) return DG_EINVAL;
    int rc;
    if ((rc = need_ws(c)) || (rc = check_ptr(c, u, "u"))) return rc;
    if (!dt_out) return dg_fail(c, DG_EINVAL, "dt_out is null");
    if (!on_host && (rc = dg_check_array(c, dt_out, sizeof(double), sizeof(double), "dt_out"))) return rc;
    if ((rc = learned_ready(c))) return rc;
    return DISPATCH(c, do_dt, c, u, dt_out, on_host);
}

template <typename T, int K>
static int do_dt_noalloc(dg_ctx *c, const void *u, double *dt_out, int on_host, double *scr)
{
    int rc = launch_project<T, K>(c, u, nullptr, scr, nullptr);
    if (rc) return rc;
    double *dst = on_host ? scr + NOALLOC_DT_SLOT : dt_out;
    rc = launch_dt_final<T, K>(c, scr, dst);
    if (rc) return rc;
    if (on_host) {
        HIPCHK(c, hipMemcpyAsync(c->pinned, dst, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        *dt_out = ((volatile double *)c->pinned)[0];
    }
    return DG_OK;
}

int dg_dt_max_noalloc(dg_ctx *c, const void *u, double *dt_out, int on_host)
{
    if (!c) return DG_EINVAL;
    if (c->cfg.flags & DG_LEARNED_SENSOR)
        return dg_fail(c, DG_EUNSUPPORTED, "dg_dt_max_noalloc: the learned sensor's viscosity lives in the workspace");
    if (c->nblk > NOALLOC_MAX_BLOCKS)
        return dg_fail(c, DG_EINVAL, "dg_dt_max_noalloc: %d cells need %d blocks of partials, the static scratch holds %d "
                                     "(%d cells)", c->nc, c->nblk, NOALLOC_MAX_BLOCKS, NOALLOC_MAX_BLOCKS * BLOCK);
    int rc;
    if ((rc = check_ptr(c, u, "u"))) return rc;
    if (!dt_out) return dg_fail(c, DG_EINVAL, "dt_out is null");
    if (!on_host && (rc = dg_check_array(c, dt_out, sizeof(double), sizeof(double), "dt_out"))) return rc;
    int dev = -1;
    HIPCHK(c, hipGetDevice(&dev));
    if (dev != c->device)
        return dg_fail(c, DG_EINVAL, "dg_dt_max_noalloc: device %d is current, the context was created on %d", dev, c->device);
    double *scr = (dev >= 0 && dev < NOALLOC_MAX_DEVICES) ? noalloc_ptr[dev] : nullptr;
    if (!scr) return dg_fail(c, DG_EHIP, "dg_dt_max_noalloc: no static scratch on device %d", dev);
    return DISPATCH(c, do_dt_noalloc, c, u, dt_out, on_host, scr);
}

template <typename T, int K>
static int do_proj(dg_ctx *c, const void *u, void *vh)
{
    return launch_project<T, K>(c, u, vh, nullptr, nullptr);
}

int dg_project_primitive(dg_ctx *c, const void *u, void *vhat)
{
    if (!c) return DG_EINVAL;
    int rc;
    if ((rc = check_ptr(c, u, "u")) || (rc = check_ptr(c, vhat, "vhat", 3))) return rc;
    return DISPATCH(c, do_proj, c, u, vhat);
}

template <typename T, int K>
static int do_limit(dg_ctx *c, void *u, long *nfail)
{
    long long *cnt = (long long *)(c->scal() + 16);
    int *fl = c->fail();
    // zero the counters with a tiny copy from pinned host zeros (no memset nodes)
    std::memset(c->pinned + 8, 0, 16);
    HIPCHK(c, hipMemcpyAsync(cnt, c->pinned + 8, 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(fl, c->pinned + 8, 4, hipMemcpyHostToDevice, c->stream));
    static const double plain[3] = {0.0, 1.0, 0.0};
    int rc = launch_stage<T, K>(c, u, u, nullptr, u, nullptr, false, plain, 0.0, cnt);
    if (rc) return rc;
    HIPCHK(c, hipMemcpyAsync(c->pinned, cnt, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (nfail) *nfail = (long)((volatile long long *)c->pinned)[0];
    return DG_OK;
}

int dg_limit(dg_ctx *c, void *u, long *nfail_host)
{
    if (!c) return DG_EINVAL;
    int rc;
    if ((rc = need_ws(c)) || (rc = check_ptr(c, u, "u"))) return rc;
    const int saved = c->cfg.flags;
    c->cfg.flags |= DG_POS_LIMITER;
    c->gen++;
    rc = DISPATCH(c, do_limit, c, u, nfail_host);
    c->cfg.flags = saved;
    return rc;
}

template <typename T, int K>
static int do_sums(dg_ctx *c, const void *u, double *out)
{
    const Mesh g{c->cfg.nx, c->cfg.ny, c->cfg.nz, c->nc};
    double *part = (double *)c->wp(c->off.part);
    hipLaunchKernelGGL((k_sums<T, K>), dim3(c->nblk), dim3(BLOCK), 0, c->stream, u, g, part);
    LAUNCHCHK(c);
    const double h3 = c->cfg.h * c->cfg.h * c->cfg.h;
    hipLaunchKernelGGL(k_final, dim3(1), dim3(BLOCK), 0, c->stream, (const double *)part, c->nblk, 0, h3, 0.0,
                       c->scal() + 24, (const int *)nullptr, (volatile long long *)nullptr, 0LL, (const double *)nullptr, 0);
    LAUNCHCHK(c);
    HIPCHK(c, hipMemcpyAsync(c->pinned, c->scal() + 24, 32, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int i = 0; i < 4; ++i) out[i] = ((volatile double *)c->pinned)[i];
    return DG_OK;
}

int dg_conserved_sums(dg_ctx *c, const void *u, double *out_host)
{
    if (!c) return DG_EINVAL;
    int rc;
    if ((rc = need_ws(c)) || (rc = check_ptr(c, u, "u"))) return rc;
    if (!out_host) return dg_fail(c, DG_EINVAL, "out_host is null");
    return DISPATCH(c, do_sums, c, u, out_host);
}
