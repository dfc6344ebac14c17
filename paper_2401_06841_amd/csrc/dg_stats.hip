// dg_stats.hip -- flow statistics of a DG state on the GPU (Sec. 4.3): the second-order
// velocity structure function from random point pairs evaluated through the cell
// expansions, and the shell-summed velocity power spectrum of the sampling grid of p
// points per cell per dimension.
//
// Pairs: pair j of bin b owns the draws 256 (b npairs + j) + t of the counter-based
// SplitMix64 stream `seed` (Steele, Lea & Flood 2014; a draw is the generator's output for
// the state seed + (i+1) 0x9E3779B97F4A7C15, a uniform double its top 53 bits times 2^-53):
// t = 0..2 the first point (uniform in the box), then direction attempts of three draws
// each, uniform in [-1,1]^3, accepted when 1e-12 < r^2 <= 1 (at most 84, else +z); the
// second point is x + l n (one fused multiply-add per axis) wrapped into the box.  Every
// decision that picks a cell is taken from correctly rounded operations only, so a pair
// lands in the same cells on any IEEE machine.
//
// Layout for the random gathers: the state is first copied to one record per cell,
// [cell][var][mode] in the state's precision (4 nb values, 16-byte aligned), so a point
// reads one contiguous record instead of 4 nb separate cache lines; the evaluation is FP64.
// The pair kernel runs one wave per block and stages the records of its 64 lanes' points
// through LDS: consecutive lanes load consecutive 16-byte pieces of the same records, so
// every cache line of a record is fetched by one instruction instead of by per-lane loads
// spread over time.  Records above 320 bytes (FP64 at degree 3) are staged in two halves
// (rho, m_x then m_y, m_z) so that 20 KB of LDS per wave keeps two waves per SIMD.  Sums are
// per lane, per wave (fixed tree) and over blocks in a fixed order, so the structure
// function is deterministic.  The spectrum bins shell energies with LDS atomics inside a block (the
// order of additions inside a block is not fixed; blocks are summed in a fixed order).
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "dg.h"
#include "dg_ctx.hpp"
#include "dg_kernels.hpp"

namespace dg {

constexpr int SF_CHUNKS = 256;      // blocks (one wave each) per bin of the pair kernel
constexpr int SFB = 64;             // threads per block of the pair kernel
constexpr int SP_BLOCKS = 1024;     // blocks of the shell kernel
constexpr int SF_MAX_BINS = 65535;  // grid y limit
constexpr int SP_MAX_SHELLS = 4096; // LDS histogram of the shell kernel (32 KiB)

struct StatsGeom {
    int nx, ny, nz;
    double h, Lx, Ly, Lz, floor;
};

__device__ __forceinline__ unsigned long long splitmix64(unsigned long long seed, unsigned long long i)
{
    unsigned long long z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double uniform01(unsigned long long seed, unsigned long long i)
{
    return (double)(splitmix64(seed, i) >> 11) * 0x1.0p-53;
}

// Lt_n(x) = sqrt(2n+1) P_n(x), n = 0..K, by the three-term recurrence of P_n
template <int K>
__device__ __forceinline__ void legendre_row(double x, double (&L)[K + 1])
{
    double pm = 1.0, p = x;
    L[0] = 1.0;
    if constexpr (K >= 1) L[1] = __builtin_sqrt(3.0) * x;
#pragma unroll
    for (int n = 1; n < K; ++n) {
        const double pn = ((2 * n + 1) * x * p - n * pm) * (1.0 / (n + 1));
        pm = p;
        p = pn;
        L[n + 1] = __builtin_sqrt(double(2 * n + 3)) * pn;
    }
}

// cell that holds x and the reference coordinates of x in it
__device__ __forceinline__ int locate(const StatsGeom &g, const double (&x)[3], double (&xi)[3])
{
    const int n[3] = {g.nx, g.ny, g.nz};
    int ijk[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double s = x[a] / g.h;
        int i = (int)floor(s);
        i = i < 0 ? 0 : (i > n[a] - 1 ? n[a] - 1 : i);
        ijk[a] = i;
        xi[a] = 2.0 * (s - i) - 1.0;
    }
    return ijk[0] + g.nx * (ijk[1] + g.ny * ijk[2]);
}

// phi_l(xi) of every mode, FP64
template <int K>
__device__ __forceinline__ void basis_at(const double (&xi)[3], double (&phi)[Shape<K>::NB])
{
    constexpr Modes<K> M = make_modes<K>();
    double Lx[K + 1], Ly[K + 1], Lz[K + 1];
    legendre_row<K>(xi[0], Lx);
    legendre_row<K>(xi[1], Ly);
    legendre_row<K>(xi[2], Lz);
#pragma unroll
    for (int l = 0; l < Shape<K>::NB; ++l) phi[l] = Lx[M.e[l][0]] * Ly[M.e[l][1]] * Lz[M.e[l][2]];
}

// [var][mode][cell] -> [cell][var][mode] (element type T) through an LDS tile of 64 cells:
// the reads run along cells and the writes along the contiguous records of the 64 cells
template <typename T, int K>
__global__ void __launch_bounds__(BLOCK) k_cell_records(const void *u_, int nc, T *cells)
{
    constexpr int NR = 4 * Shape<K>::NB;    // values per record
    constexpr int TC = 64;                  // cells per block
    __shared__ T tile[NR][TC + 1];
    const T *u = (const T *)u_;
    const int c0 = blockIdx.x * TC;
    const int ncb = nc - c0 < TC ? nc - c0 : TC;
    for (int idx = threadIdx.x; idx < NR * TC; idx += BLOCK) {
        const int i = idx / TC, t = idx - i * TC;
        if (t < ncb) tile[i][t] = u[(size_t)i * nc + c0 + t];
    }
    __syncthreads();
    T *out = cells + (size_t)c0 * NR;
    for (int q = threadIdx.x; q < NR * ncb; q += BLOCK) {
        const int t = q / NR, i = q - t * NR;
        out[q] = tile[i][t];
    }
}

// grid (chunks, bins), one wave per block: block (x, b) takes the pairs j = j0 + lane,
// j0 = x 64, x 64 + chunks 64, ...; lanes past npairs repeat the block's first pair and
// are not summed
template <int K, typename RT>
__global__ void __launch_bounds__(SFB) __attribute__((amdgpu_waves_per_eu(2))) k_sf_pairs(const RT *cells, StatsGeom g, const double *lb,
                                                  long long npairs, unsigned long long seed, double *part)
{
    constexpr int NB = Shape<K>::NB;
    constexpr int RECB = 4 * NB * (int)sizeof(RT);          // bytes per record
    constexpr int VPP = RECB > 320 ? 2 : 4;                  // variables staged per phase
    constexpr int NPH = 4 / VPP;
    constexpr int PIECES = VPP * NB * (int)sizeof(RT) / 16;  // 16-byte pieces per phase
    constexpr int RECP = RECB / 16;
    static_assert(RECB % 16 == 0 && (VPP * NB * (int)sizeof(RT)) % 16 == 0, "records in 16-byte pieces");
    __shared__ uint4 rec[SFB * PIECES];
    const int b = blockIdx.y;
    const int lane = threadIdx.x;
    const double l = lb[b];
    const double L[3] = {g.Lx, g.Ly, g.Lz};
    const uint4 *src = (const uint4 *)cells;
    double sum = 0.0;
    for (long long j0 = (long long)blockIdx.x * SFB; j0 < npairs; j0 += (long long)gridDim.x * SFB) {
        const bool act = j0 + lane < npairs;
        const unsigned long long j = (unsigned long long)(act ? j0 + lane : j0);
        const unsigned long long base = ((unsigned long long)b * (unsigned long long)npairs + j) * 256ull;
        double x[2][3];
#pragma unroll
        for (int a = 0; a < 3; ++a) x[0][a] = uniform01(seed, base + a) * L[a];
        double n0 = 0.0, n1 = 0.0, n2 = 1.0;
        for (int t = 0; t < 84; ++t) {
            const double c0 = 2.0 * uniform01(seed, base + 3 + 3 * t) - 1.0;
            const double c1 = 2.0 * uniform01(seed, base + 4 + 3 * t) - 1.0;
            const double c2 = 2.0 * uniform01(seed, base + 5 + 3 * t) - 1.0;
            const double r2 = fma(c2, c2, fma(c1, c1, c0 * c0));
            if (r2 > 1e-12 && r2 <= 1.0) {
                const double r = sqrt(r2);
                n0 = c0 / r;
                n1 = c1 / r;
                n2 = c2 / r;
                break;
            }
        }
        const double nn[3] = {n0, n1, n2};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double y = fma(l, nn[a], x[0][a]);
            if (y >= L[a]) y -= L[a];
            else if (y < 0.0) y += L[a];
            x[1][a] = y;
        }
        double v[2][3];
#pragma unroll 1
        for (int pt = 0; pt < 2; ++pt) {
            double xi[3], phi[NB];
            const int c = locate(g, x[pt], xi);
            basis_at<K>(xi, phi);
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ph = 0; ph < NPH; ++ph) {
                __syncthreads();                    // the previous records are consumed
#pragma unroll
                for (int s = 0; s < PIECES; ++s) {
                    const int item = s * SFB + lane;
                    const int r = item / PIECES, o = item - r * PIECES;
                    const int cr = __shfl(c, r, 64);
                    rec[item] = src[(size_t)cr * RECP + ph * PIECES + o];
                }
                __syncthreads();
                const RT *w = (const RT *)(rec + lane * PIECES);
#pragma unroll
                for (int vv = 0; vv < VPP; ++vv)
#pragma unroll
                    for (int m = 0; m < NB; ++m) acc[ph * VPP + vv] += (double)w[vv * NB + m] * phi[m];
            }
            const double rho = fmax(acc[0], g.floor);
            v[pt][0] = acc[1] / rho;
            v[pt][1] = acc[2] / rho;
            v[pt][2] = acc[3] / rho;
        }
        if (act)
#pragma unroll
            for (int d = 0; d < 3; ++d) sum += (v[0][d] - v[1][d]) * (v[0][d] - v[1][d]);
    }
    sum = wave_sum(sum);
    if (lane == 0) part[(size_t)b * gridDim.x + blockIdx.x] = sum;
}

// one block per bin: out[b] = (fixed-order sum over the chunks of bin b) / npairs
static __global__ void __launch_bounds__(BLOCK) k_sf_final(const double *part, int nchunks, long long npairs, double *out)
{
    __shared__ double lds[4 * 4];
    const int b = blockIdx.x;
    double t[1] = {0.0};
    for (int i = threadIdx.x; i < nchunks; i += BLOCK) t[0] += part[(size_t)b * nchunks + i];
    block_sum<1>(t, lds);
    if (threadIdx.x == 0) out[b] = t[0] / (double)npairs;
}

// v on the grid of p cell-centred sub-points per cell per dimension, [d][Z][Y][X], x fastest
template <typename T, int K>
__global__ void __launch_bounds__(BLOCK) k_velocity_grid(const void *u_, StatsGeom g, int p, double *grid)
{
    constexpr int NB = Shape<K>::NB;
    const long long X = (long long)g.nx * p, Y = (long long)g.ny * p, Z = (long long)g.nz * p;
    const long long npts = X * Y * Z;
    const long long o = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (o >= npts) return;
    const long long gg[3] = {o % X, (o / X) % Y, o / (X * Y)};
    int ijk[3];
    double xi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        ijk[a] = (int)(gg[a] / p);
        xi[a] = -1.0 + (2.0 * (double)(gg[a] % p) + 1.0) / p;
    }
    double phi[NB];
    basis_at<K>(xi, phi);
    const size_t nc = (size_t)g.nx * g.ny * g.nz;
    const size_t c = (size_t)ijk[0] + (size_t)g.nx * ((size_t)ijk[1] + (size_t)g.ny * ijk[2]);
    const T *u = (const T *)u_;
    double r = 0.0, m[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int l = 0; l < NB; ++l) {
        r += (double)u[(size_t)l * nc + c] * phi[l];
#pragma unroll
        for (int d = 0; d < 3; ++d) m[d] += (double)u[((size_t)(1 + d) * NB + l) * nc + c] * phi[l];
    }
    r = fmax(r, g.floor);
#pragma unroll
    for (int d = 0; d < 3; ++d) grid[(size_t)d * npts + o] = m[d] / r;
}

// Shell sums of 1/2 |F / npts|^2 over the half spectrum F[d][Z][Y][X/2+1] of a real X x Y x Z
// grid (the planes 0 < kx < X/2 stand for themselves and their mirror images, weight 2);
// per-block histograms to part[block][nshell]
static __global__ void __launch_bounds__(BLOCK) k_shells(const double2 *F, long long X, long long Y, long long Z,
                                                         int nshell, double *part)
{
    extern __shared__ double hist[];
    for (int s = threadIdx.x; s < nshell; s += BLOCK) hist[s] = 0.0;
    __syncthreads();
    const long long Xh = X / 2 + 1;
    const long long M = Xh * Y * Z;
    const double inv = 1.0 / ((double)X * (double)Y * (double)Z);
    for (long long o = (long long)blockIdx.x * BLOCK + threadIdx.x; o < M; o += (long long)gridDim.x * BLOCK) {
        const long long ix = o % Xh, r = o / Xh, iy = r % Y, iz = r / Y;
        const long long fy = iy < (Y + 1) / 2 ? iy : iy - Y;
        const long long fz = iz < (Z + 1) / 2 ? iz : iz - Z;
        const int shell = (int)floor(sqrt((double)(ix * ix + fy * fy + fz * fz)) + 0.5);
        const double w = (ix == 0 || (X % 2 == 0 && ix == X / 2)) ? 0.5 : 1.0;
        double e = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double2 f = F[(size_t)d * M + o];
            e += f.x * f.x + f.y * f.y;
        }
        atomicAdd(&hist[shell], w * e * inv * inv);
    }
    __syncthreads();
    for (int s = threadIdx.x; s < nshell; s += BLOCK) part[(size_t)blockIdx.x * nshell + s] = hist[s];
}

// one block per shell: fixed strided partial sums, then the fixed block tree
static __global__ void __launch_bounds__(BLOCK) k_shells_final(const double *part, int nblk, int nshell, double *out)
{
    __shared__ double lds[4 * 4];
    const int s = blockIdx.x;
    double t[1] = {0.0};
    for (int b = threadIdx.x; b < nblk; b += BLOCK) t[0] += part[(size_t)b * nshell + s];
    block_sum<1>(t, lds);
    if (threadIdx.x == 0) out[s] = t[0];
}

}  // namespace dg

using namespace dg;

namespace {

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

StatsGeom geom_of(const dg_ctx *c)
{
    StatsGeom g;
    g.nx = c->cfg.nx;
    g.ny = c->cfg.ny;
    g.nz = c->cfg.nz;
    g.h = c->cfg.h;
    g.Lx = c->cfg.nx * c->cfg.h;
    g.Ly = c->cfg.ny * c->cfg.h;
    g.Lz = c->cfg.nz * c->cfg.h;
    g.floor = c->cfg.rho_floor;
    return g;
}

struct SfLayout {
    size_t cells, lb, part, out, total;
};

SfLayout sf_layout(const dg_ctx *c, int nbins)
{
    SfLayout s;
    size_t o = 0;
    s.cells = o; o += up256((size_t)c->nc * 4 * c->nb * c->es);
    s.lb = o; o += up256((size_t)nbins * sizeof(double));
    s.part = o; o += up256((size_t)nbins * SF_CHUNKS * sizeof(double));
    s.out = o; o += up256((size_t)nbins * sizeof(double));
    s.total = o;
    return s;
}

struct SpLayout {
    long long X, Y, Z, npts, M;
    int nshell;
    size_t grid, cplx, part, out, total;
};

SpLayout sp_layout(const dg_ctx *c, int p)
{
    SpLayout s;
    s.X = (long long)c->cfg.nx * p;
    s.Y = (long long)c->cfg.ny * p;
    s.Z = (long long)c->cfg.nz * p;
    s.npts = s.X * s.Y * s.Z;
    s.M = (s.X / 2 + 1) * s.Y * s.Z;
    const double kmax = std::sqrt((double)((s.X / 2) * (s.X / 2) + (s.Y / 2) * (s.Y / 2) + (s.Z / 2) * (s.Z / 2)));
    s.nshell = (int)std::floor(kmax + 0.5) + 1;
    size_t o = 0;
    s.grid = o; o += up256((size_t)s.npts * 3 * sizeof(double));
    s.cplx = o; o += up256((size_t)s.M * 3 * 2 * sizeof(double));
    s.part = o; o += up256((size_t)SP_BLOCKS * s.nshell * sizeof(double));
    s.out = o; o += up256((size_t)s.nshell * sizeof(double));
    s.total = o;
    return s;
}

int check_state_ptr(dg_ctx *c, const void *u)
{
    return dg_check_array(c, u, dg_state_bytes(c), c->es, "u");
}

int check_scratch(dg_ctx *c, const void *scratch, size_t bytes, size_t need)
{
    if (!scratch) return dg_fail(c, DG_EINVAL, "scratch is null");
    if ((uintptr_t)scratch & 255) return dg_fail(c, DG_EINVAL, "scratch must be 256-byte aligned");
    if (bytes < need) return dg_fail(c, DG_ENOMEM, "scratch too small: %zu < %zu bytes", bytes, need);
    return dg_check_array(c, scratch, need, 256, "scratch");
}

template <typename T, int K>
int launch_sf(dg_ctx *c, const void *u, int nbins, long long npairs, unsigned long long seed, char *scr,
              const SfLayout &s, const double *lb_host)
{
    const StatsGeom g = geom_of(c);
    T *cells = (T *)(scr + s.cells);
    double *lb = (double *)(scr + s.lb);
    double *part = (double *)(scr + s.part);
    double *out = (double *)(scr + s.out);
    HIPCHK(c, hipMemcpyAsync(lb, lb_host, (size_t)nbins * sizeof(double), hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL((k_cell_records<T, K>), dim3((c->nc + 63) / 64), dim3(BLOCK), 0, c->stream, u, c->nc, cells);
    LAUNCHCHK(c);
    const long long need = (npairs + SFB - 1) / SFB;
    const int chunks = (int)(need < SF_CHUNKS ? need : SF_CHUNKS);
    hipLaunchKernelGGL((k_sf_pairs<K, T>), dim3(chunks, nbins), dim3(SFB), 0, c->stream, (const T *)cells, g,
                       (const double *)lb, npairs, seed, part);
    LAUNCHCHK(c);
    hipLaunchKernelGGL(k_sf_final, dim3(nbins), dim3(BLOCK), 0, c->stream, (const double *)part, chunks, npairs, out);
    LAUNCHCHK(c);
    return DG_OK;
}

template <typename T, int K>
int launch_grid(dg_ctx *c, const void *u, int p, double *grid, long long npts)
{
    const StatsGeom g = geom_of(c);
    hipLaunchKernelGGL((k_velocity_grid<T, K>), dim3((unsigned)((npts + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0,
                       c->stream, u, g, p, grid);
    LAUNCHCHK(c);
    return DG_OK;
}

#define STATS_DISPATCH(c, FN, ...)                                                  \
    ((c)->es == 8 ? ((c)->k == 1   ? FN<double, 1>(__VA_ARGS__)                     \
                     : (c)->k == 2 ? FN<double, 2>(__VA_ARGS__)                     \
                                   : FN<double, 3>(__VA_ARGS__))                    \
                  : ((c)->k == 1   ? FN<float, 1>(__VA_ARGS__)                      \
                     : (c)->k == 2 ? FN<float, 2>(__VA_ARGS__)                      \
                                   : FN<float, 3>(__VA_ARGS__)))

int fft_fail(dg_ctx *c, const char *what, hipfftResult r)
{
    return dg_fail(c, DG_EHIP, "%s failed: hipfftResult %d", what, (int)r);
}

// the context's real-to-complex plan for an X x Y x Z grid (made once per grid shape)
int fft_plan(dg_ctx *c, const SpLayout &s, hipfftHandle *out)
{
    if (c->fft_plan && c->fft_dims[0] == s.X && c->fft_dims[1] == s.Y && c->fft_dims[2] == s.Z) {
        *out = (hipfftHandle)c->fft_plan;
        return DG_OK;
    }
    stats_release(c);
    hipfftHandle plan;
    const hipfftResult fr = hipfftPlan3d(&plan, (int)s.Z, (int)s.Y, (int)s.X, HIPFFT_D2Z);
    if (fr != HIPFFT_SUCCESS) return fft_fail(c, "hipfftPlan3d", fr);
    c->fft_plan = (void *)plan;
    c->fft_dims[0] = s.X;
    c->fft_dims[1] = s.Y;
    c->fft_dims[2] = s.Z;
    *out = plan;
    return DG_OK;
}

}  // namespace

void stats_release(dg_ctx *c)
{
    if (c->fft_plan) {
        (void)hipStreamSynchronize(c->stream);
        hipfftDestroy((hipfftHandle)c->fft_plan);
        c->fft_plan = nullptr;
    }
}

int dg_sf_bins(const dg_ctx *c, int nbins, double *l_host)
{
    if (!c || !l_host || nbins < 1) return DG_EINVAL;
    const StatsGeom g = geom_of(c);
    const double lmax = 0.5 * std::fmin(g.Lx, std::fmin(g.Ly, g.Lz));
    const double lmin = g.h / (c->k + 1);
    for (int b = 0; b < nbins; ++b) l_host[b] = lmin * std::pow(lmax / lmin, (b + 0.5) / nbins);
    return DG_OK;
}

size_t dg_stats_scratch_bytes(const dg_ctx *c, int nbins, int p)
{
    if (!c) return 0;
    size_t need = 0;
    if (nbins > 0) need = sf_layout(c, nbins).total;
    if (p > 0) {
        const size_t s = sp_layout(c, p).total;
        need = s > need ? s : need;
    }
    return need;
}

int dg_structure_function(dg_ctx *c, const void *u, int nbins, long long npairs, unsigned long long seed,
                          void *scratch, size_t scratch_bytes, double *s2_host)
{
    if (!c) return DG_EINVAL;
    int rc;
    if ((rc = check_state_ptr(c, u))) return rc;
    if (nbins < 1 || nbins > SF_MAX_BINS) return dg_fail(c, DG_EINVAL, "nbins must be in 1..%d", SF_MAX_BINS);
    if (npairs < 1) return dg_fail(c, DG_EINVAL, "npairs must be positive");
    if ((unsigned long long)nbins * (unsigned long long)npairs > (1ull << 55))
        return dg_fail(c, DG_EINVAL, "nbins * npairs too large for the draw counters");
    if (!s2_host) return dg_fail(c, DG_EINVAL, "s2_host is null");
    const SfLayout s = sf_layout(c, nbins);
    if ((rc = check_scratch(c, scratch, scratch_bytes, s.total))) return rc;
    std::vector<double> lb(nbins);
    dg_sf_bins(c, nbins, lb.data());
    rc = STATS_DISPATCH(c, launch_sf, c, u, nbins, npairs, seed, (char *)scratch, s, lb.data());
    if (rc) return rc;
    HIPCHK(c, hipMemcpyAsync(s2_host, (char *)scratch + s.out, (size_t)nbins * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DG_OK;
}

int dg_spectrum_nshell(const dg_ctx *c, int p)
{
    if (!c || p < 1) return DG_EINVAL;
    return sp_layout(c, p).nshell;
}

int dg_velocity_spectrum(dg_ctx *c, const void *u, int p, void *scratch, size_t scratch_bytes, double *e_host)
{
    if (!c) return DG_EINVAL;
    int rc;
    if ((rc = check_state_ptr(c, u))) return rc;
    if (p < 1) return dg_fail(c, DG_EINVAL, "p must be positive");
    if (!e_host) return dg_fail(c, DG_EINVAL, "e_host is null");
    const SpLayout s = sp_layout(c, p);
    if (s.X < 2 || s.Y < 2 || s.Z < 2) return dg_fail(c, DG_EINVAL, "the sampling grid needs at least 2 points per axis");
    if (s.X > (1 << 30) || s.Y > (1 << 30) || s.Z > (1 << 30) || s.npts > (1ll << 40))
        return dg_fail(c, DG_EINVAL, "sampling grid too large");
    if (s.nshell > SP_MAX_SHELLS) return dg_fail(c, DG_EUNSUPPORTED, "more than %d shells", SP_MAX_SHELLS);
    if ((rc = check_scratch(c, scratch, scratch_bytes, s.total))) return rc;
    char *scr = (char *)scratch;
    double *grid = (double *)(scr + s.grid);
    double2 *cplx = (double2 *)(scr + s.cplx);
    double *part = (double *)(scr + s.part);
    double *out = (double *)(scr + s.out);
    rc = STATS_DISPATCH(c, launch_grid, c, u, p, grid, s.npts);
    if (rc) return rc;
    hipfftHandle plan;
    if ((rc = fft_plan(c, s, &plan))) return rc;
    hipfftResult fr = hipfftSetStream(plan, c->stream);
    for (int d = 0; d < 3 && fr == HIPFFT_SUCCESS; ++d)
        fr = hipfftExecD2Z(plan, grid + (size_t)d * s.npts, (hipfftDoubleComplex *)(cplx + (size_t)d * s.M));
    if (fr != HIPFFT_SUCCESS) {
        stats_release(c);
        return fft_fail(c, "hipfftExecD2Z", fr);
    }
    const long long need = (s.M + BLOCK - 1) / BLOCK;
    const int nblk = (int)(need < SP_BLOCKS ? need : SP_BLOCKS);
    hipLaunchKernelGGL(k_shells, dim3(nblk), dim3(BLOCK), (size_t)s.nshell * sizeof(double), c->stream,
                       (const double2 *)cplx, s.X, s.Y, s.Z, s.nshell, part);
    hipError_t le = hipGetLastError();
    if (le == hipSuccess) {
        hipLaunchKernelGGL(k_shells_final, dim3(s.nshell), dim3(BLOCK), 0, c->stream, (const double *)part, nblk,
                           s.nshell, out);
        le = hipGetLastError();
    }
    if (le == hipSuccess)
        le = hipMemcpyAsync(e_host, out, (size_t)s.nshell * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    const hipError_t se = hipStreamSynchronize(c->stream);
    if (le != hipSuccess) return dg_fail(c, DG_EHIP, "spectrum kernels failed: %s", hipGetErrorString(le));
    if (se != hipSuccess) return dg_fail(c, DG_EHIP, "hipStreamSynchronize failed: %s", hipGetErrorString(se));
    return DG_OK;
}
