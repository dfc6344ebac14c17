// dg_kernels.hpp -- gfx950 kernels of the DG right-hand side and SSP-RK3 stage.
//
// Mapping: one lane per cell, 256 cells per workgroup (4 wave64s), cells numbered
// x-fastest so that a wavefront reads 64 consecutive cells of every [var][mode] plane
// (fully coalesced 512-byte FP64 / 256-byte FP32 rows).  All quadrature tables are
// indexed with wave-uniform indices and are fetched with scalar loads; the structural
// zeros of the derivative tables (modes without an exponent along an axis) are skipped
// at compile time.  Reductions (CFL maximum, conservation and driving sums) are done in
// FP64 with a fixed tree order, so repeated runs are bitwise identical.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "dg_basis.hpp"

namespace dg {

enum : int { F_AV = 1, F_PRIM = 2, F_FORCE = 4, F_LIMIT = 8, F_LEARNED = 16, F_MEANFREE = 32, F_HLLC = 64,
             F_VOLUME_MFMA = 256 };

constexpr int BLOCK = 256;

// Workgroups are dispatched round-robin over the 8 XCDs; remap so that consecutive
// logical blocks (neighbouring slabs of cells) share one XCD and its L2.
__device__ __forceinline__ int xcd_remap(int b, int n)
{
    const int per = n >> 3;
    if (b >= (per << 3)) return b;
    return (b & 7) * per + (b >> 3);
}

// Order in which the right-hand-side kernels sweep their cell blocks: in tiles of zt
// z-planes, the planes of a tile interleaved block by block (blocks per plane bpp; identity
// when zt < 2 or blocks straddle planes).  A block's z-neighbour lines are then swept a few
// blocks before or after it, while they are still in the XCD's L2, instead of a whole plane
// of blocks later.  The partial sums stay indexed by the cell block, so every reduction is
// unchanged.
__device__ __forceinline__ int plane_tiled(int b, int bpp, int nplanes, int zt)
{
    if (zt < 2 || bpp <= 0) return b;
    const int per_tile = bpp * zt;
    const int t = b / per_tile;
    const int p0 = t * zt;
    const int tl = min(zt, nplanes - p0);
    const int r = b - t * per_tile;
    return (p0 + r % tl) * bpp + r / tl;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Sum of NV values over the 256 lanes of a block, fixed order; result valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *lds)
{
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) lds[w * NV + i] = v[i];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] = ((lds[i] + lds[NV + i]) + (lds[2 * NV + i] + lds[3 * NV + i]));
}

// totals of per-block partials part[4 i + k], i < np, over the threads of one block of
// BLOCK threads (thread t adds i = t, t + BLOCK, ... in order, then the block sum); the
// totals end in thread 0.  Every reduction of such partials uses this one order.  U: loop
// steps unrolled, so that their loads are in flight together (the order of the additions
// stays the same).
template <int U = 1>
__device__ __forceinline__ void block_partial_sums4(const double *part, int np, double (&s)[4], double *lds)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) s[k] = 0.0;
#pragma unroll U
    for (int i = threadIdx.x; i < np; i += BLOCK)
#pragma unroll
        for (int k = 0; k < 4; ++k) s[k] += part[4 * i + k];
    block_sum<4>(s, lds);
}

__device__ __forceinline__ double block_max(double v, double *lds)
{
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    v = wave_max(v);
    if (lane == 0) lds[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) v = fmax(fmax(lds[0], lds[1]), fmax(lds[2], lds[3]));
    return v;
}

struct Mesh {
    int nx, ny, nz, nc;
};

// Quadrature tables live in the constant address space: wave-uniform indices then
// compile to scalar (SMEM) loads through the scalar cache instead of per-lane loads.
template <typename T>
using ctab = const __attribute__((address_space(4))) T;

template <typename T>
__device__ __forceinline__ ctab<T> *as_tab(const void *p)
{
    return (ctab<T> *)(p);
}

// periodic neighbours of cell c: nb[0..5] = -x, +x, -y, +y, -z, +z
__device__ __forceinline__ void neighbours(const Mesh &g, int c, int (&nb)[6], int (&ijk)[3])
{
    const int i = c % g.nx;
    const int r = c / g.nx;
    const int j = r % g.ny;
    const int l = r / g.ny;
    ijk[0] = i; ijk[1] = j; ijk[2] = l;
    nb[0] = c + ((i == 0) ? g.nx - 1 : -1);
    nb[1] = c + ((i == g.nx - 1) ? 1 - g.nx : 1);
    const int sy = g.nx;
    nb[2] = c + ((j == 0) ? (g.ny - 1) * sy : -sy);
    nb[3] = c + ((j == g.ny - 1) ? (1 - g.ny) * sy : sy);
    const int sz = g.nx * g.ny;
    nb[4] = c + ((l == 0) ? (g.nz - 1) * sz : -sz);
    nb[5] = c + ((l == g.nz - 1) ? (1 - g.nz) * sz : sz);
}


// Coalesced access to element (mode plane, cell) through buffer resources: one
// descriptor (4 SGPRs) per variable block, the mode plane as a uniform SGPR offset and
// the lane part as one 32-bit byte offset shared by every access of the cell.  A block
// of nb planes must stay below 4 GiB (checked at set-up).
using rsrc_t = __amdgpu_buffer_rsrc_t;

__device__ __forceinline__ rsrc_t mkrs(const void *base)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)0xFFFFFFFF, 0x00020000);
}

// Cache policy of an access: CP_NT marks data touched once (the non-temporal hint of the
// gfx950 buffer instructions), so that it does not displace the traces that neighbouring
// cells read again from L2.
enum : int { CP_DEFAULT = 0, CP_NT = 2 };

template <typename T, int CP = CP_DEFAULT>
__device__ __forceinline__ T bld(rsrc_t r, unsigned voff, unsigned soff)
{
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, CP));
    else
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, CP));
}

template <typename T, int CP = CP_DEFAULT>
__device__ __forceinline__ void bst(rsrc_t r, unsigned voff, unsigned soff, T v)
{
    if constexpr (sizeof(T) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r,
                                              voff, soff, CP);
    else
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, CP);
}

// a [nvar][nb][nc] array viewed through one descriptor per variable
template <typename T, int NV>
struct Field {
    rsrc_t r[NV];
    unsigned pstride;   // bytes between mode planes
    __device__ __forceinline__ Field(const void *base, int nb, int nc)
    {
        pstride = (unsigned)nc * (unsigned)sizeof(T);
#pragma unroll
        for (int v = 0; v < NV; ++v) r[v] = mkrs((const char *)base + (size_t)v * nb * pstride);
    }
    // trace sources: density block of u, then the three blocks of the projected velocity
    __device__ __forceinline__ Field(const void *u, const void *vh, int nb, int nc)
    {
        pstride = (unsigned)nc * (unsigned)sizeof(T);
        r[0] = mkrs(u);
#pragma unroll
        for (int v = 1; v < NV; ++v) r[v] = mkrs((const char *)vh + (size_t)(v - 1) * nb * pstride);
    }
    __device__ __forceinline__ Field(const Field &) = default;
    __device__ __forceinline__ T get(int v, int l, unsigned boff) const { return bld<T>(r[v], boff, l * pstride); }
    __device__ __forceinline__ void put(int v, int l, unsigned boff, T x) const { bst<T>(r[v], boff, l * pstride, x); }
    // the same with the non-temporal hint (data read or written once by this kernel)
    __device__ __forceinline__ T get_nt(int v, int l, unsigned boff) const
    {
        return bld<T, CP_NT>(r[v], boff, l * pstride);
    }
    __device__ __forceinline__ void put_nt(int v, int l, unsigned boff, T x) const
    {
        bst<T, CP_NT>(r[v], boff, l * pstride, x);
    }
};

// fast reciprocal: hardware estimate refined by two Newton steps (about 1 ulp)
__device__ __forceinline__ double rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ float rcp(float x)
{
    float r = __builtin_amdgcn_rcpf(x);
    float e = fmaf(-x, r, 1.0f);
    return fmaf(r, e, r);
}

// ------------------------------------------------------------------ arguments
struct RhsArgs {
    const void *u;          // [4][NB][nc]
    const void *vh;         // [3][NB][nc] projected velocity of u
    void *out;              // [4][NB][nc] right-hand side
    const void *tab;        // quadrature tables (TabLayout)
    const void *ftab;       // driving field in pencil form (PencilLayout), element type T
    const double *modes;    // driving-mode table [nmodes][9] (direct evaluation of other tables)
    int nmodes;
    const void *nu;         // [nc] learned viscosity
    const int *fb;          // [nc] fallback flags
    double *part;           // [nblocks][4] driving partial sums (mode-0 source, mass)
    int *fail_reset;        // positivity failure flag to clear before the stages, or NULL
    // last stage of a step: decide its positivity failure here, before the stage kernel
    // writes the caller's state (pred_fail != NULL: the flag to raise; pred_un, pred_ca,
    // pred_cb, pred_cc: the stage's u^n operand and coefficients; rho_floor: the floor)
    int *pred_fail;
    const void *pred_un;
    double pred_ca, pred_cb, pred_cc, rho_floor;
    Mesh g;
    int flags;
    double h, cs, alpha, beta, dt;
    const double *dt_dev;   // the time step in device memory (a stage launched ahead), or NULL: dt
    int bpp, zt;            // block sweep order (plane_tiled): blocks per z-plane, planes per tile
    const float *mfma;      // A-operand tables of the matrix-core volume integral (MfmaTab), or NULL
    // two-lane kernel: a copy of the density weights directly in front of vh (so that density
    // and projected velocity form one [4][nb][nc] array), or NULL; and the byte distance of two
    // variable blocks (2 nb nc 8) when every lane can reach its own variables through a 32-bit
    // offset, else 0
    const void *vh_rho;
    unsigned pair_vstride;
};

// time-step bound inputs shared by the projection and stage kernels
struct ProjArgs {
    double cs, h, alpha, beta;
    int visc;           // also reduce the largest bulk viscosity of the viscous pressure
    const void *nu;     // learned per-cell bulk viscosity (element type T), or NULL
    const int *fb;      // fallback flags of the learned sensor (1 = plain sensor), or NULL;
                        // with fb set and nu NULL a learned cell adds nothing here (its
                        // viscosity is reduced where the network writes it)
};

struct StageArgs {
    const void *ui;         // stage input u^(i)
    const void *un;         // u^n, or the side combination of an earlier stage (may alias ui)
    const void *L;          // right-hand side of u^(i) (NULL: plain copy/limit of ui)
    void *out;              // u^(i+1) (may alias un)
    void *vh_out;           // projection of u^(i+1) for the next stage, or NULL
    void *rho_out;          // with vh_out: a copy of the density weights of u^(i+1), or NULL
    const int *skip_flag;   // the last stage: the failure flag (write nothing when raised), or NULL
    const void *tab;
    const double *abar;     // removed mean acceleration (3), or NULL
    const double *abar_part; // or, when not NULL: the right-hand side's per-block partials
    int abar_np;            //   (abar_np blocks of 4), reduced to it in every block
    int *fail;              // positivity failure flag
    long long *nlim;        // count of failing cells (may be NULL)
    double *part;           // with vh_out: per-block time-step maxima of u^(i+1), or NULL
    const void *w_src;      // side combination w = wa w_src + wb ui + wc dt R (w_out may alias w_src)
    void *w_out;            //   written when not NULL
    ProjArgs pa;
    Mesh g;
    int flags;
    double ca, cb, cc, dt, rho_floor, rho_floor_rel;
    double wa, wb, wc;
    const double *dt_dev;   // the time step in device memory (a stage launched ahead), or NULL: dt
    // k_limit_project: the mean-acceleration partials of the result for the next stage
    // (drive_part [nblocks][4], or NULL) and the driving field they take
    double *drive_part;
    const void *ftab;
    const double *modes;
    int nmodes;
    // a split last stage: raise *fail where the combination's mean density is at or below
    // rho_floor (before the stage kernel writes the caller's state), else 0
    int fail_on_mean;
};

// ------------------------------------------------------------------ helpers
// One coefficient of a Runge-Kutta stage, out = ca un + cb ui + cdt R, with the roundings
// fixed by explicit fused multiply-adds: the right-hand-side kernel of a last stage
// recomputes the density mean this way and must reach the stage kernel's value bit for bit.
template <typename T>
__device__ __forceinline__ T stage_value(T ca, T cb, T cdt, T un, T ui, T rhs, bool use_un)
{
    const T x = fma(cdt, rhs, cb * ui);
    return use_un ? fma(ca, un, x) : x;
}

// Positivity failure of the last stage decided from its density mean (Sec. 3.1: a cell whose
// mean is at or below the floor cannot be limited), before the stage writes the state.
template <typename T>
__device__ __forceinline__ void predict_failure(const RhsArgs &a, double dt, int c, T ui0, T rhs0)
{
    const T ca = (T)a.pred_ca, cb = (T)a.pred_cb, cdt = (T)(a.pred_cc * dt);
    const bool use_un = a.pred_ca != 0.0;
    const T un0 = use_un ? ((const T *)a.pred_un)[c] : T(0);
    const double mean = (double)stage_value<T>(ca, cb, cdt, un0, ui0, rhs0, use_un);
    if (!(mean > a.rho_floor)) atomicOr(a.pred_fail, 1);
}

template <typename T, int K, int NV>
__device__ __forceinline__ void load_field(const Field<T, NV> &f, unsigned bo, T (&W)[NV][Shape<K>::NB])
{
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int l = 0; l < Shape<K>::NB; ++l) W[v][l] = f.get(v, l, bo);
}

template <typename T, int K, int NV>
__device__ __forceinline__ void store_field(const Field<T, NV> &f, unsigned bo, const T (&W)[NV][Shape<K>::NB])
{
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int l = 0; l < Shape<K>::NB; ++l) f.put(v, l, bo, W[v][l]);
}

// projected velocity of one cell from its weights (Sec. 3.2): vh_{d,l} = 1/8 sum_q w_q phi_l v_d
template <typename T, int K>
__device__ __forceinline__ void project_cell(const T (&W)[4][Shape<K>::NB], ctab<T> *tab,
                                             T (&V)[3][Shape<K>::NB], double *smax, double cs)
{
    using S = Shape<K>;
    using TL = TabLayout<K>;
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int l = 0; l < S::NB; ++l) V[d][l] = T(0);
    double sm = 0.0;
    for (int q = 0; q < S::NQ; ++q) {
        ctab<T> *ph = tab + TL::VPHI + q * S::NB;
        T rho = T(0), m0 = T(0), m1 = T(0), m2 = T(0);
#pragma unroll
        for (int l = 0; l < S::NB; ++l) {
            const T p = ph[l];
            rho += W[0][l] * p;
            m0 += W[1][l] * p;
            m1 += W[2][l] * p;
            m2 += W[3][l] * p;
        }
        const T ir = rcp(rho);
        const T v0 = m0 * ir, v1 = m1 * ir, v2 = m2 * ir;
        if (smax) {
            const double s = (double)fabs(v0) + (double)fabs(v1) + (double)fabs(v2) + 3.0 * cs;
            sm = fmax(sm, s);
        }
        const T wq = T(0.125) * tab[TL::VW + q];
        const T a0 = wq * v0, a1 = wq * v1, a2 = wq * v2;
#pragma unroll
        for (int l = 0; l < S::NB; ++l) {
            const T p = ph[l];
            V[0][l] += a0 * p;
            V[1][l] += a1 * p;
            V[2][l] += a2 * p;
        }
    }
    if (smax) *smax = sm;
}

// Component d of the projected velocity of one cell (Sec. 3.2), same arithmetic as
// project_cell for that component; working one component at a time keeps only NB
// accumulators live.
template <typename T, int K>
__device__ __forceinline__ void project_component(const T (&W)[4][Shape<K>::NB], ctab<T> *tab, int d,
                                                  T (&V)[Shape<K>::NB])
{
    using S = Shape<K>;
    using TL = TabLayout<K>;
#pragma unroll
    for (int l = 0; l < S::NB; ++l) V[l] = T(0);
#pragma unroll 1
    for (int q = 0; q < S::NQ; ++q) {
        ctab<T> *ph = tab + TL::VPHI + q * S::NB;
        T rho = T(0), m = T(0);
#pragma unroll
        for (int l = 0; l < S::NB; ++l) {
            const T p = ph[l];
            rho += W[0][l] * p;
            m += W[1 + d][l] * p;
        }
        const T a = T(0.125) * tab[TL::VW + q] * (m * rcp(rho));
#pragma unroll
        for (int l = 0; l < S::NB; ++l) V[l] += a * ph[l];
    }
}

// project_component for d = 0 that also takes the largest signal speed sum_d |v_d| + cs
// over the points from the same point values (the time-step bound)
template <typename T, int K>
__device__ __forceinline__ void project_first_with_speed(const T (&W)[4][Shape<K>::NB], ctab<T> *tab,
                                                         T (&V)[Shape<K>::NB], double cs, double &sm)
{
    using S = Shape<K>;
    using TL = TabLayout<K>;
#pragma unroll
    for (int l = 0; l < S::NB; ++l) V[l] = T(0);
#pragma unroll 1
    for (int q = 0; q < S::NQ; ++q) {
        ctab<T> *ph = tab + TL::VPHI + q * S::NB;
        T rho = T(0), m0 = T(0), m1 = T(0), m2 = T(0);
#pragma unroll
        for (int l = 0; l < S::NB; ++l) {
            const T p = ph[l];
            rho += W[0][l] * p;
            m0 += W[1][l] * p;
            m1 += W[2][l] * p;
            m2 += W[3][l] * p;
        }
        const T ir = rcp(rho);
        const double sp = (double)fabs(m0 * ir) + (double)fabs(m1 * ir) + (double)fabs(m2 * ir) + 3.0 * cs;
        sm = fmax(sm, sp);
        const T a = T(0.125) * tab[TL::VW + q] * (m0 * ir);
#pragma unroll
        for (int l = 0; l < S::NB; ++l) V[l] += a * ph[l];
    }
}

// FP64 kernels project one velocity component at a time (fewer live registers, four
// waves per SIMD); FP32 ones have registers to spare and project all three at once
template <typename T>
constexpr bool split_projection() { return sizeof(T) == 8; }

// isothermal Rusanov flux across a face with normal +e_D between the low (L) and high
// (R) states; u = (rho, m), v = velocity (Sec. 2.2 numerical flux)
template <int D, typename T>
__device__ __forceinline__ void rusanov(T cs, T cs2, const T (&uL)[4], const T (&vL)[3], const T (&uR)[4],
                                        const T (&vR)[3], T (&F)[4])
{
    // every fused multiply-add written out and no other contraction left to the compiler:
    // the flux of a face is then the same bits whichever of its two cells computes it
#pragma clang fp contract(off)
    const T lam = fmax(fabs(vL[D]), fabs(vR[D])) + cs;
    const T hl = T(0.5) * lam;
    F[0] = fma(-hl, uR[0] - uL[0], T(0.5) * (uL[1 + D] + uR[1 + D]));
#pragma unroll
    for (int j = 0; j < 3; ++j)
        F[1 + j] = fma(-hl, uR[1 + j] - uL[1 + j], T(0.5) * fma(uL[1 + D], vL[j], uR[1 + D] * vR[j]));
    F[1 + D] = fma(T(0.5) * cs2, uL[0] + uR[0], F[1 + D]);
}

// isothermal HLLC-type flux across a face with normal +e_D (the counterpart of the HLLC
// solver of Sec. 2.2 for isothermal gas): wave speeds S_L = min(v_L, v_R) - cs and
// S_R = max(v_L, v_R) + cs of the normal velocities; density and normal momentum take the
// HLL flux, each tangential momentum is the mass flux times the upwind tangential velocity
template <int D, typename T>
__device__ __forceinline__ void hllc(T cs, T cs2, const T (&uL)[4], const T (&vL)[3], const T (&uR)[4],
                                     const T (&vR)[3], T (&F)[4])
{
    const T SL = fmin(vL[D], vR[D]) - cs;
    const T SR = fmax(vL[D], vR[D]) + cs;
    const T FL0 = uL[1 + D], FR0 = uR[1 + D];
    const T FLn = uL[1 + D] * vL[D] + cs2 * uL[0];
    const T FRn = uR[1 + D] * vR[D] + cs2 * uR[0];
    const T iw = rcp(SR - SL);
    const T sLR = SL * SR;
    T F0 = (SR * FL0 - SL * FR0 + sLR * (uR[0] - uL[0])) * iw;
    T Fn = (SR * FLn - SL * FRn + sLR * (uR[1 + D] - uL[1 + D])) * iw;
    F0 = SL >= T(0) ? FL0 : (SR <= T(0) ? FR0 : F0);
    Fn = SL >= T(0) ? FLn : (SR <= T(0) ? FRn : Fn);
    F[0] = F0;
    F[1 + D] = Fn;
#pragma unroll
    for (int t = 0; t < 3; ++t)
        if (t != D) F[1 + t] = F0 * (F0 >= T(0) ? vL[t] : vR[t]);
}

// von Neumann-Richtmyer viscous pressure at one point (Sec. 3.1)
template <typename T>
__device__ __forceinline__ T vnr_pi(T rho, T divv, T hp, T alpha, T beta, T cs, T inv_dt)
{
    const T s = -divv;
    T pi = alpha * rho * hp * hp * s * s + beta * rho * cs * hp * s;
    const T pmax = T(0.5) * rho * hp * hp * s * inv_dt;
    pi = fmin(pi, pmax);
    return s > T(0) ? pi : T(0);
}

// ---------------------------------------------------------------- face pass
// Surface integral of one face (normal axis D, side s: 0 = low, 1 = high) from the point
// fluxes in an LDS column (col: the column of the cell that stored them, [r][v] with stride
// BLOCK): the flux moments against the 2D basis of the face, M_vj = sum_r w_r F_v(r) P2_j(r),
// then per mode phi_l = Lt_{e_D}(+-1) P2_{d2(l)} on the face, so L_vl += Lt_{e_D}(+-1) M_v,d2(l)
// (the lift of every point into all NB modes takes NB multiply-adds per point and variable,
// the moments NB2).
template <typename T, int K, int D>
__device__ __forceinline__ void lift(const T *col, int s, ctab<T> *tab, T (&L)[4][Shape<K>::NB])
{
    using S = Shape<K>;
    using TL = TabLayout<K>;
    constexpr Modes<K> M = make_modes<K>();
    T Mv[4][S::NB2];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int j = 0; j < S::NB2; ++j) Mv[v][j] = T(0);
#pragma unroll 1
    for (int r = 0; r < S::NF; ++r) {
        const T wr = s ? -tab[TL::FW + r] : tab[TL::FW + r];   // outward normal
        ctab<T> *f2 = tab + TL::F2 + r * S::NB2;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const T g = wr * col[(r * 4 + v) * BLOCK];
#pragma unroll
            for (int j = 0; j < S::NB2; ++j) Mv[v][j] += g * f2[j];
        }
    }
    ctab<T> *lend = tab + TL::LEND;
#pragma unroll
    for (int l = 0; l < S::NB; ++l) {
        const T ls = lend[2 * M.e[l][D] + s];
#pragma unroll
        for (int v = 0; v < 4; ++v) L[v][l] += ls * Mv[v][M.d2[D][l]];
    }
}

// One face of the cell (normal axis D, side s): traces of the cell and its neighbour,
// the numerical flux at every face point stored in the cell's LDS column col (where the
// neighbour across a shared face reads it too), then lifted from there into L.
template <typename T, int K, int D>
__device__ __forceinline__ void face(const Field<T, 4> &src, unsigned bo, unsigned bn, int s,
                                     ctab<T> *tab, bool prim, bool use_hllc, T cs, T cs2,
                                     T (&L)[4][Shape<K>::NB], T *col)
{
    using S = Shape<K>;
    using TL = TabLayout<K>;
    constexpr Modes<K> M = make_modes<K>();
    T Co[4][S::NB2], Cn[4][S::NB2];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int j = 0; j < S::NB2; ++j) { Co[v][j] = T(0); Cn[v][j] = T(0); }
    // collapse the 3D expansions onto the face: Lt_e(+-1) along D
    ctab<T> *lend = tab + TL::LEND;
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int l = 0; l < S::NB; ++l) {
            const int e = M.e[l][D];
            const T wo = src.get(v, l, bo);
            const T wn = src.get(v, l, bn);
            Co[v][M.d2[D][l]] += wo * lend[2 * e + s];
            Cn[v][M.d2[D][l]] += wn * lend[2 * e + 1 - s];
            // keep at most one variable's loads in flight (register pressure)
            if (l == S::NB - 1) __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll 1
    for (int r = 0; r < S::NF; ++r) {
        ctab<T> *f2 = tab + TL::F2 + r * S::NB2;
        T uo[4], un[4], vo[3], vn[3];
        T ao[4] = {T(0), T(0), T(0), T(0)}, an[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int j = 0; j < S::NB2; ++j) {
            const T f = f2[j];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                ao[v] += Co[v][j] * f;
                an[v] += Cn[v][j] * f;
            }
        }
        uo[0] = ao[0];
        un[0] = an[0];
        if (prim) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                vo[d] = ao[1 + d]; uo[1 + d] = ao[0] * ao[1 + d];
                vn[d] = an[1 + d]; un[1 + d] = an[0] * an[1 + d];
            }
        } else {
            const T io = rcp(ao[0]), in = rcp(an[0]);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                uo[1 + d] = ao[1 + d]; vo[d] = ao[1 + d] * io;
                un[1 + d] = an[1 + d]; vn[d] = an[1 + d] * in;
            }
        }
        T F[4];
        if (use_hllc) {
            if (s) hllc<D>(cs, cs2, uo, vo, un, vn, F);
            else   hllc<D>(cs, cs2, un, vn, uo, vo, F);
        } else {
            if (s) rusanov<D>(cs, cs2, uo, vo, un, vn, F);
            else   rusanov<D>(cs, cs2, un, vn, uo, vo, F);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) col[(r * 4 + v) * BLOCK] = F[v];
    }
    lift<T, K, D>(col, s, tab, L);
}

// ------------------------------------------------------------ driving field
// The driving acceleration a(x) = sum_m Re[a_m exp(2 pi i n_m . x)] (Sec. 4.2) at the volume
// points of a cell.  For tables whose wavevectors have integer x components n_x in [-2, 2]
// (the driving shell 1 <= |n| <= 2), a term with n_x < 0 equals the real part of its
// conjugate (-n, conj a_m), so with X = exp(2 pi i x)
//     a_d(x, y, z) = G0_d(y, z) + Re[G1_d(y, z) X] + Re[G2_d(y, z) X^2],
// where G_nd(y, z) sums a_m,d exp(2 pi i (n_y y + n_z z)) over the modes with n_x = n.  The G
// depend only on the cell's y-z pencil (j, l) and the point's (t_y, t_z): the pencil table
// holds them (about 1 KB per pencil in FP64 at degree 2, built once per table update), and
// X = P E_t with P = exp(2 pi i (i + 1/2) h) per cell, from the table's last block (one
// (cos, sin) pair per x index i, after the pencils), and E_t = exp(pi i xi_t h) from the
// table header.  The 64 cells of a wave usually share one pencil: their G are then read with
// scalar loads.  Other tables are evaluated mode by mode at every point (k_rhs's direct form).
//
// For the mean acceleration the tables also hold moments.  The cell's source summed over its
// points, sum_q w_q rho(q) a(q) = sum_l W_l M_l with M_l = sum_q w_q phi_l(q) a(q), factors
// with phi_l = Lt_a(xi_x) phi2_j(xi_y, xi_z) (a the x degree of mode l, j its 2D mode) into
//     M_l,d = C0_jd Sx0_a + Re[C1_jd P Sx1_a] + Re[C2_jd P^2 Sx2_a],
// with the pencil's moments Cn_jd = sum_(t_y, t_z) w phi2_j Gn_d and the x factors
// Sxn_a = sum_t w_t Lt_a(xi_t) E_t^n: about 10 multiply-adds per mode and component instead of
// the field at every point.
template <int K>
struct PencilLayout {
    static constexpr int N1 = K + 1;
    static constexpr int NB2 = (K + 1) * (K + 2) / 2;
    static constexpr int HDR = 16;                  // (cos, sin)(pi xi_t h) for t < N1, padded
    static constexpr int ENT = 16;                  // per (t_y, t_z): 3 x (G0, Re G1, Im G1, Re G2, Im G2), padded
    static constexpr int STRIDE = N1 * N1 * ENT;    // reals per pencil
    static constexpr int SXN = 24;                  // per x degree a: Sx0, Sx1 (re, im), Sx2 (re, im), padded
    static constexpr int MST = NB2 * 3 * 5;         // per pencil: per 2D mode j and component d,
                                                    //   C0, C1 (re, im), C2 (re, im)
    // offset of the x phases P_i = (cos, sin)(2 pi (i + 1/2) h), after the ny nz pencils
    __host__ __device__ static size_t phases(int ny, int nz) { return HDR + (size_t)ny * nz * STRIDE; }
    // the x factors, after the phases; the pencils' moments after them
    __host__ __device__ static size_t xfactors(int nx, int ny, int nz) { return phases(ny, nz) + 2 * (size_t)nx; }
    __host__ __device__ static size_t moments(int nx, int ny, int nz) { return xfactors(nx, ny, nz) + SXN; }
    __host__ __device__ static size_t size(int nx, int ny, int nz) { return moments(nx, ny, nz) + (size_t)ny * nz * MST; }
};

// a at volume point q (q = t_x + N1 (t_y + N1 t_z)) from the pencil table: g = this pencil's
// block, (pr, pi) = the cell's phase P
// (roundings fixed by explicit fused multiply-adds: every kernel that evaluates the field gets
// the same bits)
template <typename T, int K>
__device__ __forceinline__ void pencil_accel(ctab<T> *ft, ctab<T> *g, int q, T pr, T pim, T (&acc)[3])
{
#pragma clang fp contract(off)
    using PL = PencilLayout<K>;
    const int tx = q % PL::N1, tt = q / PL::N1;
    const T er = ft[2 * tx], ei = ft[2 * tx + 1];
    const T xr = fma(pr, er, -(pim * ei));
    const T xi = fma(pr, ei, pim * er);
    const T x2r = fma(xr, xr, -(xi * xi));
    const T x2i = (T(2) * xr) * xi;
    ctab<T> *e = g + tt * PL::ENT;
#pragma unroll
    for (int d = 0; d < 3; ++d)
        acc[d] = fma(-e[5 * d + 4], x2i, fma(e[5 * d + 3], x2r, fma(-e[5 * d + 2], xi, fma(e[5 * d + 1], xr, e[5 * d]))));
}

// a at the point with reference coordinates xi of cell (i, j, l), mode by mode (any table)
template <typename T>
__device__ __forceinline__ void direct_accel(const double *modes, int nmodes, const int (&ijk)[3], T xq, T yq, T zq,
                                             double h, T (&acc)[3])
{
#pragma clang fp contract(off)
    const double x = (ijk[0] + 0.5 + 0.5 * (double)xq) * h;
    const double y = (ijk[1] + 0.5 + 0.5 * (double)yq) * h;
    const double z = (ijk[2] + 0.5 + 0.5 * (double)zq) * h;
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int m = 0; m < nmodes; ++m) {
        const double *e = modes + 9 * m;
        double sp, cp;
        sincospi(2.0 * (e[0] * x + e[1] * y + e[2] * z), &sp, &cp);
        ax += e[3] * cp - e[4] * sp;
        ay += e[5] * cp - e[6] * sp;
        az += e[7] * cp - e[8] * sp;
    }
    acc[0] = (T)ax;
    acc[1] = (T)ay;
    acc[2] = (T)az;
}

// the cell's x phase P = exp(2 pi i (i + 1/2) h) from the table's phase block px
template <typename T>
__device__ __forceinline__ void cell_phase(ctab<T> *px, int i, T &pr, T &pim)
{
    pr = px[2 * i];
    pim = px[2 * i + 1];
}

// The driving source of one volume point, s = (rho w_q) a, and the running sums of the
// cell's source for the removed mean acceleration, every rounding fixed (no contraction):
// the sums come out the same in every kernel that forms them.
template <typename T>
__device__ __forceinline__ void drive_point(T rho, T wq, const T (&ac)[3], T (&s)[3], T &fs0, T &fs1, T &fs2)
{
#pragma clang fp contract(off)
    const T rw = rho * wq;
    s[0] = rw * ac[0];
    s[1] = rw * ac[1];
    s[2] = rw * ac[2];
    fs0 = fs0 + s[0];
    fs1 = fs1 + s[1];
    fs2 = fs2 + s[2];
}

// The cell's driving source summed over its volume points, from its density weights W0 and
// the moments of its pencil (mp: MST values; sx: the x factors; (pr, pim): the cell's phase P),
// in the modal form of the pencil layout, with fixed roundings and order (2D mode, component,
// then the modes with that 2D part): every kernel that forms the mean-acceleration partials
// gets the same bits.  fs[d] = sum_l W0_l M_l,d.  Each moment is loaded once and used by the
// modes that share its 2D part.  LANE: the moments differ between lanes (vector loads), one 2D
// mode's loads in flight at a time.
template <typename T, int K, bool LANE>
__device__ __forceinline__ void drive_moments(const T (&W0)[Shape<K>::NB], ctab<T> *mp, ctab<T> *sx, T pr, T pim,
                                              T (&fs)[3])
{
#pragma clang fp contract(off)
    constexpr Modes<K> M = make_modes<K>();
    const T p2r = fma(pr, pr, -(pim * pim)), p2i = (T(2) * pr) * pim;
    T s0[K + 1], q1r[K + 1], q1i[K + 1], q2r[K + 1], q2i[K + 1];
#pragma unroll
    for (int a = 0; a <= K; ++a) {
        ctab<T> *x = sx + 5 * a;
        s0[a] = x[0];
        q1r[a] = fma(pr, x[1], -(pim * x[2]));
        q1i[a] = fma(pr, x[2], pim * x[1]);
        q2r[a] = fma(p2r, x[3], -(p2i * x[4]));
        q2i[a] = fma(p2r, x[4], p2i * x[3]);
    }
    fs[0] = fs[1] = fs[2] = T(0);
#pragma unroll
    for (int j = 0; j < Shape<K>::NB2; ++j) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            ctab<T> *cm = mp + (j * 3 + d) * 5;
            const T c0 = cm[0], c1r = cm[1], c1i = cm[2], c2r = cm[3], c2i = cm[4];
#pragma unroll
            for (int l = 0; l < Shape<K>::NB; ++l) {
                if (M.d2[0][l] != j) continue;
                const int a = M.e[l][0];
                const T m = fma(-c2i, q2i[a], fma(c2r, q2r[a], fma(-c1i, q1i[a], fma(c1r, q1r[a], c0 * s0[a]))));
                fs[d] = fma(W0[l], m, fs[d]);
            }
        }
        if constexpr (LANE) __builtin_amdgcn_sched_barrier(0);
    }
}

// drive_moments for a lane's cell (index c), the moments read with scalar loads when the
// wave's cells share one pencil.  ft: the pencil-form table.
template <typename T, int K>
__device__ __forceinline__ void drive_moment_sums(const T (&W0)[Shape<K>::NB], ctab<T> *ft, const Mesh &g, int c,
                                                  bool active, T (&fs)[3])
{
    using PL = PencilLayout<K>;
    const int pencil = c / g.nx;
    T pr, pim;
    cell_phase<T>(ft + PL::phases(g.ny, g.nz), c % g.nx, pr, pim);
    ctab<T> *sx = ft + PL::xfactors(g.nx, g.ny, g.nz);
    ctab<T> *m0 = ft + PL::moments(g.nx, g.ny, g.nz);
    const int p0 = __shfl(pencil, 0, 64);
    if (__all(!active || pencil == p0))
        drive_moments<T, K, false>(W0, m0 + (size_t)__builtin_amdgcn_readfirstlane(p0) * PL::MST, sx, pr, pim, fs);
    else
        drive_moments<T, K, true>(W0, m0 + (size_t)pencil * PL::MST, sx, pr, pim, fs);
}

// the right-hand side's partials of a cell: the three sums times 1/8 and the mean density (0
// for an inactive lane)
template <typename T>
__device__ __forceinline__ void drive_partial(const T (&fs)[3], T mass, bool active, double (&acc)[4])
{
    acc[0] = active ? 0.125 * (double)fs[0] : 0.0;
    acc[1] = active ? 0.125 * (double)fs[1] : 0.0;
    acc[2] = active ? 0.125 * (double)fs[2] : 0.0;
    acc[3] = active ? (double)mass : 0.0;
}

// Driving field forms of the right-hand-side kernels' volume loop
enum : int { FM_LANE = 0, FM_UNIFORM = 1, FM_DIRECT = 2 };

// ------------------------------------------- volume integral on the matrix cores (FP32)
// A variant of the volume integral of the FP32 degree-2 right-hand side with both dense
// contractions on v_mfma_f32_16x16x4f32, 16 cells of the wave at a time (a tile), cells
// along the N dimension of every product:
//   * evaluation at the points, U[pt][cell] = sum_l phi_l(pt) W[l][cell] for each variable:
//     A = phi (16 points x 4 modes per step, 27 points padded to 32, 10 modes to 12),
//     B = the tile's weights (4 modes x 16 cells);
//   * the divergence of the projected velocity at the points from its 4 modal coefficients;
//   * the flux and driving contraction L[l][cell] += sum_(d,pt) w ∂_d phi_l(pt) F_d(pt, cell)
//     + sum_pt (h/2) w phi_l(pt) rho a(pt): A = the weighted basis tables (16 modes x 4 points
//     per step, the modes padded from 10 to 16), B = the point fluxes (4 points x 16 cells).
// The point fluxes, the viscous pressure and the driving source are formed on the VALU in
// the accumulator layout of the evaluation: lane (g, j) = (lane / 16, lane % 16) holds points
// 16P + 4g + r (r < 4) of cell j, which is exactly the operand layout the contraction takes
// when a step's K index g stands for point 16P + 4g + r.  Padded points read point 0's
// values (finite) and carry zero weights.  The accumulators of tile t end in lane (g, j) as
// modes 4g + r of cell j; lane permutes hand them to the lane that owns the cell in the face
// pass (lane 16t + j).
//
// Measured against the one-lane VALU volume loop: see the design notes; at degree 2 the
// contraction keeps about 21 % of the matrix core's work useful (10 of 16 mode rows, 27 of
// 32 points, and per axis only 4 of 10 modes with a nonzero derivative).
typedef float f4_t __attribute__((ext_vector_type(4)));
#ifndef MFMA_WAVES
#define MFMA_WAVES 2
#endif

// A-operand tables of the matrix-core volume integral, per lane (64 lanes), FP32:
//   EV[P][s][lane]   phi_(4s+g)(pt 16P + j)                    (6 x 64)
//   DV[P][lane]      phi_g(pt 16P + j), g < 4 (divergence modes) (2 x 64)
//   CT[d][P][r][lane] w ∂_d phi_j(pt 16P + 4g + r)              (24 x 64)
//   FT[P][r][lane]   (h/2) w phi_j(pt 16P + 4g + r)             (8 x 64; h/2 applied in the kernel)
// with g = lane / 16, j = lane % 16, modes >= 10 and points >= 27 zero in CT/FT, points >= 27
// replaced by point 0 in EV/DV.
//   WQ[P][r][lane]   w(pt 16P + 4g + r), zero for points >= 27     (8 x 64)
struct MfmaTab {
    static constexpr int EV = 0, DV = EV + 6 * 64, CT = DV + 2 * 64, FT = CT + 24 * 64, WQ = FT + 8 * 64,
                         SIZE = WQ + 8 * 64;
};

__device__ __forceinline__ f4_t mfma4(float a, float b, f4_t c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}


// The volume integral of one block's FP32 degree-2 right-hand side on the matrix cores: each
// wave takes its 64 cells as four tiles of 16.  lds: the block's face-flux buffer, free until
// the face pass, holding the A tables (MfmaTab) and each wave's pencil of the driving table.
// L, fs0..fs2: the lane's own cell's accumulators and driving sums, as the VALU loop leaves them.
__device__ __forceinline__ void volume_mfma(const RhsArgs &a, ctab<float> *tab, float *lds, int blk, bool active,
                                            int pencil, float (&L)[4][10], float &fs0, float &fs1, float &fs2)
{
    using S = Shape<2>;
    using TL = TabLayout<2>;
    using PL = PencilLayout<2>;
    constexpr Modes<2> M = make_modes<2>();
    constexpr DivMap<2> DM = make_divmap<2>();
    constexpr int NB = S::NB, NQ = S::NQ;
    const int nc = a.g.nc;
    const bool av = a.flags & F_AV, force = a.flags & F_FORCE, learned_on = a.flags & F_LEARNED;
    const float cs = (float)a.cs, cs2 = (float)(a.cs * a.cs), hp = (float)(a.h / 3.0);
    const double dtv = a.dt_dev ? *a.dt_dev : a.dt;
    const float inv_dt = dtv > 0.0 ? (float)(1.0 / dtv) : 1e30f;
    const float alpha = (float)a.alpha, beta = (float)a.beta, two_h = (float)(2.0 / a.h), half_h = (float)(0.5 * a.h);
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
    // stage the A tables and, when the wave's cells share a pencil, its driving-table block
    for (int i = threadIdx.x; i < MfmaTab::SIZE; i += BLOCK) lds[i] = a.mfma[i];
    float *lgw = lds + MfmaTab::SIZE + wv * PL::STRIDE;
    ctab<float> *ft = as_tab<float>(a.ftab);
    const int p0 = __shfl(pencil, 0, 64);
    const bool uni = force && __all(!active || pencil == p0);
    if (uni)
        for (int i = lane; i < PL::STRIDE; i += 64) lgw[i] = ft[PL::HDR + (size_t)p0 * PL::STRIDE + i];
    __syncthreads();
    const Field<float, 4> U(a.u, NB, nc);
    const Field<float, 3> VH(a.vh, NB, nc);
    const int wc0 = blk * BLOCK + wv * 64;
#pragma unroll 1
    for (int t = 0; t < 4; ++t) {
        const int ct0 = wc0 + 16 * t + j;
        const bool tact = ct0 < nc;
        const int ct = tact ? ct0 : 0;
        const unsigned bt = (unsigned)ct * 4u;
        // the tile cells' weights as the B operands of the evaluation (modes 4 st + g)
        float bw[4][3];
#pragma unroll
        for (int st = 0; st < 3; ++st) {
            const int mode = 4 * st + g;
            const int mm = mode < NB ? mode : NB - 1;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float b = U.get(v, mm, bt);
                bw[v][st] = mode < NB ? b : 0.f;
            }
        }
        // divergence of the projected velocity: this lane supplies coefficient g of cell j
        float dvg = 0.f, nu = 0.f;
        bool learned = false;
        if (av) {
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int l = 0; l < NB; ++l)
                    if (M.e[l][d] >= 1) {
                        const float v = VH.get(d, l, bt);
#pragma unroll
                        for (int q = 0; q < DivMap<2>::MAXT; ++q)
                            if (DM.m[d][l][q] >= 0)
                                dvg += DM.m[d][l][q] == g ? v * float(__builtin_sqrt(double(DM.f[d][l][q]))) : 0.f;
                    }
            if (learned_on) {
                learned = a.fb[ct] == 0;
                nu = ((const float *)a.nu)[ct];
            }
        }
        // driving field: this tile cell's x phase and pencil block
        float pr = 0.f, pim = 0.f;
        const float *gb = lgw;
        if (force) {
            const int ci = ct % a.g.nx;
            cell_phase<float>(as_tab<float>(a.ftab) + PencilLayout<2>::phases(a.g.ny, a.g.nz), ci, pr, pim);
            if (!uni) gb = (const float *)(a.ftab) + PL::HDR + (size_t)(ct / a.g.nx) * PL::STRIDE;
        }
        f4_t C[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) C[v] = f4_t{0.f, 0.f, 0.f, 0.f};
        float sa0 = 0.f, sa1 = 0.f, sa2 = 0.f;
#pragma unroll
        for (int P = 0; P < 2; ++P) {
            // point values: E[v] holds points 16P + 4g + r of cell j
            f4_t E[4], Dd = f4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                E[v] = f4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int st = 0; st < 3; ++st) E[v] = mfma4(lds[MfmaTab::EV + (P * 3 + st) * 64 + lane], bw[v][st], E[v]);
            }
            if (av) Dd = mfma4(lds[MfmaTab::DV + P * 64 + lane], dvg, Dd);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int q = 16 * P + 4 * g + r;
                const int qe = q < NQ ? q : 0;
                const float rho = E[0][r];
                const float m[3] = {E[1][r], E[2][r], E[3][r]};
                float pi = 0.f;
                if (av) {
                    const float div = Dd[r] * two_h;
                    const float pv = vnr_pi<float>(rho, div, hp, alpha, beta, cs, inv_dt);
                    const float sq = -div;
                    float pl = fminf(rho * nu * sq, 0.5f * rho * hp * hp * sq * inv_dt);
                    pl = (sq > 0.f && nu > 0.f) ? pl : 0.f;
                    pi = learned ? pl : pv;
                }
                const float ir = rcp(rho);
                const float pw = cs2 * rho + pi;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const float mdr = m[d] * ir;
                    float F[4] = {m[d], mdr * m[0], mdr * m[1], mdr * m[2]};
                    F[1 + d] += pw;
                    const float ac = lds[MfmaTab::CT + ((d * 2 + P) * 4 + r) * 64 + lane];
#pragma unroll
                    for (int v = 0; v < 4; ++v) C[v] = mfma4(ac, F[v], C[v]);
                }
                if (force) {
                    const int tx = qe % 3, tt = qe / 3;
                    const float er = ft[2 * tx], ei = ft[2 * tx + 1];
                    const float xr = pr * er - pim * ei, xi = pr * ei + pim * er;
                    const float x2r = xr * xr - xi * xi, x2i = 2.f * xr * xi;
                    const float *e = gb + tt * PL::ENT;
                    float acc[3];
#pragma unroll
                    for (int d = 0; d < 3; ++d)
                        acc[d] = e[5 * d] + e[5 * d + 1] * xr - e[5 * d + 2] * xi + e[5 * d + 3] * x2r - e[5 * d + 4] * x2i;
                    const float af = lds[MfmaTab::FT + (P * 4 + r) * 64 + lane] * half_h;
                    const float wq = lds[MfmaTab::WQ + (P * 4 + r) * 64 + lane];
                    const float s0 = rho * acc[0], s1 = rho * acc[1], s2 = rho * acc[2];
                    C[1] = mfma4(af, s0, C[1]);
                    C[2] = mfma4(af, s1, C[2]);
                    C[3] = mfma4(af, s2, C[3]);
                    if (tact) { sa0 += wq * s0; sa1 += wq * s1; sa2 += wq * s2; }
                }
            }
        }
        fs0 += sa0; fs1 += sa1; fs2 += sa2;
        // hand modes 4g + r of cell j to the cell's own lane (16t + j)
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int l = 0; l < NB; ++l) {
                const float x = __shfl(C[v][l & 3], 16 * (l >> 2) + j, 64);
                L[v][l] = g == t ? x : L[v][l];
            }
    }
    __syncthreads();      // the face pass reuses the buffer
}

// ------------------------------------------------------------------ RHS kernel
// dw/dt = (1/(4h)) [ sum_q w_q grad_xi(phi) . F(q) - sum_faces +- sum_r w_r phi F*(r) ]
//         + (1/8) sum_q w_q phi rho a (Sec. 2.2 weight evolution; Sec. 3.1; Sec. 4.2)
// occupancy target (waves per SIMD) of the right-hand-side kernel: the register file
// holds the 4 NB coefficients and 4 NB accumulators of a cell per lane, so FP64 fits two
// waves and FP32 four (two at degree 3) without spilling.  FP64 at degree 3 (160 values
// of coefficients and accumulators) cannot fit 256 VGPRs: one wave per SIMD lets the
// compiler keep the overflow in accumulation registers instead of scratch memory.
template <typename T, int K, bool VMFMA = false>
constexpr int rhs_waves() { return VMFMA ? MFMA_WAVES : (sizeof(T) == 8 ? (K <= 2 ? 2 : 1) : (K <= 2 ? 4 : 2)); }

template <typename T, int K, bool UNV>
__device__ __forceinline__ void rhs_combination(const void *ui, T (&L)[4][Shape<K>::NB], T inv4h, double dt,
                                            const StageArgs &st, bool active, unsigned bo, double *lds);

// COMB: 0 stores the right-hand side (and the mean-acceleration partials); 1 and 2 go on with
// the combination of the stage st of a Runge-Kutta step for the cell (rhs_combination; 2: u^n
// enters) and store nothing of the right-hand side
template <typename T, int K, bool FDIRECT, bool VMFMA = false, int COMB = 0>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(rhs_waves<T, K, VMFMA>())))
k_rhs(RhsArgs a, StageArgs st)
{
    static_assert(!(COMB && VMFMA), "split stages: vector volume integral only");
    using S = Shape<K>;
    using TL = TabLayout<K>;
    constexpr Modes<K> M = make_modes<K>();
    constexpr int NB = S::NB, ND = S::ND;
    __shared__ double lds[4 * 4];
    __shared__ T fsh[S::NF * 4 * BLOCK];        // point fluxes of the low faces, [r][v][thread]
    ctab<T> *tab = as_tab<T>(a.tab);
    const int nc = a.g.nc;
    const int blk = plane_tiled(xcd_remap(blockIdx.x, gridDim.x), a.bpp, a.g.nz, a.zt);
    const int c0 = blk * BLOCK + threadIdx.x;
    const bool active = c0 < nc;
    const int c = active ? c0 : 0;
    if (a.fail_reset && blockIdx.x == 0 && threadIdx.x == 0) *a.fail_reset = 0;

    const bool av = a.flags & F_AV;
    const bool prim = a.flags & F_PRIM;
    const bool force = a.flags & F_FORCE;
    const bool use_hllc = a.flags & F_HLLC;
    const T cs = (T)a.cs, cs2 = (T)(a.cs * a.cs);
    const T hp = (T)(a.h / (K + 1));
    // dt <= 0: no Pi_max cap (a huge finite factor keeps 0 * cap = 0)
    const double dt = a.dt_dev ? *a.dt_dev : a.dt;
    const T inv_dt = dt > 0.0 ? (T)(1.0 / dt) : (sizeof(T) == 4 ? T(1e30f) : T(1e300));
    const T alpha = (T)a.alpha, beta = (T)a.beta;
    const T two_h = (T)(2.0 / a.h);

    const unsigned bo = (unsigned)c * sizeof(T);
    const Field<T, 4> U(a.u, NB, nc);
    const Field<T, 3> VH(a.vh, NB, nc);
    // with the projected velocity on the faces the momentum weights are read only here:
    // non-temporal, like the right-hand side written at the end
    T W[4][NB];
    if constexpr (!VMFMA) {
        if (prim) {
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int l = 0; l < NB; ++l) W[v][l] = v ? U.get_nt(v, l, bo) : U.get(v, l, bo);
        } else {
            load_field<T, K, 4>(U, bo, W);
        }
    } else {
        W[0][0] = U.get(0, 0, bo);
    }

    ctab<T> *ft = as_tab<T>(a.ftab);

    // divergence of the projected velocity (Sec. 3.1) as a degree-(K-1) polynomial:
    // its NDIV modal coefficients from the exact derivatives of the Legendre basis
    constexpr DivMap<K> DM = make_divmap<K>();
    constexpr int NDIV = DivMap<K>::NDIV;
    T Dv[NDIV];
#pragma unroll
    for (int m = 0; m < NDIV; ++m) Dv[m] = T(0);
    bool learned = false;
    T nu = T(0);
    if (av && !VMFMA) {
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int l = 0; l < NB; ++l)
                if (M.e[l][d] >= 1) {
                    const T v = VH.get(d, l, bo);
#pragma unroll
                    for (int t = 0; t < DivMap<K>::MAXT; ++t)
                        if (DM.m[d][l][t] >= 0) Dv[DM.m[d][l][t]] += v * T(__builtin_sqrt(double(DM.f[d][l][t])));
                }
        if (a.flags & F_LEARNED) {
            learned = a.fb[c] == 0;
            nu = ((const T *)a.nu)[c];
        }
    }

    T L[4][NB];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int l = 0; l < NB; ++l) L[v][l] = T(0);
    T fs0 = T(0), fs1 = T(0), fs2 = T(0);
    const T half_h = (T)(0.5 * a.h);
    // driving field: the cell's pencil (j, l) and x phase (pencil form) or indices (direct form)
    const int pencil = c / a.g.nx;
    const int cijk[3] = {c % a.g.nx, pencil % a.g.ny, pencil / a.g.ny};
    T pr = T(0), pim = T(0);
    if (force && !FDIRECT) cell_phase<T>(ft + PencilLayout<K>::phases(a.g.ny, a.g.nz), cijk[0], pr, pim);

    // ---- volume integral
    auto volume = [&](auto form, int pen) {
        constexpr int FM = decltype(form)::value;
        ctab<T> *g = ft + PencilLayout<K>::HDR + (size_t)pen * PencilLayout<K>::STRIDE;
#pragma unroll 1
        for (int q = 0; q < S::NQ; ++q) {
            ctab<T> *ph = tab + TL::VPHI + q * NB;
            ctab<T> *dph = tab + TL::VDPHI + q * 3 * ND;
            const T wq = tab[TL::VW + q];
            T rho = T(0), m[3] = {T(0), T(0), T(0)};
#pragma unroll
            for (int l = 0; l < NB; ++l) {
                const T p = ph[l];
                rho += W[0][l] * p;
                m[0] += W[1][l] * p;
                m[1] += W[2][l] * p;
                m[2] += W[3][l] * p;
            }
            T pi = T(0);
            if (av) {
                T div = T(0);
#pragma unroll
                for (int mm = 0; mm < NDIV; ++mm) div += Dv[mm] * ph[mm];
                div *= two_h;
                const T pv = vnr_pi<T>(rho, div, hp, alpha, beta, cs, inv_dt);
                // learned sensor: the cell's bulk viscosity nu in place of the vNR one,
                // Pi = rho nu s at compressed points, with the Pi_max cap of the point
                const T sq = -div;
                T pl = fmin(rho * nu * sq, T(0.5) * rho * hp * hp * sq * inv_dt);
                pl = (sq > T(0) && nu > T(0)) ? pl : T(0);
                pi = learned ? pl : pv;
            }
            const T ir = rcp(rho);
            const T pw = (cs2 * rho + pi) * wq;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const T md = m[d] * wq;
                const T mdr = md * ir;
                T F[4];
                F[0] = md;
                F[1] = mdr * m[0];
                F[2] = mdr * m[1];
                F[3] = mdr * m[2];
                F[1 + d] += pw;
#pragma unroll
                for (int l = 0; l < NB; ++l) {
                    if (M.dj[d][l] < 0) continue;
                    const T dp = dph[d * ND + M.dj[d][l]];
#pragma unroll
                    for (int v = 0; v < 4; ++v) L[v][l] += dp * F[v];
                }
            }
            if (force) {
                T ac[3];
                if constexpr (FM == FM_DIRECT)
                    direct_accel<T>(a.modes, a.nmodes, cijk, tab[TL::VXI + 3 * q], tab[TL::VXI + 3 * q + 1],
                                    tab[TL::VXI + 3 * q + 2], a.h, ac);
                else
                    pencil_accel<T, K>(ft, g, q, pr, pim, ac);
                T sp[3];
                drive_point<T>(rho, wq, ac, sp, fs0, fs1, fs2);
                const T t0 = sp[0] * half_h, t1 = sp[1] * half_h, t2 = sp[2] * half_h;
#pragma unroll
                for (int l = 0; l < NB; ++l) {
                    const T p = ph[l];
                    L[1][l] += t0 * p;
                    L[2][l] += t1 * p;
                    L[3][l] += t2 * p;
                }
            }
        }
    };
    if constexpr (VMFMA) {
        static_assert(sizeof(T) == 4 && K == 2 && !FDIRECT, "matrix-core volume integral: FP32, degree 2");
        volume_mfma(a, tab, (float *)fsh, blk, active, pencil, L, fs0, fs1, fs2);
    } else if constexpr (FDIRECT) {
        volume(std::integral_constant<int, FM_DIRECT>{}, 0);
    } else {
        // the wave's cells share one pencil (x lines of at least 64 cells): scalar table loads
        const int p0 = __shfl(pencil, 0, 64);
        if (force && __all(!active || pencil == p0))
            volume(std::integral_constant<int, FM_UNIFORM>{}, __builtin_amdgcn_readfirstlane(p0));
        else
            volume(std::integral_constant<int, FM_LANE>{}, pencil);
    }
    const T mass0 = W[0][0];

    // ---- surface integral (traces: rho and either the projected velocity or m)
    int nbr[6], ijk[3];
    neighbours(a.g, c, nbr, ijk);
    const Field<T, 4> SRC = prim ? Field<T, 4>(a.u, a.vh, NB, nc) : U;
    // Each face flux is needed by both cells.  Every cell computes its low x and y faces
    // and leaves the point fluxes in LDS; a wave whose high-side neighbours all belong to
    // this block (whole x lines per block, and y lines of the block but the last) lifts
    // those instead of recomputing the face.  The decision is a wave vote, so the branch
    // is uniform; the stored values are exactly those the cell would compute itself.
    const int base = blk * BLOCK;
    const bool xsh = __all((unsigned)(nbr[1] - base) < (unsigned)BLOCK);
    const bool ysh = __all((unsigned)(nbr[3] - base) < (unsigned)BLOCK);
    // Every face leaves its point fluxes in the cell's LDS column and lifts them from there.
    // A wave whose high neighbours all lie in the block lifts their low-face fluxes (between
    // two barriers) instead of computing its high face; a high face that is computed is
    // stored only after the second barrier, when no other wave reads the columns any more.
    T *col = fsh + threadIdx.x;
#pragma unroll 1
    for (int s = 0; s < 2; ++s) {
        if (s == 1) {
            __syncthreads();
            if (xsh) lift<T, K, 0>(fsh + (nbr[1] - base), 1, tab, L);
            __syncthreads();
            if (xsh) break;
        }
        face<T, K, 0>(SRC, bo, (unsigned)(s ? nbr[1] : nbr[0]) * sizeof(T), s, tab, prim, use_hllc, cs, cs2, L, col);
    }
#pragma unroll 1
    for (int s = 0; s < 2; ++s) {
        if (s == 1) {
            __syncthreads();
            if (ysh) lift<T, K, 1>(fsh + (nbr[3] - base), 1, tab, L);
            __syncthreads();
            if (ysh) break;
        }
        face<T, K, 1>(SRC, bo, (unsigned)(s ? nbr[3] : nbr[2]) * sizeof(T), s, tab, prim, use_hllc, cs, cs2, L, col);
    }
#pragma unroll 1
    for (int s = 0; s < 2; ++s)
        face<T, K, 2>(SRC, bo, (unsigned)(s ? nbr[5] : nbr[4]) * sizeof(T), s, tab, prim, use_hllc, cs, cs2, L, col);

    const T inv4h = (T)(0.25 / a.h);
    if constexpr (COMB != 0) {
        (void)mass0;
        __shared__ double lds_st[20];
        rhs_combination<T, K, COMB == 2>(a.u, L, inv4h, dt, st, active, bo, lds_st);
    } else {
        (void)st;
        if (active) {
            const Field<T, 4> O(a.out, NB, nc);
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int l = 0; l < NB; ++l) O.put_nt(v, l, bo, L[v][l] * inv4h);
            if (a.pred_fail) predict_failure<T>(a, dt, c, mass0, L[0][0] * inv4h);
        }
        if (force && a.part) {
            const bool fsok = active || VMFMA;     // the matrix-core sums are masked per tile cell
            double acc[4] = {fsok ? 0.125 * (double)fs0 : 0.0, fsok ? 0.125 * (double)fs1 : 0.0,
                             fsok ? 0.125 * (double)fs2 : 0.0, active ? (double)mass0 : 0.0};
            block_sum<4>(acc, lds);
            if (threadIdx.x == 0)
#pragma unroll
                for (int i = 0; i < 4; ++i) a.part[blk * 4 + i] = acc[i];
        }
    }
}

// ------------------------------------------- RHS kernel, FP64, two lanes per cell
// The FP64 kernel above keeps all 4 NB coefficients and 4 NB accumulators of a cell in one
// lane, which at degree 3 fits only one wave per SIMD.  Here the lanes 2i and 2i+1 of a wave share
// cell i: lane h owns variables 2h and 2h+1 (coefficients, accumulators, face traces), and
// the partner's point values come across in registers (a DPP lane swap).  The flux at a
// point, which needs all four variables, is formed in both lanes; each lane contracts and
// lifts its own two variables.  Buffer resources are uniform over the wave: a lane reaches
// its variable 2h+i through the buffer of variable i and a lane offset of two variable
// blocks (LSEL: when that offset fits 32 bits, with the projected traces read from one
// array that holds a copy of the density weights in front of the projected velocity);
// otherwise it loads variables i and 2+i and keeps its own.

// the value held by the other lane of the pair (lane ^ 1)
__device__ __forceinline__ double pair_swap(double x)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)(b & 0xffffffffull), 0xB1, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), 0xB1, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// all four variables from the own pair (a0, a1) and the partner's pair (b0, b1): lane 0
// owns variables 0 and 1, lane 1 variables 2 and 3
__device__ __forceinline__ void pair_assemble(int h, double a0, double a1, double b0, double b1, double (&x)[4])
{
    x[0] = h ? b0 : a0;
    x[1] = h ? b1 : a1;
    x[2] = h ? a0 : b0;
    x[3] = h ? a1 : b1;
}

// Surface integral of one face (normal axis D, side s) from the point fluxes in an LDS column
// (col: the column of the cell that stored them, [r][v] with stride CB): the flux moments
// against the 2D basis of the face, M_j = sum_r w_r F(r) P2_j(r), then per mode
// phi_l = Lt_{e_D}(+-1) P2_{d2(l)} on the face
template <int K, int D, int CB>
__device__ __forceinline__ void lift_pair(const double *col, int h, int s, ctab<double> *tab,
                                          double (&L)[2][Shape<K>::NB])
{
    using S = Shape<K>;
    using TL = TabLayout<K>;
    constexpr Modes<K> M = make_modes<K>();
    double M2[2][S::NB2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < S::NB2; ++j) M2[i][j] = 0.0;
#pragma unroll 1
    for (int r = 0; r < S::NF; ++r) {
        const double wr = s ? -tab[TL::FW + r] : tab[TL::FW + r];   // outward normal
        ctab<double> *f2 = tab + TL::F2 + r * S::NB2;
        const double g0 = wr * col[(r * 4 + 2 * h) * CB];
        const double g1 = wr * col[(r * 4 + 2 * h + 1) * CB];
#pragma unroll
        for (int j = 0; j < S::NB2; ++j) {
            M2[0][j] += g0 * f2[j];
            M2[1][j] += g1 * f2[j];
        }
    }
    ctab<double> *lend = tab + TL::LEND;
#pragma unroll
    for (int l = 0; l < S::NB; ++l) {
        const double ls = lend[2 * M.e[l][D] + s];
        L[0][l] += ls * M2[0][M.d2[D][l]];
        L[1][l] += ls * M2[1][M.d2[D][l]];
    }
}

// one face of the cell for the lane's two variables; src[i] points at variable 2h+i of
// the trace field (mode planes nc apart), c and cn the own and the neighbour cell
template <int K, int D, int CB, bool LSEL>
__device__ __forceinline__ void face_pair(const Field<double, 4> &src, unsigned bo, unsigned bn, int s, int h,
                                          unsigned hoff, ctab<double> *tab, bool prim, bool use_hllc, double cs,
                                          double cs2, double (&L)[2][Shape<K>::NB], double *col)
{
    using S = Shape<K>;
    using TL = TabLayout<K>;
    constexpr Modes<K> M = make_modes<K>();
    double Co[2][S::NB2], Cn[2][S::NB2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < S::NB2; ++j) { Co[i][j] = 0.0; Cn[i][j] = 0.0; }
    ctab<double> *lend = tab + TL::LEND;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int l = 0; l < S::NB; ++l) {
            const int e = M.e[l][D];
            double wo, wn;
            if constexpr (LSEL) {
                // variable 2h+i: the buffer of variable i, two variable blocks further in lane 1
                wo = src.get(i, l, bo + hoff);
                wn = src.get(i, l, bn + hoff);
            } else {
                // through the uniform per-variable buffers: both candidates, then the lane's own
                const double wo0 = src.get(i, l, bo), wo1 = src.get(2 + i, l, bo);
                const double wn0 = src.get(i, l, bn), wn1 = src.get(2 + i, l, bn);
                wo = h ? wo1 : wo0;
                wn = h ? wn1 : wn0;
            }
            Co[i][M.d2[D][l]] += wo * lend[2 * e + s];
            Cn[i][M.d2[D][l]] += wn * lend[2 * e + 1 - s];
            // keep at most one variable's loads in flight (register pressure)
            if (l == S::NB - 1) __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll 1
    for (int r = 0; r < S::NF; ++r) {
        ctab<double> *f2 = tab + TL::F2 + r * S::NB2;
        double ao[2] = {0.0, 0.0}, an[2] = {0.0, 0.0};
#pragma unroll
        for (int j = 0; j < S::NB2; ++j) {
            const double f = f2[j];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                ao[i] += Co[i][j] * f;
                an[i] += Cn[i][j] * f;
            }
        }
        double xo[4], xn[4];
        pair_assemble(h, ao[0], ao[1], pair_swap(ao[0]), pair_swap(ao[1]), xo);
        pair_assemble(h, an[0], an[1], pair_swap(an[0]), pair_swap(an[1]), xn);
        double uo[4], un[4], vo[3], vn[3];
        uo[0] = xo[0];
        un[0] = xn[0];
        if (prim) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                vo[d] = xo[1 + d]; uo[1 + d] = xo[0] * xo[1 + d];
                vn[d] = xn[1 + d]; un[1 + d] = xn[0] * xn[1 + d];
            }
        } else {
            const double io = rcp(xo[0]), in = rcp(xn[0]);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                uo[1 + d] = xo[1 + d]; vo[d] = xo[1 + d] * io;
                un[1 + d] = xn[1 + d]; vn[d] = xn[1 + d] * in;
            }
        }
        double F[4];
        if (use_hllc) {
            if (s) hllc<D>(cs, cs2, uo, vo, un, vn, F);
            else   hllc<D>(cs, cs2, un, vn, uo, vo, F);
        } else {
            if (s) rusanov<D>(cs, cs2, uo, vo, un, vn, F);
            else   rusanov<D>(cs, cs2, un, vn, uo, vo, F);
        }
        col[(r * 4 + 2 * h) * CB] = h ? F[2] : F[0];
        col[(r * 4 + 2 * h + 1) * CB] = h ? F[3] : F[1];
    }
    lift_pair<K, D, CB>(col, h, s, tab, L);
}

template <int K>
constexpr int rhs_pair_waves() { return K <= 2 ? 3 : 2; }   // at K = 3: 256 VGPRs, 14 of them spilled

template <int K, bool FDIRECT, bool LSEL>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(rhs_pair_waves<K>()))) k_rhs_pair(RhsArgs a)
{
    using S = Shape<K>;
    using TL = TabLayout<K>;
    constexpr Modes<K> M = make_modes<K>();
    constexpr int NB = S::NB, ND = S::ND;
    constexpr int CB = BLOCK / 2;                  // cells per block
    __shared__ double lds[4 * 4];
    __shared__ double fsh[S::NF * 4 * CB];          // point fluxes of the low faces, [r][v][cell]
    ctab<double> *tab = as_tab<double>(a.tab);
    const int nc = a.g.nc;
    const size_t ncs = (size_t)nc;
    const int blk = plane_tiled(xcd_remap(blockIdx.x, gridDim.x), a.bpp, a.g.nz, a.zt);
    const int h = threadIdx.x & 1;                 // variables 2h and 2h+1
    const int cb = threadIdx.x >> 1;
    const int c0 = blk * CB + cb;
    const bool active = c0 < nc;
    const int c = active ? c0 : 0;

    const bool av = a.flags & F_AV;
    const bool prim = a.flags & F_PRIM;
    const bool force = a.flags & F_FORCE;
    const bool use_hllc = a.flags & F_HLLC;
    const double cs = a.cs, cs2 = a.cs * a.cs;
    const double hp = a.h / (K + 1);
    const double dt = a.dt_dev ? *a.dt_dev : a.dt;
    const double inv_dt = dt > 0.0 ? 1.0 / dt : 1e300;
    const double alpha = a.alpha, beta = a.beta;
    const double two_h = 2.0 / a.h;

    const unsigned bo = (unsigned)c * 8u;
    const Field<double, 4> U(a.u, NB, nc);
    const unsigned hoff = h ? a.pair_vstride : 0u;
    double W[2][NB];
    // with the projected velocity on the faces the momentum weights are read only here:
    // non-temporal, like the right-hand side written at the end
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int l = 0; l < NB; ++l) {
            if constexpr (LSEL) {
                W[i][l] = (i && prim) ? U.get_nt(i, l, bo + hoff) : U.get(i, l, bo + hoff);
            } else {
                const double w0 = (i && prim) ? U.get_nt(i, l, bo) : U.get(i, l, bo);
                const double w1 = prim ? U.get_nt(2 + i, l, bo) : U.get(2 + i, l, bo);
                W[i][l] = h ? w1 : w0;
            }
        }

    constexpr DivMap<K> DM = make_divmap<K>();
    constexpr int NDIV = DivMap<K>::NDIV;
    double Dv[NDIV];
#pragma unroll
    for (int m = 0; m < NDIV; ++m) Dv[m] = 0.0;
    bool learned = false;
    double nu = 0.0;
    const Field<double, 3> VH(a.vh, NB, nc);
    if (av) {
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int l = 0; l < NB; ++l)
                if (M.e[l][d] >= 1) {
                    const double v = VH.get(d, l, bo);
#pragma unroll
                    for (int t = 0; t < DivMap<K>::MAXT; ++t)
                        if (DM.m[d][l][t] >= 0) Dv[DM.m[d][l][t]] += v * __builtin_sqrt(double(DM.f[d][l][t]));
                }
        if (a.flags & F_LEARNED) {
            learned = a.fb[c] == 0;
            nu = ((const double *)a.nu)[c];
        }
    }

    double L[2][NB];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int l = 0; l < NB; ++l) L[i][l] = 0.0;
    // driving source sums of the lane's own momentum components: lane 0 the x one (fsa),
    // lane 1 the y and z ones (fsa, fsb)
    double fsa = 0.0, fsb = 0.0;
    const double half_h = 0.5 * a.h;
    const int pencil = c / a.g.nx;
    const int cijk[3] = {c % a.g.nx, pencil % a.g.ny, pencil / a.g.ny};
    double pr = 0.0, pim = 0.0;
    ctab<double> *ft = as_tab<double>(a.ftab);
    if (force && !FDIRECT) cell_phase<double>(ft + PencilLayout<K>::phases(a.g.ny, a.g.nz), cijk[0], pr, pim);

    // ---- volume integral
    auto volume = [&](auto form, int pen) {
        constexpr int FM = decltype(form)::value;
        ctab<double> *g = ft + PencilLayout<K>::HDR + (size_t)pen * PencilLayout<K>::STRIDE;
#pragma unroll 1
        for (int q = 0; q < S::NQ; ++q) {
            ctab<double> *ph = tab + TL::VPHI + q * NB;
            ctab<double> *dph = tab + TL::VDPHI + q * 3 * ND;
            const double wq = tab[TL::VW + q];
            double x0 = 0.0, x1 = 0.0;
#pragma unroll
            for (int l = 0; l < NB; ++l) {
                x0 += W[0][l] * ph[l];
                x1 += W[1][l] * ph[l];
            }
            double xv[4];
            pair_assemble(h, x0, x1, pair_swap(x0), pair_swap(x1), xv);
            const double rho = xv[0];
            const double m[3] = {xv[1], xv[2], xv[3]};
            double pi = 0.0;
            if (av) {
                double div = 0.0;
#pragma unroll
                for (int mm = 0; mm < NDIV; ++mm) div += Dv[mm] * ph[mm];
                div *= two_h;
                const double pv = vnr_pi<double>(rho, div, hp, alpha, beta, cs, inv_dt);
                const double sq = -div;
                double pl = fmin(rho * nu * sq, 0.5 * rho * hp * hp * sq * inv_dt);
                pl = (sq > 0.0 && nu > 0.0) ? pl : 0.0;
                pi = learned ? pl : pv;
            }
            const double ir = rcp(rho);
            const double pw = (cs2 * rho + pi) * wq;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double md = m[d] * wq;
                const double mdr = md * ir;
                // lane 0: (rho, m_x) fluxes; lane 1: (m_y, m_z)
                const double fa = h ? mdr * m[1] + (d == 1 ? pw : 0.0) : md;
                const double fb = h ? mdr * m[2] + (d == 2 ? pw : 0.0) : mdr * m[0] + (d == 0 ? pw : 0.0);
#pragma unroll
                for (int l = 0; l < NB; ++l) {
                    if (M.dj[d][l] < 0) continue;
                    const double dp = dph[d * ND + M.dj[d][l]];
                    L[0][l] += dp * fa;
                    L[1][l] += dp * fb;
                }
            }
            if (force) {
                double ac[3];
                if constexpr (FM == FM_DIRECT)
                    direct_accel<double>(a.modes, a.nmodes, cijk, tab[TL::VXI + 3 * q], tab[TL::VXI + 3 * q + 1],
                                         tab[TL::VXI + 3 * q + 2], a.h, ac);
                else
                    pencil_accel<double, K>(ft, g, q, pr, pim, ac);
                const double rw = rho * wq;
                const double sa = rw * (h ? ac[1] : ac[0]);
                const double sb = h ? rw * ac[2] : 0.0;
                fsa += sa;
                fsb += sb;
                const double ta = h ? sa * half_h : 0.0;
                const double tb = h ? sb * half_h : sa * half_h;
#pragma unroll
                for (int l = 0; l < NB; ++l) {
                    const double p = ph[l];
                    L[0][l] += ta * p;
                    L[1][l] += tb * p;
                }
            }
        }
    };
    if constexpr (FDIRECT) {
        volume(std::integral_constant<int, FM_DIRECT>{}, 0);
    } else {
        const int p0 = __shfl(pencil, 0, 64);
        if (force && __all(!active || pencil == p0))
            volume(std::integral_constant<int, FM_UNIFORM>{}, __builtin_amdgcn_readfirstlane(p0));
        else
            volume(std::integral_constant<int, FM_LANE>{}, pencil);
    }
    const double mass0 = W[0][0];                   // cell mean density (lane 0)

    // ---- surface integral, with the low x and y face fluxes shared through LDS as in the
    // one-lane kernel (cells of the block: CB consecutive cells)
    int nbr[6], ijk[3];
    neighbours(a.g, c, nbr, ijk);
    // trace sources: density and projected velocity (one array when the density copy is
    // there), or the weights
    const Field<double, 4> SRC = !prim ? U
                                 : (LSEL ? Field<double, 4>(a.vh_rho, NB, nc) : Field<double, 4>(a.u, a.vh, NB, nc));
    const int base = blk * CB;
    const bool xsh = __all((unsigned)(nbr[1] - base) < (unsigned)CB);
    const bool ysh = __all((unsigned)(nbr[3] - base) < (unsigned)CB);
    // Every face leaves its point fluxes in the cell's LDS column and lifts them from there.
    // The low x and y faces are the high faces of the neighbours below: a wave whose
    // neighbours above all lie in the block lifts theirs (between two barriers) instead of
    // computing its high face; a high face that is computed is stored only after the second
    // barrier, when no other wave reads the columns any more.
    double *col = fsh + cb;
#pragma unroll 1
    for (int s = 0; s < 2; ++s) {
        if (s == 1) {
            __syncthreads();
            if (xsh) lift_pair<K, 0, CB>(fsh + (nbr[1] - base), h, 1, tab, L);
            __syncthreads();
            if (xsh) break;
        }
        face_pair<K, 0, CB, LSEL>(SRC, bo, (unsigned)(s ? nbr[1] : nbr[0]) * 8u, s, h, hoff, tab, prim, use_hllc, cs,
                                  cs2, L, col);
    }
#pragma unroll 1
    for (int s = 0; s < 2; ++s) {
        if (s == 1) {
            __syncthreads();
            if (ysh) lift_pair<K, 1, CB>(fsh + (nbr[3] - base), h, 1, tab, L);
            __syncthreads();
            if (ysh) break;
        }
        face_pair<K, 1, CB, LSEL>(SRC, bo, (unsigned)(s ? nbr[3] : nbr[2]) * 8u, s, h, hoff, tab, prim, use_hllc, cs,
                                  cs2, L, col);
    }
#pragma unroll 1
    for (int s = 0; s < 2; ++s)
        face_pair<K, 2, CB, LSEL>(SRC, bo, (unsigned)(s ? nbr[5] : nbr[4]) * 8u, s, h, hoff, tab, prim, use_hllc, cs,
                                  cs2, L, col);

    const double inv4h = 0.25 / a.h;
    if (active) {
        double *ob = (double *)a.out;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int l = 0; l < NB; ++l)
                __builtin_nontemporal_store(L[i][l] * inv4h, &ob[((size_t)(2 * h + i) * NB + l) * ncs + c]);
        if (a.pred_fail && h == 0) predict_failure<double>(a, dt, c, mass0, L[0][0] * inv4h);
    }
    if (force && a.part) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        if (active) {
            acc[0] = h ? 0.0 : 0.125 * fsa;
            acc[1] = h ? 0.125 * fsa : 0.0;
            acc[2] = h ? 0.125 * fsb : 0.0;
            acc[3] = h ? 0.0 : mass0;
        }
        block_sum<4>(acc, lds);
        if (threadIdx.x == 0)
#pragma unroll
            for (int i = 0; i < 4; ++i) a.part[blk * 4 + i] = acc[i];
    }
}

// Projected velocity of one cell (Sec. 3.2; stored when vh is not null) and, when part is
// not null, the per-block maxima for the time step: signal speed sum_d |v_d| + cs over the
// interior points, and bulk viscosity alpha (h/p)^2 |div v| + beta cs h/p at compressing
// points (or the learned cell viscosity where the learned sensor is in use), written to
// part[2 blk] and part[2 blk + 1].  With part set every thread of the block must call it.
template <typename T, int K, bool SPLIT = split_projection<T>()>
__device__ __forceinline__ void project_and_bounds(const T (&W)[4][Shape<K>::NB], ctab<T> *tab, void *vh, int nc,
                                                   unsigned bo, int c, bool active, const ProjArgs &pa,
                                                   double *part, int blk, double *lds)
{
    using S = Shape<K>;
    using TL = TabLayout<K>;
    constexpr Modes<K> M = make_modes<K>();
    constexpr int NB = S::NB;
    double sm = 0.0;
    // the projection takes the signal speed along from its own point values
    const bool speed_in_projection = vh || (part && pa.visc);
    if (part && !speed_in_projection) {
        // largest signal speed sum_d |v_d| + cs over the interior points
#pragma unroll 1
        for (int q = 0; q < S::NQ; ++q) {
            ctab<T> *ph = tab + TL::VPHI + q * NB;
            T rho = T(0), m0 = T(0), m1 = T(0), m2 = T(0);
#pragma unroll
            for (int l = 0; l < NB; ++l) {
                const T p = ph[l];
                rho += W[0][l] * p;
                m0 += W[1][l] * p;
                m1 += W[2][l] * p;
                m2 += W[3][l] * p;
            }
            const T ir = rcp(rho);
            const double s = (double)fabs(m0 * ir) + (double)fabs(m1 * ir) + (double)fabs(m2 * ir) + 3.0 * pa.cs;
            sm = fmax(sm, s);
        }
    }
    // projected velocity, component by component: stored, and folded into the modal
    // coefficients of its divergence (a degree-(K-1) polynomial) for the viscous bound
    constexpr DivMap<K> DM = make_divmap<K>();
    constexpr int NDIV = DivMap<K>::NDIV;
    const bool visc = part && pa.visc;
    T Dv[NDIV];
#pragma unroll
    for (int m = 0; m < NDIV; ++m) Dv[m] = T(0);
    if (vh || visc) {
        const Field<T, 3> VO(vh ? vh : (const void *)tab, NB, nc);
        auto fold = [&](int d, const T (&V)[NB]) {
#pragma unroll
            for (int l = 0; l < NB; ++l)
                if (M.e[l][d] >= 1)
#pragma unroll
                    for (int t = 0; t < DivMap<K>::MAXT; ++t)
                        if (DM.m[d][l][t] >= 0) Dv[DM.m[d][l][t]] += V[l] * T(__builtin_sqrt(double(DM.f[d][l][t])));
        };
        if constexpr (SPLIT) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                T V[NB];
                if (d == 0 && part)
                    project_first_with_speed<T, K>(W, tab, V, pa.cs, sm);
                else
                    project_component<T, K>(W, tab, d, V);
                if (vh && active)
#pragma unroll
                    for (int l = 0; l < NB; ++l) VO.put(d, l, bo, V[l]);
                if (visc) fold(d, V);
            }
        } else {
            T V[3][NB];
            if (part)   // two calls, so that sm stays in registers
                project_cell<T, K>(W, tab, V, &sm, pa.cs);
            else
                project_cell<T, K>(W, tab, V, nullptr, pa.cs);
            if (vh && active) store_field<T, K, 3>(VO, bo, V);
            if (visc)
#pragma unroll
                for (int d = 0; d < 3; ++d) fold(d, V[d]);
        }
    }
    if (part) {
        double nm = 0.0;
        if (visc) {
            // most negative divergence of the projected velocity over the interior points
            const double hp = pa.h / (K + 1);
            double smin = 0.0;
#pragma unroll 1
            for (int q = 0; q < S::NQ; ++q) {
                ctab<T> *ph = tab + TL::VPHI + q * NB;
                T div = T(0);
#pragma unroll
                for (int m = 0; m < NDIV; ++m) div += Dv[m] * ph[m];
                smin = fmin(smin, (double)div);
            }
            const double s = -smin * (2.0 / pa.h);
            if (s > 0.0) nm = pa.alpha * hp * hp * s + pa.beta * pa.cs * hp;
            if (pa.fb && pa.fb[c] == 0) nm = pa.nu ? fmax((double)((const T *)pa.nu)[c], 0.0) : 0.0;
        }
        __syncthreads();
        sm = block_max(active ? sm : 0.0, lds);
        __syncthreads();
        nm = block_max(active ? nm : 0.0, lds);
        if (threadIdx.x == 0) {
            part[2 * blk] = sm;
            part[2 * blk + 1] = nm;
        }
    }
}

// The driving source of a cell summed over its volume points (times 1/8) and its mean
// density, from its density weights W0, for tables off the driving shell (the field mode by
// mode at each point), with the arithmetic of the right-hand side's volume loop: the point
// densities summed mode by mode in the same order, the source through drive_point and
// direct_accel.  acc[0..2]: source, acc[3]: mean density (all 0 for an inactive lane).
template <typename T, int K>
__device__ __forceinline__ void drive_sums_direct(const T (&W0)[Shape<K>::NB], ctab<T> *tab, const double *modes,
                                                  int nmodes, const Mesh &g, double h, int c, bool active,
                                                  double (&acc)[4])
{
    using S = Shape<K>;
    using TL = TabLayout<K>;
    constexpr int NB = S::NB;
    const int pencil = c / g.nx;
    const int cijk[3] = {c % g.nx, pencil % g.ny, pencil / g.ny};
    T fs0 = T(0), fs1 = T(0), fs2 = T(0);
    // three points per loop step: their table loads in flight together (the same sums)
#pragma unroll 3
    for (int q = 0; q < S::NQ; ++q) {
        ctab<T> *ph = tab + TL::VPHI + q * NB;
        const T wq = tab[TL::VW + q];
        T rho = T(0);
#pragma unroll
        for (int l = 0; l < NB; ++l) rho += W0[l] * ph[l];
        T ac[3];
        direct_accel<T>(modes, nmodes, cijk, tab[TL::VXI + 3 * q], tab[TL::VXI + 3 * q + 1], tab[TL::VXI + 3 * q + 2],
                        h, ac);
        T sp[3];
        drive_point<T>(rho, wq, ac, sp, fs0, fs1, fs2);
    }
    acc[0] = active ? 0.125 * (double)fs0 : 0.0;
    acc[1] = active ? 0.125 * (double)fs1 : 0.0;
    acc[2] = active ? 0.125 * (double)fs2 : 0.0;
    acc[3] = active ? (double)W0[0] : 0.0;
}

// --------------------------------------------------------------- stage kernel
// The removed mean acceleration of a stage (Sec. 4.2, mean-free driving): given in abar, or
// reduced here from the per-block partials of the stage input (every thread of the block
// must call it then), or zero.
template <typename T>
__device__ __forceinline__ void stage_abar(const StageArgs &a, T (&ab)[3], double *lds_ab)
{
    ab[0] = ab[1] = ab[2] = T(0);
    if (a.abar) { ab[0] = (T)a.abar[0]; ab[1] = (T)a.abar[1]; ab[2] = (T)a.abar[2]; }
    if (a.abar_part) {
        // the mass-weighted mean acceleration, as k_final computes it
        double sum[4];
        block_partial_sums4(a.abar_part, a.abar_np, sum, lds_ab);
        if (threadIdx.x == 0)
#pragma unroll
            for (int k = 0; k < 3; ++k) lds_ab[16 + k] = sum[k] / sum[3];
        __syncthreads();
        ab[0] = (T)lds_ab[16];
        ab[1] = (T)lds_ab[17];
        ab[2] = (T)lds_ab[18];
    }
}

// Positivity limiter of one cell after a stage (Sec. 3.1; target minimum
// max(floor, rel * mean)) with FP64 comparisons.  With a.nlim set every thread of the block
// must call it.
template <typename T, int K>
__device__ __forceinline__ bool stage_limit(T (&U)[4][Shape<K>::NB], ctab<T> *tab, const StageArgs &a, bool active,
                                            double *lds)
{
    using S = Shape<K>;
    using TL = TabLayout<K>;
    constexpr Modes<K> M = make_modes<K>();
    constexpr int NB = S::NB;
    const double mean = (double)U[0][0];
    const double fl = a.rho_floor;
    const double target = fmax(fl, a.rho_floor_rel * mean);
    // The density at any point of the cell differs from the mean by at most
    // dev = sum_{l>0} |W_l| max|phi_l|, with max|phi_l| = prod_a sqrt(2 e_a + 1) (the
    // normalised Legendre polynomials peak at the cell faces).  When mean - dev clears
    // the target with a margin for the rounding of the point sums, the minimum below
    // cannot fall short of the target and the limiter leaves the cell as it is; a wave
    // whose cells all clear it skips the point evaluations (same result).
    double dev = 0.0;
#pragma unroll
    for (int l = 1; l < NB; ++l) {
        double pm = 1.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) pm *= __builtin_sqrt(2.0 * M.e[l][d] + 1.0);
        dev += fabs((double)U[0][l]) * pm;
    }
    constexpr double EPS = sizeof(T) == 8 ? 1e-13 : 1e-5;
    const bool clear = !active || mean - dev - EPS * (fabs(mean) + dev) >= target;
    // minimum density over the volume and face Gauss points
    T rmin = T(__builtin_huge_valf());
    if (!__all(clear)) {
#pragma unroll 1
        for (int q = 0; q < S::NQ; ++q) {
            ctab<T> *ph = tab + TL::VPHI + q * NB;
            T r = T(0);
#pragma unroll
            for (int l = 0; l < NB; ++l) r += U[0][l] * ph[l];
            rmin = fmin(rmin, r);
        }
        ctab<T> *lend = tab + TL::LEND;
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                T C[S::NB2];
#pragma unroll
                for (int j = 0; j < S::NB2; ++j) C[j] = T(0);
#pragma unroll
                for (int l = 0; l < NB; ++l) C[M.d2[d][l]] += U[0][l] * lend[2 * M.e[l][d] + s];
#pragma unroll 1
                for (int r = 0; r < S::NF; ++r) {
                    ctab<T> *f2 = tab + TL::F2 + r * S::NB2;
                    T val = T(0);
#pragma unroll
                    for (int j = 0; j < S::NB2; ++j) val += C[j] * f2[j];
                    rmin = fmin(rmin, val);
                }
            }
    }
    const double rm = (double)rmin;
    int bad = 0;
    bool changed = false;
    if (!(mean > fl)) {
        bad = active ? 1 : 0;
    } else if (rm < target) {
        const T theta = (T)((mean - target) / (mean - rm));
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int l = 1; l < NB; ++l) U[v][l] *= theta;
        changed = true;
    }
    if (bad) atomicOr(a.fail, 1);
    if (a.nlim) {
        double cnt[1] = {(double)bad};
        block_sum<1>(cnt, lds);
        if (threadIdx.x == 0 && cnt[0] > 0.0) atomicAdd((unsigned long long *)a.nlim, (unsigned long long)cnt[0]);
    }
    return changed;
}

// What follows the combination in every stage: the limiter, the new weights, their density
// copy and their projected velocity (with the time-step maxima when a.part is set).  SPLIT:
// project one velocity component at a time (fewer live registers; the same bits).
template <typename T, int K, bool SPLIT = split_projection<T>()>
__device__ __forceinline__ void stage_finish(T (&U)[4][Shape<K>::NB], ctab<T> *tab, const StageArgs &a, unsigned bo,
                                             int c, bool active, int blk, double *lds)
{
    constexpr int NB = Shape<K>::NB;
    const int nc = a.g.nc;
    if (a.flags & F_LIMIT) stage_limit<T, K>(U, tab, a, active, lds);
    if (active) store_field<T, K, 4>(Field<T, 4>(a.out, NB, nc), bo, U);
    if (a.rho_out && active)
#pragma unroll
        for (int l = 0; l < NB; ++l) ((T *)a.rho_out)[(size_t)l * nc + c] = U[0][l];
    if (a.vh_out) project_and_bounds<T, K, SPLIT>(U, tab, a.vh_out, nc, bo, c, active, a.pa, a.part, blk, lds);
}

// out = ca*un + cb*ui + cc*dt*R with R = L - abar W_rho (one stage of an SSP Runge-Kutta
// scheme in Shu-Osher form), optionally a side combination w = wa*w_src + wb*ui + wc*dt*R
// of the same operands, then the positivity limiter (Sec. 3.1; target minimum
// max(floor, rel * mean)) with FP64 comparisons, then the projected velocity of the
// result for the next stage.
// occupancy of the stage kernel (waves per SIMD), pinned at what its registers allow so that
// small code changes cannot silently drop a wave (FP64 at degree 2: 128 VGPRs for 4 waves)
template <typename T, int K>
constexpr int stage_waves() { return sizeof(T) == 8 ? (K == 1 ? 7 : (K == 2 ? 4 : 2)) : (K == 1 ? 7 : (K == 2 ? 5 : 3)); }

template <typename T, int K, bool UNV, bool SIDE>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(stage_waves<T, K>()))) k_stage(StageArgs a)
{
    using S = Shape<K>;
    constexpr int NB = S::NB;
    __shared__ double lds[4];
    __shared__ double lds_ab[20];
    const int nc = a.g.nc;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int c0 = blk * BLOCK + threadIdx.x;
    const bool active = c0 < nc;
    // With the side combination, lanes past the mesh take its last cell: in the wave that holds
    // that cell they read, form and store exactly what its own lane does (every load of the
    // wave before its store), so the side combination is stored without a per-lane branch,
    // which made the compiler spill (233 VGPRs in FP64 at degree 3); a wave with no cell of the
    // mesh leaves the combination out.
    const int c = active ? c0 : (SIDE ? nc - 1 : 0);
    const unsigned bo = (unsigned)c * sizeof(T);
    ctab<T> *tab = as_tab<T>(a.tab);

    // the last stage writes the caller's state: nothing at all once the step has failed (the
    // flag is final here: earlier stages and this stage's right-hand side have raised it)
    if (a.skip_flag && *a.skip_flag) return;
    T U[4][NB];
    load_field<T, K, 4>(Field<T, 4>(a.ui, NB, nc), bo, U);
    if (a.L) {
        const Field<T, 4> LF(a.L, NB, nc);
        const Field<T, 4> UN(a.un, NB, nc);
        const double dt = a.dt_dev ? *a.dt_dev : a.dt;
        const T ca = (T)a.ca, cb = (T)a.cb, cdt = (T)(a.cc * dt);
        T ab[3];
        stage_abar<T>(a, ab, lds_ab);
        const Field<T, 4> WS(SIDE ? a.w_src : a.ui, NB, nc);
        const Field<T, 4> WO(SIDE ? a.w_out : a.ui, NB, nc);
        const T wa = (T)a.wa, wb = (T)a.wb, wcdt = (T)(a.wc * dt);
        const bool wave_has_cell = __builtin_amdgcn_ballot_w64(active) != 0;
        // The combination of every weight, momentum first (the removed mean acceleration
        // multiplies the input density).  Whether u^n and the side combination enter is a
        // template choice (UNV, SIDE): with a branch per weight the compiler waited for each
        // weight's loads in turn.  The roundings are those of the combination k_rhs forms for a split stage.
        // Weights in chunks of CH, each chunk's loads issued together before its arithmetic:
        // with a whole variable's right-hand side and u^n in flight the FP64 kernel at degree 2
        // does not fit its registers (128 VGPRs for 4 waves), and the compiler then issued one
        // load at a time, each waiting for the last.  At degree 3 (2 waves) a whole variable's
        // loads fit and go out together (chunks of 5 measured 1 % slower per step).
        constexpr int CH = (sizeof(T) == 8 && K == 2) ? 5 : NB;
        if constexpr (!SIDE) {
#pragma unroll
            for (int v = 3; v >= 0; --v)
#pragma unroll
                for (int l0 = 0; l0 < NB; l0 += CH) {
                    // the right-hand side and u^n are read once (non-temporal)
                    T rl[CH], nl[UNV ? CH : 1];
#pragma unroll
                    for (int j = 0; j < CH; ++j)
                        if (l0 + j < NB) {
                            rl[j] = LF.get_nt(v, l0 + j, bo);
                            if constexpr (UNV) nl[j] = UN.get_nt(v, l0 + j, bo);
                        }
#pragma unroll
                    for (int j = 0; j < CH; ++j)
                        if (l0 + j < NB) {
                            const int l = l0 + j;
                            T rhs = rl[j];
                            if (v > 0) rhs = fma(-ab[v - 1], U[0][l], rhs);
                            const T ui = U[v][l];
                            // stage_value, written out: u^n is loaded only where it enters
                            const T x = fma(cdt, rhs, cb * ui);
                            if constexpr (UNV) U[v][l] = fma(ca, nl[j], x);
                            else U[v][l] = x;
                        }
                    __builtin_amdgcn_sched_barrier(0);
                }
        } else if (wave_has_cell) {
            // The same with the side combination stored as it is formed.  The loads of a chunk
            // of weights come before its stores: the compiler cannot tell that the side
            // combination's array does not overlap the other inputs, so a load placed after a
            // store was issued only once the store's own loads had returned.  Chunks of 5 in
            // FP64 from degree 2 (the third operand does not fit otherwise).
            constexpr int CS = (sizeof(T) == 8 && K >= 2) ? 5 : NB;
#pragma unroll
            for (int v = 3; v >= 0; --v)
#pragma unroll
                for (int l0 = 0; l0 < NB; l0 += CS) {
                    T rl[CS], wl[CS], nl[UNV ? CS : 1];
#pragma unroll
                    for (int j = 0; j < CS; ++j)
                        if (l0 + j < NB) {
                            rl[j] = LF.get_nt(v, l0 + j, bo);
                            wl[j] = WS.get(v, l0 + j, bo);
                            if constexpr (UNV) nl[j] = UN.get_nt(v, l0 + j, bo);
                        }
#pragma unroll
                    for (int j = 0; j < CS; ++j)
                        if (l0 + j < NB) {
                            const int l = l0 + j;
                            T rhs = rl[j];
                            if (v > 0) rhs = fma(-ab[v - 1], U[0][l], rhs);
                            const T ui = U[v][l];
                            WO.put(v, l, bo, wa * wl[j] + wb * ui + wcdt * rhs);
                            const T x = fma(cdt, rhs, cb * ui);
                            if constexpr (UNV) U[v][l] = fma(ca, nl[j], x);
                            else U[v][l] = x;
                        }
                    __builtin_amdgcn_sched_barrier(0);
                }
        }
    }
    stage_finish<T, K>(U, tab, a, bo, c, active, blk, lds);
}

// The combination of a stage formed in the right-hand-side kernel (k_rhs with COMB): k_stage's
// u^(i+1) = ca un + cb ui + cdt (L - abar W_rho) for the cell whose right-hand side the kernel
// has just formed, with 4h dw/dt in L (it becomes the new weights) in place of the stored
// right-hand side and the same roundings, stored into st.out unlimited.  k_limit_project then
// limits and projects the result, so that the two kernels write the bits of the separate
// right-hand side and stage kernels.  The input weights are read again (they are not kept
// through the surface integral).  Every thread of the block calls it.
template <typename T, int K, bool UNV>
__device__ __forceinline__ void rhs_combination(const void *ui, T (&L)[4][Shape<K>::NB], T inv4h, double dt,
                                            const StageArgs &st, bool active, unsigned bo, double *lds)
{
    constexpr int NB = Shape<K>::NB;
    const int nc = st.g.nc;
    T ab[3];
    stage_abar<T>(st, ab, lds);
    const Field<T, 4> UI(ui, NB, nc);
    const Field<T, 4> UN(st.un, NB, nc);
    const T ca = (T)st.ca, cb = (T)st.cb, cdt = (T)(st.cc * dt);
    const Field<T, 4> UO(st.out, NB, nc);
    T R0[NB];
#pragma unroll
    for (int l = 0; l < NB; ++l) R0[l] = UI.get(0, l, bo);
    // variable by variable, each stored as soon as it is formed (its registers are free then).
    // All of a variable's loads come before its stores: the compiler cannot tell that the output
    // does not overlap the inputs, so a load placed after a store was issued only once the
    // store's own load had returned (one memory latency per weight).
#pragma unroll
    for (int v = 3; v >= 0; --v) {
        T ui[NB], un[UNV ? NB : 1];
#pragma unroll
        for (int l = 0; l < NB; ++l) {
            ui[l] = v ? UI.get_nt(v, l, bo) : R0[l];
            if constexpr (UNV) un[l] = UN.get_nt(v, l, bo);
        }
#pragma unroll
        for (int l = 0; l < NB; ++l) {
            // the value the separate right-hand side stores
            T rhs = L[v][l] * inv4h;
            if (v > 0) rhs = fma(-ab[v - 1], R0[l], rhs);
            const T x = fma(cdt, rhs, cb * ui[l]);
            T w;
            if constexpr (UNV) w = fma(ca, un[l], x);
            else w = x;
            if (active) UO.put(v, l, bo, w);
            // a last stage's failure, from its mean density as the stage kernel's limiter
            // decides it (Sec. 3.1: a cell whose mean is at or below the floor cannot be limited)
            if (v == 0 && l == 0 && st.fail_on_mean && active && !((double)w > st.rho_floor)) atomicOr(st.fail, 1);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// The rest of a stage whose combination the right-hand-side kernel has stored (a.out,
// unlimited): the positivity limiter in place (a cell is written back only where it changes),
// the projected velocity of the result (a.vh_out; project_cell's arithmetic, all three
// components in one pass over the points), and with DRIVE the mean-acceleration partials of the
// result for the next stage (block b: cells b BLOCK + t), in the modal form the right-hand
// side uses (driving table in the pencil form).
#ifndef LP_W64K2D
#define LP_W64K2D 3
#endif
template <typename T, int K, bool DRIVE>
constexpr int limit_project_waves()
{
    return sizeof(T) == 8 ? (K == 1 ? (DRIVE ? 5 : 6) : (K == 2 ? (DRIVE ? LP_W64K2D : 3) : 2))
                          : (K == 1 ? 7 : (K == 2 ? 5 : 3));
}

template <typename T, int K, bool DRIVE>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(limit_project_waves<T, K, DRIVE>())))
k_limit_project(StageArgs a)
{
    using S = Shape<K>;
    using TL = TabLayout<K>;
    constexpr int NB = S::NB;
    __shared__ double lds[16];
    const int nc = a.g.nc;
    const int blk = blockIdx.x;
    const int c0 = blk * BLOCK + threadIdx.x;
    const bool active = c0 < nc;
    const int c = active ? c0 : 0;
    const unsigned bo = (unsigned)c * sizeof(T);
    ctab<T> *tab = as_tab<T>(a.tab);
    const Field<T, 4> UO(a.out, NB, nc);
    T U[4][NB];
    load_field<T, K, 4>(UO, bo, U);
    if (a.flags & F_LIMIT) {
        const bool changed = stage_limit<T, K>(U, tab, a, active, lds);
        if (changed && active) store_field<T, K, 4>(UO, bo, U);
    }
    T V[3][NB];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int l = 0; l < NB; ++l) V[d][l] = T(0);
#pragma unroll 1
    for (int q = 0; q < S::NQ; ++q) {
        ctab<T> *ph = tab + TL::VPHI + q * NB;
        T rho = T(0), m0 = T(0), m1 = T(0), m2 = T(0);
#pragma unroll
        for (int l = 0; l < NB; ++l) {
            const T p = ph[l];
            rho += U[0][l] * p;
            m0 += U[1][l] * p;
            m1 += U[2][l] * p;
            m2 += U[3][l] * p;
        }
        const T ir = rcp(rho);
        const T v0 = m0 * ir, v1 = m1 * ir, v2 = m2 * ir;
        const T wq = T(0.125) * tab[TL::VW + q];
        const T a0 = wq * v0, a1 = wq * v1, a2 = wq * v2;
#pragma unroll
        for (int l = 0; l < NB; ++l) {
            const T p = ph[l];
            V[0][l] += a0 * p;
            V[1][l] += a1 * p;
            V[2][l] += a2 * p;
        }
    }
    if (active) store_field<T, K, 3>(Field<T, 3>(a.vh_out, NB, nc), bo, V);
    if constexpr (DRIVE) {
        double acc[4];
        T fs[3];
        drive_moment_sums<T, K>(U[0], as_tab<T>(a.ftab), a.g, c, active, fs);
        drive_partial<T>(fs, U[0][0], active, acc);
        block_sum<4>(acc, lds);
        if (threadIdx.x == 0)
#pragma unroll
            for (int i = 0; i < 4; ++i) a.drive_part[blk * 4 + i] = acc[i];
    }
}

// Per-block partial sums of the removed mean acceleration of a state alone (Sec. 4.2,
// mean-free driving): the cell's driving source rho w_q a summed over the volume points (times
// 1/8) and its mean density, at the block index the right-hand-side kernel uses (block b holds
// cells b BLOCK + t): in the modal form of the pencil table (drive_moment_sums, as
// k_limit_project forms them), or for tables off the driving shell with the right-hand side's
// own point sums (drive_sums_direct).  A split stage needs the mean of its input before its
// kernel has formed any right-hand side: this kernel runs first.  a.fail_reset: the failure
// flag to clear, or NULL.
template <typename T, int K, bool FDIRECT>
__global__ void __launch_bounds__(BLOCK) k_drive_parts(RhsArgs a)
{
    constexpr int NB = Shape<K>::NB;
    __shared__ double lds[16];
    const int nc = a.g.nc;
    const int blk = blockIdx.x;
    const int c0 = blk * BLOCK + threadIdx.x;
    const bool active = c0 < nc;
    const int c = active ? c0 : 0;
    if (a.fail_reset && blk == 0 && threadIdx.x == 0) *a.fail_reset = 0;
    const unsigned bo = (unsigned)c * sizeof(T);
    const Field<T, 1> U(a.u, NB, nc);
    T W0[NB];
#pragma unroll
    for (int l = 0; l < NB; ++l) W0[l] = U.get(0, l, bo);
    double acc[4];
    if constexpr (FDIRECT) {
        drive_sums_direct<T, K>(W0, as_tab<T>(a.tab), a.modes, a.nmodes, a.g, a.h, c, active, acc);
    } else {
        T fs[3];
        drive_moment_sums<T, K>(W0, as_tab<T>(a.ftab), a.g, c, active, fs);
        drive_partial<T>(fs, W0[0], active, acc);
    }
    block_sum<4>(acc, lds);
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < 4; ++i) a.part[blk * 4 + i] = acc[i];
}

// ------------------------------------------------------------ projection kernel

// vhat of u and, optionally, the per-block time-step maxima and a reset of the failure flag
template <typename T, int K>
__global__ void __launch_bounds__(BLOCK) k_project(const void *u_, void *vh_, const void *tab_, Mesh g, ProjArgs pa,
                                                   double *part, int *fail, void *rho_out)
{
    using S = Shape<K>;
    constexpr int NB = S::NB;
    __shared__ double lds[4];
    const int nc = g.nc;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int c0 = blk * BLOCK + threadIdx.x;
    const bool active = c0 < nc;
    const int c = active ? c0 : 0;
    const unsigned bo = (unsigned)c * sizeof(T);
    if (fail && blockIdx.x == 0 && threadIdx.x == 0) *fail = 0;
    ctab<T> *tab = as_tab<T>(tab_);
    T W[4][NB];
    load_field<T, K, 4>(Field<T, 4>(u_, NB, nc), bo, W);
    if (rho_out && active)
#pragma unroll
        for (int l = 0; l < NB; ++l) ((T *)rho_out)[(size_t)l * nc + c] = W[0][l];
    project_and_bounds<T, K>(W, tab, vh_, nc, bo, c, active, pa, part, blk, lds);
}

// Pencil table of the driving field (see PencilLayout): one thread per pencil and (t_y, t_z)
// point pair; the header (thread 0) holds (cos, sin)(pi xi_t h).  Modes with n_x < 0 enter as
// their conjugates; their y-z phase is evaluated directly, so n_y and n_z may be any reals.
// Only tables whose every n_x is an integer in [-2, 2] take this form.
template <typename T, int K>
__global__ void __launch_bounds__(BLOCK) k_forcing_pencils(void *ft_, const double *modes, int nmodes,
                                                           const void *tab_, Mesh g, double h)
{
    using TL = TabLayout<K>;
    using PL = PencilLayout<K>;
    constexpr int N1 = PL::N1;
    ctab<T> *tab = as_tab<T>(tab_);
    T *ft = (T *)ft_;
    const long long t = (long long)blockIdx.x * BLOCK + threadIdx.x;
    const long long nt = (long long)g.ny * g.nz * N1 * N1;
    if (t == 0)
        for (int k = 0; k < N1; ++k) {
            double sp, cp;
            sincospi((double)tab[TL::VXI + 3 * k] * h, &sp, &cp);      // xi of the 1D point k
            ft[2 * k] = (T)cp;
            ft[2 * k + 1] = (T)sp;
        }
    if (t < g.nx) {
        double sp, cp;
        sincospi(2.0 * ((double)t + 0.5) * h, &sp, &cp);
        T *px = ft + PL::phases(g.ny, g.nz);
        px[2 * t] = (T)cp;
        px[2 * t + 1] = (T)sp;
    }
    if (t >= nt) return;
    const int pen = (int)(t / (N1 * N1)), tt = (int)(t % (N1 * N1));
    const int j = pen % g.ny, l = pen / g.ny;
    const int ty = tt % N1, tz = tt / N1;
    const double y = (j + 0.5 + 0.5 * (double)tab[TL::VXI + 3 * ty]) * h;
    const double z = (l + 0.5 + 0.5 * (double)tab[TL::VXI + 3 * tz]) * h;
    double G[3][5] = {};
    for (int m = 0; m < nmodes; ++m) {
        const double *e = modes + 9 * m;
        const double sg = e[0] < 0.0 ? -1.0 : 1.0;       // conjugate term for n_x < 0
        const int nx = (int)(sg * e[0]);
        double sp, cp;
        sincospi(2.0 * sg * (e[1] * y + e[2] * z), &sp, &cp);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double ar = e[3 + 2 * d], ai = sg * e[4 + 2 * d];
            const double cr = ar * cp - ai * sp, ci = ar * sp + ai * cp;
            G[d][0] += nx == 0 ? cr : 0.0;
            G[d][1] += nx == 1 ? cr : 0.0;
            G[d][2] += nx == 1 ? ci : 0.0;
            G[d][3] += nx == 2 ? cr : 0.0;
            G[d][4] += nx == 2 ? ci : 0.0;
        }
    }
    T *o = ft + PL::HDR + (size_t)pen * PL::STRIDE + tt * PL::ENT;
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int k = 0; k < 5; ++k) o[5 * d + k] = (T)G[d][k];
    o[15] = T(0);
}

// The moments of the pencil form (see PencilLayout), from the pencil values k_forcing_pencils
// has written: one thread per pencil, 2D mode j and component d; thread 0 also writes the x
// factors.  Sums in FP64 over the table values, stored in the element type.
template <typename T, int K>
__global__ void __launch_bounds__(BLOCK) k_forcing_moments(void *ft_, const void *tab_, Mesh g)
{
    using TL = TabLayout<K>;
    using PL = PencilLayout<K>;
    using S = Shape<K>;
    constexpr int N1 = PL::N1;
    ctab<T> *tab = as_tab<T>(tab_);
    T *ft = (T *)ft_;
    const long long t = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (t == 0) {
        T *sx = ft + PL::xfactors(g.nx, g.ny, g.nz);
        for (int a = 0; a <= K; ++a) {
            double s0 = 0.0, s1r = 0.0, s1i = 0.0, s2r = 0.0, s2i = 0.0;
            for (int p = 0; p < N1; ++p) {
                const double wl = (double)tab[TL::WLT + p * (K + 1) + a];
                const double er = (double)ft[2 * p], ei = (double)ft[2 * p + 1];
                s0 += wl;
                s1r += wl * er;
                s1i += wl * ei;
                s2r += wl * (er * er - ei * ei);
                s2i += wl * (2.0 * er * ei);
            }
            sx[5 * a] = (T)s0;
            sx[5 * a + 1] = (T)s1r;
            sx[5 * a + 2] = (T)s1i;
            sx[5 * a + 3] = (T)s2r;
            sx[5 * a + 4] = (T)s2i;
        }
    }
    const long long nt = (long long)g.ny * g.nz * PL::NB2 * 3;
    if (t >= nt) return;
    const int pen = (int)(t / (PL::NB2 * 3)), r = (int)(t % (PL::NB2 * 3));
    const int j = r / 3, d = r % 3;
    const T *gp = ft + PL::HDR + (size_t)pen * PL::STRIDE;
    double cm[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int tt = 0; tt < S::NF; ++tt) {
        const double w = (double)tab[TL::FW + tt] * (double)tab[TL::F2 + tt * S::NB2 + j];
        const T *e = gp + tt * PL::ENT + 5 * d;
#pragma unroll
        for (int k = 0; k < 5; ++k) cm[k] += w * (double)e[k];
    }
    T *o = ft + PL::moments(g.nx, g.ny, g.nz) + (size_t)pen * PL::MST + (j * 3 + d) * 5;
#pragma unroll
    for (int k = 0; k < 5; ++k) o[k] = (T)cm[k];
}

// per-block sums of the cell means (conservation totals, Sec. 2.2: w_0 is the mean)
template <typename T, int K>
__global__ void __launch_bounds__(BLOCK) k_sums(const void *u_, Mesh g, double *part)
{
    constexpr int NB = Shape<K>::NB;
    __shared__ double lds[16];
    const int nc = g.nc;
    const int c0 = blockIdx.x * BLOCK + threadIdx.x;
    const bool active = c0 < nc;
    const int c = active ? c0 : 0;
    const T *u = (const T *)u_;
    double v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = active ? (double)u[(i * NB) * (size_t)nc + c] : 0.0;
    block_sum<4>(v, lds);
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < 4; ++i) part[blockIdx.x * 4 + i] = v[i];
}

// single-block fixed-order reductions of per-block partials
// mode 0: out[i] = scale * sum part[.][i], i < 4
// mode 1: out[0..2] = sum part[.][0..2] / sum part[.][3]   (mass-weighted mean acceleration)
// mode 2: out[0] = min(scale / max part[.][0], scale2 / max part[.][1])   (time step; the
//         second term only when scale2 > 0 and the maximum is positive); the second
//         maximum also runs over part2[0 .. np2) when part2 is not null
// Publication (mode 2, pub != null): the time step and the step's failure flag are also
// stored into pub (pinned host memory: pub[1] = the bits of dt, pub[2] = *fail), and then
// pub[0] = seq, each store made visible to the host before the next; the host waits for
// pub[0] == seq instead of copying the values back and synchronising the stream.  The flag
// is also kept in out[1] (device memory), because a stage launched behind this kernel may
// clear *fail before the host reads it.
static __global__ void __launch_bounds__(BLOCK) k_final(const double *part, int np, int mode, double scale, double scale2,
                                                 double *out, const int *fail, volatile long long *pub,
                                                 long long seq, const double *part2, int np2)
{
    __shared__ double lds[16];
    if (mode == 2) {
        double m = 0.0, n = 0.0;
#pragma unroll 16
        for (int i = threadIdx.x; i < np; i += BLOCK) {
            m = fmax(m, part[2 * i]);
            n = fmax(n, part[2 * i + 1]);
        }
        if (part2)
            for (int i = threadIdx.x; i < np2; i += BLOCK) n = fmax(n, part2[i]);
        m = block_max(m, lds);
        __syncthreads();
        n = block_max(n, lds);
        if (threadIdx.x == 0) {
            double dt = scale / m;
            if (scale2 > 0.0 && n > 0.0) dt = fmin(dt, scale2 / n);
            out[0] = dt;
            if (pub) {
                const int f = *fail;
                out[1] = (double)f;
                pub[1] = __double_as_longlong(dt);
                pub[2] = f;
                __threadfence_system();
                pub[0] = seq;
                __threadfence_system();
            }
        }
        return;
    }
    double s[4];
    block_partial_sums4<16>(part, np, s, lds);
    if (threadIdx.x == 0) {
        if (mode == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) out[k] = scale * s[k];
        } else {
            out[0] = s[0] / s[3];
            out[1] = s[1] / s[3];
            out[2] = s[2] / s[3];
        }
    }
}

// *f = 0 (a flag cleared on the stream, without a memset node)
static __global__ void k_clear_flag(int *f) { *f = 0; }

// dudt_m -= abar W_rho (mean-free driving applied to a stand-alone right-hand side)
template <typename T, int K>
__global__ void __launch_bounds__(BLOCK) k_meanfree(const void *u_, void *dudt_, const double *abar, int nc)
{
    constexpr int NB = Shape<K>::NB;
    const int c = blockIdx.x * BLOCK + threadIdx.x;
    if (c >= nc) return;
    const T *u = (const T *)u_;
    T *o = (T *)dudt_;
    const T ab[3] = {(T)abar[0], (T)abar[1], (T)abar[2]};
    // every load before the first store: o and u may overlap as far as the compiler can tell,
    // so a load placed after a store was issued only once that store's value had arrived
    T r[NB], x[3][NB];
#pragma unroll
    for (int l = 0; l < NB; ++l) r[l] = u[l * (size_t)nc + c];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int l = 0; l < NB; ++l) x[d][l] = o[((1 + d) * NB + l) * (size_t)nc + c];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int l = 0; l < NB; ++l) o[((1 + d) * NB + l) * (size_t)nc + c] = x[d][l] - ab[d] * r[l];
}

}  // namespace dg
