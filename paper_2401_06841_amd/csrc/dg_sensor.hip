// dg_sensor.hip -- learned shock sensor: per-cell features, plain-sensor labels, the
// 20-64-64-1 GELU network on the bf16 matrix cores (forward, gradient, Adam) and the
// judge that sends cells back to the plain sensor.  The network is not in the paper; it
// stands in for the compression sensor of Sec. 3.1 and is trained on that sensor's output.
//
// Matrix-core mapping (v_mfma_f32_16x16x32_bf16, one wave64 per 16-row tile): lane
// 16 g + i holds A[i][8g .. 8g+7], B[8g .. 8g+7][i] and accumulates D[4g .. 4g+3][i].
// Activations are rounded to bf16 only where they feed a matrix instruction; bias, GELU,
// the last layer and all accumulations are FP32.  Gradients are reduced per wave, then
// summed over waves in a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "dg.h"
#include "dg_ctx.hpp"
#include "dg_kernels.hpp"

namespace dg {

constexpr int NIN = DG_MLP_NIN, NH = DG_MLP_NHID, NPARAM = DG_MLP_NPARAM;
constexpr int OFF_W1 = 0, OFF_B1 = NH * NIN, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH;
constexpr int MLP_WAVES = MLP_PART_ROWS;  // waves of the gradient kernel: one per SIMD at its occupancy of 1
constexpr double NU0 = 1e-3;            // nu scale of the target t = log(1 + nu/nu0)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_d(float z)
{
    const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
    return cdf + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void wave_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// sum over the 16 lanes of a lane group (same g)
__device__ __forceinline__ float group_sum(float v)
{
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// sum over the 4 lane groups (same i)
__device__ __forceinline__ float across_groups(float v)
{
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

// network weights of one wave in matrix-operand form
struct Net {
    bf16x8 b1[4];        // layer 1, tile t: W1[16t+i][8g+j] (k >= 20: 0)
    bf16x8 b2[2][4];     // layer 2, (k-step s, tile t): W2[16t+i][32s+8g+j]
    float bias1[4], bias2[4], w3[4];
    float b3;
};

__device__ __forceinline__ void load_net(const float *__restrict__ P, Net &w)
{
    const int lane = threadIdx.x & 63, i = lane & 15, g = lane >> 4;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = 8 * g + j;
            w.b1[t][j] = (__bf16)(k < NIN ? P[OFF_W1 + (16 * t + i) * NIN + k] : 0.0f);
        }
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int j = 0; j < 8; ++j) w.b2[s][t][j] = (__bf16)P[OFF_W2 + (16 * t + i) * NH + 32 * s + 8 * g + j];
        w.bias1[t] = P[OFF_B1 + 16 * t + i];
        w.bias2[t] = P[OFF_B2 + 16 * t + i];
        w.w3[t] = P[OFF_W3 + 16 * t + i];
    }
    w.b3 = P[OFF_B3];
}

// per-wave LDS scratch of one tile (bf16)
struct alignas(16) TileLds {
    __bf16 h1[16 * NH];     // H1 row-major [row][n]
    __bf16 h1t[NH * 16];    // H1 transposed [n][row]
    __bf16 g2[16 * NH];     // G2 row-major
    __bf16 g2t[NH * 16];    // G2 transposed
    __bf16 g1t[NH * 16];    // G1 transposed
    __bf16 xt[32 * 16];     // X transposed [m][row] (m >= 20: 0)
};

// forward pass of the 16-row tile starting at row0 (rows >= n are zero inputs).
// z1, z2: pre-activations in the D layout (rows 4g+j, column 16t+i); y[j]: output of row
// 4g+j (valid in every lane of the group).
__device__ __forceinline__ void forward_tile(const float *__restrict__ x, int row0, int n, const Net &w, TileLds &L,
                                             bool keep, float (&z1)[4][4], float (&z2)[4][4], float (&y)[4])
{
    const int lane = threadIdx.x & 63, i = lane & 15, g = lane >> 4;
    const int r = row0 + i;
    bf16x8 a;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int k = 8 * g + j;
        const float v = (r < n && k < NIN) ? x[(size_t)r * NIN + k] : 0.0f;
        a[j] = (__bf16)v;
        if (keep) L.xt[(8 * g + j) * 16 + i] = (__bf16)v;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f32x4 d = mfma(a, w.b1[t], f32x4{0.0f, 0.0f, 0.0f, 0.0f});
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            z1[t][j] = d[j] + w.bias1[t];
            const __bf16 h = (__bf16)gelu(z1[t][j]);
            L.h1[(4 * g + j) * NH + 16 * t + i] = h;
            if (keep) L.h1t[(16 * t + i) * 16 + 4 * g + j] = h;
        }
    }
    wave_fence();
    bf16x8 a2[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) a2[s] = *(const bf16x8 *)&L.h1[i * NH + 32 * s + 8 * g];
    float p[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f32x4 d = mfma(a2[0], w.b2[0][t], f32x4{0.0f, 0.0f, 0.0f, 0.0f});
        d = mfma(a2[1], w.b2[1][t], d);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            z2[t][j] = d[j] + w.bias2[t];
            p[j] += gelu(z2[t][j]) * w.w3[t];
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) y[j] = group_sum(p[j]) + w.b3;
    wave_fence();
}

// ------------------------------------------------------------------ forward
// y[n] from x[n][20]; with nu != nullptr the output is the viscosity
// nu = nu0 (exp(y) - 1), clipped at zero, stored in the state's element type.  With vmax
// != nullptr each block also writes vmax[block] = the largest stored viscosity of its cells
// whose fallback flag fb is 0 (0 if none): the learned cells' part of the viscous time-step
// bound.
template <typename T>
__global__ void __launch_bounds__(256) k_mlp_forward(const float *__restrict__ P, const float *__restrict__ x, int n,
                                                     float *__restrict__ y, T *__restrict__ nu,
                                                     const int *__restrict__ fb, double *__restrict__ vmax)
{
    __shared__ double bmax[4];
    double vm = 0.0;
    __shared__ TileLds lds[4];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, i = lane & 15, g = lane >> 4;
    Net w;
    load_net(P, w);
    const int ntile = (n + 15) / 16;
    const int nw = gridDim.x * 4;
    for (int tile = blockIdx.x * 4 + wave; tile < ntile; tile += nw) {
        float z1[4][4], z2[4][4], yy[4];
        forward_tile(x, tile * 16, n, w, lds[wave], false, z1, z2, yy);
        if (i == 0) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = tile * 16 + 4 * g + j;
                if (r >= n) continue;
                if (y) y[r] = yy[j];
                if (nu) {
                    const T v = (T)fmax(NU0 * expm1((double)yy[j]), 0.0);
                    nu[r] = v;
                    if (vmax && fb[r] == 0) vm = fmax(vm, fmax((double)v, 0.0));
                }
            }
        }
    }
    if (vmax) {
        vm = wave_max(vm);
        if (lane == 0) bmax[wave] = vm;
        __syncthreads();
        if (threadIdx.x == 0) vmax[blockIdx.x] = fmax(fmax(bmax[0], bmax[1]), fmax(bmax[2], bmax[3]));
    }
}

// --------------------------------------------------------------- gradient
// Mean-squared-error loss L = (1/n) sum (y - t)^2 and dL/dparams; each wave writes its
// partial sums to part[wave][NPARAM + 1] (the last entry is the partial loss sum).
__global__ void __launch_bounds__(256) k_mlp_grad(const float *__restrict__ P, const float *__restrict__ x,
                                                  const float *__restrict__ tgt, int n, float *__restrict__ part)
{
    __shared__ TileLds lds[4];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, i = lane & 15, g = lane >> 4;
    const int gw = blockIdx.x * 4 + wave;
    const int nw = gridDim.x * 4;
    TileLds &L = lds[wave];
    Net w;
    load_net(P, w);
    // layer-2 weights as the B operand of G2 W2: W2[32s+8g+j][16t+i]
    bf16x8 bw2[2][4];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int j = 0; j < 8; ++j) bw2[s][t][j] = (__bf16)P[OFF_W2 + (32 * s + 8 * g + j) * NH + 16 * t + i];

    f32x4 aw2[4][4], aw1[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int b = 0; b < 4; ++b) aw2[a][b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int b = 0; b < 2; ++b) aw1[a][b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    }
    float gb1[4] = {0, 0, 0, 0}, gb2[4] = {0, 0, 0, 0}, gw3[4] = {0, 0, 0, 0};
    float gb3 = 0.0f, loss = 0.0f;
    const float inv_n = 1.0f / (float)n;
    const int ntile = (n + 15) / 16;
    const bf16x8 zero8 = {};

    for (int tile = gw; tile < ntile; tile += nw) {
        float z1[4][4], z2[4][4], y[4];
        forward_tile(x, tile * 16, n, w, L, true, z1, z2, y);
        float g3[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = tile * 16 + 4 * g + j;
            const float e = r < n ? y[j] - tgt[r] : 0.0f;
            g3[j] = 2.0f * inv_n * e;
            if (i == 0) loss += e * e;
            if (i == 0) gb3 += g3[j];
        }
        // last layer and G2 = g3 W3 gelu'(z2)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                gw3[t] += g3[j] * gelu(z2[t][j]);
                const float v = g3[j] * w.w3[t] * gelu_d(z2[t][j]);
                gb2[t] += v;
                const __bf16 b = (__bf16)v;
                L.g2[(4 * g + j) * NH + 16 * t + i] = b;
                L.g2t[(16 * t + i) * 16 + 4 * g + j] = b;
            }
        wave_fence();
        // dW2[n][k] += sum_rows G2[row][n] H1[row][k]  (K = 16 rows, upper half zero)
        bf16x8 ag[4], bh[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            ag[t] = g < 2 ? *(const bf16x8 *)&L.g2t[(16 * t + i) * 16 + 8 * g] : zero8;
            bh[t] = g < 2 ? *(const bf16x8 *)&L.h1t[(16 * t + i) * 16 + 8 * g] : zero8;
        }
#pragma unroll
        for (int tn = 0; tn < 4; ++tn)
#pragma unroll
            for (int tk = 0; tk < 4; ++tk) aw2[tn][tk] = mfma(ag[tn], bh[tk], aw2[tn][tk]);
        // G1 = (G2 W2) gelu'(z1)
        bf16x8 a2[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) a2[s] = *(const bf16x8 *)&L.g2[i * NH + 32 * s + 8 * g];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            f32x4 d = mfma(a2[0], bw2[0][t], f32x4{0.0f, 0.0f, 0.0f, 0.0f});
            d = mfma(a2[1], bw2[1][t], d);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float v = d[j] * gelu_d(z1[t][j]);
                gb1[t] += v;
                L.g1t[(16 * t + i) * 16 + 4 * g + j] = (__bf16)v;
            }
        }
        wave_fence();
        // dW1[k][m] += sum_rows G1[row][k] X[row][m]
        bf16x8 bx[2];
#pragma unroll
        for (int tm = 0; tm < 2; ++tm) bx[tm] = g < 2 ? *(const bf16x8 *)&L.xt[(16 * tm + i) * 16 + 8 * g] : zero8;
#pragma unroll
        for (int tk = 0; tk < 4; ++tk) {
            const bf16x8 a1 = g < 2 ? *(const bf16x8 *)&L.g1t[(16 * tk + i) * 16 + 8 * g] : zero8;
#pragma unroll
            for (int tm = 0; tm < 2; ++tm) aw1[tk][tm] = mfma(a1, bx[tm], aw1[tk][tm]);
        }
        wave_fence();
    }
    // write this wave's partial gradient
    float *pw = part + (size_t)gw * (NPARAM + 1);
#pragma unroll
    for (int tn = 0; tn < 4; ++tn)
#pragma unroll
        for (int tk = 0; tk < 4; ++tk)
#pragma unroll
            for (int j = 0; j < 4; ++j) pw[OFF_W2 + (16 * tn + 4 * g + j) * NH + 16 * tk + i] = aw2[tn][tk][j];
#pragma unroll
    for (int tk = 0; tk < 4; ++tk)
#pragma unroll
        for (int tm = 0; tm < 2; ++tm)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int m = 16 * tm + i;
                if (m < NIN) pw[OFF_W1 + (16 * tk + 4 * g + j) * NIN + m] = aw1[tk][tm][j];
            }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const float s1 = across_groups(gb1[t]);
        const float s2 = across_groups(gb2[t]);
        const float s3 = across_groups(gw3[t]);
        if (g == 0) {
            pw[OFF_B1 + 16 * t + i] = s1;
            pw[OFF_B2 + 16 * t + i] = s2;
            pw[OFF_W3 + 16 * t + i] = s3;
        }
    }
    const float sb3 = across_groups(gb3);
    const float sl = across_groups(loss);
    if (lane == 0) {
        pw[OFF_B3] = sb3;
        pw[NPARAM] = sl;
    }
}

// fixed-order sum of the per-wave partials: grad[p] and loss = sum / n.  A block takes 64
// entries; its wave w sums the rows w, w+4, w+8, ... in order, and the four wave sums are
// added in wave order.
__global__ void __launch_bounds__(256) k_mlp_reduce(const float *__restrict__ part, int nwaves, int n,
                                                    float *__restrict__ grad, float *__restrict__ loss)
{
    __shared__ float lds[4][64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int p = blockIdx.x * 64 + lane;
    float s = 0.0f;
    if (p <= NPARAM)
#pragma unroll 8
        for (int wv = w; wv < nwaves; wv += 4) s += part[(size_t)wv * (NPARAM + 1) + p];
    lds[w][lane] = s;
    __syncthreads();
    if (w == 0 && p <= NPARAM) {
        const float t = ((lds[0][lane] + lds[1][lane]) + lds[2][lane]) + lds[3][lane];
        if (p < NPARAM) grad[p] = t;
        else loss[0] = t / (float)n;
    }
}

// Adam (Kingma & Ba 2015), beta1 0.9, beta2 0.999, eps 1e-8
__global__ void __launch_bounds__(256) k_mlp_adam(float *__restrict__ P, const float *__restrict__ G,
                                                  float *__restrict__ m, float *__restrict__ v, int step, float lr)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= NPARAM) return;
    const float b1 = 0.9f, b2 = 0.999f;
    const float gg = G[p];
    const float mm = b1 * m[p] + (1.0f - b1) * gg;
    const float vv = b2 * v[p] + (1.0f - b2) * gg * gg;
    m[p] = mm;
    v[p] = vv;
    const float mh = mm / (1.0f - powf(b1, (float)step));
    const float vh = vv / (1.0f - powf(b2, (float)step));
    P[p] -= lr * mh / (sqrtf(vh) + 1e-8f);
}

// ------------------------------------------------------------ features
// x[cell][20] (degree 2, modes in graded order 0:(000) 1:(100) 2:(010) 3:(001) 4:(200)
// 5:(110) 6:(101) 7:(020) 8:(011) 9:(002)):
//   [0..5]   density shape W_rho,l/W_rho,0 for l = 1, 2, 3, 4, 7, 9
//   [6]      log10 W_rho,0
//   [7..15]  cell-mean velocity gradient (2 sqrt(3)/h) vhat_{d,(e)}, scaled by (h/3)/cs
//   [16..18] slopes of div vhat across the cell: with d/dxi Lt_1 = sqrt(3) and
//            d/dxi Lt_2 = 3 sqrt(5) xi the divergence is D0 + sum_i D_i xi_i with
//            D_1 = 3 sqrt(5) V_x,(200) + 3 V_y,(110) + 3 V_z,(101) (and cyclic), times 2/h,
//            scaled by (h/3)/cs
//   [19]     |mean velocity|/cs
// vhat: the projected velocity of u already at hand (same arithmetic as project_cell), used
// unless *fail is raised (then u is not the state vhat belongs to); NULL: project here.
template <typename T>
__global__ void __launch_bounds__(BLOCK) k_features(const void *u_, float *__restrict__ x, const void *tab_, Mesh g,
                                                    double cs, const void *vhat, const int *fail)
{
    constexpr int K = 2, NB = Shape<K>::NB;
    const int nc = g.nc;
    const int c0 = blockIdx.x * BLOCK + threadIdx.x;
    const bool active = c0 < nc;
    const int c = active ? c0 : 0;
    const unsigned bo = (unsigned)c * sizeof(T);
    T W[4][NB];
    T V[3][NB];
    if (vhat && !*fail) {
#pragma unroll
        for (int l = 0; l < NB; ++l) W[0][l] = Field<T, 1>(u_, NB, nc).get(0, l, bo);
        load_field<T, K, 3>(Field<T, 3>(vhat, NB, nc), bo, V);
    } else {
        load_field<T, K, 4>(Field<T, 4>(u_, NB, nc), bo, W);
        project_cell<T, K>(W, as_tab<T>(tab_), V, nullptr, 0.0);
    }
    if (!active) return;
    const double r0 = (double)W[0][0];
    float *xc = x + (size_t)c * NIN;
    constexpr int dmode[6] = {1, 2, 3, 4, 7, 9};
#pragma unroll
    for (int i = 0; i < 6; ++i) xc[i] = (float)((double)W[0][dmode[i]] / r0);
    xc[6] = (float)log10(r0);
    const double fac = 2.0 * 1.7320508075688772 / (3.0 * cs);
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int e = 0; e < 3; ++e) xc[7 + 3 * d + e] = (float)(fac * (double)V[d][1 + e]);
    const double r5 = 3.0 * 2.23606797749979;     // 3 sqrt(5)
    const double sfac = 2.0 / (3.0 * cs);         // (h/3)/cs * 2/h
    xc[16] = (float)(sfac * (r5 * (double)V[0][4] + 3.0 * (double)V[1][5] + 3.0 * (double)V[2][6]));
    xc[17] = (float)(sfac * (3.0 * (double)V[0][5] + r5 * (double)V[1][7] + 3.0 * (double)V[2][8]));
    xc[18] = (float)(sfac * (3.0 * (double)V[0][6] + 3.0 * (double)V[1][8] + r5 * (double)V[2][9]));
    const double vm = sqrt((double)V[0][0] * V[0][0] + (double)V[1][0] * V[1][0] + (double)V[2][0] * V[2][0]);
    xc[19] = (float)(vm / cs);
}

// plain-sensor label: the vNR bulk viscosity nu(s) = alpha (h/p)^2 s + beta cs (h/p)
// (Pi = rho nu s without the cap, Sec. 3.1) averaged over the compressed interior points
// (s = -div v > 0) with weights omega s: nu = alpha (h/p)^2 sum(w s^2)/sum(w s) + beta cs h/p
// OUT = double: the label nu itself; OUT = float: the training target log(1 + nu/nu0)
template <typename T, int K, typename OUT>
__global__ void __launch_bounds__(BLOCK) k_labels(const void *u_, OUT *__restrict__ nu, const void *tab_, Mesh g,
                                                  double h, double cs, double alpha, double beta)
{
    using S = Shape<K>;
    using TL = TabLayout<K>;
    constexpr Modes<K> M = make_modes<K>();
    constexpr int NB = S::NB, ND = S::ND;
    const int nc = g.nc;
    const int c0 = blockIdx.x * BLOCK + threadIdx.x;
    const bool active = c0 < nc;
    const int c = active ? c0 : 0;
    const unsigned bo = (unsigned)c * sizeof(T);
    ctab<T> *tab = as_tab<T>(tab_);
    T W[4][NB];
    load_field<T, K, 4>(Field<T, 4>(u_, NB, nc), bo, W);
    T V[3][NB];
    project_cell<T, K>(W, tab, V, nullptr, 0.0);
    double s1 = 0.0, s2 = 0.0;
#pragma unroll 1
    for (int q = 0; q < S::NQ; ++q) {
        ctab<T> *dph = tab + TL::VDPHI + q * 3 * ND;
        T div = T(0);
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int l = 0; l < NB; ++l)
                if (M.dj[d][l] >= 0) div += V[d][l] * dph[d * ND + M.dj[d][l]];
        const double sq = -(double)div * (2.0 / h);
        if (sq > 0.0) {
            const double w = (double)tab[TL::VW + q];
            s1 += w * sq;
            s2 += w * sq * sq;
        }
    }
    if (!active) return;
    const double hp = h / (K + 1);
    const double v = s1 > 0.0 ? alpha * hp * hp * (s2 / s1) + beta * cs * hp : 0.0;
    if (sizeof(OUT) == 8) nu[c] = (OUT)v;
    else nu[c] = (OUT)log1p(v / NU0);
}

// judge: fallback flag where |nu_learned - nu_plain| / (nu_plain + nu0) > tau; counts the flags
template <typename T>
__global__ void __launch_bounds__(BLOCK) k_judge(const T *__restrict__ nul, const double *__restrict__ nup, int nc,
                                                 double tau, int *__restrict__ fb, unsigned long long *__restrict__ count)
{
    __shared__ double lds[4];
    const int c = blockIdx.x * BLOCK + threadIdx.x;
    int flag = 0;
    if (c < nc) {
        const double a = (double)nul[c], b = nup[c];
        flag = fabs(a - b) / (b + NU0) > tau ? 1 : 0;
        fb[c] = flag;
    }
    double v[1] = {(double)flag};
    block_sum<1>(v, lds);
    if (threadIdx.x == 0 && v[0] > 0.0) atomicAdd(count, (unsigned long long)v[0]);
}

__global__ void k_fill_int(int *__restrict__ p, int n, int value)
{
    const int c = blockIdx.x * BLOCK + threadIdx.x;
    if (c < n) p[c] = value;
}

}  // namespace dg

using namespace dg;

// gradient: at most MLP_WAVES waves, one partial-sum row each
static int mlp_blocks(int n)
{
    const int ntile = (n + 15) / 16;
    int nw = ntile < MLP_WAVES ? ntile : MLP_WAVES;
    return (nw + 3) / 4;
}

// forward: one full round of waves at the kernel's occupancy (3 waves per SIMD), each wave
// looping over its share of the 16-row tiles (the network is loaded into registers once per
// wave, and no wave waits for a second round)
static int fwd_blocks(const dg_ctx *c, int n)
{
    const long ntile = ((long)n + 15) / 16;
    const long round = (long)c->ncu * 4 * 3;
    const long nw = ntile < round ? ntile : round;
    return (int)((nw + 3) / 4);
}

static float *mlp_part(dg_ctx *c) { return (float *)c->wp(c->off.mlp); }

static int need_k2(dg_ctx *c)
{
    if (c->k != 2) return dg_fail(c, DG_EUNSUPPORTED, "the learned sensor is defined for degree 2");
    if (!c->ws) return dg_fail(c, DG_ENOMEM, "no workspace set (dg_set_workspace)");
    return DG_OK;
}

int dg_mlp_forward(dg_ctx *c, const float *P, const float *x, int n, float *y)
{
    if (!c) return DG_EINVAL;
    if (!P || !x || !y || n < 0) return dg_fail(c, DG_EINVAL, "bad network arguments");
    if (n == 0) return DG_OK;
    int rc;
    if ((rc = dg_check_array(c, P, sizeof(float) * NPARAM, sizeof(float), "params")) ||
        (rc = dg_check_array(c, x, sizeof(float) * NIN * (size_t)n, sizeof(float), "x")) ||
        (rc = dg_check_array(c, y, sizeof(float) * (size_t)n, sizeof(float), "y")))
        return rc;
    hipLaunchKernelGGL((k_mlp_forward<float>), dim3(fwd_blocks(c, n)), dim3(256), 0, c->stream, P, x, n, y,
                       (float *)nullptr, (const int *)nullptr, (double *)nullptr);
    LAUNCHCHK(c);
    return DG_OK;
}

int dg_mlp_grad(dg_ctx *c, const float *P, const float *x, const float *t, int n, float *grad, float *loss)
{
    if (!c) return DG_EINVAL;
    if (!P || !x || !t || !grad || !loss || n <= 0) return dg_fail(c, DG_EINVAL, "bad network arguments");
    if (dg_check_array(c, P, sizeof(float) * NPARAM, sizeof(float), "params") ||
        dg_check_array(c, x, sizeof(float) * NIN * (size_t)n, sizeof(float), "x") ||
        dg_check_array(c, t, sizeof(float) * (size_t)n, sizeof(float), "t") ||
        dg_check_array(c, grad, sizeof(float) * NPARAM, sizeof(float), "grad") ||
        dg_check_array(c, loss, sizeof(float), sizeof(float), "loss"))
        return DG_EINVAL;
    if (!c->ws) return dg_fail(c, DG_ENOMEM, "no workspace set (dg_set_workspace)");
    const int nb = mlp_blocks(n);
    hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(256), 0, c->stream, P, x, t, n, mlp_part(c));
    LAUNCHCHK(c);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((NPARAM + 1 + 63) / 64), dim3(256), 0, c->stream, (const float *)mlp_part(c),
                       nb * 4, n, grad, loss);
    LAUNCHCHK(c);
    return DG_OK;
}

int dg_mlp_adam(dg_ctx *c, float *P, const float *G, float *m, float *v, int step, float lr)
{
    if (!c) return DG_EINVAL;
    if (!P || !G || !m || !v || step < 1 || !(lr > 0.0f)) return dg_fail(c, DG_EINVAL, "bad Adam arguments");
    if (dg_check_array(c, P, sizeof(float) * NPARAM, sizeof(float), "params") ||
        dg_check_array(c, G, sizeof(float) * NPARAM, sizeof(float), "grad") ||
        dg_check_array(c, m, sizeof(float) * NPARAM, sizeof(float), "m") ||
        dg_check_array(c, v, sizeof(float) * NPARAM, sizeof(float), "v"))
        return DG_EINVAL;
    hipLaunchKernelGGL(k_mlp_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, c->stream, P, G, m, v, step, lr);
    LAUNCHCHK(c);
    return DG_OK;
}

int dg_sensor_set_params(dg_ctx *c, const float *P)
{
    if (!c) return DG_EINVAL;
    c->spec_valid = false;          // the viscosity or flags a launched next stage used change
    if (int rc = dg_check_array(c, P, sizeof(float) * NPARAM, sizeof(float), "params")) return rc;
    HIPCHK(c, hipMemcpyAsync(c->mlp_bf16, P, sizeof(float) * NPARAM, hipMemcpyDeviceToDevice, c->stream));
    c->have_params = true;
    return DG_OK;
}

static int launch_features(dg_ctx *c, const void *u, float *x, const void *vhat)
{
    const Mesh g{c->cfg.nx, c->cfg.ny, c->cfg.nz, c->nc};
    const int *fail = (const int *)c->fail();
    if (c->es == 8)
        hipLaunchKernelGGL((k_features<double>), dim3(c->nblk), dim3(BLOCK), 0, c->stream, u, x, c->tab, g, c->cfg.cs,
                           vhat, fail);
    else
        hipLaunchKernelGGL((k_features<float>), dim3(c->nblk), dim3(BLOCK), 0, c->stream, u, x, c->tab, g, c->cfg.cs,
                           vhat, fail);
    LAUNCHCHK(c);
    return DG_OK;
}

int dg_sensor_features(dg_ctx *c, const void *u, float *x)
{
    if (!c) return DG_EINVAL;
    int rc = need_k2(c);
    if (rc) return rc;
    if ((rc = dg_check_array(c, u, dg_state_bytes(c), c->es, "u")) ||
        (rc = dg_check_array(c, x, sizeof(float) * NIN * (size_t)c->nc, sizeof(float), "x")))
        return rc;
    return launch_features(c, u, x, nullptr);
}

template <typename T, int K, typename OUT>
static void launch_labels(dg_ctx *c, const void *u, OUT *nu)
{
    const Mesh g{c->cfg.nx, c->cfg.ny, c->cfg.nz, c->nc};
    hipLaunchKernelGGL((k_labels<T, K, OUT>), dim3(c->nblk), dim3(BLOCK), 0, c->stream, u, nu, c->tab, g, c->cfg.h,
                       c->cfg.cs, c->cfg.alpha_visc, c->cfg.beta_visc);
}

template <typename OUT>
static int labels_any(dg_ctx *c, const void *u, OUT *nu)
{
    if (!c) return DG_EINVAL;
    if (int rc = dg_check_array(c, u, dg_state_bytes(c), c->es, "u")) return rc;
    if (int rc = dg_check_array(c, nu, sizeof(OUT) * (size_t)c->nc, sizeof(OUT), "output")) return rc;
    if (c->es == 8) {
        if (c->k == 1) launch_labels<double, 1>(c, u, nu);
        else if (c->k == 2) launch_labels<double, 2>(c, u, nu);
        else launch_labels<double, 3>(c, u, nu);
    } else {
        if (c->k == 1) launch_labels<float, 1>(c, u, nu);
        else if (c->k == 2) launch_labels<float, 2>(c, u, nu);
        else launch_labels<float, 3>(c, u, nu);
    }
    LAUNCHCHK(c);
    return DG_OK;
}

int dg_sensor_labels(dg_ctx *c, const void *u, double *nu) { return labels_any(c, u, nu); }

int dg_sensor_targets(dg_ctx *c, const void *u, float *t)
{
    if (!c) return DG_EINVAL;
    int rc = need_k2(c);
    if (rc) return rc;
    return labels_any(c, u, t);
}

int sensor_infer_impl(dg_ctx *c, const void *u, int *nvmax, const void *vhat)
{
    int rc = need_k2(c);
    if (rc) return rc;
    if (!c->have_params) return dg_fail(c, DG_ESTATE, "no network parameters (dg_sensor_set_params)");
    float *x = (float *)c->wp(c->off.feat);
    if ((rc = dg_check_array(c, u, dg_state_bytes(c), c->es, "u"))) return rc;
    rc = launch_features(c, u, x, vhat);
    if (rc) return rc;
    const int nblk = fwd_blocks(c, c->nc);
    const int *fb = nvmax ? (const int *)c->wp(c->off.fb) : nullptr;
    double *vmax = nvmax ? (double *)c->wp(c->off.mlp) : nullptr;
    if (c->es == 8)
        hipLaunchKernelGGL((k_mlp_forward<double>), dim3(nblk), dim3(256), 0, c->stream, (const float *)c->mlp_bf16,
                           (const float *)x, c->nc, (float *)nullptr, (double *)c->wp(c->off.nu), fb, vmax);
    else
        hipLaunchKernelGGL((k_mlp_forward<float>), dim3(nblk), dim3(256), 0, c->stream, (const float *)c->mlp_bf16,
                           (const float *)x, c->nc, (float *)nullptr, (float *)c->wp(c->off.nu), fb, vmax);
    LAUNCHCHK(c);
    if (nvmax) *nvmax = nblk;
    c->have_nu = true;
    return DG_OK;
}

int dg_sensor_infer(dg_ctx *c, const void *u)
{
    if (!c) return DG_EINVAL;
    c->spec_valid = false;          // the viscosity or flags a launched next stage used change
    if (int rc = dg_check_array(c, u, dg_state_bytes(c), c->es, "u")) return rc;
    return sensor_infer_impl(c, u);
}

int dg_sensor_judge(dg_ctx *c, const void *u, double tau, long *nfallback)
{
    if (!c) return DG_EINVAL;
    c->spec_valid = false;          // the viscosity or flags a launched next stage used change
    if (!u || !(tau >= 0.0)) return dg_fail(c, DG_EINVAL, "bad judge arguments");
    if (int rc = dg_check_array(c, u, dg_state_bytes(c), c->es, "u")) return rc;
    int rc = sensor_infer_impl(c, u);
    if (rc) return rc;
    double *lab = (double *)c->wp(c->off.lab);
    rc = dg_sensor_labels(c, u, lab);
    if (rc) return rc;
    unsigned long long *cnt = (unsigned long long *)(c->scal() + 32);
    std::memset(c->pinned + 8, 0, 8);
    HIPCHK(c, hipMemcpyAsync(cnt, c->pinned + 8, 8, hipMemcpyHostToDevice, c->stream));
    int *fb = (int *)c->wp(c->off.fb);
    if (c->es == 8)
        hipLaunchKernelGGL((k_judge<double>), dim3(c->nblk), dim3(BLOCK), 0, c->stream,
                           (const double *)c->wp(c->off.nu), (const double *)lab, c->nc, tau, fb, cnt);
    else
        hipLaunchKernelGGL((k_judge<float>), dim3(c->nblk), dim3(BLOCK), 0, c->stream,
                           (const float *)c->wp(c->off.nu), (const double *)lab, c->nc, tau, fb, cnt);
    LAUNCHCHK(c);
    HIPCHK(c, hipMemcpyAsync(c->pinned, cnt, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (nfallback) *nfallback = (long)((volatile unsigned long long *)c->pinned)[0];
    return DG_OK;
}

int dg_sensor_set_nu(dg_ctx *c, const void *nu, const int32_t *fb)
{
    if (!c) return DG_EINVAL;
    c->spec_valid = false;          // the viscosity or flags a launched next stage used change
    int rc = need_k2(c);
    if (rc) return rc;
    if (nu && (rc = dg_check_array(c, nu, c->es * (size_t)c->nc, c->es, "nu"))) return rc;
    if (fb && (rc = dg_check_array(c, fb, 4 * (size_t)c->nc, 4, "fallback"))) return rc;
    if (nu) {
        HIPCHK(c, hipMemcpyAsync(c->wp(c->off.nu), nu, c->es * (size_t)c->nc, hipMemcpyDeviceToDevice, c->stream));
        c->have_nu = true;
    }
    if (fb) HIPCHK(c, hipMemcpyAsync(c->wp(c->off.fb), fb, 4 * (size_t)c->nc, hipMemcpyDeviceToDevice, c->stream));
    return DG_OK;
}

// clear the fallback flags of a fresh workspace (every cell starts on the learned sensor)
int sensor_reset_flags(dg_ctx *c)
{
    hipLaunchKernelGGL(k_fill_int, dim3(c->nblk), dim3(BLOCK), 0, c->stream, (int *)c->wp(c->off.fb), c->nc, 0);
    LAUNCHCHK(c);
    return DG_OK;
}
