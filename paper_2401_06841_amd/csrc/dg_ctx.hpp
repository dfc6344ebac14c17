// dg_ctx.hpp -- the opaque context behind the C ABI (host-side bookkeeping only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "dg.h"

// rows of per-wave partial network gradients in the workspace (waves of the gradient kernel)
constexpr int MLP_PART_ROWS = 1024;

struct dg_offsets {
    size_t stA, stB, stC, L, vh0, vh1, ftab, nu, fb, feat, lab, mlp, part, spart, dpart, scal, iflags;
};

struct dg_ctx {
    dg_config cfg{};
    int k = 0, nb = 0, nq = 0, nc = 0, nblk = 0;
    int rhs_nblk = 0;              // blocks of the last right-hand-side launch (its partial sums)
    int ncu = 256;                 // compute units of the device (grid sizing of persistent-style kernels)
    int device = 0;                // HIP device current at dg_init
    size_t es = 8;                 // element size of the state (8 = FP64, 4 = FP32)
    hipStream_t stream = nullptr;
    void *tab = nullptr;           // quadrature tables (element type of the state)
    double *modes_dev = nullptr;   // driving mode table [64][9]
    double modes_host[64 * 9] = {};
    int nmodes = 0;
    bool modes_sep = false;        // every n_x an integer in [-2, 2] (pencil form of the driving field)
    bool forcing_dirty = false;
    // pinned staging slots of the asynchronous table uploads, each with the event of its copy
    static constexpr int MODE_SLOTS = 4;
    double *modes_stage = nullptr;
    hipEvent_t modes_ev[MODE_SLOTS] = {};
    int modes_slot = 0;
    double *pinned = nullptr;      // 256 bytes of pinned host memory for read-backs
    // pinned[PUB..PUB+2]: the step's published {sequence number, time step bits, failure
    // flag} written by the device (k_final), and the last sequence number issued
    static constexpr int PUB = 16;
    long long pub_seq = 0;
    double wait_limit_s = 300.0;   // wall-clock bound of the host wait for a published step
    char *ws = nullptr;            // caller's workspace
    size_t ws_need = 0;
    dg_offsets off{};
    // Ornstein-Uhlenbeck driving state: 16 modes x 3 complex components
    double ou_tc = 0.0, ou_sigma = 0.0;
    double ou_x[16 * 6] = {};
    int ou_ready = 0;
    // learned sensor
    void *mlp_bf16 = nullptr;      // device copy of the parameters (fp32 master + bf16 weights)
    float *mfma_tab = nullptr;     // A-operand tables of the matrix-core volume integral (DG_VOLUME_MFMA)
    bool have_params = false;
    bool have_nu = false;
    bool learned_bounds_later = false;   // see proj_args
    bool abar_in_stage = false;          // see launch_stage
    // kernel timing (dg_profile)
    static constexpr int NEV = 64;
    int prof = 0;                      // 0 off, 1 first-stage right-hand sides, 2 every launch
    bool prof_first = false;           // the launch being issued belongs to a first stage
    bool prof_last = false;            // the right-hand side being issued belongs to a last stage
    hipEvent_t ev[2 * NEV][2] = {};    // [slot][start/stop]
    int ev_kind[2 * NEV] = {};         // 0 = rhs kernel, 1 = stage kernel
    int nev = 0;
    double prof_ms[2] = {0.0, 0.0};
    long prof_n[2] = {0, 0};
    char err[512] = {0};
    // projection of the state left in vh0 by the last dg_rk_step_next (valid while no other
    // state-changing call has been made: gen counts such calls)
    unsigned long gen = 0;
    const void *vh_cache_u = nullptr;
    unsigned long vh_cache_gen = 0;
    // the first stage of the next step launched ahead by dg_rk_step_next_ahead: for array
    // spec_u with time step spec_dt, valid while nothing it depends on has changed
    bool spec_valid = false;
    const void *spec_u = nullptr;
    double spec_dt = 0.0;

    // cached hipFFT plan of the velocity spectrum (a hipfftHandle) and its grid X, Y, Z
    void *fft_plan = nullptr;
    long long fft_dims[3] = {0, 0, 0};

    void *wp(size_t o) const { return ws + o; }
    double *scal() const { return (double *)(ws + off.scal); }
    double *abar() const { return scal(); }          // scal[0..2]
    int *fail() const { return (int *)(ws + off.iflags); }
};

int dg_fail(dg_ctx *ctx, int code, const char *fmt, ...);

// a device array of `bytes` bytes at p, checked before any launch reads or writes it: not
// null, aligned to `align`, and inside one allocation the HIP runtime tracks (DG_EINVAL
// otherwise)
int dg_check_array(dg_ctx *ctx, const void *p, size_t bytes, size_t align, const char *name);
// the state array [nvar][modes][cells] in the context's precision
inline size_t dg_state_bytes(const dg_ctx *c, int nvar = 4) { return (size_t)nvar * c->nb * c->nc * c->es; }

// return a DG_EHIP error with the failing call and its place from a host function
#define HIPCHK(ctx, call)                                                                         \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return dg_fail((ctx), DG_EHIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                           __FILE__, __LINE__);                                                   \
    } while (0)

#define LAUNCHCHK(ctx)                                                                            \
    do {                                                                                          \
        hipError_t e_ = hipGetLastError();                                                        \
        if (e_ != hipSuccess)                                                                     \
            return dg_fail((ctx), DG_EHIP, "kernel launch failed: %s (%s:%d)", hipGetErrorString(e_), \
                           __FILE__, __LINE__);                                                   \
    } while (0)

// nvmax != NULL: the forward pass also writes the learned cells' largest viscosity per block
// into the mlp region (as doubles) and *nvmax = the number of blocks; vhat != NULL: the
// projected velocity of u, used by the features unless the step's failure flag is raised
int sensor_infer_impl(dg_ctx *c, const void *u, int *nvmax = nullptr, const void *vhat = nullptr);
void stats_release(dg_ctx *c);
int sensor_reset_flags(dg_ctx *c);
