// ssm.hip -- libssm: host runtime and C ABI (include/ssm.h) of the SSM
// particle step on MI355X (gfx950).  See ssm_kernels.hpp for the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/ssm.h"
#include "ssm_surrogate.hpp"
#include "ssm_small.hpp"

using namespace ssm;

static constexpr int kRedBlocks = 256;  // blocks of the fixed-order moment / rMSE reductions
static constexpr int64_t kSmallTicksPerLaunch = 4096;  // ticks per persistent launch, at most
static constexpr double kLog2e = 1.4426950408889634073599246810018921;  // log2(e)

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

static ssm_status fail(ssm_status st, const std::string& msg)
{
    g_last_error = msg;
    return st;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(SSM_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));  \
    } while (0)

extern "C" const char* ssm_last_error(void) { return g_last_error.c_str(); }

// ---------------------------------------------------------------------------
// kernels of the kernel-level entry points
// ---------------------------------------------------------------------------
namespace ssm {

template <int D>
__global__ void k_brownian(int64_t N, uint64_t seed, int32_t ens, int64_t n0, int32_t r, double sqrt_hf,
                           double* __restrict__ dW)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double zs[kMaxD] = {0.0, 0.0, 0.0, 0.0};
    const uint64_t q0 = (uint64_t)n0 * D;
    stream_sum<D>(seed, (uint64_t)i, (uint64_t)ens, q0, q0 + (uint64_t)r * D, q0 / 4, 1, zs);
    for (int k = 0; k < D; ++k) dW[(int64_t)k * N + i] = sqrt_hf * zs[k];
}

__global__ void k_philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                         uint64_t k1, int64_t count, uint64_t* __restrict__ out)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    const Block4 b = philox4x64_10(c0 + (uint64_t)q, c1, c2, c3, k0, k1);
    for (int w = 0; w < 4; ++w) out[4 * q + w] = b.w[w];
}

template <int D>
__global__ void k_implicit_plain(int64_t N, const double* __restrict__ X, double h, double rho,
                                 double a, double kappa, double lam, double xb0, double xb1,
                                 double xb2, double xb3, double m2, int max_iter,
                                 double* __restrict__ Y, int32_t* __restrict__ iters)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double xbar[kMaxD] = {xb0, xb1, xb2, xb3};
    double w[D], y[D];
    for (int k = 0; k < D; ++k) w[k] = X[(int64_t)k * N + i] + h * lam * xbar[k];
    const int it = implicit_radial<D>(w, 1.0 - h * (rho - kappa * m2), h * a, max_iter, y);
    for (int k = 0; k < D; ++k) Y[(int64_t)k * N + i] = y[k];
    if (iters) iters[i] = it;
}

}  // namespace ssm

// ---------------------------------------------------------------------------
// kernel dispatch tables (d, R, precision)
// ---------------------------------------------------------------------------
// Symmetric scheme: one workgroup per item.
template <typename T, int D>
static void launch_pair_sym_D(int R, bool kahan, int n, hipStream_t st, const PairItem* items, const SysDev* sys,
                              const T* Ys, int64_t P, T* Bp, T* Bpj, int jrow_base)
{
    dim3 grid((unsigned)n), block(64 * kWaves);
    if constexpr (sizeof(T) == sizeof(double)) {
        // FP64: no compensation; R * d bounded by the LDS row
        (void)kahan;
        switch (R) {
            case 1: hipLaunchKernelGGL((k_pair_sym<T, D, 1, false>), grid, block, 0, st, items, sys, Ys, P, Bp, Bpj, jrow_base); break;
            case 2: if constexpr (D <= 3) hipLaunchKernelGGL((k_pair_sym<T, D, 2, false>), grid, block, 0, st, items, sys, Ys, P, Bp, Bpj, jrow_base); break;
            case 4: if constexpr (D == 1) hipLaunchKernelGGL((k_pair_sym<T, D, 4, false>), grid, block, 0, st, items, sys, Ys, P, Bp, Bpj, jrow_base); break;
            default: break;
        }
    } else {
#define SSM_SYM_CASE(RR)                                                                                      \
    case RR:                                                                                                  \
        if (kahan)                                                                                            \
            hipLaunchKernelGGL((k_pair_sym<T, D, RR, true>), grid, block, 0, st, items, sys, Ys, P, Bp, Bpj,   \
                               jrow_base);                                                                    \
        else                                                                                                  \
            hipLaunchKernelGGL((k_pair_sym<T, D, RR, false>), grid, block, 0, st, items, sys, Ys, P, Bp, Bpj,  \
                               jrow_base);                                                                    \
        break;
        switch (R) {
            SSM_SYM_CASE(1)
            SSM_SYM_CASE(2)
            SSM_SYM_CASE(4)
            SSM_SYM_CASE(8)
            default: break;
        }
#undef SSM_SYM_CASE
    }
}

template <typename T, int D>
static void launch_pair_T(int R, bool kahan, dim3 grid, hipStream_t st, const PairItem* items,
                          int n, const SysDev* sys, const T* Ys, int64_t P, T* Bp)
{
    dim3 block(64 * kWaves);
#define SSM_PAIR_CASE(RR)                                                                      \
    case RR:                                                                                   \
        if (kahan)                                                                             \
            hipLaunchKernelGGL((k_pair<T, D, RR, true>), grid, block, 0, st, items, n, sys, Ys, P, Bp); \
        else                                                                                   \
            hipLaunchKernelGGL((k_pair<T, D, RR, false>), grid, block, 0, st, items, n, sys, Ys, P, Bp); \
        break;
    switch (R) {
        SSM_PAIR_CASE(1)
        SSM_PAIR_CASE(2)
        SSM_PAIR_CASE(4)
        SSM_PAIR_CASE(8)
        default: break;
    }
#undef SSM_PAIR_CASE
}

// Pair kernel launch: ordered scheme one wavefront per item (kWaves items per
// workgroup), symmetric scheme one workgroup per item.
template <typename T>
static void launch_pair(int d, int R, bool kahan, dim3 grid, hipStream_t st, const PairItem* items,
                        int n, const SysDev* sys, const T* Ys, int64_t P, T* Bp, T* Bpj, bool sym,
                        bool kpair = false, int jrow_base = 0)
{
    if constexpr (sizeof(T) == sizeof(float)) {
        if (kpair) {
            dim3 block(64 * kWaves);
#define SSM_KPAIR_CASE(DD, RR)                                                                                  \
    if (d == DD && R == RR) {                                                                                   \
        hipLaunchKernelGGL((k_pair_kpair<DD, RR>), grid, block, 0, st, items, n, sys, Ys, P, Bp);               \
        return;                                                                                                 \
    }
            SSM_KPAIR_CASE(1, 1) SSM_KPAIR_CASE(1, 2) SSM_KPAIR_CASE(1, 4) SSM_KPAIR_CASE(1, 8)
            SSM_KPAIR_CASE(2, 1) SSM_KPAIR_CASE(2, 2) SSM_KPAIR_CASE(2, 4) SSM_KPAIR_CASE(2, 8)
            SSM_KPAIR_CASE(3, 1) SSM_KPAIR_CASE(3, 2) SSM_KPAIR_CASE(3, 4) SSM_KPAIR_CASE(3, 8)
            SSM_KPAIR_CASE(4, 1) SSM_KPAIR_CASE(4, 2) SSM_KPAIR_CASE(4, 4) SSM_KPAIR_CASE(4, 8)
#undef SSM_KPAIR_CASE
            return;
        }
    }
    if (sym) {
        switch (d) {
            case 1: launch_pair_sym_D<T, 1>(R, kahan, n, st, items, sys, Ys, P, Bp, Bpj, jrow_base); break;
            case 2: launch_pair_sym_D<T, 2>(R, kahan, n, st, items, sys, Ys, P, Bp, Bpj, jrow_base); break;
            case 3: launch_pair_sym_D<T, 3>(R, kahan, n, st, items, sys, Ys, P, Bp, Bpj, jrow_base); break;
            case 4: launch_pair_sym_D<T, 4>(R, kahan, n, st, items, sys, Ys, P, Bp, Bpj, jrow_base); break;
            default: break;
        }
        return;
    }
    switch (d) {
        case 1: launch_pair_T<T, 1>(R, kahan, grid, st, items, n, sys, Ys, P, Bp); break;
        case 2: launch_pair_T<T, 2>(R, kahan, grid, st, items, n, sys, Ys, P, Bp); break;
        case 3: launch_pair_T<T, 3>(R, kahan, grid, st, items, n, sys, Ys, P, Bp); break;
        case 4: launch_pair_T<T, 4>(R, kahan, grid, st, items, n, sys, Ys, P, Bp); break;
        default: break;
    }
}

// A symmetric target group (kWaves x 64 R particles) times d fits the LDS row.
static bool sym_fits(bool fp64, int R, int d) { return (int64_t)64 * R * kWaves * d <= sym_lds_for(fp64, d); }

#define SSM_DISPATCH_D(d, KERNEL_CALL)       \
    switch (d) {                             \
        case 1: { constexpr int D = 1; KERNEL_CALL; } break; \
        case 2: { constexpr int D = 2; KERNEL_CALL; } break; \
        case 3: { constexpr int D = 3; KERNEL_CALL; } break; \
        case 4: { constexpr int D = 4; KERNEL_CALL; } break; \
        default: break;                      \
    }

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct SysHost {
    int64_t N;
    int32_t ens;
    double h;
    int64_t stride;  // ticks per step
    int64_t r;       // fine increments per step
    int64_t off;     // slot offset
    int64_t blk0, nblk;
    int64_t splits;
    int64_t steps_done;
    int64_t win_off = -1;  // offset of its path group's Brownian window (-1: none)
};

struct ssm_ctx {
    int d = 1;
    int prec = SSM_FP64;
    bool fused = true;
    bool has_pair = false;
    Coef coef{};
    std::vector<SysHost> sys;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool x_bound = false;      // X lives in a caller-owned buffer (ssm_bind_state)
    ssm_config cfg{};          // the creating config (system arrays below), for training runs
    std::vector<int64_t> cfg_N;
    std::vector<int32_t> cfg_ens;
    std::vector<double> cfg_h;
    int64_t P = 0;          // padded slots
    int64_t nblk_tot = 0;
    int64_t max_stride = 1;
    int64_t tick = 0, ticks_total = 0;
    int R = 4;
    int64_t L = 0;          // sources per pair item
    int64_t max_splits = 1;
    // device buffers
    void* X = nullptr;
    void* Y = nullptr;
    void* Ys = nullptr;
    void* Bp = nullptr;        // i-side partials [max_splits][d][P] in the storage precision
    void* Bpj = nullptr;       // symmetric scheme: j-side partials [nb_max][d][P] (pair precision)
    double* pairsum = nullptr; // [d][P] scaled pair term of the last exact tick (k_combine)
    bool sym = false;          // symmetric pair scheme
    int64_t band = 0;          // symmetric scheme: target groups per band of j-side rows (0: not banded)
    int64_t n_bands = 1;
    double* jtot = nullptr;    // banded: [d][P] running total of a particle's j-side sums (k_jfold)
    std::vector<std::vector<int64_t>> pair_band_off;  // per phase: first item of each band, and the end
    bool kpair = false;        // FP32-compensated with every pair term compensated (kahan_span = 1)
    int64_t nb_max = 0;
    double* psumX = nullptr;
    double* psumY = nullptr;
    SysDev* dsys = nullptr;
    PairItem* dpair = nullptr;
    BlkItem* dblk = nullptr;
    Flags* dflags = nullptr;
    int32_t* dnmax = nullptr;      // [nblk_tot][kSlotsPerBlk] largest Newton iteration count
    double* dstage = nullptr;  // staging for state copies / moments
    double* dred = nullptr;    // [kMaxD][kRedBlocks] partial sums of the moment / rMSE reductions
    double* dsq = nullptr;     // [systems] squared differences of ssm_rmse
    int64_t bytes = 0;
    // per phase (tick % max_stride) work lists: offsets into dpair / dblk
    std::vector<int64_t> pair_off, pair_cnt, blk_off, blk_cnt;
    std::vector<int64_t> all_blk_off;  // blocks of every system (init / set_state)
    int64_t all_blk_cnt = 0;
    std::vector<int64_t> sys_blk_off;  // per system: first of its blocks in the all-blocks list
    // learned surrogate of the pair term
    bool surr_loaded = false;
    int32_t surr_check_every = 0;  // 0: surrogate off
    double surr_tol = 1e-3;
    bool surr_fallback = false;
    int64_t surr_checks = 0, surr_fallback_ticks = 0, surr_ticks = 0;
    bool surr_recheck = false;     // in a fallback, every tick where all systems step is a check
    int64_t surr_rechecks = 0;     // checks made by that rule
    double surr_last_err = 0.0, surr_max_err = 0.0, surr_last_raw_err = 0.0;
    double surr_gain[kMaxD] = {1.0, 1.0, 1.0, 1.0};
    int32_t surr_mode = SSM_SURR_GAIN;
    bool surr_res_valid = false;   // residuals stored by a check since enabling
    float* surr_res = nullptr;     // [d][P] residual p - (s - mean s) of the last check
    MlpPacked* dmlp = nullptr;
    float* surr = nullptr;         // [d][P] surrogate pair term
    double* rff_part = nullptr;    // [nblk_tot][2K]
    float* mom = nullptr;          // [n_sys][2K]
    double* err_part = nullptr;    // [nblk_tot][2]
    double* smean_part = nullptr;  // [nblk_tot][kMaxD]
    float* smean = nullptr;        // [n_sys][kMaxD]
    int32_t* dsys_list = nullptr;  // per phase: active systems
    std::vector<int64_t> sys_list_off, sys_list_cnt;
    RffFreq rff{};
    double ell = 1.0;
    // device tick counter read by the update kernels; HIP graphs of one tick
    // per phase (tick % max_stride), built on first use and replayed
    int64_t* dtick = nullptr;
    bool dtick_valid = true;  // device counter equals the host tick
    double* dW = nullptr;  // [d][P] Brownian increments of the current tick
    bool needs_ybar = false;   // b or sigma uses the mean of mu^Y
    double* ymean = nullptr;   // [n_sys][kMaxD] mean of mu^Y of the current step (k_prep / k_brownian_sum)
    int bm_lanes = 1;      // lanes per particle in k_brownian_sum
    // shared Brownian windows of path groups (systems of one ensemble and size)
    double* win = nullptr;      // [groups][max_stride][d][N_g] per-tick normal sums
    BlkItem* dwin_items = nullptr;
    int64_t win_items = 0;      // blocks of one member per group
    int64_t r_min = 1;          // fine increments per tick
    int win_lanes = 1;          // lanes per particle in k_bm_window
    bool use_graphs = false;
    std::vector<hipGraphExec_t> phase_graph;
    // kernel timing: event pairs recorded around launches while profiling
    bool profiling = false;
    int32_t profile_every = 1;     // bracket the launches of ticks with tick % profile_every == 0
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pair, ev_update;
    std::vector<hipEvent_t> ev_pool;
    // persistent runs of small systems (ssm_small.hpp)
    bool small_ok = false;          // eligible: ticks without surrogate, profiling or graphs use it
    SmallTile* dtiles = nullptr;    // [small_grid] workgroup -> (system, tile)
    int64_t small_grid = 0;         // tiles of 64 particles = workgroups per launch
    double* sumY = nullptr;         // [2][d][small_grid] tile sums of Y*
    double* sumX = nullptr;         // [d + 1][small_grid] tile sums of the new X and |X|^2
    uint64_t* dbar = nullptr;       // [n_sys][kBarLine] barrier counters
    uint64_t small_epoch = 0;       // barriers every system has passed
    int64_t small_wait_limit = 0;   // wall-clock counts a barrier wait may take
    int64_t small_launches = 0, small_ticks = 0;
    int small_lanes = 1;            // lanes per particle of the persistent draws (every system draws its own)
    bool psum_stale = false;        // after persistent ticks: psumY and the current window lag
    bool broken = false;            // a persistent run was aborted
};

static hipEvent_t take_event(ssm_ctx* c)
{
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    // timing only (read after the stream is synchronized): no system-scope
    // fence, whose cache writeback cost about 3 us per timed tick and slowed
    // the launch after it
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

static void recycle_events(ssm_ctx* c, std::vector<std::pair<hipEvent_t, hipEvent_t>>& v)
{
    for (auto& p : v) {
        if (p.first) c->ev_pool.push_back(p.first);
        if (p.second) c->ev_pool.push_back(p.second);
    }
    v.clear();
}

// Sum of elapsed times of recorded event pairs (the stream must be synchronized).
static double elapsed_ms(const std::vector<std::pair<hipEvent_t, hipEvent_t>>& v)
{
    double tot = 0.0;
    for (auto& p : v) {
        float ms = 0.0f;
        if (p.first && p.second && hipEventElapsedTime(&ms, p.first, p.second) == hipSuccess) tot += ms;
    }
    return tot;
}

static size_t elt(int prec) { return prec == SSM_FP64 ? sizeof(double) : sizeof(float); }

static ssm_status dev_alloc(ssm_ctx* c, void** p, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(SSM_ERR_OOM, std::string("hipMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e));
    }
    c->bytes += (int64_t)bytes;
    return SSM_OK;
}

static void free_ctx(ssm_ctx* c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    void* bufs[] = {c->x_bound ? nullptr : c->X, c->Y, c->Ys, c->Bp, c->Bpj, c->pairsum, c->psumX, c->psumY, c->dsys, c->dpair, c->dblk, c->dflags, c->dstage,
                    c->dmlp, c->surr, c->rff_part, c->mom, c->err_part, c->dsys_list, c->smean_part, c->smean,
                    c->dtick, c->dW, c->surr_res, c->dnmax, c->dred, c->dsq, c->win, c->dwin_items, c->ymean,
                    c->jtot, c->dtiles, c->sumY, c->sumX, c->dbar};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    recycle_events(c, c->ev_pair);
    recycle_events(c, c->ev_update);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    for (hipGraphExec_t g : c->phase_graph)
        if (g) (void)hipGraphExecDestroy(g);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

static bool is_int_ratio(double a, double b, int64_t* out)
{
    const double q = a / b;
    const double rq = std::nearbyint(q);
    if (!(rq >= 1.0) || std::fabs(q - rq) > 1e-9 * rq || rq > 4e18) return false;
    *out = (int64_t)rq;
    return true;
}

// Work items of one system's pair sums.
//  Ordered-pair scheme: tiles of 64 R targets x source ranges of L sources;
//    i-side partial q = source range q.
//  Symmetric scheme: target groups of G = kWaves x 64 R particles
//    (one workgroup); group a has a diagonal item (its own sources, ordered
//    pairs, partial 0) and items over the later sources [G (a+1), N) in ranges
//    of L (partial 1, 2, ...), each also writing j-side partial row a.  Every
//    unordered pair is visited once.
// Each item carries a cost estimate (VALU issue slots) for ordering.
static int64_t plan_system(int s, int64_t N, int R, bool sym, int64_t L,
                           std::vector<std::pair<int64_t, PairItem>>& out, int64_t* nb_out)
{
    const int64_t tile = 64 * (int64_t)R;
    const int64_t tiles = (N + tile - 1) / tile;
    int64_t isplits = 0;
    if (!sym) {
        isplits = (N + L - 1) / L;
        for (int64_t q = 0; q < isplits; ++q) {
            const int64_t j0 = q * L;
            const int64_t nj = std::min<int64_t>(L, N - j0);
            for (int64_t t = 0; t < tiles; ++t) {
                PairItem it{};
                it.sys = s;
                it.tgt0 = (int32_t)(t * tile);
                it.src0 = (int32_t)j0;
                it.nsrc = (int32_t)nj;
                it.split = (int32_t)q;
                it.jrow = -1;
                out.push_back({5 * nj * std::min<int64_t>(tile, N - t * tile), it});
            }
        }
        if (nb_out) *nb_out = 0;
        return isplits;
    }
    // symmetric: target groups of kWaves blocks, one workgroup per item
    const int64_t group = tile * kWaves;
    const int64_t groups = (N + group - 1) / group;
    for (int64_t a = 0; a < groups; ++a) {
        const int64_t t0 = a * group;
        const int64_t nt = std::min<int64_t>(group, N - t0);
        PairItem dg{};
        dg.sys = s;
        dg.tgt0 = (int32_t)t0;
        dg.src0 = (int32_t)t0;
        dg.nsrc = (int32_t)nt;
        dg.split = 0;
        dg.jrow = -1;
        out.push_back({5 * nt * nt, dg});
        int64_t q = 1;
        for (int64_t j0 = t0 + group; j0 < N; j0 += L, ++q) {
            PairItem it{};
            it.sys = s;
            it.tgt0 = (int32_t)t0;
            it.src0 = (int32_t)j0;
            it.nsrc = (int32_t)std::min<int64_t>(L, N - j0);
            it.split = (int32_t)q;
            it.jrow = (int32_t)a;
            out.push_back({6 * (int64_t)it.nsrc * group + 64 * group, it});
        }
        isplits = std::max(isplits, q);
    }
    if (nb_out) *nb_out = groups;
    return isplits;
}

// Longest first (stable), so that big items start early.
static void order_items(std::vector<std::pair<int64_t, PairItem>>& tmp, std::vector<PairItem>& out)
{
    std::stable_sort(tmp.begin(), tmp.end(),
                     [](const std::pair<int64_t, PairItem>& a, const std::pair<int64_t, PairItem>& b) {
                         return a.first > b.first;
                     });
    for (auto& p : tmp) out.push_back(p.second);
}

// The items of the listed systems, longest first; banded (symmetric scheme
// with j-side bands), band by band: band_off receives the first item of each
// band and the end.
static void build_pair_items(const ssm_ctx* c, const std::vector<int>& systems, std::vector<PairItem>& out,
                             std::vector<int64_t>* band_off)
{
    std::vector<std::pair<int64_t, PairItem>> tmp;
    for (int s : systems) plan_system(s, c->sys[s].N, c->R, c->sym, c->L, tmp, nullptr);
    if (!band_off) {
        order_items(tmp, out);
        return;
    }
    const int64_t group = 64 * (int64_t)c->R * kWaves;
    std::vector<std::vector<std::pair<int64_t, PairItem>>> per(c->n_bands);
    for (auto& p : tmp) {
        const int64_t a = p.second.jrow >= 0 ? p.second.jrow : p.second.tgt0 / group;
        per[a / c->band].push_back(p);
    }
    band_off->clear();
    for (auto& v : per) {
        band_off->push_back((int64_t)out.size());
        order_items(v, out);
    }
    band_off->push_back((int64_t)out.size());
}

// Default sources per item: about 16384 wavefront items per tick (16 per
// SIMD) over the given sizes; at least 512 (ordered) / 256 (symmetric)
// sources, a multiple of 64 / 16.  (Measured on MI355X: shorter items beat
// longer ones down to this size for d = 1..3.)
// Default targets per lane: 4 for d = 1, 2 for d >= 2 (measured fastest at
// full size), halved while the largest work item (a symmetric group's
// diagonal item, (256 R)^2 / 2 pair evaluations; an ordered item, 64 R x 512)
// exceeds the average work of a resident workgroup slot (about 1024 of them),
// so that small runs spread over the chip instead of a few long items.
static int default_R(int d, const std::vector<int64_t>& Ns, bool sym)
{
    int R = d == 1 ? 4 : 2;
    double total = 0.0;
    for (int64_t N : Ns) total += (double)N * (double)N;
    const double per_slot = (sym ? 0.5 : 1.0) * total / 1024.0;
    while (R > 1) {
        const double g = sym ? 256.0 * R : 64.0 * R;
        const double item = sym ? 0.5 * g * g : g * 512.0;
        if (item <= per_slot) break;
        R /= 2;
    }
    return R;
}

static int64_t default_L(const std::vector<int64_t>& Ns, int R, bool sym, int d)
{
    const int64_t tile = 64 * (int64_t)R;
    if (sym) {
        // ~6600 workgroup items per tick (about 8.6 per resident workgroup
        // slot at R = 4: small enough a tail, few enough i-side partials;
        // measured best at d = 1, N = 2^16 among 4000..16000 items)
        const double group = (double)(tile * kWaves);
        double work = 0.0;
        for (int64_t N : Ns) work += 0.5 * (double)N * (double)N / group;
        const int64_t L = (int64_t)std::ceil(work / 6600.0 / 16.0) * 16;
        (void)d;
        return std::max<int64_t>(L, 128);
    }
    double work = 0.0;
    for (int64_t N : Ns) work += (double)((N + tile - 1) / tile) * (double)N;
    const double per_item = work / 16384.0;
    return std::max<int64_t>((int64_t)std::ceil(per_item / 64.0) * 64, 512);
}

static void build_blk_items(const ssm_ctx* c, const std::vector<int>& systems, std::vector<BlkItem>& out)
{
    // largest systems first: their blocks also reduce the longest block-sum lists
    std::vector<int> order(systems);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return c->sys[a].N > c->sys[b].N; });
    for (int s : order)
        for (int64_t b = 0; b < c->sys[s].nblk; ++b) out.push_back(BlkItem{s, (int32_t)b});
}

// The pair sums of phase ph's items into the partial-sum buffers: one launch,
// or (banded j-side rows) one launch per band followed by the fold of that
// band's rows into jtot for every stepping particle.
template <typename T>
static ssm_status launch_pairs(ssm_ctx* c, int64_t ph)
{
    const int d = c->d;
    const int64_t np = c->pair_cnt[ph];
    const PairItem* items = c->dpair + c->pair_off[ph];
    if (c->band == 0) {
        const dim3 grid((unsigned)(c->sym ? np : (np + kWaves - 1) / kWaves));
        launch_pair<T>(d, c->R, c->prec == SSM_FP32_KAHAN, grid, c->stream, items, (int)np, c->dsys, (const T*)c->Ys,
                       c->P, (T*)c->Bp, (T*)c->Bpj, c->sym, c->kpair);
        HIP_TRY(hipGetLastError());
        return SSM_OK;
    }
    const std::vector<int64_t>& off = c->pair_band_off[ph];
    const BlkItem* blks = c->dblk + c->blk_off[ph];
    const unsigned nb = (unsigned)c->blk_cnt[ph];
    for (int64_t b = 0; b < c->n_bands; ++b) {
        const int64_t n = off[b + 1] - off[b];
        if (n == 0) continue;  // no system has groups in this band: no particle reads its rows
        const int a0 = (int)(b * c->band), a1 = (int)((b + 1) * c->band);
        // off[] holds positions in the whole item list (dpair)
        launch_pair<T>(d, c->R, c->prec == SSM_FP32_KAHAN, dim3((unsigned)n), c->stream, c->dpair + off[b], (int)n,
                       c->dsys, (const T*)c->Ys, c->P, (T*)c->Bp, (T*)c->Bpj, true, false, a0);
        HIP_TRY(hipGetLastError());
        SSM_DISPATCH_D(d, hipLaunchKernelGGL((k_jfold<T, D>), dim3(nb), dim3(kBlk), 0, c->stream, blks, c->dsys, c->P,
                                             (const T*)c->Bpj, a0, a1, b == 0 ? 1 : 0, c->jtot));
        HIP_TRY(hipGetLastError());
    }
    return SSM_OK;
}

template <typename T>
static ssm_status launch_surrogate(ssm_ctx* c, int64_t ph)
{
    const int d = c->d;
    const BlkItem* items = c->dblk + c->blk_off[ph];
    const int64_t nb = c->blk_cnt[ph];
    SSM_DISPATCH_D(d, hipLaunchKernelGGL((k_rff_partial<T, D>), dim3((unsigned)nb), dim3(kBlk), 0, c->stream, items,
                                         c->dsys, c->P, (const T*)c->Y, c->rff, c->rff_part));
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_rff_final, dim3((unsigned)c->sys_list_cnt[ph], 2 * kRff), dim3(kBlk), 0, c->stream,
                       c->dsys_list + c->sys_list_off[ph], c->dsys, c->rff_part, c->mom);
    HIP_TRY(hipGetLastError());
    // one workgroup per 256-particle block (its weights load is a small part of it):
    // 71.8 us at N = 2^20 against 75.6 us with 2048 workgroups of two blocks each
    const unsigned grid = (unsigned)std::min<int64_t>(nb, 1 << 20);
    SSM_DISPATCH_D(d, hipLaunchKernelGGL((k_mlp_infer<T, D>), dim3(grid), dim3(256), 0, c->stream, items, (int)nb,
                                         c->dsys, c->P, (const T*)c->Y, c->mom, c->dmlp, c->surr));
    HIP_TRY(hipGetLastError());
    SSM_DISPATCH_D(d, hipLaunchKernelGGL((k_surr_partial<D>), dim3((unsigned)nb), dim3(kBlk), 0, c->stream, items,
                                         c->dsys, c->P, c->surr, c->smean_part));
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_surr_final, dim3((unsigned)c->sys_list_cnt[ph], d), dim3(kBlk), 0, c->stream,
                       c->dsys_list + c->sys_list_off[ph], c->dsys, c->smean_part, c->smean);
    HIP_TRY(hipGetLastError());
    return SSM_OK;
}

// The path groups' Brownian windows for ticks t0 .. t0 + max_stride - 1
// (t0 = *tdev when tdev is given).
template <typename T>
static ssm_status launch_window(ssm_ctx* c, int64_t t0, const int64_t* tdev)
{
    const int d = c->d;
    const dim3 gw((unsigned)(c->win_items * c->win_lanes), (unsigned)c->max_stride);
#define SSM_WIN(LPV)                                                                                                   \
    SSM_DISPATCH_D(d, hipLaunchKernelGGL((k_bm_window<D, LPV, (sizeof(T) == 4)>), gw, dim3(kBlk), 0, c->stream,      \
                                         c->dwin_items, c->dsys, c->coef, c->r_min, t0, tdev, c->win))
    switch (c->win_lanes) {
        case 16: SSM_WIN(16); break;
        case 8: SSM_WIN(8); break;
        case 4: SSM_WIN(4); break;
        case 2: SSM_WIN(2); break;
        default: SSM_WIN(1); break;
    }
#undef SSM_WIN
    HIP_TRY(hipGetLastError());
    return SSM_OK;
}

template <typename T>
static ssm_status launch_tick(ssm_ctx* c, bool capture)
{
    // eager launches pass the tick by value; a captured tick reads (and at its
    // end advances) the device counter so that the graph can be replayed
    const int64_t* tdev = capture ? c->dtick : nullptr;
    const int64_t ph = c->tick % c->max_stride;
    const int64_t np = c->pair_cnt[ph], nb = c->blk_cnt[ph];
    T* X = (T*)c->X;
    T* Y = (T*)c->Y;
    T* Ys = (T*)c->Ys;
    const int d = c->d;
    const bool surr_on = c->surr_check_every > 0 && c->has_pair;
    // scheduled checks every surr_check_every ticks; with surr_recheck, a
    // fallback tick on which every system steps is a check too (its exact
    // term is computed anyway, and the network is judged on it)
    const bool recheck = surr_on && c->surr_recheck && c->surr_fallback && c->tick % c->surr_check_every != 0 &&
                         c->tick % c->max_stride == 0;
    const bool check = surr_on && (c->tick % c->surr_check_every == 0 || recheck);
    const bool run_exact = !surr_on || check || c->surr_fallback;
    const bool run_surr = surr_on && (check || !c->surr_fallback);
    const bool prof = c->profiling && c->tick % c->profile_every == 0;
    if (ph == 0 && c->win_items > 0 && nb > 0) {
        ssm_status st = launch_window<T>(c, c->tick, tdev);
        if (st != SSM_OK) return st;
    }
    if (c->has_pair && np > 0 && run_exact) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (prof) {
            e0 = take_event(c);
            e1 = take_event(c);
            if (e0) HIP_TRY(hipEventRecord(e0, c->stream));
        }
        ssm_status st = launch_pairs<T>(c, ph);
        if (st != SSM_OK) return st;
        if (prof) {
            if (e1) HIP_TRY(hipEventRecord(e1, c->stream));
            c->ev_pair.push_back({e0, e1});
        }
    }
    if (run_surr && nb > 0) {
        ssm_status st = launch_surrogate<T>(c, ph);
        if (st != SSM_OK) return st;
    }
    const int use_surr = (run_surr && !check) ? 1 : 0;
    if (nb > 0) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (prof) {
            e0 = take_event(c);
            e1 = take_event(c);
            if (e0) HIP_TRY(hipEventRecord(e0, c->stream));
        }
        const BlkItem* items = c->dblk + c->blk_off[ph];
        // Brownian sums of the step, and on exact ticks the combine of the pair
        // partials in the same launch (k_prep)
        const bool comb = c->has_pair && run_exact;
        const int ncb = comb ? (int)(nb * 4) : 0;
        const int n_main = (int)(ncb + nb * c->bm_lanes);
        // the stepping systems' means of mu^Y, when b or sigma needs them
        const YMeanJob job{c->dsys_list + c->sys_list_off[ph], c->needs_ybar ? (int)c->sys_list_cnt[ph] : 0,
                           c->psumY, c->nblk_tot, c->ymean};
        const unsigned gb = (unsigned)(n_main + job.n);
#define SSM_BM(LPV)                                                                                                   \
    if (comb) {                                                                                                       \
        SSM_DISPATCH_D(d, hipLaunchKernelGGL((k_prep<T, D, LPV>), dim3(gb), dim3(kBlk), 0, c->stream, ncb, n_main,    \
                                             items, c->dsys, c->coef, c->P, (const T*)c->Bp, (const T*)c->Bpj,        \
                                             (const double*)c->jtot, c->pairsum, c->tick, tdev, (const double*)c->win, \
                                             c->dW, job));                                                            \
    } else {                                                                                                          \
        SSM_DISPATCH_D(d, hipLaunchKernelGGL((k_brownian_sum<D, LPV, (sizeof(T) == 4)>), dim3(gb), dim3(kBlk), 0,    \
                                             c->stream, n_main,                                                       \
                                             items, c->dsys, c->coef, c->P, c->tick, tdev, (const double*)c->win,     \
                                             c->dW, job));                                                            \
    }
        switch (c->bm_lanes) {
            case 16: SSM_BM(16); break;
            case 8: SSM_BM(8); break;
            case 4: SSM_BM(4); break;
            case 2: SSM_BM(2); break;
            default: SSM_BM(1); break;
        }
#undef SSM_BM
        HIP_TRY(hipGetLastError());
        SSM_DISPATCH_D(d, hipLaunchKernelGGL((k_update<T, D>), dim3((unsigned)nb), dim3(kBlk), 0, c->stream,
                                             items, c->dsys, c->coef, c->P, c->tick, tdev, X, Y, Ys, c->pairsum, c->surr,
                                             c->smean, use_surr,
                                             make_float4((float)c->surr_gain[0], (float)c->surr_gain[1],
                                                         (float)c->surr_gain[2], (float)c->surr_gain[3]),
                                             (use_surr && c->surr_mode == SSM_SURR_RESIDUAL && c->surr_res_valid)
                                                 ? c->surr_res : nullptr,
                                             c->dW, c->needs_ybar ? (const double*)c->ymean : nullptr,
                                             c->psumX, c->psumY, c->nblk_tot, c->dflags, c->dnmax));
        HIP_TRY(hipGetLastError());
        if (!c->fused) {
            SSM_DISPATCH_D(d, hipLaunchKernelGGL((k_newton<T, D>), dim3((unsigned)nb), dim3(kBlk), 0, c->stream,
                                                 items, c->dsys, c->coef, c->P, c->tick, tdev, X, Y, Ys,
                                                 c->psumX, c->psumY, c->nblk_tot, c->dflags, c->dnmax));
            HIP_TRY(hipGetLastError());
        }
        if (prof) {
            if (e1) HIP_TRY(hipEventRecord(e1, c->stream));
            c->ev_update.push_back({e0, e1});
        }
    }
    if (check && nb > 0) {
        // check statistics (and, in residual mode, the new residuals) from this
        // tick's exact term and surrogate; k_update of this tick used the exact term
        const BlkItem* items = c->dblk + c->blk_off[ph];
        const bool resid = c->surr_mode == SSM_SURR_RESIDUAL;
        SSM_DISPATCH_D(d, hipLaunchKernelGGL((k_surr_err<T, D>), dim3((unsigned)nb), dim3(kBlk), 0, c->stream, items,
                                             c->dsys, c->P, c->pairsum, c->surr, c->smean, c->surr_res,
                                             (resid && c->surr_res_valid) ? 1 : 0, resid ? 1 : 0, c->err_part));
        HIP_TRY(hipGetLastError());
    }
    if (capture) {
        hipLaunchKernelGGL(k_tick_advance, dim3(1), dim3(64), 0, c->stream, c->dtick);
        HIP_TRY(hipGetLastError());
    }
    if (surr_on) {
        if (use_surr) c->surr_ticks++;
        if (!check && c->surr_fallback) c->surr_fallback_ticks++;
    }
    if (check && nb > 0) {
        // Gain mode: least-squares gain per component from the check's exact
        // and surrogate terms, then the relative error of the gained surrogate.
        // Residual mode: the error of the prediction with the residuals of the
        // previous check (the kernel has stored this check's residuals).
        // Over the stepping systems, the error decides whether the ticks until
        // the next check use the prediction or the exact sums.
        std::vector<double> h(kErrStats * nb);
        HIP_TRY(hipMemcpyAsync(h.data(), c->err_part, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        double se = 0.0, sb = 0.0, sr = 0.0, sps[kMaxD] = {0, 0, 0, 0}, sss[kMaxD] = {0, 0, 0, 0};
        for (int64_t q = 0; q < nb; ++q) {
            const double* r = &h[kErrStats * q];
            se += r[0];
            sb += r[1];
            sr += r[2 + 2 * kMaxD];
            for (int k = 0; k < d; ++k) {
                sps[k] += r[2 + 2 * k];
                sss[k] += r[3 + 2 * k];
            }
        }
        double se_q = se;
        if (c->surr_mode == SSM_SURR_GAIN) {
            se_q = sb;  // |g s - p|^2 = g^2 |s|^2 - 2 g s.p + |p|^2, per component
            for (int k = 0; k < d; ++k) {
                const double g = sss[k] > 0.0 ? sps[k] / sss[k] : 1.0;
                c->surr_gain[k] = g;
                se_q += g * g * sss[k] - 2.0 * g * sps[k];
            }
            se_q = std::max(se_q, 0.0);
        } else {
            c->surr_res_valid = true;
        }
        const double err = sb > 0.0 ? std::sqrt(se_q / sb) : (se_q > 0.0 ? INFINITY : 0.0);
        c->surr_last_raw_err = sb > 0.0 ? std::sqrt(sr / sb) : 0.0;
        c->surr_last_err = err;
        c->surr_max_err = std::max(c->surr_max_err, err);
        c->surr_checks++;
        if (recheck) c->surr_rechecks++;
        c->surr_fallback = !(err <= c->surr_tol);
    }
    return SSM_OK;
}

static void advance_host(ssm_ctx* c)
{
    for (auto& S : c->sys)
        if (c->tick % S.stride == 0) S.steps_done++;
    c->tick++;
}

// One tick: eager launches, or (graphs on, no profiling, no surrogate) the
// replay of this phase's captured graph.
template <typename T>
static ssm_status run_tick(ssm_ctx* c)
{
    const bool graph_ok = c->use_graphs && !c->profiling && c->surr_check_every == 0;
    if (!graph_ok) {
        ssm_status st = launch_tick<T>(c, false);
        if (st != SSM_OK) return st;
        advance_host(c);
        c->dtick_valid = false;
        return SSM_OK;
    }
    const int64_t ph = c->tick % c->max_stride;
    if (!c->dtick_valid) {
        // the device counter lags after eager ticks: set it (value copied at the call)
        const int64_t t = c->tick;
        HIP_TRY(hipMemcpyAsync(c->dtick, &t, sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        c->dtick_valid = true;
    }
    if (!c->phase_graph[ph]) {
        hipGraph_t g = nullptr;
        HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        ssm_status st = launch_tick<T>(c, true);
        hipError_t he = hipStreamEndCapture(c->stream, &g);
        if (st != SSM_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (he != hipSuccess) return fail(SSM_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(he));
        hipGraphExec_t ex = nullptr;
        he = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (he != hipSuccess) return fail(SSM_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(he));
        c->phase_graph[ph] = ex;
    }
    HIP_TRY(hipGraphLaunch(c->phase_graph[ph], c->stream));
    advance_host(c);
    return SSM_OK;
}

// ---------------------------------------------------------------------------
// persistent runs of small systems (ssm_small.hpp)
// ---------------------------------------------------------------------------
static const void* small_kernel(int prec, int d)
{
#define SSM_SMALL_K(T, KH)                                                  \
    switch (d) {                                                            \
        case 1: return reinterpret_cast<const void*>(&k_small<T, 1, KH>);   \
        case 2: return reinterpret_cast<const void*>(&k_small<T, 2, KH>);   \
        case 3: return reinterpret_cast<const void*>(&k_small<T, 3, KH>);   \
        case 4: return reinterpret_cast<const void*>(&k_small<T, 4, KH>);   \
        default: return nullptr;                                            \
    }
    if (prec == SSM_FP64) { SSM_SMALL_K(double, false) }
    if (prec == SSM_FP32) { SSM_SMALL_K(float, false) }
    SSM_SMALL_K(float, true)
#undef SSM_SMALL_K
}

// Why a context can never run persistent ticks ("" if it can): the default
// compensation, each system's staged positions within the LDS budget, and
// every tile's workgroup co-resident with the others.
static std::string small_ineligible(const ssm_ctx* c, int64_t tiles)
{
    if (c->kpair) return "kahan_span = 1";
    for (auto& S : c->sys)
        if ((int64_t)c->d * small_row(S.N) * (int64_t)elt(c->prec) > kSmallLdsBytes)
            return "a system's positions (d x N) exceed " + std::to_string(kSmallLdsBytes / 1024) + " KiB";
    int dev = 0, cus = 0, coop = 0, occ = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, small_kernel(c->prec, c->d), kSmallThreads, 0) != hipSuccess) {
        (void)hipGetLastError();
        return "device query failed";
    }
    if (!coop) return "the device has no cooperative launch";
    if (tiles > (int64_t)occ * cus)
        return std::to_string(tiles) + " tiles of 64 particles, more than the " + std::to_string((int64_t)occ * cus) +
               " co-resident workgroups";
    return "";
}

static int device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return cus;
}

// The default's choice between the two paths: estimated tick times in
// microseconds, coefficients from MI355X measurements.  Persistent: a fixed
// latency (staging, update, the barrier) plus the ordered pairs of the
// largest system's tile, 64 targets x N sources on one compute unit (64
// lane-slots per clock at 2.4 GHz, about 77 % issued), at 3d + 2 issue slots
// per pair (FP64: 16 more for its exponential).  Multi-launch: three
// dependent launches plus the symmetric pair sums over the whole chip
// (3.93e13 lane-slots/s, about 90 % issued), 2d + 1 slots per unordered pair
// (FP64: about 2d + 20).  Small case, FP32: 9.2 against 17.4 (measured 8.9
// and 18.2); FP64: 19.4 against 33 (18.8 and 31.7).
static bool small_preferred(const ssm_ctx* c)
{
    const bool f64 = c->prec == SSM_FP64;
    const double d = (double)c->d;
    double maxN = 0.0, sumN2 = 0.0;  // pairs per tick: each system steps every stride ticks
    for (auto& S : c->sys) {
        maxN = std::max(maxN, (double)S.N);
        sumN2 += (double)S.N * (double)S.N / (double)S.stride;
    }
    double pers = f64 ? 8.0 : 6.5, multi = f64 ? 30.0 : 17.0;
    if (c->has_pair) {
        pers += maxN * (3.0 * d + 2.0 + (f64 ? 16.0 : 0.0)) / 1850.0;
        multi += 0.5 * sumN2 * (f64 ? 2.0 * d + 20.0 : 2.0 * d + 1.0) / 3.5e7;
    }
    return pers < multi;
}

static bool small_usable(const ssm_ctx* c)
{
    return c->small_ok && c->surr_check_every == 0 && !c->profiling && !c->use_graphs;
}

// n ticks in one cooperative launch.
template <typename T>
static ssm_status launch_small(ssm_ctx* c, int64_t n)
{
    SmallArgs<T> a{};
    a.tiles = c->dtiles;
    a.sys = c->dsys;
    a.cf = c->coef;
    a.P = c->P;
    a.t0 = c->tick;
    a.n = n;
    a.ntile_tot = c->small_grid;
    a.X = (T*)c->X;
    a.Y = (T*)c->Y;
    a.Ys = (T*)c->Ys;
    a.sumY = c->sumY;
    a.sumX = c->sumX;
    a.bar = c->dbar;
    a.epoch0 = c->small_epoch;
    a.flags = c->dflags;
    a.nmax = c->dnmax;
    a.bm_lanes = c->small_lanes;
    a.needs_ybar = c->needs_ybar ? 1 : 0;
    a.wait_limit = c->small_wait_limit;
    void* args[] = {&a};
    HIP_TRY(hipLaunchCooperativeKernel(small_kernel(c->prec, c->d), dim3((unsigned)c->small_grid), dim3(kSmallThreads),
                                       args, 0, c->stream));
    c->small_epoch += small_barriers(c->fused, n);
    c->small_launches++;
    c->small_ticks += n;
    for (int64_t t = 0; t < n; ++t) advance_host(c);
    c->dtick_valid = false;
    c->psum_stale = true;
    return SSM_OK;
}

// What the multi-launch path reads from earlier ticks, after persistent ticks
// (which keep tile sums of their own and draw their increments directly): the
// block sums of Y*, and, in the middle of a window of path groups, the
// window's normal sums.
template <typename T>
static ssm_status refresh_after_small(ssm_ctx* c)
{
    const int64_t ph = c->tick % c->max_stride;
    if (ph != 0 && c->win_items > 0) {
        ssm_status st = launch_window<T>(c, c->tick - ph, nullptr);
        if (st != SSM_OK) return st;
    }
    const BlkItem* items = c->dblk + c->all_blk_off[0];
    const dim3 g((unsigned)c->all_blk_cnt);
    // k_ysums takes the steps done from the tick before: (tick - 1) / stride + 1
    const int64_t tick_arg = c->tick - 1;
    if (c->prec == SSM_FP64) {
        SSM_DISPATCH_D(c->d, hipLaunchKernelGGL((k_ysums<double, D>), g, dim3(kBlk), 0, c->stream, items, c->dsys,
                                                c->P, tick_arg, (const double*)c->Y, c->psumY, c->nblk_tot));
    } else {
        SSM_DISPATCH_D(c->d, hipLaunchKernelGGL((k_ysums<float, D>), g, dim3(kBlk), 0, c->stream, items, c->dsys,
                                                c->P, tick_arg, (const float*)c->Y, c->psumY, c->nblk_tot));
    }
    HIP_TRY(hipGetLastError());
    c->psum_stale = false;
    return SSM_OK;
}

template <typename T>
static ssm_status launch_init(ssm_ctx* c)
{
    const BlkItem* items = c->dblk + c->all_blk_off[0];
    const unsigned nb = (unsigned)c->all_blk_cnt;
    SSM_DISPATCH_D(c->d, hipLaunchKernelGGL((k_init<T, D>), dim3(nb), dim3(kBlk), 0, c->stream, items, c->dsys,
                                            c->coef, c->P, (T*)c->X, (T*)c->Y, (T*)c->Ys, c->psumX,
                                            c->nblk_tot));
    HIP_TRY(hipGetLastError());
    SSM_DISPATCH_D(c->d, hipLaunchKernelGGL((k_newton<T, D>), dim3(nb), dim3(kBlk), 0, c->stream, items, c->dsys,
                                            c->coef, c->P, (int64_t)-1, (const int64_t*)nullptr, (const T*)c->X, (T*)c->Y, (T*)c->Ys,
                                            c->psumX, c->psumY, c->nblk_tot, c->dflags, c->dnmax));
    HIP_TRY(hipGetLastError());
    return SSM_OK;
}

static ssm_status validate(const ssm_config* cfg)
{
    if (!cfg) return fail(SSM_ERR_INVALID, "cfg is NULL");
    if (cfg->d < 1 || cfg->d > SSM_MAX_D) return fail(SSM_ERR_INVALID, "d must be in 1..4");
    if (cfg->n_sys < 1 || !cfg->N || !cfg->ens || !cfg->h) return fail(SSM_ERR_INVALID, "need n_sys >= 1 and N, ens, h arrays");
    if (cfg->precision < SSM_FP64 || cfg->precision > SSM_FP32_KAHAN) return fail(SSM_ERR_INVALID, "unknown precision");
    if (!(cfg->T > 0.0) || !std::isfinite(cfg->T)) return fail(SSM_ERR_INVALID, "T must be > 0");
    if (!(cfg->h_fine > 0.0)) return fail(SSM_ERR_INVALID, "h_fine must be > 0");
    if (!(cfg->v_a >= 0.0)) return fail(SSM_ERR_INVALID, "v_a must be >= 0 (one-sided Lipschitz v)");
    if (!(cfg->v_kappa >= 0.0)) return fail(SSM_ERR_INVALID, "v_kappa must be >= 0");
    for (int k = 0; k < cfg->d; ++k)
        if (!(cfg->v_ak[k] >= 0.0)) return fail(SSM_ERR_INVALID, "v_ak must be >= 0 (one-sided Lipschitz v)");
    if (cfg->b_g != 0.0 && !(cfg->b_ell > 0.0)) return fail(SSM_ERR_INVALID, "b_ell must be > 0");
    if (cfg->targets_per_lane != 0 && cfg->targets_per_lane != 1 && cfg->targets_per_lane != 2 &&
        cfg->targets_per_lane != 4 && cfg->targets_per_lane != 8)
        return fail(SSM_ERR_INVALID, "targets_per_lane must be 0, 1, 2, 4 or 8");
    if (cfg->sources_per_item != 0 && cfg->sources_per_item < 64)
        return fail(SSM_ERR_INVALID, "sources_per_item must be 0 or >= 64");
    if (cfg->jside_band_groups < 0) return fail(SSM_ERR_INVALID, "jside_band_groups must be >= 0");
    if (cfg->persistent < -1 || cfg->persistent > 1) return fail(SSM_ERR_INVALID, "persistent must be -1, 0 or 1");
    for (int s = 0; s < cfg->n_sys; ++s) {
        const double h = cfg->h[s];
        if (cfg->N[s] < 1 || cfg->N[s] > 0x7fffffff - 1024) return fail(SSM_ERR_INVALID, "N out of range");
        if (!(h > 0.0)) return fail(SSM_ERR_INVALID, "h must be > 0");
        int64_t m, r;
        if (!is_int_ratio(cfg->T, h, &m)) return fail(SSM_ERR_INVALID, "T / h must be an integer");
        if (!is_int_ratio(h, cfg->h_fine, &r)) return fail(SSM_ERR_INVALID, "h / h_fine must be an integer >= 1");
        if (r > 0x7fffffff) return fail(SSM_ERR_INVALID, "h / h_fine too large");
        if (!(1.0 - h * cfg->v_rho > 0.0)) return fail(SSM_ERR_INVALID, "1 - h v_rho <= 0: the implicit step has no unique root (Lemma 4.1)");
        if (!cfg->allow_unstable_h && !(1.0 - h * (2.0 * cfg->v_rho + 1.0) > 0.0))
            return fail(SSM_ERR_INVALID, "h violates 1 - h (2 L_v + 1) > 0 (Theorem 2.6); set allow_unstable_h to override");
    }
    return SSM_OK;
}

// Largest j-side partial-sum buffer the symmetric scheme may take: 40 % of the
// device's free memory, or 32 GiB if the runtime cannot say.
static double jside_cap()
{
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess || free_b == 0) {
        (void)hipGetLastError();
        return 32.0 * (double)(1ull << 30);
    }
    return 0.4 * (double)free_b;
}

extern "C" ssm_status ssm_init(const ssm_config* cfg, ssm_ctx** out)
{
    if (!out) return fail(SSM_ERR_INVALID, "out is NULL");
    *out = nullptr;
    ssm_status st = validate(cfg);
    if (st != SSM_OK) return st;

    ssm_ctx* c = new (std::nothrow) ssm_ctx();
    if (!c) return fail(SSM_ERR_OOM, "host allocation failed");
    c->cfg = *cfg;
    c->cfg_N.assign(cfg->N, cfg->N + cfg->n_sys);
    c->cfg_ens.assign(cfg->ens, cfg->ens + cfg->n_sys);
    c->cfg_h.assign(cfg->h, cfg->h + cfg->n_sys);
    c->d = cfg->d;
    c->prec = cfg->precision;
    c->fused = (cfg->v_kappa == 0.0 && cfg->v_lam == 0.0);
    c->has_pair = cfg->b_g != 0.0;
    Coef& cf = c->coef;
    cf.v_rho = cfg->v_rho; cf.v_a = cfg->v_a; cf.v_kappa = cfg->v_kappa; cf.v_lam = cfg->v_lam;
    cf.b_c0 = cfg->b_c0; cf.b_lam = cfg->b_lam;
    for (int k = 0; k < kMaxD; ++k) {
        const bool in = k < cfg->d;
        cf.s0[k] = in ? cfg->s0[k] : 0.0; cf.s1[k] = in ? cfg->s1[k] : 0.0; cf.s2[k] = in ? cfg->s2[k] : 0.0;
        cf.x0_mean[k] = in ? cfg->x0_mean[k] : 0.0; cf.x0_std[k] = in ? cfg->x0_std[k] : 0.0;
    }
    c->needs_ybar = cfg->b_lam != 0.0;
    for (int k = 0; k < cfg->d; ++k)
        if (cfg->s2[k] != 0.0 || cfg->b_mean[k] != 0.0) c->needs_ybar = true;
    const double ell = c->has_pair ? cfg->b_ell : 1.0;
    c->ell = ell;
    cf.coord_scale = std::sqrt(kLog2e / (2.0 * ell * ell));
    cf.sqrt_hf = std::sqrt(cfg->h_fine);
    cf.seed = cfg->seed;
    cf.newton_max_iter = cfg->newton_max_iter > 0 ? cfg->newton_max_iter : 64;
    cf.has_pair = c->has_pair ? 1 : 0;
    cf.fused = c->fused ? 1 : 0;
    cf.v_cw = cfg->v_componentwise ? 1 : 0;
    cf.has_lin = 0;
    for (int k = 0; k < kMaxD; ++k) {
        const bool in = k < cfg->d;
        cf.v_ak[k] = in ? cfg->v_ak[k] : 0.0;
        cf.b_const[k] = in ? cfg->b_const[k] : 0.0;
        cf.b_mean[k] = in ? cfg->b_mean[k] : 0.0;
        if (cf.b_mean[k] != 0.0) cf.has_lin = 1;
        for (int l = 0; l < kMaxD; ++l) {
            cf.b_mat[k * kMaxD + l] = (in && l < cfg->d) ? cfg->b_mat[k * SSM_MAX_D + l] : 0.0;
            if (cf.b_mat[k * kMaxD + l] != 0.0) cf.has_lin = 1;
        }
        if (cf.b_const[k] != 0.0) cf.has_lin = 1;
    }

    // systems, strides, padding
    double h_min = cfg->h[0];
    for (int s = 1; s < cfg->n_sys; ++s) h_min = std::min(h_min, cfg->h[s]);
    int64_t off = 0, blk = 0;
    for (int s = 0; s < cfg->n_sys; ++s) {
        SysHost S{};
        S.N = cfg->N[s];
        S.ens = cfg->ens[s];
        S.h = cfg->h[s];
        if (!is_int_ratio(S.h, h_min, &S.stride)) { free_ctx(c); return fail(SSM_ERR_INVALID, "every h must be an integer multiple of the smallest h"); }
        is_int_ratio(S.h, cfg->h_fine, &S.r);
        S.off = off;
        S.nblk = (S.N + kBlk - 1) / kBlk;
        S.blk0 = blk;
        off += S.nblk * kBlk;
        blk += S.nblk;
        c->max_stride = std::max(c->max_stride, S.stride);
        c->sys.push_back(S);
    }
    for (auto& S : c->sys)
        if (c->max_stride % S.stride != 0) { free_ctx(c); return fail(SSM_ERR_INVALID, "every h / h_min must divide the largest such ratio"); }
    if (c->max_stride > 4096) { free_ctx(c); return fail(SSM_ERR_INVALID, "h_max / h_min larger than 4096"); }
    c->P = off;
    c->nblk_tot = blk;
    // path groups: systems of one ensemble and size step on the same Brownian
    // paths; with several step sizes, such a group draws each tick's normals
    // once into a window of max_stride ticks that all its members sum from
    std::vector<BlkItem> win_items;
    int64_t win_doubles = 0;
    if (c->max_stride > 1) {
        std::map<std::pair<int64_t, int32_t>, std::vector<int>> groups;
        for (int s = 0; s < (int)c->sys.size(); ++s) groups[{c->sys[s].N, c->sys[s].ens}].push_back(s);
        for (auto& kv : groups) {
            if (kv.second.size() < 2) continue;
            for (int s : kv.second) c->sys[s].win_off = win_doubles;
            const SysHost& R0 = c->sys[kv.second[0]];
            for (int64_t b = 0; b < R0.nblk; ++b) win_items.push_back(BlkItem{kv.second[0], (int32_t)b});
            win_doubles += c->max_stride * (int64_t)cfg->d * R0.N;
        }
        is_int_ratio(h_min, cfg->h_fine, &c->r_min);
        const int64_t wb = (c->r_min * cfg->d + 3) / 4;
        c->win_lanes = wb >= 16 ? 16 : wb >= 8 ? 8 : wb >= 4 ? 4 : wb >= 2 ? 2 : 1;
    }
    c->win_items = (int64_t)win_items.size();
    is_int_ratio(cfg->T, h_min, &c->ticks_total);

    // pair tiling: R targets per lane, L sources per item, scheme
    const bool f64 = c->prec == SSM_FP64;
    if (cfg->kahan_span != 0 && cfg->kahan_span != 1) { free_ctx(c); return fail(SSM_ERR_INVALID, "kahan_span must be 0 or 1"); }
    if (cfg->kahan_span == 1 && c->prec != SSM_FP32_KAHAN) { free_ctx(c); return fail(SSM_ERR_INVALID, "kahan_span = 1 needs the FP32-compensated precision"); }
    if (cfg->kahan_span == 1 && cfg->pair_scheme == 2) { free_ctx(c); return fail(SSM_ERR_INVALID, "kahan_span = 1 runs the ordered pair scheme only"); }
    c->kpair = cfg->kahan_span == 1;
    c->sym = cfg->pair_scheme != 1 && !c->kpair;
    {
        std::vector<int64_t> Ns;
        for (auto& S : c->sys) Ns.push_back(S.N);
        c->R = cfg->targets_per_lane > 0 ? cfg->targets_per_lane : default_R(c->d, Ns, c->sym);
    }
    // a target group's j-side sums must fit the kernel's LDS buffer
    if (c->sym && cfg->targets_per_lane <= 0)
        while (c->R > 1 && !sym_fits(f64, c->R, c->d)) c->R /= 2;
    if (c->sym && !sym_fits(f64, c->R, c->d)) {
        if (cfg->pair_scheme == 2) { free_ctx(c); return fail(SSM_ERR_INVALID, "symmetric scheme: targets_per_lane too large for this d and precision (64 x R x 4 x d must be <= " + std::to_string(sym_lds_for(f64, c->d)) + ")"); }
        c->sym = false;
    }
    for (int attempt = 0; attempt < 2; ++attempt) {
        std::vector<int64_t> Ns;
        for (auto& S : c->sys) Ns.push_back(S.N);
        // the symmetric scheme's j-side partials: one row of d x P elements of
        // the pair precision per target group (the groups of the largest
        // system); past 40 % of the device's free memory (115 GB of an idle
        // MI355X's 288 GB; 32 GiB when it cannot be queried) they run in bands
        // (k_jfold) of as many groups as fit 16 GiB (every row is read once per
        // tick either way, so larger bands would save only launches), or in
        // the requested bands
        c->band = 0;
        c->n_bands = 1;
        if (c->sym) {
            const int64_t group = 64 * (int64_t)c->R * kWaves;
            int64_t groups = 0;
            for (int64_t N : Ns) groups = std::max(groups, (N + group - 1) / group);
            const double row_bytes = (double)c->d * (double)c->P * elt(c->prec);
            int64_t band = 0;
            if (cfg->jside_band_groups > 0) {
                band = std::min<int64_t>(cfg->jside_band_groups, groups);
            } else if ((double)groups * row_bytes > jside_cap()) {
                band = (int64_t)(std::min(jside_cap(), 16.0 * (double)(1ull << 30)) / row_bytes);
                if (band < 1) {
                    if (cfg->pair_scheme == 2) { free_ctx(c); return fail(SSM_ERR_INVALID, "symmetric scheme: one j-side row does not fit 40 % of the free device memory; use ordered pairs"); }
                    c->sym = false;
                    continue;
                }
            }
            if (band > 0 && band < groups) {
                c->band = band;
                c->n_bands = (groups + band - 1) / band;
            }
        }
        if (cfg->sources_per_item > 0) {
            c->L = c->sym ? (cfg->sources_per_item + 15) / 16 * 16 : cfg->sources_per_item;
        } else {
            c->L = default_L(Ns, c->R, c->sym, c->d);
            // banded, each band's launch takes about the item count of an
            // unbanded one (enough workgroups to fill the chip)
            if (c->n_bands > 1) c->L = std::max<int64_t>(128, (c->L / c->n_bands + 15) / 16 * 16);
        }
        c->max_splits = 1;
        c->nb_max = 0;
        for (int s = 0; s < (int)c->sys.size(); ++s) {
            std::vector<std::pair<int64_t, PairItem>> scratch;
            int64_t nb = 0;
            c->sys[s].splits = plan_system(s, c->sys[s].N, c->R, c->sym, c->L, scratch, &nb);
            c->max_splits = std::max(c->max_splits, c->sys[s].splits);
            c->nb_max = std::max(c->nb_max, nb);
        }
        break;
    }

    // stream
    if (cfg->stream) {
        c->stream = (hipStream_t)cfg->stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) { free_ctx(c); return fail(SSM_ERR_HIP, "hipStreamCreate failed"); }
        c->own_stream = true;
    }

    // persistent runs of small systems: one workgroup per tile of 64 particles
    std::vector<SmallTile> tiles;
    if (cfg->persistent >= 0) {
        int64_t ntiles = 0;
        for (auto& S : c->sys) ntiles += (S.N + kSmallTile - 1) / kSmallTile;
        const std::string why = small_ineligible(c, ntiles);
        if (cfg->persistent == 1 && !why.empty()) { free_ctx(c); return fail(SSM_ERR_INVALID, "persistent = 1: " + why); }
        // default: at most one tile per compute unit, where the estimate
        // says the multi-launch tick is slower (bound by launch latency),
        // unless a tiling of the multi-launch pair kernels was asked for
        const bool tiled = cfg->targets_per_lane != 0 || cfg->sources_per_item != 0 || cfg->pair_scheme != 0 ||
                           cfg->jside_band_groups != 0;
        c->small_ok = why.empty() &&
                      (cfg->persistent == 1 || (!tiled && ntiles <= device_cus() && small_preferred(c)));
        if (c->small_ok) {
            for (int s = 0; s < (int)c->sys.size(); ++s) {
                const int32_t nt = (int32_t)((c->sys[s].N + kSmallTile - 1) / kSmallTile);
                const int32_t g0 = (int32_t)tiles.size();
                for (int32_t q = 0; q < nt; ++q) tiles.push_back(SmallTile{s, q, g0, nt});
            }
            c->small_grid = (int64_t)tiles.size();
            int64_t bmax = 1;
            for (auto& S : c->sys) bmax = std::max<int64_t>(bmax, (S.r * c->d + 3) / 4);
            c->small_lanes = bmax >= 16 ? 16 : bmax >= 8 ? 8 : bmax >= 4 ? 4 : bmax >= 2 ? 2 : 1;
            int dev = 0, khz = 0;
            if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) {
                (void)hipGetLastError();
                khz = 100000;  // the 100 MHz counter of gfx9
            }
            c->small_wait_limit = (int64_t)khz * 1000 * 4;  // 4 s per barrier wait
            if (const char* env = std::getenv("SSM_PERSISTENT_WAIT_US")) {
                const long long us = std::atoll(env);
                if (us >= 0) c->small_wait_limit = (int64_t)khz * us / 1000;
            }
        }
    }

    // work lists per phase
    std::vector<PairItem> pairs;
    std::vector<BlkItem> blks;
    std::vector<int32_t> sys_lists;
    {
        // per step and particle: about r d / 4 Philox blocks, or (path groups)
        // `stride` window entries, four per lane
        int64_t bmax = 1;
        for (auto& S : c->sys)
            bmax = std::max<int64_t>(bmax, S.win_off >= 0 ? (S.stride + 3) / 4 : (S.r * c->d + 3) / 4);
        c->bm_lanes = bmax >= 16 ? 16 : bmax >= 8 ? 8 : bmax >= 4 ? 4 : bmax >= 2 ? 2 : 1;
    }
    c->phase_graph.assign(c->max_stride, nullptr);
    c->use_graphs = cfg->graphs != 0;
    c->pair_off.resize(c->max_stride);
    c->pair_cnt.resize(c->max_stride);
    c->blk_off.resize(c->max_stride);
    c->blk_cnt.resize(c->max_stride);
    for (int64_t ph = 0; ph < c->max_stride; ++ph) {
        std::vector<int> act;
        for (int s = 0; s < (int)c->sys.size(); ++s)
            if (ph % c->sys[s].stride == 0) act.push_back(s);
        c->pair_off[ph] = (int64_t)pairs.size();
        std::vector<int64_t> boff;
        if (c->has_pair) build_pair_items(c, act, pairs, c->band > 0 ? &boff : nullptr);
        c->pair_cnt[ph] = (int64_t)pairs.size() - c->pair_off[ph];
        c->pair_band_off.push_back(boff);
        c->blk_off[ph] = (int64_t)blks.size();
        build_blk_items(c, act, blks);
        c->blk_cnt[ph] = (int64_t)blks.size() - c->blk_off[ph];
        c->sys_list_off.push_back((int64_t)sys_lists.size());
        for (int s : act) sys_lists.push_back(s);
        c->sys_list_cnt.push_back((int64_t)act.size());
    }
    {
        std::vector<int> all;
        for (int s = 0; s < (int)c->sys.size(); ++s) all.push_back(s);
        c->all_blk_off.push_back((int64_t)blks.size());
        build_blk_items(c, all, blks);
        c->all_blk_cnt = (int64_t)blks.size() - c->all_blk_off[0];
        // each system's blocks are consecutive in that list (ascending block order)
        c->sys_blk_off.assign(c->sys.size(), -1);
        for (int64_t q = c->all_blk_off[0]; q < (int64_t)blks.size(); ++q)
            if (blks[q].blk == 0) c->sys_blk_off[blks[q].sys] = q;
    }

    // device state
    const size_t e = elt(c->prec);
    const size_t field = (size_t)c->d * (size_t)c->P * e;
    std::vector<SysDev> sd;
    for (auto& S : c->sys) {
        SysDev x{};
        x.off = S.off;
        x.N = (int32_t)S.N;
        x.ens = S.ens;
        x.stride = (int32_t)S.stride;
        x.r = (int32_t)S.r;
        x.blk0 = (int32_t)S.blk0;
        x.nblk = (int32_t)S.nblk;
        x.splits = (int32_t)S.splits;
        x.sym_B = c->sym ? 64 * c->R * kWaves : 0;
        x.sym_L = c->sym ? (int32_t)c->L : 0;
        x.h = S.h;
        x.win_off = S.win_off >= 0 ? S.win_off : 0;
        x.win_W = S.win_off >= 0 ? (int32_t)c->max_stride : 0;
        x.pair_scale = c->has_pair ? cfg->b_g / ((double)S.N * cf.coord_scale) : 0.0;
        sd.push_back(x);
    }
#define ALLOC(ptr, bytes) do { st = dev_alloc(c, (void**)&(ptr), (bytes)); if (st != SSM_OK) { free_ctx(c); return st; } } while (0)
    ALLOC(c->X, field);
    ALLOC(c->Y, field);
    ALLOC(c->Ys, field);
    ALLOC(c->Bp, c->has_pair ? (size_t)c->max_splits * c->d * c->P * elt(c->prec) : 0);
    ALLOC(c->pairsum, c->has_pair ? (size_t)c->d * c->P * sizeof(double) : 0);
    ALLOC(c->Bpj, (c->has_pair && c->sym) ? (size_t)(c->band > 0 ? c->band : c->nb_max) * c->d * c->P * elt(c->prec) : 0);
    if (c->band > 0) ALLOC(c->jtot, (size_t)c->d * c->P * sizeof(double));
    ALLOC(c->psumX, 2 * (size_t)(c->d + 1) * c->nblk_tot * sizeof(double));
    ALLOC(c->psumY, 2 * (size_t)c->d * c->nblk_tot * sizeof(double));
    ALLOC(c->dsys, sd.size() * sizeof(SysDev));
    ALLOC(c->dpair, std::max<size_t>(pairs.size(), 1) * sizeof(PairItem));
    ALLOC(c->dblk, blks.size() * sizeof(BlkItem));
    ALLOC(c->dflags, sizeof(Flags));
    ALLOC(c->dnmax, (size_t)c->nblk_tot * kSlotsPerBlk * sizeof(int32_t));
    ALLOC(c->dtick, sizeof(int64_t));
    ALLOC(c->dW, (size_t)c->d * c->P * sizeof(double));
    ALLOC(c->dsys_list, sys_lists.size() * sizeof(int32_t));
    int64_t maxN = 0;
    for (auto& S : c->sys) maxN = std::max(maxN, S.N);
    ALLOC(c->dstage, std::max<size_t>((size_t)c->d * maxN * sizeof(double), 2 * kMaxD * sizeof(double)));
    ALLOC(c->dred, (size_t)kMaxD * kRedBlocks * sizeof(double));
    if (c->win_items > 0) {
        ALLOC(c->win, (size_t)win_doubles * sizeof(double));
        ALLOC(c->dwin_items, (size_t)c->win_items * sizeof(BlkItem));
    }
    ALLOC(c->dsq, c->sys.size() * sizeof(double));
    ALLOC(c->ymean, c->sys.size() * kMaxD * sizeof(double));
    if (c->small_ok) {
        ALLOC(c->dtiles, tiles.size() * sizeof(SmallTile));
        ALLOC(c->sumY, 2 * (size_t)c->d * c->small_grid * sizeof(double));
        ALLOC(c->sumX, (size_t)(c->d + 1) * c->small_grid * sizeof(double));
        ALLOC(c->dbar, c->sys.size() * kBarLine * sizeof(uint64_t));
    }
#undef ALLOC
    hipError_t he = hipMemcpyAsync(c->dsys, sd.data(), sd.size() * sizeof(SysDev), hipMemcpyHostToDevice, c->stream);
    if (he == hipSuccess && !pairs.empty()) he = hipMemcpyAsync(c->dpair, pairs.data(), pairs.size() * sizeof(PairItem), hipMemcpyHostToDevice, c->stream);
    if (he == hipSuccess) he = hipMemcpyAsync(c->dblk, blks.data(), blks.size() * sizeof(BlkItem), hipMemcpyHostToDevice, c->stream);
    if (he == hipSuccess) he = hipMemcpyAsync(c->dsys_list, sys_lists.data(), sys_lists.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream);
    if (he == hipSuccess && c->win_items > 0)
        he = hipMemcpyAsync(c->dwin_items, win_items.data(), win_items.size() * sizeof(BlkItem), hipMemcpyHostToDevice, c->stream);
    if (he == hipSuccess) he = hipMemsetAsync(c->dflags, 0, sizeof(Flags), c->stream);
    if (he == hipSuccess) he = hipMemsetAsync(c->dnmax, 0, (size_t)c->nblk_tot * kSlotsPerBlk * sizeof(int32_t), c->stream);
    if (he == hipSuccess) he = hipMemsetAsync(c->dtick, 0, sizeof(int64_t), c->stream);
    if (he == hipSuccess && c->small_ok) he = hipMemcpyAsync(c->dtiles, tiles.data(), tiles.size() * sizeof(SmallTile), hipMemcpyHostToDevice, c->stream);
    if (he == hipSuccess && c->small_ok) he = hipMemsetAsync(c->dbar, 0, c->sys.size() * kBarLine * sizeof(uint64_t), c->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);  // host vectors go out of scope
    if (he != hipSuccess) { std::string m = hipGetErrorString(he); free_ctx(c); return fail(SSM_ERR_HIP, "upload: " + m); }

    st = (c->prec == SSM_FP64) ? launch_init<double>(c) : launch_init<float>(c);
    if (st != SSM_OK) { free_ctx(c); return st; }
    *out = c;
    return SSM_OK;
}

extern "C" ssm_status ssm_step(ssm_ctx* c, int64_t n_ticks)
{
    if (!c) return fail(SSM_ERR_INVALID, "ctx is NULL");
    if (c->broken) return fail(SSM_ERR_STATE, "a persistent run of this context was aborted; the context is unusable");
    if (n_ticks < 0) return fail(SSM_ERR_INVALID, "n_ticks < 0");
    if (c->tick + n_ticks > c->ticks_total) return fail(SSM_ERR_STATE, "stepping past T");
    if (n_ticks == 0) return SSM_OK;
    if (small_usable(c)) {
        // launches of at most kSmallTicksPerLaunch ticks, so that one call
        // does not hold the GPU for an unbounded time (a run split over
        // launches equals one launch bit for bit)
        for (int64_t done = 0; done < n_ticks;) {
            const int64_t n = std::min<int64_t>(n_ticks - done, kSmallTicksPerLaunch);
            ssm_status st = (c->prec == SSM_FP64) ? launch_small<double>(c, n) : launch_small<float>(c, n);
            if (st != SSM_OK) return st;
            done += n;
        }
        return SSM_OK;
    }
    if (c->psum_stale) {
        ssm_status st = (c->prec == SSM_FP64) ? refresh_after_small<double>(c) : refresh_after_small<float>(c);
        if (st != SSM_OK) return st;
    }
    for (int64_t t = 0; t < n_ticks; ++t) {
        ssm_status st = (c->prec == SSM_FP64) ? run_tick<double>(c) : run_tick<float>(c);
        if (st != SSM_OK) return st;
    }
    return SSM_OK;
}

extern "C" ssm_status ssm_sync(ssm_ctx* c)
{
    if (!c) return fail(SSM_ERR_INVALID, "ctx is NULL");
    HIP_TRY(hipStreamSynchronize(c->stream));
    Flags f{};
    HIP_TRY(hipMemcpy(&f, c->dflags, sizeof(Flags), hipMemcpyDeviceToHost));
    if (f.abort) {
        c->broken = true;
        return fail(SSM_ERR_HIP, "a persistent run was aborted: a barrier wait ran out of time");
    }
    if (f.newton_fail) return fail(SSM_ERR_NEWTON, std::to_string(f.newton_fail) + " implicit solves did not converge");
    if (f.nonfinite) return fail(SSM_ERR_NONFINITE, std::to_string(f.nonfinite) + " particles became non-finite");
    return SSM_OK;
}

extern "C" ssm_status ssm_run(ssm_ctx* c)
{
    if (!c) return fail(SSM_ERR_INVALID, "ctx is NULL");
    ssm_status st = ssm_step(c, c->ticks_total - c->tick);
    if (st != SSM_OK) return st;
    return ssm_sync(c);
}

// ---------------------------------------------------------------------------
// moments, state access, rMSE
// ---------------------------------------------------------------------------
// Reductions over one system's particles in a fixed order: block b of a
// grid of nb <= kRedBlocks blocks adds the particles b kBlk + t + m nb kBlk
// per thread and then over the block (tree), and one block adds the nb
// partials in block order.

static unsigned red_blocks(int64_t N)
{
    return (unsigned)std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, (N + kBlk - 1) / kBlk));
}

// Partial sums per component k of X_k (mean == nullptr) or of (X_k - mean[k])^2.
template <typename T>
__global__ void k_moments_part(const T* __restrict__ X, int64_t P, int64_t off, int64_t N, int d,
                               const double* __restrict__ mean, double* __restrict__ part)
{
    __shared__ double red[kBlk];
    for (int k = 0; k < d; ++k) {
        const double m = mean ? mean[k] : 0.0;
        double s = 0.0;
        for (int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x; i < N; i += (int64_t)gridDim.x * kBlk) {
            const double x = (double)X[k * P + off + i];
            s += mean ? (x - m) * (x - m) : x;
        }
        const double t = block_sum(s, red);
        if (threadIdx.x == 0) part[k * gridDim.x + blockIdx.x] = t;
    }
}

// out[k] = scale * (sum over b < nb of part[k nb + b]), one block.
__global__ void k_red_final(const double* __restrict__ part, int nb, int d, double scale, double* __restrict__ out)
{
    __shared__ double red[kBlk];
    for (int k = 0; k < d; ++k) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nb; b += kBlk) s += part[k * nb + b];
        const double t = block_sum(s, red);
        if (threadIdx.x == 0) out[k] = t * scale;
    }
}

template <typename T>
__global__ void k_gather(const T* __restrict__ X, int64_t P, int64_t off, int64_t N, int d, double* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    for (int k = 0; k < d; ++k) out[(int64_t)k * N + i] = (double)X[k * P + off + i];
}

template <typename T>
__global__ void k_scatter(const double* __restrict__ in, int64_t P, int64_t off, int64_t N, int d, T* __restrict__ X)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    for (int k = 0; k < d; ++k) X[k * P + off + i] = (T)in[(int64_t)k * N + i];
}

// Partial sums of |A^i - B^i|^2 (same grid rule as k_moments_part).
template <typename TA, typename TB>
__global__ void k_sqdiff_part(const TA* __restrict__ A, int64_t PA, int64_t offA, const TB* __restrict__ B, int64_t PB,
                              int64_t offB, int64_t N, int d, double* __restrict__ part)
{
    __shared__ double red[kBlk];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x; i < N; i += (int64_t)gridDim.x * kBlk)
        for (int k = 0; k < d; ++k) {
            const double c = (double)A[k * PA + offA + i] - (double)B[k * PB + offB + i];
            s += c * c;
        }
    const double t = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// one system of a against one system of b; result in dout (device), async on a's stream
static ssm_status launch_sqdiff(ssm_ctx* a, int sa, ssm_ctx* b, int sb, double* dout)
{
    const SysHost& A = a->sys[sa];
    const SysHost& B = b->sys[sb];
    const bool fa = a->prec == SSM_FP64, fb = b->prec == SSM_FP64;
    const unsigned nb = red_blocks(A.N);
#define SQD(TA, TB) hipLaunchKernelGGL((k_sqdiff_part<TA, TB>), dim3(nb), dim3(kBlk), 0, a->stream, (const TA*)a->X, a->P, \
                                       A.off, (const TB*)b->X, b->P, B.off, A.N, a->d, a->dred)
    if (fa && fb) SQD(double, double);
    else if (fa) SQD(double, float);
    else if (fb) SQD(float, double);
    else SQD(float, float);
#undef SQD
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_red_final, dim3(1), dim3(kBlk), 0, a->stream, (const double*)a->dred, (int)nb, 1, 1.0, dout);
    HIP_TRY(hipGetLastError());
    return SSM_OK;
}

extern "C" ssm_status ssm_moments(ssm_ctx* c, int32_t sys, double* mean, double* var)
{
    if (!c || !mean || !var) return fail(SSM_ERR_INVALID, "NULL argument");
    if (sys < 0 || sys >= (int32_t)c->sys.size()) return fail(SSM_ERR_INVALID, "sys out of range");
    const SysHost& S = c->sys[sys];
    // two passes (mean, then the mean square deviation about it), each a
    // fixed-order partial-sum launch and a final one-block sum into dstage
    const unsigned nb = red_blocks(S.N);
    const double inv_n = 1.0 / (double)S.N;
    for (int pass = 0; pass < 2; ++pass) {
        const double* mean = pass ? c->dstage : nullptr;
        if (c->prec == SSM_FP64)
            hipLaunchKernelGGL(k_moments_part<double>, dim3(nb), dim3(kBlk), 0, c->stream, (const double*)c->X, c->P, S.off,
                               S.N, c->d, mean, c->dred);
        else
            hipLaunchKernelGGL(k_moments_part<float>, dim3(nb), dim3(kBlk), 0, c->stream, (const float*)c->X, c->P, S.off,
                               S.N, c->d, mean, c->dred);
        HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_red_final, dim3(1), dim3(kBlk), 0, c->stream, (const double*)c->dred, (int)nb, c->d, inv_n,
                           c->dstage + pass * kMaxD);
        HIP_TRY(hipGetLastError());
    }
    double buf[2 * kMaxD];
    HIP_TRY(hipMemcpyAsync(buf, c->dstage, sizeof(buf), hipMemcpyDeviceToHost, c->stream));
    ssm_status st = ssm_sync(c);
    for (int k = 0; k < c->d; ++k) {
        mean[k] = buf[k];
        var[k] = buf[kMaxD + k];
    }
    return st;
}

extern "C" ssm_status ssm_get_state(ssm_ctx* c, int32_t sys, int32_t which, double* host, int64_t* step)
{
    if (!c || !host) return fail(SSM_ERR_INVALID, "NULL argument");
    if (sys < 0 || sys >= (int32_t)c->sys.size()) return fail(SSM_ERR_INVALID, "sys out of range");
    if (which != 0 && which != 1) return fail(SSM_ERR_INVALID, "which must be 0 (X) or 1 (Y*)");
    const SysHost& S = c->sys[sys];
    const void* src = which == 0 ? c->X : c->Y;
    const unsigned g = (unsigned)((S.N + kBlk - 1) / kBlk);
    if (c->prec == SSM_FP64)
        hipLaunchKernelGGL(k_gather<double>, dim3(g), dim3(kBlk), 0, c->stream, (const double*)src, c->P, S.off, S.N, c->d, c->dstage);
    else
        hipLaunchKernelGGL(k_gather<float>, dim3(g), dim3(kBlk), 0, c->stream, (const float*)src, c->P, S.off, S.N, c->d, c->dstage);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(host, c->dstage, (size_t)c->d * S.N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    ssm_status st = ssm_sync(c);
    if (step) *step = S.steps_done;
    return st;
}

// Recompute Y* = F_h(X) and its block sums for system sys after X was
// written from outside the step loop (the parity of the system's step count
// selects the double-buffered sums).  When v depends on mu^X, the block sums
// of X (mean and second moment) are recomputed first, into the parity slot
// the implicit solve reads.  Asynchronous on the context's stream.
static ssm_status refresh_implicit(ssm_ctx* c, int32_t sys)
{
    const SysHost& S = c->sys[sys];
    const BlkItem* items = c->dblk + c->sys_blk_off[sys];
    const dim3 g((unsigned)S.nblk);
    // k_newton derives the step count from the tick: tick = (steps_done - 1) * stride
    const int64_t tick_arg = S.steps_done == 0 ? -1 : (S.steps_done - 1) * S.stride;
    if (c->prec == SSM_FP64) {
        if (!c->fused)
            SSM_DISPATCH_D(c->d, hipLaunchKernelGGL((k_xsums<double, D>), g, dim3(kBlk), 0, c->stream, items, c->dsys,
                                                    c->P, tick_arg, (const double*)c->X, c->psumX, c->nblk_tot));
        SSM_DISPATCH_D(c->d, hipLaunchKernelGGL((k_newton<double, D>), g, dim3(kBlk), 0, c->stream,
                                                items, c->dsys, c->coef, c->P, tick_arg, (const int64_t*)nullptr, (const double*)c->X, (double*)c->Y,
                                                (double*)c->Ys, c->psumX, c->psumY, c->nblk_tot, c->dflags, c->dnmax));
    } else {
        if (!c->fused)
            SSM_DISPATCH_D(c->d, hipLaunchKernelGGL((k_xsums<float, D>), g, dim3(kBlk), 0, c->stream, items, c->dsys,
                                                    c->P, tick_arg, (const float*)c->X, c->psumX, c->nblk_tot));
        SSM_DISPATCH_D(c->d, hipLaunchKernelGGL((k_newton<float, D>), g, dim3(kBlk), 0, c->stream,
                                                items, c->dsys, c->coef, c->P, tick_arg, (const int64_t*)nullptr, (const float*)c->X, (float*)c->Y,
                                                (float*)c->Ys, c->psumX, c->psumY, c->nblk_tot, c->dflags, c->dnmax));
    }
    HIP_TRY(hipGetLastError());
    return SSM_OK;
}

// The surrogate's stored residuals and fitted gains belong to the state and
// weights they were taken from: after a change of either, the ticks up to the
// next check use the exact pair sums (as after a failed check).
static void surrogate_invalidate(ssm_ctx* c)
{
    c->surr_res_valid = false;
    c->surr_fallback = true;
    for (int k = 0; k < kMaxD; ++k) c->surr_gain[k] = 1.0;
}

// Move the context to tick t (a step boundary of every system): each system's
// step count becomes ceil(t / stride), and every system's Y* is recomputed at
// the new parity of its step count.
static ssm_status seek_tick(ssm_ctx* c, int64_t t)
{
    c->tick = t;
    for (auto& S : c->sys) S.steps_done = (t + S.stride - 1) / S.stride;
    c->dtick_valid = false;
    for (int32_t s = 0; s < (int32_t)c->sys.size(); ++s) {
        ssm_status st = refresh_implicit(c, s);
        if (st != SSM_OK) return st;
    }
    return SSM_OK;
}

extern "C" ssm_status ssm_set_state(ssm_ctx* c, int32_t sys, const double* host, int64_t step)
{
    if (!c || !host) return fail(SSM_ERR_INVALID, "NULL argument");
    if (sys < 0 || sys >= (int32_t)c->sys.size()) return fail(SSM_ERR_INVALID, "sys out of range");
    const SysHost& S = c->sys[sys];
    int64_t t = -1;
    if (step >= 0) {
        if (step > (c->ticks_total + S.stride - 1) / S.stride) return fail(SSM_ERR_INVALID, "step past T");
        t = step * S.stride;
        if (t % c->max_stride != 0)
            return fail(SSM_ERR_INVALID, "step x (h / h_min) must be a multiple of h_max / h_min "
                                         "(a step boundary of every system)");
        if (t > c->ticks_total) return fail(SSM_ERR_INVALID, "step past T");
    } else if (step != -1) {
        return fail(SSM_ERR_INVALID, "step must be >= 0, or -1 to keep the step count");
    }
    HIP_TRY(hipStreamSynchronize(c->stream));  // dstage may still be read by earlier work
    surrogate_invalidate(c);
    HIP_TRY(hipMemcpyAsync(c->dstage, host, (size_t)c->d * S.N * sizeof(double), hipMemcpyHostToDevice, c->stream));
    const unsigned g = (unsigned)((S.N + kBlk - 1) / kBlk);
    if (c->prec == SSM_FP64)
        hipLaunchKernelGGL(k_scatter<double>, dim3(g), dim3(kBlk), 0, c->stream, c->dstage, c->P, S.off, S.N, c->d, (double*)c->X);
    else
        hipLaunchKernelGGL(k_scatter<float>, dim3(g), dim3(kBlk), 0, c->stream, c->dstage, c->P, S.off, S.N, c->d, (float*)c->X);
    HIP_TRY(hipGetLastError());
    ssm_status st = (t >= 0 && t != c->tick) ? seek_tick(c, t) : refresh_implicit(c, sys);
    if (st != SSM_OK) return st;
    return ssm_sync(c);
}

extern "C" ssm_status ssm_state_layout(ssm_ctx* c, int64_t* P, int64_t* offsets, int32_t* elt_bytes)
{
    if (!c || !P) return fail(SSM_ERR_INVALID, "NULL argument");
    *P = c->P;
    if (offsets)
        for (size_t s = 0; s < c->sys.size(); ++s) offsets[s] = c->sys[s].off;
    if (elt_bytes) *elt_bytes = (int32_t)elt(c->prec);
    return SSM_OK;
}

extern "C" ssm_status ssm_bind_state(ssm_ctx* c, void* dev, size_t bytes)
{
    if (!c || !dev) return fail(SSM_ERR_INVALID, "NULL argument");
    const size_t need = (size_t)c->d * (size_t)c->P * elt(c->prec);
    if (bytes < need) return fail(SSM_ERR_INVALID, "buffer smaller than d x P elements of the storage precision");
    if ((uintptr_t)dev % 16 != 0) return fail(SSM_ERR_INVALID, "buffer must be 16-byte aligned");
    if (dev == c->X) return SSM_OK;
    // the current state (padding slots included) moves into the buffer in stream order
    HIP_TRY(hipMemcpyAsync(dev, c->X, need, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (!c->x_bound) {
        (void)hipFree(c->X);
        c->bytes -= (int64_t)need;
    }
    c->X = dev;
    c->x_bound = true;
    // captured tick graphs hold the old address
    for (auto& g : c->phase_graph)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    return ssm_sync(c);
}

extern "C" ssm_status ssm_state_refresh(ssm_ctx* c, int32_t sys)
{
    if (!c) return fail(SSM_ERR_INVALID, "ctx is NULL");
    if (sys < -1 || sys >= (int32_t)c->sys.size()) return fail(SSM_ERR_INVALID, "sys out of range");
    ssm_status st = ssm_sync(c);
    if (st != SSM_OK) return st;
    surrogate_invalidate(c);
    for (int32_t s = (sys < 0 ? 0 : sys); s < (sys < 0 ? (int32_t)c->sys.size() : sys + 1); ++s) {
        st = refresh_implicit(c, s);
        if (st != SSM_OK) return st;
    }
    return ssm_sync(c);
}

extern "C" ssm_status ssm_rmse(ssm_ctx* a, ssm_ctx* b, double* per_sys, double* rmse)
{
    if (!a || !b || !rmse) return fail(SSM_ERR_INVALID, "NULL argument");
    if (a->d != b->d || a->sys.size() != b->sys.size()) return fail(SSM_ERR_INVALID, "contexts differ in layout");
    for (size_t s = 0; s < a->sys.size(); ++s)
        if (a->sys[s].N != b->sys[s].N) return fail(SSM_ERR_INVALID, "contexts differ in layout");
    ssm_status st = ssm_sync(b);
    if (st != SSM_OK) return st;
    const int n = (int)a->sys.size();
    for (int s = 0; s < n && st == SSM_OK; ++s) st = launch_sqdiff(a, s, b, s, a->dsq + s);
    if (st != SSM_OK) return st;
    std::vector<double> h(n);
    hipError_t he = hipMemcpyAsync(h.data(), a->dsq, n * sizeof(double), hipMemcpyDeviceToHost, a->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(a->stream);
    if (he != hipSuccess) return fail(SSM_ERR_HIP, std::string("rmse: ") + hipGetErrorString(he));
    double tot = 0.0;
    int64_t cnt = 0;
    for (int s = 0; s < n; ++s) {
        if (per_sys) per_sys[s] = h[s];
        tot += h[s];
        cnt += a->sys[s].N;
    }
    *rmse = std::sqrt(tot / (double)cnt);
    return ssm_sync(a);
}

extern "C" ssm_status ssm_sqdiff(ssm_ctx* a, int32_t sys_a, ssm_ctx* b, int32_t sys_b, double* out)
{
    if (!a || !b || !out) return fail(SSM_ERR_INVALID, "NULL argument");
    if (sys_a < 0 || sys_a >= (int32_t)a->sys.size() || sys_b < 0 || sys_b >= (int32_t)b->sys.size())
        return fail(SSM_ERR_INVALID, "sys out of range");
    if (a->d != b->d || a->sys[sys_a].N != b->sys[sys_b].N) return fail(SSM_ERR_INVALID, "systems differ in d or N");
    ssm_status st = ssm_sync(b);
    if (st != SSM_OK) return st;
    st = launch_sqdiff(a, sys_a, b, sys_b, a->dstage);
    if (st != SSM_OK) return st;
    HIP_TRY(hipMemcpyAsync(out, a->dstage, sizeof(double), hipMemcpyDeviceToHost, a->stream));
    return ssm_sync(a);
}

extern "C" ssm_status ssm_info(ssm_ctx* c, ssm_info_t* out)
{
    if (!c || !out) return fail(SSM_ERR_INVALID, "NULL argument");
    HIP_TRY(hipStreamSynchronize(c->stream));
    Flags f{};
    HIP_TRY(hipMemcpy(&f, c->dflags, sizeof(Flags), hipMemcpyDeviceToHost));
    out->tick = c->tick;
    out->ticks_total = c->ticks_total;
    std::vector<int32_t> nmax((size_t)c->nblk_tot * kSlotsPerBlk);
    HIP_TRY(hipMemcpy(nmax.data(), c->dnmax, nmax.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    out->newton_max_seen = nmax.empty() ? 0 : *std::max_element(nmax.begin(), nmax.end());
    out->newton_failures = f.newton_fail;
    out->nonfinite = f.nonfinite;
    out->n_pair_items = (int32_t)c->pair_cnt[0];
    out->targets_per_lane = c->R;
    out->sources_per_item = (int32_t)c->L;
    out->symmetric = c->sym ? 1 : 0;
    out->jside_band_groups = (int32_t)c->band;
    out->device_bytes = c->bytes;
    out->pair_launches = (int64_t)c->ev_pair.size();
    out->pair_ms = elapsed_ms(c->ev_pair);
    out->update_launches = (int64_t)c->ev_update.size();
    out->update_ms = elapsed_ms(c->ev_update);
    out->surr_checks = c->surr_checks;
    out->surr_ticks = c->surr_ticks;
    out->surr_fallback_ticks = c->surr_fallback_ticks;
    out->surr_rechecks = c->surr_rechecks;
    out->surr_last_err = c->surr_last_err;
    out->surr_max_err = c->surr_max_err;
    out->surr_last_raw_err = c->surr_last_raw_err;
    for (int k = 0; k < SSM_MAX_D; ++k) out->surr_gain[k] = c->surr_gain[k];
    out->persistent = c->small_ok ? 1 : 0;
    out->persistent_tiles = (int32_t)(c->small_ok ? c->small_grid : 0);
    out->persistent_launches = c->small_launches;
    out->persistent_ticks = c->small_ticks;
    return SSM_OK;
}

extern "C" ssm_status ssm_profile(ssm_ctx* c, int32_t every)
{
    if (!c) return fail(SSM_ERR_INVALID, "ctx is NULL");
    if (every < 0) return fail(SSM_ERR_INVALID, "every must be >= 0");
    HIP_TRY(hipStreamSynchronize(c->stream));
    recycle_events(c, c->ev_pair);
    recycle_events(c, c->ev_update);
    c->profiling = every > 0;
    c->profile_every = every > 0 ? every : 1;
    return SSM_OK;
}

extern "C" void ssm_destroy(ssm_ctx* c) { free_ctx(c); }

// ---------------------------------------------------------------------------
// kernel-level entry points
// ---------------------------------------------------------------------------

// Plan of the kernel-level pair sum over one system of N particles.
struct KPlan {
    bool sym;
    int R;
    int64_t L, isplits, nb;
    std::vector<PairItem> items;
};

static KPlan kernel_plan(int32_t d, int64_t N, int32_t precision)
{
    KPlan p{};
    p.sym = true;
    p.R = default_R(d, std::vector<int64_t>{N}, p.sym);
    while (p.R > 1 && !sym_fits(precision == SSM_FP64, p.R, d)) p.R /= 2;
    p.L = default_L(std::vector<int64_t>{N}, p.R, p.sym, d);
    std::vector<std::pair<int64_t, PairItem>> tmp;
    p.isplits = plan_system(0, N, p.R, p.sym, p.L, tmp, &p.nb);
    order_items(tmp, p.items);
    return p;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static size_t kernel_ws_bytes(int32_t d, int64_t N, int32_t precision, const KPlan& p)
{
    return align256(sizeof(SysDev)) + align256(p.items.size() * sizeof(PairItem)) +
           align256((size_t)d * N * elt(precision)) + align256((size_t)p.isplits * d * N * elt(precision)) +
           align256((size_t)std::max<int64_t>(p.nb, 1) * d * N * elt(precision));
}

extern "C" size_t ssm_pair_workspace_bytes(int32_t d, int64_t N, int32_t precision)
{
    if (d < 1 || d > SSM_MAX_D || N < 1 || N > 0x7fffffff - 1024) return 0;
    if (precision < SSM_FP64 || precision > SSM_FP32_KAHAN) return 0;
    return kernel_ws_bytes(d, N, precision, kernel_plan(d, N, precision));
}

extern "C" ssm_status ssm_pair_sum(int32_t d, int64_t N, int32_t precision, const void* Y, double ell,
                                   double* K, void* workspace, size_t workspace_bytes, void* stream)
{
    if (d < 1 || d > SSM_MAX_D) return fail(SSM_ERR_INVALID, "d must be in 1..4");
    if (N < 1 || N > 0x7fffffff - 1024) return fail(SSM_ERR_INVALID, "N out of range");
    if (precision < SSM_FP64 || precision > SSM_FP32_KAHAN) return fail(SSM_ERR_INVALID, "unknown precision");
    if (!Y || !K || !workspace) return fail(SSM_ERR_INVALID, "NULL pointer");
    if (!(ell > 0.0)) return fail(SSM_ERR_INVALID, "ell must be > 0");
    const KPlan plan = kernel_plan(d, N, precision);
    const size_t need = kernel_ws_bytes(d, N, precision, plan);
    if (workspace_bytes < need) return fail(SSM_ERR_INVALID, "workspace too small: need " + std::to_string(need));
    hipStream_t st = (hipStream_t)stream;
    SysDev S{};
    S.off = 0;
    S.N = (int32_t)N;
    S.stride = 1;
    S.r = 1;
    S.nblk = (int32_t)((N + kBlk - 1) / kBlk);
    S.splits = (int32_t)plan.isplits;
    S.sym_B = plan.sym ? 64 * plan.R * kWaves : 0;
    S.sym_L = plan.sym ? (int32_t)plan.L : 0;
    const double c = std::sqrt(kLog2e / (2.0 * ell * ell));
    S.pair_scale = 1.0 / ((double)N * c);  // unscaled sums of the scaled coordinates -> (1/N) sum
    char* w = (char*)workspace;
    SysDev* dS = (SysDev*)w; w += align256(sizeof(SysDev));
    PairItem* dI = (PairItem*)w; w += align256(plan.items.size() * sizeof(PairItem));
    void* dYs = (void*)w; w += align256((size_t)d * N * elt(precision));
    void* dBp = (void*)w; w += align256((size_t)plan.isplits * d * N * elt(precision));
    void* dBpj = (void*)w;
    HIP_TRY(hipMemcpyAsync(dS, &S, sizeof(S), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(dI, plan.items.data(), plan.items.size() * sizeof(PairItem), hipMemcpyHostToDevice, st));
    const int64_t n = (int64_t)d * N;
    const dim3 g1((unsigned)((n + 255) / 256));
    const dim3 gp((unsigned)(plan.sym ? plan.items.size() : (plan.items.size() + kWaves - 1) / kWaves));
    if (precision == SSM_FP64) {
        hipLaunchKernelGGL(k_scale_copy<double>, g1, dim3(256), 0, st, (const double*)Y, (double*)dYs, n, c);
        launch_pair<double>(d, plan.R, false, gp, st, dI, (int)plan.items.size(), dS, (const double*)dYs, N, (double*)dBp, (double*)dBpj, plan.sym);
    } else {
        hipLaunchKernelGGL(k_scale_copy<float>, g1, dim3(256), 0, st, (const float*)Y, (float*)dYs, n, c);
        launch_pair<float>(d, plan.R, precision == SSM_FP32_KAHAN, gp, st, dI, (int)plan.items.size(), dS, (const float*)dYs, N, (float*)dBp, (float*)dBpj, plan.sym);
    }
    const dim3 gc((unsigned)(4 * ((N + kBlk - 1) / kBlk)));
    if (precision == SSM_FP64) {
        SSM_DISPATCH_D(d, hipLaunchKernelGGL((k_combine<double, D>), gc, dim3(64 * kCombineWaves), 0, st,
                                             (const BlkItem*)nullptr, dS, N, (const double*)dBp, (const double*)dBpj,
                                             (const double*)nullptr, K));
    } else {
        SSM_DISPATCH_D(d, hipLaunchKernelGGL((k_combine<float, D>), gc, dim3(64 * kCombineWaves), 0, st,
                                             (const BlkItem*)nullptr, dS, N, (const float*)dBp, (const float*)dBpj,
                                             (const double*)nullptr, K));
    }
    HIP_TRY(hipGetLastError());
    // the host-side plan must outlive the asynchronous copies
    HIP_TRY(hipStreamSynchronize(st));
    return SSM_OK;
}

extern "C" ssm_status ssm_implicit_solve(int32_t d, int64_t N, const double* X, double h, double v_rho,
                                         double v_a, double v_kappa, double v_lam, const double* xbar,
                                         double m2, int32_t max_iter, double* Y, int32_t* iters, void* stream)
{
    if (d < 1 || d > SSM_MAX_D || N < 1) return fail(SSM_ERR_INVALID, "bad d or N");
    if (!X || !Y) return fail(SSM_ERR_INVALID, "NULL pointer");
    if (!(v_a >= 0.0) || !(v_kappa >= 0.0)) return fail(SSM_ERR_INVALID, "v_a, v_kappa must be >= 0");
    if (!(1.0 - h * (v_rho - v_kappa * m2) > 0.0)) return fail(SSM_ERR_INVALID, "no unique implicit root (1 - h L_v <= 0)");
    double xb[kMaxD] = {0.0, 0.0, 0.0, 0.0};
    if (xbar)
        for (int k = 0; k < d; ++k) xb[k] = xbar[k];
    const dim3 g((unsigned)((N + 255) / 256));
    hipStream_t st = (hipStream_t)stream;
    const int mi = max_iter > 0 ? max_iter : 64;
    SSM_DISPATCH_D(d, hipLaunchKernelGGL((k_implicit_plain<D>), g, dim3(256), 0, st, N, X, h, v_rho, v_a, v_kappa, v_lam,
                                         xb[0], xb[1], xb[2], xb[3], m2, mi, Y, iters));
    HIP_TRY(hipGetLastError());
    return SSM_OK;
}

extern "C" ssm_status ssm_brownian(int32_t d, int64_t N, uint64_t seed, int32_t ens, int64_t n0, int32_t r,
                                   double h_fine, double* dW, void* stream)
{
    if (d < 1 || d > SSM_MAX_D || N < 1 || r < 1 || n0 < 0 || !dW || !(h_fine > 0.0))
        return fail(SSM_ERR_INVALID, "bad argument");
    SSM_DISPATCH_D(d, hipLaunchKernelGGL((k_brownian<D>), dim3((unsigned)((N + 255) / 256)), dim3(256), 0,
                                         (hipStream_t)stream, N, seed, ens, n0, r, std::sqrt(h_fine), dW));
    HIP_TRY(hipGetLastError());
    return SSM_OK;
}

extern "C" ssm_status ssm_philox_blocks(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1,
                                        int64_t count, uint64_t* out, void* stream)
{
    if (count < 1 || !out) return fail(SSM_ERR_INVALID, "bad argument");
    hipLaunchKernelGGL(k_philox, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, (hipStream_t)stream, c0, c1, c2, c3,
                       k0, k1, count, out);
    HIP_TRY(hipGetLastError());
    return SSM_OK;
}

// ---------------------------------------------------------------------------
// learned surrogate
// ---------------------------------------------------------------------------
namespace ssm {

__global__ void k_rff_freq(uint64_t seed, int d, double ell, RffFreq* out)
{
    const int q = threadIdx.x;
    if (q >= kRff) return;
    double z[kMaxD];
    normals(seed, 3u, (uint64_t)q, 0ull, 0ull, 4, z);
    for (int k = 0; k < kMaxD; ++k) out->w[q][k] = (k < d) ? (float)(z[k] / ell) : 0.0f;
}

__global__ void k_loss_reduce(const float* __restrict__ part, int nb, int B, float* __restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int q = 0; q < nb; ++q) s += part[q];
    out[0] = (float)(s / (double)B);
}

}  // namespace ssm

extern "C" int64_t ssm_mlp_num_params(int32_t d)
{
    if (d < 1 || d > SSM_MAX_D) return 0;
    return mlp_params(d);
}

static ssm_status ensure_surrogate_buffers(ssm_ctx* c)
{
    if (c->dmlp) return SSM_OK;
    ssm_status st;
    // each buffer only once (a call after a failed one resumes); dmlp last, as
    // it marks the set complete
#define ALLOC2(ptr, bytes) do { if (!(ptr)) { st = dev_alloc(c, (void**)&(ptr), (bytes)); if (st != SSM_OK) return st; } } while (0)
    ALLOC2(c->surr, (size_t)c->d * c->P * sizeof(float));
    ALLOC2(c->surr_res, (size_t)c->d * c->P * sizeof(float));
    ALLOC2(c->rff_part, (size_t)c->nblk_tot * 2 * kRff * sizeof(double));
    ALLOC2(c->mom, c->sys.size() * 2 * kRff * sizeof(float));
    ALLOC2(c->err_part, (size_t)c->nblk_tot * kErrStats * sizeof(double));
    ALLOC2(c->smean_part, (size_t)c->nblk_tot * kMaxD * sizeof(double));
    ALLOC2(c->smean, c->sys.size() * kMaxD * sizeof(float));
    RffFreq* dfq = nullptr;
    HIP_TRY(hipMalloc((void**)&dfq, sizeof(RffFreq)));
    hipLaunchKernelGGL(k_rff_freq, dim3(1), dim3(64), 0, c->stream, c->coef.seed, c->d, c->ell, dfq);
    hipError_t he = hipGetLastError();
    if (he == hipSuccess) he = hipMemcpyAsync(&c->rff, dfq, sizeof(RffFreq), hipMemcpyDeviceToHost, c->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
    (void)hipFree(dfq);
    if (he != hipSuccess) return fail(SSM_ERR_HIP, std::string("rff frequencies: ") + hipGetErrorString(he));
    ALLOC2(c->dmlp, sizeof(MlpPacked));
#undef ALLOC2
    return SSM_OK;
}

static ssm_status pack_weights(const float* master_dev, int d, MlpPacked* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_pack, dim3((kHid * kStride + 255) / 256), dim3(256), 0, st, master_dev, d, out);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_mlp_pack_infer, dim3(64), dim3(256), 0, st, master_dev, d, &out->inf);
    HIP_TRY(hipGetLastError());
    return SSM_OK;
}

extern "C" ssm_status ssm_surrogate_load(ssm_ctx* c, const float* master_host, int64_t n)
{
    if (!c || !master_host) return fail(SSM_ERR_INVALID, "NULL argument");
    if (!c->has_pair) return fail(SSM_ERR_STATE, "the surrogate replaces the pairwise term; b_g is 0");
    if (n != mlp_params(c->d)) return fail(SSM_ERR_INVALID, "expected " + std::to_string(mlp_params(c->d)) + " parameters");
    ssm_status st = ensure_surrogate_buffers(c);
    if (st != SSM_OK) return st;
    float* dm = nullptr;
    HIP_TRY(hipMalloc((void**)&dm, n * sizeof(float)));
    hipError_t he = hipMemcpyAsync(dm, master_host, n * sizeof(float), hipMemcpyHostToDevice, c->stream);
    if (he == hipSuccess) {
        st = pack_weights(dm, c->d, c->dmlp, c->stream);
        he = hipStreamSynchronize(c->stream);
    }
    (void)hipFree(dm);
    if (st != SSM_OK) return st;
    if (he != hipSuccess) return fail(SSM_ERR_HIP, std::string("surrogate_load: ") + hipGetErrorString(he));
    c->surr_loaded = true;
    surrogate_invalidate(c);  // residuals and gains of other weights
    return SSM_OK;
}

extern "C" ssm_status ssm_surrogate_enable(ssm_ctx* c, int32_t check_every, double tol, int32_t mode)
{
    if (!c) return fail(SSM_ERR_INVALID, "ctx is NULL");
    if (check_every < 0 || !(tol > 0.0)) return fail(SSM_ERR_INVALID, "check_every >= 0 and tol > 0 required");
    if (mode != SSM_SURR_GAIN && mode != SSM_SURR_RESIDUAL) return fail(SSM_ERR_INVALID, "unknown surrogate mode");
    if (check_every > 0 && !c->surr_loaded) return fail(SSM_ERR_STATE, "load surrogate weights first");
    if (check_every > 0 && mode == SSM_SURR_RESIDUAL && check_every % c->max_stride != 0)
        return fail(SSM_ERR_INVALID, "residual mode: check_every must be a multiple of " +
                                         std::to_string(c->max_stride) + " (every system steps on check ticks)");
    c->surr_check_every = check_every;
    c->surr_tol = tol;
    c->surr_mode = mode;
    c->surr_fallback = false;
    c->surr_res_valid = false;
    for (int k = 0; k < kMaxD; ++k) c->surr_gain[k] = 1.0;
    return SSM_OK;
}

extern "C" ssm_status ssm_surrogate_recheck(ssm_ctx* c, int32_t on)
{
    if (!c) return fail(SSM_ERR_INVALID, "ctx is NULL");
    if (on != 0 && on != 1) return fail(SSM_ERR_INVALID, "on must be 0 or 1");
    c->surr_recheck = on == 1;
    return SSM_OK;
}

extern "C" ssm_status ssm_surrogate_predict(ssm_ctx* c, int32_t sys, double* out, float* moments)
{
    if (!c || !out) return fail(SSM_ERR_INVALID, "NULL argument");
    if (sys < 0 || sys >= (int32_t)c->sys.size()) return fail(SSM_ERR_INVALID, "sys out of range");
    if (!c->surr_loaded) return fail(SSM_ERR_STATE, "load surrogate weights first");
    // the tick's own launches (phase 0 lists every system) on the current Y*
    ssm_status st = (c->prec == SSM_FP64) ? launch_surrogate<double>(c, 0) : launch_surrogate<float>(c, 0);
    if (st != SSM_OK) return st;
    const SysHost& S = c->sys[sys];
    hipLaunchKernelGGL(k_gather<float>, dim3((unsigned)((S.N + kBlk - 1) / kBlk)), dim3(kBlk), 0, c->stream,
                       (const float*)c->surr, c->P, S.off, S.N, c->d, c->dstage);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(out, c->dstage, (size_t)c->d * S.N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (moments)
        HIP_TRY(hipMemcpyAsync(moments, c->mom + (int64_t)sys * 2 * kRff, 2 * kRff * sizeof(float),
                               hipMemcpyDeviceToHost, c->stream));
    return ssm_sync(c);
}

extern "C" ssm_status ssm_surrogate_samples(ssm_ctx* c, int32_t sys, int64_t n, uint64_t seed, float* U, float* Tt)
{
    if (!c || !U || !Tt || n < 1) return fail(SSM_ERR_INVALID, "bad argument");
    if (sys < 0 || sys >= (int32_t)c->sys.size()) return fail(SSM_ERR_INVALID, "sys out of range");
    if (!c->has_pair) return fail(SSM_ERR_STATE, "b_g is 0: no pairwise term to sample");
    ssm_status st = ensure_surrogate_buffers(c);
    if (st != SSM_OK) return st;
    // exact pair sums and RFF moments of the current Y* of every system (phase-0 lists hold all)
    const int64_t np = c->pair_cnt[0], nb = c->blk_cnt[0];
    const int d = c->d;
    (void)np;
    if (c->prec == SSM_FP64) {
        st = launch_pairs<double>(c, 0);
        if (st != SSM_OK) return st;
        SSM_DISPATCH_D(d, hipLaunchKernelGGL((k_rff_partial<double, D>), dim3((unsigned)nb), dim3(kBlk), 0, c->stream, c->dblk + c->blk_off[0], c->dsys, c->P, (const double*)c->Y, c->rff, c->rff_part));
    } else {
        st = launch_pairs<float>(c, 0);
        if (st != SSM_OK) return st;
        SSM_DISPATCH_D(d, hipLaunchKernelGGL((k_rff_partial<float, D>), dim3((unsigned)nb), dim3(kBlk), 0, c->stream, c->dblk + c->blk_off[0], c->dsys, c->P, (const float*)c->Y, c->rff, c->rff_part));
    }
    HIP_TRY(hipGetLastError());
    if (c->prec == SSM_FP64) {
        SSM_DISPATCH_D(d, hipLaunchKernelGGL((k_combine<double, D>), dim3((unsigned)(nb * 4)), dim3(64 * kCombineWaves), 0,
                                             c->stream, c->dblk + c->blk_off[0], c->dsys, c->P, (const double*)c->Bp,
                                             (const double*)c->Bpj, (const double*)c->jtot, c->pairsum));
    } else {
        SSM_DISPATCH_D(d, hipLaunchKernelGGL((k_combine<float, D>), dim3((unsigned)(nb * 4)), dim3(64 * kCombineWaves), 0,
                                             c->stream, c->dblk + c->blk_off[0], c->dsys, c->P, (const float*)c->Bp,
                                             (const float*)c->Bpj, (const double*)c->jtot, c->pairsum));
    }
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_rff_final, dim3((unsigned)c->sys_list_cnt[0], 2 * kRff), dim3(kBlk), 0, c->stream, c->dsys_list + c->sys_list_off[0], c->dsys, c->rff_part, c->mom);
    HIP_TRY(hipGetLastError());
    const dim3 g((unsigned)((n + 255) / 256));
    if (c->prec == SSM_FP64) {
        SSM_DISPATCH_D(d, hipLaunchKernelGGL((k_gather_samples<double, D>), g, dim3(256), 0, c->stream, c->dsys, sys, c->P, (const double*)c->Y, c->pairsum, c->mom, n, seed, U, Tt));
    } else {
        SSM_DISPATCH_D(d, hipLaunchKernelGGL((k_gather_samples<float, D>), g, dim3(256), 0, c->stream, c->dsys, sys, c->P, (const float*)c->Y, c->pairsum, c->mom, n, seed, U, Tt));
    }
    HIP_TRY(hipGetLastError());
    return ssm_sync(c);
}

extern "C" ssm_status ssm_mlp_forward(int32_t d, const float* master, const float* U, int64_t n, float* out, void* stream)
{
    if (d < 1 || d > SSM_MAX_D || !master || !U || !out || n < 1) return fail(SSM_ERR_INVALID, "bad argument");
    hipStream_t st = (hipStream_t)stream;
    MlpPacked* W = nullptr;
    HIP_TRY(hipMalloc((void**)&W, sizeof(MlpPacked)));
    ssm_status s = pack_weights(master, d, W, st);
    if (s == SSM_OK) {
        const unsigned grid = (unsigned)std::min<int64_t>((n + 127) / 128, 4096);
        SSM_DISPATCH_D(d, hipLaunchKernelGGL((k_mlp_apply<D>), dim3(grid), dim3(256), 0, st, U, n, W, out));
        hipError_t he = hipGetLastError();
        if (he == hipSuccess) he = hipStreamSynchronize(st);
        if (he != hipSuccess) s = fail(SSM_ERR_HIP, std::string("mlp_forward: ") + hipGetErrorString(he));
    }
    (void)hipFree(W);
    return s;
}

// ---------------------------------------------------------------------------
// Network output without allocation: the packed weights go to a file-scope
// device buffer (one per GPU, held until the process ends) instead of a
// hipMalloc'd one.  Host code never passes `scratch` itself (in host code it
// names a host-side stand-in, not the device copy): the device address comes
// from hipGetSymbolAddress, taken once per device with that device current.
// ---------------------------------------------------------------------------
static __device__ __align__(256) MlpPacked scratch;

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static ssm_status scratch_for_current_device(MlpPacked** out)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SSM_ERR_INVALID, "device index beyond the library's table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SSM_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = (MlpPacked*)g_scratch_ptr[dev];
    return SSM_OK;
}

extern "C" ssm_status ssm_mlp_forward_noalloc(int32_t d, const float* master, const float* U, int64_t n, float* out,
                                              void* stream)
{
    if (d < 1 || d > SSM_MAX_D)
        return fail(SSM_ERR_INVALID, "d must be in 1..4 (the static weight buffer holds a network for d <= 4)");
    if (n < 1 || n > ((int64_t)1 << 31))
        return fail(SSM_ERR_INVALID, "n must be in 1..2^31 rows");
    if (!master || !U || !out) return fail(SSM_ERR_INVALID, "NULL pointer");
    MlpPacked* W = nullptr;
    ssm_status s = scratch_for_current_device(&W);
    if (s != SSM_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    s = pack_weights(master, d, W, st);
    if (s != SSM_OK) return s;
    const unsigned grid = (unsigned)std::min<int64_t>((n + 127) / 128, 4096);
    SSM_DISPATCH_D(d, hipLaunchKernelGGL((k_mlp_apply<D>), dim3(grid), dim3(256), 0, st, U, n, W, out));
    HIP_TRY(hipGetLastError());
    return SSM_OK;
}

struct TrainWork {
    TrainBufs tb{};
    void* base = nullptr;
    MlpPacked* W = nullptr;
};

static ssm_status alloc_train(int B, TrainWork* w)
{
    const size_t feat = (size_t)kKpad * B * sizeof(__bf16);
    const size_t out = (size_t)kOutPad * B * sizeof(__bf16);
    const size_t bytes = 4 * feat + 3 * feat + out + (size_t)(B / 64) * sizeof(float) + sizeof(MlpPacked) + 1024;
    HIP_TRY(hipMalloc(&w->base, bytes));
    char* p = (char*)w->base;
    for (int q = 0; q < 4; ++q) { w->tb.act[q] = (__bf16*)p; p += feat; }
    for (int q = 0; q < 3; ++q) { w->tb.delta[q] = (__bf16*)p; p += feat; }
    w->tb.delta[3] = (__bf16*)p; p += out;
    w->W = (MlpPacked*)p; p += (sizeof(MlpPacked) + 255) & ~(size_t)255;
    w->tb.loss_part = (float*)p;
    return SSM_OK;
}

extern "C" ssm_status ssm_mlp_loss_grad(int32_t d, const float* master, const float* U, const float* Tt, int64_t n,
                                        float* grad, double* loss, void* stream)
{
    if (d < 1 || d > SSM_MAX_D || !master || !U || !Tt || !grad) return fail(SSM_ERR_INVALID, "bad argument");
    if (n < 64 || n % 64 != 0 || n > (1 << 24)) return fail(SSM_ERR_INVALID, "n must be a positive multiple of 64");
    hipStream_t st = (hipStream_t)stream;
    TrainWork w;
    ssm_status s = alloc_train((int)n, &w);
    if (s != SSM_OK) return s;
    s = pack_weights(master, d, w.W, st);
    hipError_t he = hipSuccess;
    std::vector<float> lp(n / 64);
    if (s == SSM_OK) {
        hipLaunchKernelGGL(k_train_fwdbwd, dim3((unsigned)(n / 64)), dim3(256), 0, st, w.W, U, Tt, n, d, (int)n, 0ull, (int64_t)0, 1, w.tb);
        hipLaunchKernelGGL(k_train_wgrad, dim3(52), dim3(64), 0, st, w.tb, d, (int)n, grad);
        he = hipGetLastError();
        if (he == hipSuccess) he = hipMemcpyAsync(lp.data(), w.tb.loss_part, lp.size() * sizeof(float), hipMemcpyDeviceToHost, st);
        if (he == hipSuccess) he = hipStreamSynchronize(st);
    }
    (void)hipFree(w.base);
    if (s != SSM_OK) return s;
    if (he != hipSuccess) return fail(SSM_ERR_HIP, std::string("mlp_loss_grad: ") + hipGetErrorString(he));
    if (loss) {
        double t = 0.0;
        for (float v : lp) t += v;
        *loss = t / (double)n;
    }
    return SSM_OK;
}

extern "C" ssm_status ssm_mlp_train(int32_t d, const float* U, const float* Tt, int64_t n_samples,
                                    const ssm_train_cfg* cfg, float* master, float* loss_hist, void* stream)
{
    if (d < 1 || d > SSM_MAX_D || !U || !Tt || !master || !cfg || n_samples < 1) return fail(SSM_ERR_INVALID, "bad argument");
    const int B = cfg->batch;
    if (B < 64 || B % 64 != 0 || B > (1 << 20)) return fail(SSM_ERR_INVALID, "batch must be a positive multiple of 64");
    if (cfg->steps < 1 || !(cfg->lr > 0.0f)) return fail(SSM_ERR_INVALID, "steps >= 1 and lr > 0 required");
    hipStream_t st = (hipStream_t)stream;
    const int64_t P = mlp_params(d);
    TrainWork w;
    ssm_status s = alloc_train(B, &w);
    if (s != SSM_OK) return s;
    float *m = nullptr, *g = nullptr, *lh = nullptr;
    hipError_t he = hipMalloc((void**)&m, 3 * P * sizeof(float) + cfg->steps * sizeof(float));
    if (he != hipSuccess) { (void)hipFree(w.base); return fail(SSM_ERR_OOM, "mlp_train workspace"); }
    float* v = m + P;
    g = v + P;
    lh = g + P;
    he = hipMemsetAsync(m, 0, 2 * P * sizeof(float), st);
    const float b1 = cfg->beta1 > 0.0f ? cfg->beta1 : 0.9f, b2 = cfg->beta2 > 0.0f ? cfg->beta2 : 0.999f;
    const float eps = cfg->eps > 0.0f ? cfg->eps : 1e-8f;
    double c1 = 1.0, c2 = 1.0;
    for (int64_t t = 0; t < cfg->steps && he == hipSuccess; ++t) {
        c1 *= b1;
        c2 *= b2;
        s = pack_weights(master, d, w.W, st);
        if (s != SSM_OK) break;
        hipLaunchKernelGGL(k_train_fwdbwd, dim3((unsigned)(B / 64)), dim3(256), 0, st, w.W, U, Tt, n_samples, d, B, cfg->seed, t, 0, w.tb);
        hipLaunchKernelGGL(k_train_wgrad, dim3(52), dim3(64), 0, st, w.tb, d, B, g);
        hipLaunchKernelGGL(k_loss_reduce, dim3(1), dim3(64), 0, st, w.tb.loss_part, B / 64, B, lh + t);
        hipLaunchKernelGGL(k_adam, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, master, m, v, g, P, cfg->lr, b1, b2,
                           eps, (float)(1.0 - c1), (float)(1.0 - c2));
        he = hipGetLastError();
    }
    if (he == hipSuccess && loss_hist) he = hipMemcpyAsync(loss_hist, lh, cfg->steps * sizeof(float), hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    (void)hipFree(m);
    (void)hipFree(w.base);
    if (s != SSM_OK) return s;
    if (he != hipSuccess) return fail(SSM_ERR_HIP, std::string("mlp_train: ") + hipGetErrorString(he));
    return SSM_OK;
}

extern "C" ssm_status ssm_surrogate_train(ssm_ctx* c, const ssm_surrogate_train_cfg* tc, const float* init,
                                          float* master_out, float* loss_hist)
{
    if (!c || !tc) return fail(SSM_ERR_INVALID, "NULL argument");
    if (!c->has_pair) return fail(SSM_ERR_STATE, "the surrogate replaces the pairwise term; b_g is 0");
    if (tc->n_ens < 1 || tc->snapshots < 1 || tc->N < 0 || tc->n_samples < 1 ||
        tc->n_samples % ((int64_t)tc->n_ens * tc->snapshots) != 0)
        return fail(SSM_ERR_INVALID, "need n_ens >= 1, snapshots >= 1, N >= 0 and n_samples a multiple of n_ens x snapshots");
    const int d = c->d;
    const int64_t np = mlp_params(d), per = tc->n_samples / ((int64_t)tc->n_ens * tc->snapshots);
    const int64_t Ntr = tc->N > 0 ? tc->N : c->cfg_N[0];
    const double h0 = c->cfg_h[0];
    int64_t M = 0;
    if (!is_int_ratio(c->cfg.T, h0, &M)) return fail(SSM_ERR_INVALID, "T / h of system 0 is not an integer");
    if (tc->snapshots > M) return fail(SSM_ERR_INVALID, "more snapshots than steps");
    // device rows, weights
    float *U = nullptr, *Tt = nullptr, *master = nullptr;
    auto release = [&]() {
        if (U) (void)hipFree(U);
        if (Tt) (void)hipFree(Tt);
        if (master) (void)hipFree(master);
    };
    if (hipMalloc((void**)&U, (size_t)tc->n_samples * raw_in(d) * sizeof(float)) != hipSuccess ||
        hipMalloc((void**)&Tt, (size_t)tc->n_samples * d * sizeof(float)) != hipSuccess ||
        hipMalloc((void**)&master, (size_t)np * sizeof(float)) != hipSuccess) {
        release();
        return fail(SSM_ERR_OOM, "surrogate_train: training rows");
    }
    hipError_t he = hipSuccess;
    if (init) {
        he = hipMemcpyAsync(master, init, (size_t)np * sizeof(float), hipMemcpyHostToDevice, c->stream);
    } else {
        hipLaunchKernelGGL(k_mlp_init, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, c->stream, tc->seed, d, master);
        he = hipGetLastError();
    }
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
    if (he != hipSuccess) { release(); return fail(SSM_ERR_HIP, std::string("surrogate_train: ") + hipGetErrorString(he)); }
    // exact runs of systems like system 0 (ensembles ens0 ..), rows drawn at
    // ticks k M / snapshots
    ssm_config cfg = c->cfg;
    cfg.n_sys = 1;
    cfg.stream = c->stream;
    cfg.graphs = 0;
    ssm_status st = SSM_OK;
    for (int32_t e = 0; e < tc->n_ens && st == SSM_OK; ++e) {
        int64_t Nn = Ntr;
        int32_t ens = tc->ens0 + e;
        double h = h0;
        cfg.N = &Nn;
        cfg.ens = &ens;
        cfg.h = &h;
        ssm_ctx* r = nullptr;
        st = ssm_init(&cfg, &r);
        int64_t at = 0;
        for (int32_t k = 0; k < tc->snapshots && st == SSM_OK; ++k) {
            const int64_t tick = (int64_t)k * M / tc->snapshots;
            st = ssm_step(r, tick - at);
            at = tick;
            const int64_t row = ((int64_t)e * tc->snapshots + k) * per;
            if (st == SSM_OK)
                st = ssm_surrogate_samples(r, 0, per, tc->seed + 1000003ull * (uint64_t)(e * tc->snapshots + k + 1),
                                           U + row * raw_in(d), Tt + row * d);
        }
        ssm_destroy(r);
    }
    if (st == SSM_OK) st = ssm_mlp_train(d, U, Tt, tc->n_samples, &tc->train, master, loss_hist, c->stream);
    if (st == SSM_OK) st = ensure_surrogate_buffers(c);
    if (st == SSM_OK) st = pack_weights(master, d, c->dmlp, c->stream);
    if (st == SSM_OK && master_out) {
        he = hipMemcpyAsync(master_out, master, (size_t)np * sizeof(float), hipMemcpyDeviceToHost, c->stream);
        if (he != hipSuccess) st = fail(SSM_ERR_HIP, std::string("surrogate_train: ") + hipGetErrorString(he));
    }
    if (st == SSM_OK) {
        he = hipStreamSynchronize(c->stream);
        if (he != hipSuccess) st = fail(SSM_ERR_HIP, std::string("surrogate_train: ") + hipGetErrorString(he));
    }
    release();
    if (st != SSM_OK) return st;
    c->surr_loaded = true;
    surrogate_invalidate(c);  // residuals and gains of other weights
    return SSM_OK;
}
