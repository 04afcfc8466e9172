// ssm_small.hpp -- whole runs of small systems in one launch ("persistent" mode).
//
// For systems of a few thousand particles a tick is bound by latency, not by
// work: three dependent launches (pair sums, combine + increments, update)
// cost far more than their arithmetic.  Here one cooperative launch runs every
// tick of an ssm_step call.  Each workgroup (8 wavefronts) owns a tile of 64
// particles of one system and, per tick:
//   1. stages the system's scaled positions Ys in LDS;
//   2. sums the interaction over every ordered pair (i, j) of its targets,
//      the 8 wavefronts taking 8 consecutive source ranges, the ranges'
//      partial sums added in double in ascending order (the self term is 0);
//   3. applies the update (2.4) and the implicit step (2.3) of the next step,
//      and writes the tile's sums of Y* (fixed-order wavefront reduction);
//   4. arrives at its system's barrier (all tiles of the system), draws the
//      next tick's Brownian increments (the same stream sums as the
//      multi-launch path draws for a system without a shared window), and
//      waits, so that the next tick sees the whole new cloud.
// When v depends on mu^X the update and the implicit step are separated by a
// second barrier (the moments of the new X are needed first).  The means of
// mu^Y and mu^X are the tile sums added in ascending tile order.  Systems are
// independent: each waits only for its own tiles.  A system steps on the
// ticks t with t % stride == 0 and draws its own increments (no shared
// windows); on its other ticks its workgroups only take part in the barriers.
//
// Every barrier wait is bounded in wall-clock time; a wait that runs out sets
// the abort flag, every workgroup leaves at its next barrier, and the host
// reports the failure (the context is then unusable).
#pragma once

#include "ssm_kernels.hpp"

namespace ssm {

constexpr int kSmallWaves = 8;                  // wavefronts per tile workgroup
constexpr int kSmallThreads = 64 * kSmallWaves;
constexpr int kSmallTile = 64;                  // particles per tile
constexpr int kSmallLdsBytes = 32768;           // staged positions: d x N4 elements, N4 = N rounded up to 4
constexpr int kBarLine = 32;                    // uint64 per barrier counter (one 256-byte line)

// Staged rows hold N rounded up to a multiple of 4 (16-byte source reads).
__host__ __device__ constexpr int64_t small_row(int64_t N) { return (N + 3) & ~(int64_t)3; }

struct SmallTile {
    int32_t sys;    // system
    int32_t tile;   // system-local tile: particles 64 tile .. 64 tile + 63
    int32_t gtile;  // first global tile of the system (its tiles are gtile .. gtile + ntile - 1)
    int32_t ntile;  // tiles of the system (the members of its barrier)
};

template <typename T>
struct SmallArgs {
    const SmallTile* tiles;  // [grid]
    const SysDev* sys;
    Coef cf;
    int64_t P;
    int64_t t0, n;           // ticks t0 .. t0 + n - 1
    int64_t ntile_tot;
    T* X;
    T* Y;
    T* Ys;
    double* sumY;            // [2][D][ntile_tot]: tile sums of Y* before step n of a system (slot n & 1)
    double* sumX;            // [D + 1][ntile_tot]: tile sums of the new X and |X|^2 (v depends on mu^X)
    uint64_t* bar;           // per system: counter at bar[s * kBarLine]
    uint64_t epoch0;         // barriers every system has passed before this launch
    Flags* flags;
    int32_t* nmax;
    int bm_lanes;            // lanes per particle of the Brownian sums (each system draws its own)
    int needs_ybar;
    int64_t wait_limit;      // wall-clock counts a barrier wait may take
};

// Lane permutations within each row of 16 lanes (gfx9 DPP controls):
// exchange with lane ^ 1 and lane ^ 2 (quad_perm), mirror within 8 and 16.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

template <int CTRL>
__device__ __forceinline__ double dpp64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double readlane64(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes of a wavefront in a fixed order; every lane gets it.
// Within each row of 16 lanes, four DPP steps (pairs, quads, eights,
// sixteens) leave the row's sum in all its lanes; the four row sums are then
// read and added as (row 0 + row 1) + (row 2 + row 3).  DPP instead of LDS
// shuffles: this sum sits on the latency chain of the update.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp64<kDppXor1>(v);
    v += dpp64<kDppXor2>(v);
    v += dpp64<kDppHalfMirror>(v);
    v += dpp64<kDppMirror>(v);
    return (readlane64(v, 0) + readlane64(v, 16)) + (readlane64(v, 32) + readlane64(v, 48));
}

// Largest value over the lanes of a wavefront, the same way.
__device__ __forceinline__ int wave_max(int v)
{
    v = max(v, __builtin_amdgcn_update_dpp(0, v, kDppXor1, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, kDppXor2, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, kDppHalfMirror, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, kDppMirror, 0xF, 0xF, false));
    return max(max(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               max(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

// Split-phase barrier of the `members` workgroups of one system.  Arrive:
// one release increment of the system's counter by thread 0.  Wait: until the
// counter reaches members x epoch, then an acquire fence by thread 0 (it
// invalidates the compute unit's caches for every wavefront) and a workgroup
// barrier.  Work between the two must not write what other workgroups read.
// Wait returns false (in every thread) when the run is being aborted.
// The release covers the global writes of thread 0's own wavefront only (the
// workgroup barrier before it waits for LDS traffic, not for other
// wavefronts' stores): in k_small every global write that another workgroup
// reads (Ys, Y*, X, the tile sums) is made by wavefront 0; the other
// wavefronts write only LDS.
__device__ __forceinline__ void small_arrive(uint64_t* ctr)
{
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(ctr, (uint64_t)1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool small_wait(uint64_t* ctr, uint64_t target, Flags* flags, int64_t limit, int* ok_lds)
{
    if (threadIdx.x == 0) {
        int ok = 1;
        const uint64_t start = wall_clock64();
        int n = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if ((int64_t)(wall_clock64() - start) > limit) {
                __hip_atomic_store(&flags->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            if ((++n & 15) == 0 && __hip_atomic_load(&flags->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                ok = 0;
                break;
            }
        }
        if (ok && __hip_atomic_load(&flags->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *ok_lds = ok;
    }
    __syncthreads();
    const int ok = *ok_lds;
    __syncthreads();  // the flag's LDS word is reused by the next wait
    return ok != 0;
}

// Mean over a system's tiles of tile sums sums[k * ntile_tot + g0 + q], added
// in ascending tile order per lane (q = lane, lane + 64, ...) and then by the
// wavefront tree; every lane gets the same value.
__device__ __forceinline__ double tile_mean(const double* __restrict__ sums, int64_t ntile_tot, int g0, int ntile,
                                            int k, double N)
{
    const int lane = threadIdx.x & 63;
    double part = 0.0;
    for (int q = lane; q < ntile; q += 64) part += sums[(int64_t)k * ntile_tot + g0 + q];
    return wave_sum(part) / N;
}

// The ordered-pair sums of target y against sources [j0, j1) of the staged
// rows (row c at src + c * row), in T; KAHAN: plain over chunks of
// kKahanChunk sources, the chunk sums added by Neumaier's method, the pair
// rounded once to T.
template <typename T, int D, bool KAHAN>
__device__ __forceinline__ void small_pairs(const T* src, int64_t row, int j0, int j1, const T (&yi)[D],
                                            T (&out)[D])
{
    using V4 = T __attribute__((ext_vector_type(4)));
    T hi[D], lo[D];
#pragma unroll
    for (int c = 0; c < D; ++c) hi[c] = lo[c] = (T)0;
    for (int c0 = j0; c0 < j1; c0 += kKahanChunk) {
        const int c1 = min(c0 + kKahanChunk, j1);
        T acc[D];
#pragma unroll
        for (int c = 0; c < D; ++c) acc[c] = (T)0;
        int j = c0;
        for (; j + 4 <= c1; j += 4) {
            V4 s[D];
#pragma unroll
            for (int c = 0; c < D; ++c) s[c] = *reinterpret_cast<const V4*>(src + c * row + j);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                T z[D];
                T t = (T)0;
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    z[c] = s[c][u] - yi[c];
                    t = (c == 0) ? z[c] * z[c] : fma_t(z[c], z[c], t);
                }
                const T e = exp2_fast<T>(-t);
#pragma unroll
                for (int c = 0; c < D; ++c) acc[c] = fma_t(z[c], e, acc[c]);
            }
        }
        for (; j < c1; ++j) {
            T z[D];
            T t = (T)0;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                z[c] = src[c * row + j] - yi[c];
                t = (c == 0) ? z[c] * z[c] : fma_t(z[c], z[c], t);
            }
            const T e = exp2_fast<T>(-t);
#pragma unroll
            for (int c = 0; c < D; ++c) acc[c] = fma_t(z[c], e, acc[c]);
        }
        if constexpr (KAHAN) {
#pragma unroll
            for (int c = 0; c < D; ++c) {
                const T a = acc[c];
                const T sm = hi[c] + a;
                lo[c] += (fabs(hi[c]) >= fabs(a)) ? (hi[c] - sm) + a : (a - sm) + hi[c];
                hi[c] = sm;
            }
        } else {
#pragma unroll
            for (int c = 0; c < D; ++c) hi[c] += acc[c];
        }
    }
#pragma unroll
    for (int c = 0; c < D; ++c) out[c] = KAHAN ? (T)((double)hi[c] + (double)lo[c]) : hi[c];
}

// The tile's Brownian sums: LP lanes per particle, as brownian_block (same
// stream_sum and butterfly, so the same increments bit for bit), in passes
// of kSmallThreads / LP particles; lane q = 0 of each particle writes dw[k][p].
template <int D, int LP, bool F32>
__device__ __forceinline__ void small_brownian(const SysDev& S, const Coef& cf, int tile0, int64_t t,
                                               double (*dw)[kSmallTile])
{
    constexpr int kPer = kSmallThreads / LP < kSmallTile ? kSmallThreads / LP : kSmallTile;
    // whole wavefronts leave (kPer LP is a multiple of 64)
    if ((int)threadIdx.x >= kPer * LP) return;
    const int q = threadIdx.x % LP;
    const int64_t n = t / S.stride;
    for (int base = 0; base < kSmallTile; base += kPer) {
        const int p = base + (int)threadIdx.x / LP;
        const int i = tile0 + p;
        double zs[kMaxD] = {0.0, 0.0, 0.0, 0.0};
        if (i < S.N) {
            const uint64_t q0 = (uint64_t)n * (uint64_t)S.r * D;
            const uint64_t q1 = q0 + (uint64_t)S.r * D;
            stream_sum<D, F32>(cf.seed, (uint64_t)i, (uint64_t)S.ens, q0, q1, q0 / 4 + q, LP, zs);
        }
        lane_butterfly<LP, D>(zs);
        if (q == 0)
#pragma unroll
            for (int k = 0; k < D; ++k) dw[k][p] = cf.sqrt_hf * zs[k];
    }
}

// Implicit step (2.3) of one particle (wavefront 0 of the tile), as
// solve_and_store; the tile's Y* sums go to sumY_out[k][gt], the stored Y*
// (as double) to yout, and the wavefront's largest Newton count into nrun.
template <typename T, int D>
__device__ __forceinline__ void small_solve(const SysDev& S, const Coef& cf, bool valid, const double (&x)[kMaxD],
                                            const double (&xbar)[kMaxD], double m2, int64_t slot, int64_t P,
                                            T* __restrict__ Y, T* __restrict__ Ys, double* __restrict__ sumY_out,
                                            int64_t ntile_tot, int64_t gt, Flags* flags, int& nrun,
                                            double (&yout)[kMaxD])
{
    double w[D], y[D];
#pragma unroll
    for (int k = 0; k < D; ++k) w[k] = x[k] + S.h * cf.v_lam * xbar[k];
    const double alpha = 1.0 - S.h * (cf.v_rho - cf.v_kappa * m2);
    int it = 0;
    bool nonfin = false;
    if (valid) {
        if (cf.v_cw) {
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const int ik = implicit_radial<1>(&w[k], alpha, S.h * cf.v_ak[k], cf.newton_max_iter, &y[k]);
                if (ik == -2) nonfin = true;
                else it = (it < 0 || ik < 0) ? -1 : max(it, ik);
            }
        } else {
            it = implicit_radial<D>(w, alpha, S.h * cf.v_a, cf.newton_max_iter, y);
            if (it == -2) {
                nonfin = true;
                it = 0;
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < D; ++k) y[k] = 0.0;
    }
    const uint64_t fails = __ballot(it < 0);
    const uint64_t bad = __ballot(nonfin);
    const int itmax = wave_max(it);
    if ((threadIdx.x & 63) == 0) {
        if (fails) atomicAdd(&flags->newton_fail, (int)__popcll(fails));
        if (bad) atomicAdd(&flags->nonfinite, (int)__popcll(bad));
    }
    nrun = max(nrun, itmax);
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const T yt = (T)y[k];
        if (valid) {
            Y[k * P + slot] = yt;
            Ys[k * P + slot] = (T)(cf.coord_scale * (double)yt);
        }
        yout[k] = valid ? (double)yt : 0.0;
        const double s = wave_sum(yout[k]);
        if ((threadIdx.x & 63) == 0) sumY_out[(int64_t)k * ntile_tot + gt] = s;
    }
}

template <int D, bool F32>
__device__ __forceinline__ void small_draw(int lanes, const SysDev& S, const Coef& cf, int tile0, int64_t t,
                                           double (*dw)[kSmallTile])
{
    switch (lanes) {
        case 16: small_brownian<D, 16, F32>(S, cf, tile0, t, dw); break;
        case 8: small_brownian<D, 8, F32>(S, cf, tile0, t, dw); break;
        case 4: small_brownian<D, 4, F32>(S, cf, tile0, t, dw); break;
        case 2: small_brownian<D, 2, F32>(S, cf, tile0, t, dw); break;
        default: small_brownian<D, 1, F32>(S, cf, tile0, t, dw); break;
    }
}

// Barriers per launch of n ticks: one after the tile sums of the first Y*
// (two when v depends on mu^X: the first Y* is solved again at the tile sums'
// moments), one after every tick but the last (the end of the launch orders
// the last), and one more per tick between the update and the implicit step
// when v depends on mu^X.
__host__ __device__ constexpr uint64_t small_barriers(bool fused, int64_t n)
{
    return fused ? (uint64_t)n : 2 * (uint64_t)n + 1;
}

template <typename T, int D, bool KAHAN>
__global__ __launch_bounds__(kSmallThreads) void k_small(SmallArgs<T> a)
{
    constexpr int kRowElems = kSmallLdsBytes / (int)sizeof(T);
    constexpr bool F32 = sizeof(T) == 4;
    __shared__ __align__(32) T src[kRowElems];
    __shared__ T part[kSmallWaves][D][kSmallTile];
    __shared__ double dw[D][kSmallTile];
    __shared__ int ok_lds;

    const SmallTile tl = a.tiles[blockIdx.x];
    const SysDev S = a.sys[tl.sys];
    const Coef& cf = a.cf;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int tile0 = tl.tile * kSmallTile;
    const int i = tile0 + lane;               // wavefront 0's particle
    const bool valid = i < S.N;
    const int64_t slot = S.off + i;
    const int64_t gt = tl.gtile + tl.tile;    // global tile
    const int64_t nslot = (int64_t)(S.blk0 + tl.tile / kSlotsPerBlk) * kSlotsPerBlk + tl.tile % kSlotsPerBlk;
    const int64_t row = small_row(S.N);
    // wavefront 0 keeps its particles' Y* and its largest Newton count in
    // registers for the whole launch (the slot is stored at the end)
    double yv[kMaxD] = {0.0, 0.0, 0.0, 0.0};
    int nrun = 0;
    if (wave == 0) nrun = a.nmax[nslot];
    uint64_t* ctr = a.bar + (int64_t)tl.sys * kBarLine;
    uint64_t epoch = a.epoch0;
    const uint64_t members = (uint64_t)tl.ntile;
    // source ranges of the wavefronts: kSmallWaves consecutive ranges of Ls (a multiple of 4)
    const int Ls = (int)((((int64_t)S.N + kSmallWaves - 1) / kSmallWaves + 3) & ~3);
    const int j0 = min(S.N, wave * Ls), j1 = min(S.N, (wave + 1) * Ls);

    // The system steps on ticks t with t % stride == 0, as step t / stride;
    // its tile sums of Y* alternate between two slots by the parity of the
    // step (par0: the slot its first step in this launch reads).
    const int par0 = (int)(((a.t0 + S.stride - 1) / S.stride) & 1);

    // Y* of the first tick and its tile sums.  When v depends on mu^X, Y* is
    // solved again here at the tile sums' moments of X, so that a run split
    // over several launches (or resumed from a saved state) takes the same
    // values as one launch; otherwise Y* = F_h(X) is already in place.
    if (!cf.fused) {
        if (wave == 0) {
            double xv[kMaxD] = {0.0, 0.0, 0.0, 0.0};
            double n2 = 0.0;
            if (valid) {
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    xv[k] = (double)a.X[k * a.P + slot];
                    n2 += xv[k] * xv[k];
                }
            }
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const double s = wave_sum(valid ? xv[k] : 0.0);
                if (lane == 0) a.sumX[(int64_t)k * a.ntile_tot + gt] = s;
            }
            const double s2 = wave_sum(valid ? n2 : 0.0);
            if (lane == 0) a.sumX[(int64_t)D * a.ntile_tot + gt] = s2;
        }
        small_arrive(ctr);
        if (!small_wait(ctr, members * ++epoch, a.flags, a.wait_limit, &ok_lds)) return;
        if (wave == 0) {
            double xbar[kMaxD] = {0.0, 0.0, 0.0, 0.0};
            double m2 = 0.0;
            if (cf.v_lam != 0.0) {
#pragma unroll
                for (int k = 0; k < D; ++k) xbar[k] = tile_mean(a.sumX, a.ntile_tot, tl.gtile, tl.ntile, k, (double)S.N);
            }
            if (cf.v_kappa != 0.0) m2 = tile_mean(a.sumX, a.ntile_tot, tl.gtile, tl.ntile, D, (double)S.N);
            double x[kMaxD] = {0.0, 0.0, 0.0, 0.0};
            if (valid) {
#pragma unroll
                for (int k = 0; k < D; ++k) x[k] = (double)a.X[k * a.P + slot];
            }
            small_solve<T, D>(S, cf, valid, x, xbar, m2, slot, a.P, a.Y, a.Ys,
                              a.sumY + (int64_t)par0 * D * a.ntile_tot, a.ntile_tot, gt, a.flags, nrun, yv);
        }
    } else if (wave == 0) {
        const int par = par0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            yv[k] = valid ? (double)a.Y[k * a.P + slot] : 0.0;
            const double s = wave_sum(yv[k]);
            if (lane == 0) a.sumY[((int64_t)par * D + k) * a.ntile_tot + gt] = s;
        }
    }
    // the first tick's increments are drawn while the other tiles arrive
    small_arrive(ctr);
    if (a.t0 % S.stride == 0) small_draw<D, F32>(a.bm_lanes, S, cf, tile0, a.t0, dw);
    if (!small_wait(ctr, members * ++epoch, a.flags, a.wait_limit, &ok_lds)) return;

    for (int64_t t = a.t0; t < a.t0 + a.n; ++t) {
        // every system takes part in every barrier; one that does not step
        // on this tick only waits
        const bool stepping = t % S.stride == 0;
        const int par = (int)((t / S.stride) & 1);
        if (stepping) {
            // 1. stage the system's scaled positions (loads issued four at a time);
            //    wavefront 0 also loads its particles' Y* and its share of the tile
            //    sums of mu^Y
            if (cf.has_pair) {
                const int64_t tot = (int64_t)D * row;
                for (int64_t q0 = threadIdx.x; q0 < tot; q0 += 4 * kSmallThreads) {
                    T v[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int64_t q = q0 + (int64_t)u * kSmallThreads;
                        const int c = (int)(q / row);
                        const int j = (int)(q - (int64_t)c * row);
                        v[u] = (q < tot && j < S.N) ? a.Ys[c * a.P + S.off + j] : (T)0;
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int64_t q = q0 + (int64_t)u * kSmallThreads;
                        if (q < tot) src[q] = v[u];
                    }
                }
            }
            double ypart[kMaxD] = {0.0, 0.0, 0.0, 0.0};
            if (wave == 0) {
                if (a.needs_ybar) {
                    const double* sy = a.sumY + (int64_t)par * D * a.ntile_tot + tl.gtile;
#pragma unroll
                    for (int k = 0; k < D; ++k)
                        for (int q = lane; q < tl.ntile; q += 64) ypart[k] += sy[(int64_t)k * a.ntile_tot + q];
                }
            }
            __syncthreads();
            // 2. ordered-pair sums of the tile's targets over the wavefront's source range
            if (cf.has_pair) {
                T yi[D], ps[D];
#pragma unroll
                for (int c = 0; c < D; ++c) yi[c] = valid ? src[c * row + i] : (T)0;
                small_pairs<T, D, KAHAN>(src, row, j0, j1, yi, ps);
#pragma unroll
                for (int c = 0; c < D; ++c) part[wave][c][lane] = ps[c];
                __syncthreads();
            }
            // 3. update (2.4) and the next implicit step, wavefront 0
            if (wave == 0) {
                double ybar[kMaxD] = {0.0, 0.0, 0.0, 0.0};
                if (a.needs_ybar) {
#pragma unroll
                    for (int k = 0; k < D; ++k) ybar[k] = wave_sum(ypart[k]) / (double)S.N;
                }
                double xn[kMaxD] = {0.0, 0.0, 0.0, 0.0};
                if (valid) {
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        const double y = yv[k];
                        double pair = 0.0;
                        if (cf.has_pair) {
                            double tot = 0.0;
#pragma unroll
                            for (int w = 0; w < kSmallWaves; ++w) tot += (double)part[w][k][lane];
                            pair = tot * S.pair_scale;
                        }
                        double b = cf.b_c0 * y + cf.b_lam * ybar[k] + pair;
                        if (cf.has_lin) {
                            b += cf.b_const[k];
#pragma unroll
                            for (int l = 0; l < D; ++l) b += cf.b_mat[k * kMaxD + l] * yv[l];
                            b += cf.b_mean[k] * ybar[k];
                        }
                        const double sig = cf.s0[k] + cf.s1[k] * y + cf.s2[k] * ybar[k];
                        xn[k] = (y + S.h * b) + sig * dw[k][lane];
                    }
                }
                double n2 = 0.0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const T xs = (T)xn[k];
                    if (valid) a.X[k * a.P + slot] = xs;
                    xn[k] = (double)xs;
                    n2 += xn[k] * xn[k];
                }
                if (cf.fused) {
                    const double zero[kMaxD] = {0.0, 0.0, 0.0, 0.0};
                    small_solve<T, D>(S, cf, valid, xn, zero, 0.0, slot, a.P, a.Y, a.Ys,
                                      a.sumY + (int64_t)(par ^ 1) * D * a.ntile_tot, a.ntile_tot, gt, a.flags, nrun, yv);
                } else {
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        const double s = wave_sum(valid ? xn[k] : 0.0);
                        if (lane == 0) a.sumX[(int64_t)k * a.ntile_tot + gt] = s;
                    }
                    const double s2 = wave_sum(valid ? n2 : 0.0);
                    if (lane == 0) a.sumX[(int64_t)D * a.ntile_tot + gt] = s2;
                }
            }
        }
        const bool last = t + 1 == a.t0 + a.n;
        if (!cf.fused) {
            // the implicit step at mu^X of the new cloud
            small_arrive(ctr);
            if (!small_wait(ctr, members * ++epoch, a.flags, a.wait_limit, &ok_lds)) return;
            if (stepping && wave == 0) {
                double xbar[kMaxD] = {0.0, 0.0, 0.0, 0.0};
                double m2 = 0.0;
                if (cf.v_lam != 0.0) {
#pragma unroll
                    for (int k = 0; k < D; ++k)
                        xbar[k] = tile_mean(a.sumX, a.ntile_tot, tl.gtile, tl.ntile, k, (double)S.N);
                }
                if (cf.v_kappa != 0.0) m2 = tile_mean(a.sumX, a.ntile_tot, tl.gtile, tl.ntile, D, (double)S.N);
                double x[kMaxD] = {0.0, 0.0, 0.0, 0.0};
                if (valid) {
#pragma unroll
                    for (int k = 0; k < D; ++k) x[k] = (double)a.X[k * a.P + slot];
                }
                small_solve<T, D>(S, cf, valid, x, xbar, m2, slot, a.P, a.Y, a.Ys,
                                  a.sumY + (int64_t)(par ^ 1) * D * a.ntile_tot, a.ntile_tot, gt, a.flags, nrun, yv);
            }
        }
        if (last) {
            // the end of the launch orders the last tick
            if (wave == 0 && lane == 0) a.nmax[nslot] = nrun;
            break;
        }
        // the next tick's increments are drawn while the other tiles arrive
        small_arrive(ctr);
        if ((t + 1) % S.stride == 0) small_draw<D, F32>(a.bm_lanes, S, cf, tile0, t + 1, dw);
        if (!small_wait(ctr, members * ++epoch, a.flags, a.wait_limit, &ok_lds)) return;
    }
}

// k_ysums: block sums of Y* of the listed blocks into the parity slot that the
// multi-launch path reads at the tick after tick_arg (as k_newton writes them),
// for a Y* computed by the persistent kernel.
template <typename T, int D>
__global__ __launch_bounds__(kBlk) void k_ysums(const BlkItem* __restrict__ items, const SysDev* __restrict__ sys,
                                                int64_t P, int64_t tick_arg, const T* __restrict__ Y,
                                                double* __restrict__ psumY, int64_t nblk_tot)
{
    __shared__ double red[kBlk];
    const BlkItem it = items[blockIdx.x];
    const SysDev S = sys[it.sys];
    const int64_t done = tick_arg < 0 ? 0 : tick_arg / S.stride + 1;
    double* pY = psumY + (int64_t)(done & 1) * D * nblk_tot;
    const int i = it.blk * kBlk + threadIdx.x;
    const bool valid = i < S.N;
    const int64_t gb = S.blk0 + it.blk;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double s = block_sum(valid ? (double)Y[k * P + S.off + i] : 0.0, red);
        if (threadIdx.x == 0) pY[(int64_t)k * nblk_tot + gb] = s;
    }
}

}  // namespace ssm
