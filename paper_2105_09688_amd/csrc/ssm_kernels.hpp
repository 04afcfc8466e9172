// ssm_kernels.hpp -- the kernels of one SSM time step on gfx950.
//
// A tick runs, for the systems that step on it:
//   k_pair   : the O(N^2) interaction sums at mu^Y (eq. (2.4) drift), one
//              wavefront per (target tile, source range) work item, partial
//              sums per source range written to a scratch buffer;
//   k_update : per particle, combines the partial sums in a fixed order,
//              evaluates b and sigma at mu^Y, draws dW and applies (2.4);
//              then (when v does not depend on mu^X) solves the implicit step
//              (2.3) of the next step in the same thread;
//   k_newton : the implicit step on its own (first step, and every step when
//              v depends on mu^X, whose moments need the whole new cloud).
// Layout: component-major [d][P] arrays over all systems, each system starting
// at a multiple of kBlk particles (padding slots are zero and never read as
// sources).
#pragma once

#include "ssm_device.hpp"

namespace ssm {

constexpr int kBlk = 256;      // particles per update block (and system alignment)
constexpr int kWaves = 4;      // wavefronts per pair block
constexpr int kUnroll = 8;     // sources per inner-loop iteration
constexpr int kKahanChunk = 128;  // sources summed plainly before a compensated add

struct SysDev {
    int64_t off;        // first slot of the system in [P]
    int32_t N;          // particles
    int32_t ens;        // ensemble id (Philox counter word 2)
    int32_t stride;     // ticks per step
    int32_t r;          // fine Brownian increments per step
    int32_t blk0;       // first global update block of the system
    int32_t nblk;       // update blocks of the system
    int32_t splits;     // source ranges of the pair sum (partials to combine)
    int32_t pad;
    double h;           // time step
    double pair_scale;  // b_g / (N c): scaled pair sums -> b's pair term
};

struct PairItem {
    int32_t sys;
    int32_t tgt0;   // first target (system-local)
    int32_t src0;   // first source (system-local)
    int32_t nsrc;   // sources in this item
    int32_t split;  // which partial buffer
    int32_t pad;
};

struct BlkItem {
    int32_t sys;
    int32_t blk;    // system-local block
};

struct Coef {
    double v_rho, v_a, v_kappa, v_lam;
    double b_c0, b_lam;
    double s0[kMaxD], s1[kMaxD], s2[kMaxD];
    double x0_mean[kMaxD], x0_std[kMaxD];
    double coord_scale;  // c = sqrt(log2(e) / (2 ell^2)): Ys = c Y, exp(-|dy|^2/(2ell^2)) = exp2(-|c dy|^2)
    double sqrt_hf;      // sqrt(h_fine)
    uint64_t seed;
    int32_t newton_max_iter;
    int32_t has_pair;    // b_g != 0
    int32_t fused;       // v independent of mu^X: the implicit solve runs inside k_update
    int32_t pad;
};

struct Flags {
    int32_t newton_fail;
    int32_t nonfinite;
    int32_t newton_max;
    int32_t pad;
};

template <typename T>
__device__ __forceinline__ T exp2_fast(T x);

template <>
__device__ __forceinline__ float exp2_fast<float>(float x)
{
    return __builtin_amdgcn_exp2f(x);  // v_exp_f32
}

template <>
__device__ __forceinline__ double exp2_fast<double>(double x)
{
    return exp2(x);
}

// Fixed-order tree sum of one double per thread over a kBlk-thread block.
// Returns the block total in every thread.  `red` is kBlk doubles of LDS.
__device__ __forceinline__ double block_sum(double v, double* red)
{
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
#pragma unroll
    for (int s = kBlk / 2; s > 0; s >>= 1) {
        if (t < s) red[t] = red[t] + red[t + s];
        __syncthreads();
    }
    const double total = red[0];
    __syncthreads();
    return total;
}

// ---------------------------------------------------------------------------
// k_init: X_0 = x0_mean + x0_std * Z(1, i, 0, ens); zero padding; block sums
// of x_k and |x|^2 (for measure-dependent v).
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ __launch_bounds__(kBlk) void k_init(const BlkItem* __restrict__ items,
                                               const SysDev* __restrict__ sys, Coef cf, int64_t P,
                                               T* __restrict__ X, T* __restrict__ Y,
                                               T* __restrict__ Ys, double* __restrict__ psumX,
                                               int64_t nblk_tot)
{
    __shared__ double red[kBlk];
    const BlkItem it = items[blockIdx.x];
    const SysDev S = sys[it.sys];
    const int i = it.blk * kBlk + threadIdx.x;
    const bool valid = i < S.N;
    double x[kMaxD] = {0.0, 0.0, 0.0, 0.0};
    if (valid) {
        double z[kMaxD];
        normals(cf.seed, 1u, (uint64_t)i, 0ull, (uint64_t)S.ens, D, z);
#pragma unroll
        for (int k = 0; k < D; ++k) x[k] = cf.x0_mean[k] + cf.x0_std[k] * z[k];
    }
    const int64_t slot = S.off + i;
    double n2 = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const T xs = (T)x[k];
        X[k * P + slot] = xs;
        Y[k * P + slot] = (T)0;
        Ys[k * P + slot] = (T)0;
        n2 += (double)xs * (double)xs;
    }
    // parity 0 block sums (step count 0)
    const int64_t gb = S.blk0 + it.blk;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double s = block_sum(valid ? (double)X[k * P + slot] : 0.0, red);
        if (threadIdx.x == 0) psumX[(int64_t)k * nblk_tot + gb] = s;
    }
    const double s2 = block_sum(valid ? n2 : 0.0, red);
    if (threadIdx.x == 0) psumX[(int64_t)D * nblk_tot + gb] = s2;
}

// Mean of mu over system S from its block sums (fixed order, block-cooperative).
template <int D>
__device__ __forceinline__ void system_means(const SysDev& S, const double* __restrict__ psum,
                                             int64_t nblk_tot, int ncomp, double* out,
                                             double* red)
{
    for (int k = 0; k < ncomp; ++k) {
        double part = 0.0;
        for (int b = threadIdx.x; b < S.nblk; b += kBlk) part += psum[(int64_t)k * nblk_tot + S.blk0 + b];
        out[k] = block_sum(part, red) / (double)S.N;
    }
}

// Implicit solve + writes of Y, Ys and the block sums of Y for one particle
// (all threads of the block must call it: it contains block reductions).
template <typename T, int D>
__device__ __forceinline__ void solve_and_store(const SysDev& S, const Coef& cf, bool valid,
                                                const double x[kMaxD], const double* xbar,
                                                double m2, int64_t slot, int64_t P,
                                                T* __restrict__ Y, T* __restrict__ Ys,
                                                double* __restrict__ psumY_out, int64_t gb,
                                                int64_t nblk_tot, Flags* flags, double* red)
{
    double w[D], y[D];
#pragma unroll
    for (int k = 0; k < D; ++k) w[k] = x[k] + S.h * cf.v_lam * xbar[k];
    const double alpha = 1.0 - S.h * (cf.v_rho - cf.v_kappa * m2);
    int it = 0;
    if (valid) {
        it = implicit_radial<D>(w, alpha, S.h * cf.v_a, cf.newton_max_iter, y);
        if (it < 0) atomicAdd(&flags->newton_fail, 1);
        else if (it > 0) atomicMax(&flags->newton_max, it);
    } else {
#pragma unroll
        for (int k = 0; k < D; ++k) y[k] = 0.0;
    }
    double ysum[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const T yt = (T)y[k];
        Y[k * P + slot] = yt;
        Ys[k * P + slot] = (T)(cf.coord_scale * (double)yt);
        ysum[k] = valid ? (double)yt : 0.0;
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double s = block_sum(ysum[k], red);
        if (threadIdx.x == 0) psumY_out[(int64_t)k * nblk_tot + gb] = s;
    }
}

// ---------------------------------------------------------------------------
// k_newton: Y* = F_h(X) for the listed blocks.  `done` is the number of steps
// each listed system has completed: (tick / stride) + 1 after an update on
// `tick`, or 0 at initialisation (tick < 0).
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ __launch_bounds__(kBlk) void k_newton(const BlkItem* __restrict__ items,
                                                 const SysDev* __restrict__ sys, Coef cf,
                                                 int64_t P, int64_t tick,
                                                 const T* __restrict__ X, T* __restrict__ Y,
                                                 T* __restrict__ Ys,
                                                 const double* __restrict__ psumX,
                                                 double* __restrict__ psumY, int64_t nblk_tot,
                                                 Flags* flags)
{
    __shared__ double red[kBlk];
    const BlkItem it = items[blockIdx.x];
    const SysDev S = sys[it.sys];
    const int64_t done = tick < 0 ? 0 : tick / S.stride + 1;
    const int par = (int)(done & 1);
    const double* pX = psumX + (int64_t)par * (D + 1) * nblk_tot;
    double* pY = psumY + (int64_t)par * D * nblk_tot;
    double xbar[kMaxD] = {0.0, 0.0, 0.0, 0.0};
    double m2 = 0.0;
    if (cf.v_lam != 0.0) system_means<D>(S, pX, nblk_tot, D, xbar, red);
    if (cf.v_kappa != 0.0) {
        double tmp[1];
        system_means<1>(S, pX + (int64_t)D * nblk_tot, nblk_tot, 1, tmp, red);
        m2 = tmp[0];
    }
    const int i = it.blk * kBlk + threadIdx.x;
    const bool valid = i < S.N;
    const int64_t slot = S.off + i;
    double x[kMaxD] = {0.0, 0.0, 0.0, 0.0};
    if (valid) {
#pragma unroll
        for (int k = 0; k < D; ++k) x[k] = (double)X[k * P + slot];
    }
    solve_and_store<T, D>(S, cf, valid, x, xbar, m2, slot, P, Y, Ys, pY, S.blk0 + it.blk, nblk_tot,
                          flags, red);
}

// ---------------------------------------------------------------------------
// k_update: eq. (2.4) for the listed blocks at `tick`, then (fused) the
// implicit step (2.3) of the next step.
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ __launch_bounds__(kBlk) void k_update(const BlkItem* __restrict__ items,
                                                 const SysDev* __restrict__ sys, Coef cf,
                                                 int64_t P, int64_t tick, T* __restrict__ X,
                                                 T* __restrict__ Y, T* __restrict__ Ys,
                                                 const double* __restrict__ Bp,
                                                 const float* __restrict__ surr,
                                                 const float* __restrict__ surr_mean, int use_surr,
                                                 float4 surr_gain,
                                                 double* __restrict__ psumX,
                                                 double* __restrict__ psumY, int64_t nblk_tot,
                                                 Flags* flags)
{
    __shared__ double red[kBlk];
    const BlkItem it = items[blockIdx.x];
    const SysDev S = sys[it.sys];
    const int64_t n = tick / S.stride;  // step index of this update
    const int par_in = (int)(n & 1);
    const int par_out = par_in ^ 1;
    // mean of mu^Y_n
    double ybar[kMaxD] = {0.0, 0.0, 0.0, 0.0};
    system_means<D>(S, psumY + (int64_t)par_in * D * nblk_tot, nblk_tot, D, ybar, red);

    const int i = it.blk * kBlk + threadIdx.x;
    const bool valid = i < S.N;
    const int64_t slot = S.off + i;
    double xn[kMaxD] = {0.0, 0.0, 0.0, 0.0};
    if (valid) {
        double zs[kMaxD] = {0.0, 0.0, 0.0, 0.0};
        const uint64_t nf0 = (uint64_t)n * (uint64_t)S.r;
        for (int m = 0; m < S.r; ++m) {
            double z[kMaxD];
            normals(cf.seed, 0u, (uint64_t)i, nf0 + (uint64_t)m, (uint64_t)S.ens, D, z);
#pragma unroll
            for (int k = 0; k < D; ++k) zs[k] += z[k];
        }
        bool bad = false;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double y = (double)Y[k * P + slot];
            double pair = 0.0;
            if (use_surr) {
                // learned surrogate of the pair term, projected to zero net force and
                // scaled by the gain fitted at the last check
                const float gk = k == 0 ? surr_gain.x : k == 1 ? surr_gain.y : k == 2 ? surr_gain.z : surr_gain.w;
                pair = (double)gk * ((double)surr[k * P + slot] - (double)surr_mean[(int64_t)it.sys * kMaxD + k]);
            } else if (cf.has_pair) {
                for (int q = 0; q < S.splits; ++q) pair += Bp[((int64_t)q * D + k) * P + slot];
                pair *= S.pair_scale;
            }
            const double b = cf.b_c0 * y + cf.b_lam * ybar[k] + pair;
            const double sig = cf.s0[k] + cf.s1[k] * y + cf.s2[k] * ybar[k];
            const double dW = cf.sqrt_hf * zs[k];
            xn[k] = (y + S.h * b) + sig * dW;
            bad |= !isfinite(xn[k]);
        }
        if (bad) atomicAdd(&flags->nonfinite, 1);
    }
    double n2 = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const T xs = (T)xn[k];
        if (valid) X[k * P + slot] = xs;
        xn[k] = (double)xs;
        n2 += xn[k] * xn[k];
    }
    const int64_t gb = S.blk0 + it.blk;
    if (cf.fused) {
        const double zero[kMaxD] = {0.0, 0.0, 0.0, 0.0};
        solve_and_store<T, D>(S, cf, valid, xn, zero, 0.0, slot, P, Y, Ys,
                              psumY + (int64_t)par_out * D * nblk_tot, gb, nblk_tot, flags, red);
    } else {
        double* pX = psumX + (int64_t)par_out * (D + 1) * nblk_tot;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double s = block_sum(valid ? xn[k] : 0.0, red);
            if (threadIdx.x == 0) pX[(int64_t)k * nblk_tot + gb] = s;
        }
        const double s2 = block_sum(valid ? n2 : 0.0, red);
        if (threadIdx.x == 0) pX[(int64_t)D * nblk_tot + gb] = s2;
    }
}

// ---------------------------------------------------------------------------
// k_pair: one wavefront per work item.  Lane l holds R targets
// i = tgt0 + l + 64 r; the wavefront sweeps the item's sources j, which are
// wave-uniform (scalar loads), and accumulates
//   acc_k(i) += (Ys_k^j - Ys_k^i) * exp2(-|Ys^j - Ys^i|^2)
// in T.  KAHAN: plain sums over chunks of kKahanChunk sources, each chunk
// total added into a (hi, lo) pair with Neumaier's compensated summation.
// Writes Bp[split][k][slot] (double).
// ---------------------------------------------------------------------------
template <typename T, int D, int R>
__device__ __forceinline__ void pair_block(const T* __restrict__ src, int64_t P, int j0, int j1,
                                           const T (&yi)[R][D], T (&acc)[R][D])
{
    int j = j0;
    for (; j + kUnroll <= j1; j += kUnroll) {
        T s[kUnroll][D];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int k = 0; k < D; ++k) s[u][k] = src[k * P + j + u];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                T z[D];
                T t = (T)0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    z[k] = s[u][k] - yi[r][k];
                    t = (k == 0) ? z[k] * z[k] : fma(z[k], z[k], t);
                }
                const T e = exp2_fast<T>(-t);
#pragma unroll
                for (int k = 0; k < D; ++k) acc[r][k] = fma(z[k], e, acc[r][k]);
            }
        }
    }
    for (; j < j1; ++j) {
        T s[D];
#pragma unroll
        for (int k = 0; k < D; ++k) s[k] = src[k * P + j];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            T z[D];
            T t = (T)0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                z[k] = s[k] - yi[r][k];
                t = (k == 0) ? z[k] * z[k] : fma(z[k], z[k], t);
            }
            const T e = exp2_fast<T>(-t);
#pragma unroll
            for (int k = 0; k < D; ++k) acc[r][k] = fma(z[k], e, acc[r][k]);
        }
    }
}

template <typename T, int D, int R, bool KAHAN>
__global__ __launch_bounds__(64 * kWaves) void k_pair(const PairItem* __restrict__ items,
                                                      int n_items,
                                                      const SysDev* __restrict__ sys,
                                                      const T* __restrict__ Ys, int64_t P,
                                                      double* __restrict__ Bp)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int idx = blockIdx.x * kWaves + wave;
    if (idx >= n_items) return;
    const PairItem it = items[idx];
    const SysDev S = sys[it.sys];
    const T* __restrict__ base = Ys + S.off;

    T yi[R][D];
    bool valid[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = it.tgt0 + lane + 64 * r;
        valid[r] = i < S.N;
#pragma unroll
        for (int k = 0; k < D; ++k) yi[r][k] = valid[r] ? base[k * P + i] : (T)0;
    }
    T acc[R][D];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < D; ++k) acc[r][k] = (T)0;

    const int j0 = it.src0;
    const int j1 = it.src0 + it.nsrc;
    if constexpr (!KAHAN) {
        pair_block<T, D, R>(base, P, j0, j1, yi, acc);
    } else {
        T hi[R][D], lo[R][D];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < D; ++k) {
                hi[r][k] = (T)0;
                lo[r][k] = (T)0;
            }
        for (int c0 = j0; c0 < j1; c0 += kKahanChunk) {
            const int c1 = min(c0 + kKahanChunk, j1);
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int k = 0; k < D; ++k) acc[r][k] = (T)0;
            pair_block<T, D, R>(base, P, c0, c1, yi, acc);
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    // Neumaier: s = hi + a; the rounding error goes to lo
                    const T a = acc[r][k];
                    const T s = hi[r][k] + a;
                    const T err = (fabs(hi[r][k]) >= fabs(a)) ? (hi[r][k] - s) + a : (a - s) + hi[r][k];
                    lo[r][k] += err;
                    hi[r][k] = s;
                }
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < D; ++k) acc[r][k] = hi[r][k];
        // the compensation is added in double at the store below
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = it.tgt0 + lane + 64 * r;
            if (!valid[r]) continue;
#pragma unroll
            for (int k = 0; k < D; ++k)
                Bp[((int64_t)it.split * D + k) * P + S.off + i] = (double)hi[r][k] + (double)lo[r][k];
        }
        return;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = it.tgt0 + lane + 64 * r;
        if (!valid[r]) continue;
#pragma unroll
        for (int k = 0; k < D; ++k) Bp[((int64_t)it.split * D + k) * P + S.off + i] = (double)acc[r][k];
    }
}

// ---------------------------------------------------------------------------
// Helpers of the kernel-level entry points.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_scale_copy(const T* __restrict__ in, T* __restrict__ out, int64_t n, double c)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n) out[g] = (T)(c * (double)in[g]);
}

__global__ void k_combine(const double* __restrict__ Bp, int splits, int d, int64_t P, int64_t N,
                          double scale, double* __restrict__ K);

__global__ void k_brownian(int d, int64_t N, uint64_t seed, int32_t ens, int64_t n0, int32_t r,
                           double sqrt_hf, double* __restrict__ dW);

__global__ void k_philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                         uint64_t k1, int64_t count, uint64_t* __restrict__ out);

}  // namespace ssm
