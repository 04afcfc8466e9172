// ssm_kernels.hpp -- the kernels of one SSM time step on gfx950.
//
// An exact tick runs, for the systems that step on it:
//   k_pair_sym / k_pair : the O(N^2) interaction sums at mu^Y (eq. (2.4)
//              drift).  FP32: each unordered pair once (the kernel is odd),
//              one workgroup per (target group, source range) item, i-side
//              and j-side partial sums to scratch.  FP64 (or on request):
//              every ordered pair, one wavefront per (target tile, source
//              range) item, i-side partials only;
//   k_prep   : the partial sums combined in a fixed order into the scaled
//              pair term, and (same launch) the step's Brownian increments;
//   k_update : per particle, b and sigma at mu^Y and the update (2.4); then
//              (when v does not depend on mu^X) the implicit step (2.3) of
//              the next step in the same thread;
//   k_newton : the implicit step on its own (first step, and every step when
//              v depends on mu^X, whose moments need the whole new cloud).
// A surrogate tick replaces the first two by the network's kernels
// (ssm_surrogate.hpp) and k_brownian_sum.
// Layout: component-major [d][P] arrays over all systems, each system starting
// at a multiple of kBlk particles (padding slots are zero and never read as
// sources).
#pragma once

#include "ssm_device.hpp"

namespace ssm {

constexpr int kBlk = 256;      // particles per update block (and system alignment)
constexpr int kWaves = 4;      // wavefronts per pair block
constexpr int kUnroll = 8;     // sources per inner-loop iteration
// Sources summed plainly (per lane and target) before a compensated add: 256
// ran 0.65 % faster than 128 at d = 1, N = 2^16, with the same pathwise
// distance to the FP64 path (float storage of the state dominates it).
constexpr int kKahanChunk = 256;
// Floats of LDS j-side buffer per wavefront in the symmetric scheme: a
// target group times d must fit (the diagonal item's j-side sums).  d = 3
// takes 3072 (1024 sources per flush instead of 682: 1.5 % faster at
// N = 2^18); d = 1, 2 measured slower with it.  A d = 3 row has 64 more
// floats, where the lanes that store no j-side sum write (no branch around
// the store: 1 % faster at d = 3, slower at d = 1, 2).
__host__ __device__ constexpr int sym_lds(int D) { return D == 3 ? 3072 : 2048; }
__host__ __device__ constexpr int sym_row(int D) { return sym_lds(D) + (D == 3 ? 64 : 0); }
// The same buffer in FP64: 1024 doubles (1536 at d = 3, where a target group
// of 2 x 256 particles fills it), sources per flush a multiple of 16.
__host__ __device__ constexpr int sym_lds_f64(int D) { return D == 3 ? 1536 : 1024; }
// The buffer's capacity for a pair precision (fp64 or float storage).
__host__ __device__ constexpr int sym_lds_for(bool fp64, int D) { return fp64 ? sym_lds_f64(D) : sym_lds(D); }

struct SysDev {
    int64_t off;        // first slot of the system in [P]
    int32_t N;          // particles
    int32_t ens;        // ensemble id (Philox counter word 2)
    int32_t stride;     // ticks per step
    int32_t r;          // fine Brownian increments per step
    int32_t blk0;       // first global update block of the system
    int32_t nblk;       // update blocks of the system
    int32_t splits;     // i-side partial sums to combine (ordered-pair scheme)
    int32_t sym_B;      // symmetric scheme: target block size (0: ordered-pair scheme)
    int32_t sym_L;      // symmetric scheme: sources per off-diagonal work item
    int32_t pad;
    double h;           // time step
    double pair_scale;  // b_g / (N c): scaled pair sums -> b's pair term
    int64_t win_off;    // shared Brownian window of the system's path group (win_W > 0)
    int32_t win_W;      // ticks per window (0: the system draws its own increments)
    int32_t pad2;
};

struct PairItem {
    int32_t sys;
    int32_t tgt0;   // first target (system-local)
    int32_t src0;   // first source (system-local)
    int32_t nsrc;   // sources in this item
    int32_t split;  // which i-side partial buffer
    int32_t jrow;   // symmetric item: j-side partial row (target block index); -1: ordered pairs only
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
    int32_t v_cw;        // component-wise cubic -v_ak[k] y_k^3 (else radial -v_a |y|^2 y)
    int32_t has_lin;     // b += b_const + b_mat y + b_mean o ybar
    int32_t pad;
    double v_ak[kMaxD];
    double b_const[kMaxD];
    double b_mat[kMaxD * kMaxD];  // row-major [k][l]
    double b_mean[kMaxD];         // b_k += b_mean[k] mean_k(mu_Y)
};

// Error counters (atomics: they fire only when something goes wrong).
struct Flags {
    int32_t newton_fail;
    int32_t nonfinite;
    int32_t abort;  // a persistent run's barrier wait ran out of time (ssm_small.hpp)
    int32_t pad;
};

// Largest Newton iteration count per wavefront slot: slot gb * kSlotsPerBlk + w
// for global block gb, wavefront w (plain stores by the owning wavefront; a
// device-wide atomic per wavefront on one address serializes across the XCDs).
constexpr int kSlotsPerBlk = kBlk / 64;

template <typename T>
__device__ __forceinline__ T exp2_fast(T x);

template <>
__device__ __forceinline__ float exp2_fast<float>(float x)
{
    return __builtin_amdgcn_exp2f(x);  // v_exp_f32
}

// FP64 2^x for x <= 0, the pair kernels' argument -|c dy|^2 (NaN passes through).
// x = n + r with n = rint(x) and |r| <= 1/2 exact; 2^r is the degree-11
// polynomial that interpolates 2^r at the 12 Chebyshev nodes of [-1/2, 1/2]
// (interpolation error 4.2e-18 relative; coefficients rounded to double from
// 60-digit values; 0.80 ulp worst case with Horner's rounding); 2^n by ldexp,
// n clamped at -1100 so that every x below the double range, the padding's
// -4e30 included, gives exactly 0.  16 instructions, none of them range tests
// (the device library's exp2 took about 20: d = 1, N = 2^16 symmetric pair
// kernel 1.48 -> 1.29 ms per launch, timed the same way).
__device__ __forceinline__ double exp2_poly_coef(int k)
{
    constexpr double c[12] = {0x1.0000000000000p+0,  0x1.62e42fefa39efp-1, 0x1.ebfbdff82c5aep-3,
                              0x1.c6b08d704a0c6p-5,  0x1.3b2ab6fb9f1a5p-7, 0x1.5d87fe78a3f9cp-10,
                              0x1.430913112c61bp-13, 0x1.ffcbfc6da6ed1p-17, 0x1.62bfc2c86d700p-20,
                              0x1.b524ebd13a55fp-24, 0x1.e6228acd1c6e5p-28, 0x1.e9ec1fcb69a7fp-32};
    return c[k];
}

template <>
__device__ __forceinline__ double exp2_fast<double>(double x)
{
    const double n = rint(x);
    const double r = x - n;
    double p = exp2_poly_coef(11);
#pragma unroll
    for (int k = 10; k >= 0; --k) p = fma(p, r, exp2_poly_coef(k));
    return ldexp(p, (int)fmax(n, -1100.0));
}

// The partial-sum rows of particle i of system S, in their fixed order:
// ni i-side rows (Bp[q][k][P] in the storage precision: the target tile's or group's work
// items) then, in the symmetric scheme, nj j-side rows (same precision, Bpj[a][k][P]:
// every earlier group and the particle's own group).
struct PairRows {
    int ni, nj;
};

__device__ __forceinline__ PairRows pair_rows(const SysDev& S, int i)
{
    if (!S.sym_B) return PairRows{S.splits, 0};
    const int a = i / S.sym_B;
    const int rest = S.N - S.sym_B * (a + 1);
    return PairRows{1 + (rest > 0 ? (rest + S.sym_L - 1) / S.sym_L : 0), a + 1};
}

// Sum, in ascending order, of the rows r = w, w + W, w + 2W, ... (r < ni + nj)
// of component k at slot; loads are issued four at a time.
template <int D, int W, typename PT>
__device__ __forceinline__ double sum_rows(const PT* __restrict__ Bp, const PT* __restrict__ Bpj,
                                           PairRows pr, int k, int64_t P, int64_t slot, int w)
{
    double acc = 0.0;
    int r = w;
    for (; r + 3 * W < pr.ni; r += 4 * W) {
        PT v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = Bp[((int64_t)(r + u * W) * D + k) * P + slot];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += (double)v[u];
    }
    for (; r < pr.ni; r += W) acc += (double)Bp[((int64_t)r * D + k) * P + slot];
    int q = r - pr.ni;
    for (; q + 3 * W < pr.nj; q += 4 * W) {
        PT v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = Bpj[((int64_t)(q + u * W) * D + k) * P + slot];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += (double)v[u];
    }
    for (; q < pr.nj; q += W) acc += (double)Bpj[((int64_t)q * D + k) * P + slot];
    return acc;
}

// ---------------------------------------------------------------------------
// k_combine: the scaled pair term of every particle of the listed blocks,
// out[k][slot] = pair_scale * (sum of the particle's partial rows).  Four
// blocks of 64 particles per 256-particle block item (items
// null: system 0, block blockIdx.x / 4); wavefront w of a block adds the rows
// w, w + 4, ... and the four sums are added in wavefront order, so the result
// does not depend on the launch.
// ---------------------------------------------------------------------------
constexpr int kCombineWaves = 4;

// jtot (banded j-side, see k_jfold): when given, the particle's j-side sums
// are that one double instead of its j-side rows; it is added last.
template <typename PT, int D>
__device__ __forceinline__ void combine_block(int vb, const BlkItem* __restrict__ items,
                                              const SysDev* __restrict__ sys, int64_t P, const PT* __restrict__ Bp,
                                              const PT* __restrict__ Bpj, const double* __restrict__ jtot,
                                              double* __restrict__ out, double (*part)[D][64])
{
    const int q4 = vb & 3;
    const BlkItem it = items ? items[vb >> 2] : BlkItem{0, (int32_t)(vb >> 2)};
    const SysDev S = sys[it.sys];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int i = it.blk * kBlk + q4 * 64 + lane;
    const bool valid = i < S.N;
    const int64_t slot = S.off + i;
    PairRows pr = valid ? pair_rows(S, i) : PairRows{0, 0};
    if (jtot) pr.nj = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) part[wave][k][lane] = sum_rows<D, kCombineWaves, PT>(Bp, Bpj, pr, k, P, slot, wave);
    __syncthreads();
    if (wave == 0 && valid) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            double t = part[0][k][lane];
#pragma unroll
            for (int w = 1; w < kCombineWaves; ++w) t += part[w][k][lane];
            if (jtot) t += jtot[k * P + slot];
            out[k * P + slot] = t * S.pair_scale;
        }
    }
}

// ---------------------------------------------------------------------------
// k_jfold: banded j-side sums.  When the symmetric scheme's j-side rows (one
// per target group) would not fit the memory budget, the pair sums run in
// bands of target groups [a0, a1), each band writing its rows to rows
// a - a0 of Bpj; after each band, every particle adds the rows its own band
// holds for it (groups a0 .. min(a1, g + 1) - 1, g the particle's group, in
// ascending order) to its running total jtot (first band: from zero).  The
// order of the additions is fixed, so runs stay bitwise reproducible.
// One thread per particle of the listed blocks.
// ---------------------------------------------------------------------------
template <typename PT, int D>
__global__ __launch_bounds__(kBlk) void k_jfold(const BlkItem* __restrict__ items, const SysDev* __restrict__ sys,
                                                int64_t P, const PT* __restrict__ Bpj, int a0, int a1, int first,
                                                double* __restrict__ jtot)
{
    const BlkItem it = items[blockIdx.x];
    const SysDev S = sys[it.sys];
    const int i = it.blk * kBlk + threadIdx.x;
    if (i >= S.N || !S.sym_B) return;
    const int64_t slot = S.off + i;
    const int hi = min(a1, i / S.sym_B + 1);
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double t = first ? 0.0 : jtot[k * P + slot];
        for (int a = a0; a < hi; ++a) t += (double)Bpj[((int64_t)(a - a0) * D + k) * P + slot];
        jtot[k * P + slot] = t;
    }
}

template <typename PT, int D>
__global__ __launch_bounds__(64 * kCombineWaves) void k_combine(const BlkItem* __restrict__ items,
                                                               const SysDev* __restrict__ sys, int64_t P,
                                                               const PT* __restrict__ Bp,
                                                               const PT* __restrict__ Bpj,
                                                               const double* __restrict__ jtot,
                                                               double* __restrict__ out)
{
    __shared__ double part[kCombineWaves][D][64];
    combine_block<PT, D>(blockIdx.x, items, sys, P, Bp, Bpj, jtot, out, part);
}

// The tick a per-tick kernel works on: the context's device counter when
// given (graph replays), else the value passed at launch.
__device__ __forceinline__ int64_t tick_of(const int64_t* tick_dev, int64_t tick_arg)
{
    return tick_dev ? *tick_dev : tick_arg;
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
                                                int64_t nblk_tot, Flags* flags, int32_t* __restrict__ nmax,
                                                double* red)
{
    double w[D], y[D];
#pragma unroll
    for (int k = 0; k < D; ++k) w[k] = x[k] + S.h * cf.v_lam * xbar[k];
    const double alpha = 1.0 - S.h * (cf.v_rho - cf.v_kappa * m2);
    int it = 0;
    bool nonfin = false;  // a non-finite particle (from the update, or written by the caller)
    if (valid) {
        if (cf.v_cw) {
            // one scalar cubic per component: alpha y_k + h a_k y_k^3 = w_k
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
    // failures and non-finite particles: one atomic per wavefront that has
    // any; iteration counts: the wavefront's maximum into its own slot
    const uint64_t fails = __ballot(it < 0);
    const uint64_t bad = __ballot(nonfin);
    int itmax = it;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) itmax = max(itmax, __shfl_xor(itmax, off, 64));
    if ((threadIdx.x & 63) == 0) {
        if (fails) atomicAdd(&flags->newton_fail, (int)__popcll(fails));
        if (bad) atomicAdd(&flags->nonfinite, (int)__popcll(bad));
        int32_t* slot = nmax + gb * kSlotsPerBlk + (threadIdx.x >> 6);
        if (itmax > *slot) *slot = itmax;
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
// `tick`, or 0 at initialisation (tick < 0).  The tick is *tick_dev (the
// context's device tick counter) when tick_dev is non-null, else tick_arg.
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ __launch_bounds__(kBlk) void k_newton(const BlkItem* __restrict__ items,
                                                 const SysDev* __restrict__ sys, Coef cf,
                                                 int64_t P, int64_t tick_arg,
                                                 const int64_t* __restrict__ tick_dev,
                                                 const T* __restrict__ X, T* __restrict__ Y,
                                                 T* __restrict__ Ys,
                                                 const double* __restrict__ psumX,
                                                 double* __restrict__ psumY, int64_t nblk_tot,
                                                 Flags* flags, int32_t* __restrict__ nmax)
{
    __shared__ double red[kBlk];
    const BlkItem it = items[blockIdx.x];
    const SysDev S = sys[it.sys];
    const int64_t tick = tick_of(tick_dev, tick_arg);
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
                          flags, nmax, red);
}

// ---------------------------------------------------------------------------
// k_xsums: block sums of x_k and |x|^2 of the listed blocks into the parity
// slot that k_newton reads for the same `tick_arg` (the moments of mu^X that a
// measure-dependent v needs), computed as k_update computes them, for a state
// X written from outside the step loop.
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ __launch_bounds__(kBlk) void k_xsums(const BlkItem* __restrict__ items,
                                                const SysDev* __restrict__ sys, int64_t P,
                                                int64_t tick_arg, const T* __restrict__ X,
                                                double* __restrict__ psumX, int64_t nblk_tot)
{
    __shared__ double red[kBlk];
    const BlkItem it = items[blockIdx.x];
    const SysDev S = sys[it.sys];
    const int64_t done = tick_arg < 0 ? 0 : tick_arg / S.stride + 1;
    double* pX = psumX + (int64_t)(done & 1) * (D + 1) * nblk_tot;
    const int i = it.blk * kBlk + threadIdx.x;
    const bool valid = i < S.N;
    double xn[kMaxD] = {0.0, 0.0, 0.0, 0.0};
    if (valid) {
#pragma unroll
        for (int k = 0; k < D; ++k) xn[k] = (double)X[k * P + S.off + i];
    }
    double n2 = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) n2 += xn[k] * xn[k];
    const int64_t gb = S.blk0 + it.blk;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double s = block_sum(valid ? xn[k] : 0.0, red);
        if (threadIdx.x == 0) pX[(int64_t)k * nblk_tot + gb] = s;
    }
    const double s2 = block_sum(valid ? n2 : 0.0, red);
    if (threadIdx.x == 0) pX[(int64_t)D * nblk_tot + gb] = s2;
}

// ---------------------------------------------------------------------------
// k_update: eq. (2.4) for the listed blocks at the tick *tick_dev (the
// context's device tick counter), with the Brownian increments of
// k_brownian_sum, then (fused) the implicit step (2.3) of the next step.
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ __launch_bounds__(kBlk) void k_update(const BlkItem* __restrict__ items,
                                                 const SysDev* __restrict__ sys, Coef cf,
                                                 int64_t P, int64_t tick_arg,
                                                 const int64_t* __restrict__ tick_dev,
                                                 T* __restrict__ X,
                                                 T* __restrict__ Y, T* __restrict__ Ys,
                                                 const double* __restrict__ pairsum,
                                                 const float* __restrict__ surr,
                                                 const float* __restrict__ surr_mean, int use_surr,
                                                 float4 surr_gain, const float* __restrict__ surr_res,
                                                 const double* __restrict__ dWbuf,
                                                 const double* __restrict__ ymean,
                                                 double* __restrict__ psumX,
                                                 double* __restrict__ psumY, int64_t nblk_tot,
                                                 Flags* flags, int32_t* __restrict__ nmax)
{
    __shared__ double red[kBlk];
    const BlkItem it = items[blockIdx.x];
    const SysDev S = sys[it.sys];
    const int64_t n = tick_of(tick_dev, tick_arg) / S.stride;  // step index of this update
    const int par_in = (int)(n & 1);
    const int par_out = par_in ^ 1;
    // mean of mu^Y_n, reduced by the tick's preceding launch (null: the
    // coefficients do not use it)
    double ybar[kMaxD] = {0.0, 0.0, 0.0, 0.0};
    if (ymean) {
#pragma unroll
        for (int k = 0; k < D; ++k) ybar[k] = ymean[(int64_t)it.sys * kMaxD + k];
    }
    (void)par_in;

    const int i = it.blk * kBlk + threadIdx.x;
    const bool valid = i < S.N;
    const int64_t slot = S.off + i;
    double xn[kMaxD] = {0.0, 0.0, 0.0, 0.0};
    if (valid) {
        double yv[D];
#pragma unroll
        for (int k = 0; k < D; ++k) yv[k] = (double)Y[k * P + slot];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double y = yv[k];
            double pair = 0.0;
            if (use_surr) {
                // learned surrogate of the pair term, projected to zero net force,
                // scaled by the gain fitted at the last check and (residual mode)
                // corrected by the particle's residual stored at the last check
                const float gk = k == 0 ? surr_gain.x : k == 1 ? surr_gain.y : k == 2 ? surr_gain.z : surr_gain.w;
                pair = (double)gk * ((double)surr[k * P + slot] - (double)surr_mean[(int64_t)it.sys * kMaxD + k]);
                if (surr_res) pair += (double)surr_res[k * P + slot];
            } else if (cf.has_pair) {
                pair = pairsum[k * P + slot];
            }
            double b = cf.b_c0 * y + cf.b_lam * ybar[k] + pair;
            if (cf.has_lin) {
                // the linear extension b_const + b_mat y + b_mean o ybar, terms in ascending l
                b += cf.b_const[k];
#pragma unroll
                for (int l = 0; l < D; ++l) b += cf.b_mat[k * kMaxD + l] * yv[l];
                b += cf.b_mean[k] * ybar[k];
            }
            const double sig = cf.s0[k] + cf.s1[k] * y + cf.s2[k] * ybar[k];
            const double dW = dWbuf[k * P + slot];
            xn[k] = (y + S.h * b) + sig * dW;
        }
    }
    // a non-finite new state is flagged by the implicit solve that follows
    // (here when fused, else in k_newton), on the value as stored
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
                              psumY + (int64_t)par_out * D * nblk_tot, gb, nblk_tot, flags, nmax, red);
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
// Brownian increments.  The normals of particle i (ensemble e) form one
// stream: normal q is component q % 4 of Philox block q / 4 of stream tag 0.
// Fine step m, component k of a d-dimensional increment is normal m d + k, so
// a step of r fine increments uses normals [n r d, (n + 1) r d).
// stream_sum adds the normals of [q0, q1) that fall in the blocks
// b = b_first, b_first + stride, ... (a lane's share), per component.
// ---------------------------------------------------------------------------
// F32: the FP32 transform (the FP32 precision modes); the sums stay in double.
template <int D, bool F32 = false>
__device__ __forceinline__ void stream_sum(uint64_t seed, uint64_t i, uint64_t e, uint64_t q0, uint64_t q1,
                                           uint64_t b_first, uint64_t stride, double zs[kMaxD])
{
    for (uint64_t b = b_first; b * 4 < q1; b += stride) {
        double z[kMaxD];
        if constexpr (F32) {
            float zf[4];
            normals4_f32(seed, 0u, i, b, e, zf);
#pragma unroll
            for (int s = 0; s < 4; ++s) z[s] = (double)zf[s];
        } else {
            normals(seed, 0u, i, b, e, 4, z);
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const uint64_t q = 4 * b + s;
            if (q >= q0 && q < q1) {
                const int k = (int)((q - q0) % (uint64_t)D);
#pragma unroll
                for (int c = 0; c < D; ++c)
                    if (c == k) zs[c] += z[s];
            }
        }
    }
}

// k_brownian_sum: dW_n^i = sqrt(h_fine) x (sum of the step's normals) for the
// listed blocks at the tick *tick_dev (or tick_arg).  LP lanes (a power of two
// <= 16) share one particle and take every LP-th Philox block of the step;
// their partial sums are combined by a fixed butterfly.  Block g of the grid
// handles sub-block g % LP of item g / LP (256 / LP particles).
// A system of a path group (systems of one ensemble and size at several step
// sizes, so on the same Brownian paths) reads its normals' sums from the
// group's window instead: win[win_off + (p D + k) N + i] holds the sum of
// particle i's normals of component k over tick p of the current window of
// win_W ticks (k_bm_window), and a step of `stride` ticks starting at window
// tick p0 adds the entries p0 .. p0 + stride - 1 (lane q takes p0 + q,
// p0 + q + LP, ...).  Each normal is then drawn once per window, not once
// per step size.
template <int LP, int D>
__device__ __forceinline__ void lane_butterfly(double (&zs)[kMaxD])
{
#pragma unroll
    for (int w = LP / 2; w > 0; w >>= 1)
#pragma unroll
        for (int k = 0; k < D; ++k) zs[k] += __shfl_xor(zs[k], w, 64);
}

template <int D, int LP, bool F32>
__device__ __forceinline__ void brownian_block(int vb, const BlkItem* __restrict__ items,
                                               const SysDev* __restrict__ sys, const Coef& cf, int64_t P,
                                               int64_t tick_arg, const int64_t* __restrict__ tick_dev,
                                               const double* __restrict__ win, double* __restrict__ dW)
{
    const BlkItem it = items[vb / LP];
    const int sub = vb % LP;
    const SysDev S = sys[it.sys];
    const int q = threadIdx.x % LP;
    const int i = it.blk * kBlk + sub * (kBlk / LP) + threadIdx.x / LP;
    const int64_t t = tick_of(tick_dev, tick_arg);
    const int64_t n = t / S.stride;
    double zs[kMaxD] = {0.0, 0.0, 0.0, 0.0};
    if (i < S.N) {
        if (S.win_W > 0) {
            const int p0 = (int)(t % S.win_W);
            const double* __restrict__ w = win + S.win_off;
            for (int p = p0 + q; p < p0 + S.stride; p += LP)
#pragma unroll
                for (int k = 0; k < D; ++k) zs[k] += w[((int64_t)p * D + k) * S.N + i];
        } else {
            const uint64_t q0 = (uint64_t)n * (uint64_t)S.r * D;
            const uint64_t q1 = q0 + (uint64_t)S.r * D;
            stream_sum<D, F32>(cf.seed, (uint64_t)i, (uint64_t)S.ens, q0, q1, q0 / 4 + q, LP, zs);
        }
    }
    lane_butterfly<LP, D>(zs);
    if (q == 0 && i < S.N) {
#pragma unroll
        for (int k = 0; k < D; ++k) dW[k * P + S.off + i] = cf.sqrt_hf * zs[k];
    }
}

// The mean of mu^Y_n of one stepping system (listed system q of the tick),
// reduced once from its block sums in a fixed order into ymean[s][k] for
// k_update (which would otherwise reduce all of the system's block sums in
// every one of its blocks: 4096 x 4096 x d reads at N = 2^20).
struct YMeanJob {
    const int32_t* sys_list;  // the tick's stepping systems
    int n;                    // how many (0: the coefficients do not use the mean)
    const double* psumY;
    int64_t nblk_tot;
    double* ymean;            // [n_sys][kMaxD]
};

template <int D>
__device__ __forceinline__ void ymean_block(int q, const YMeanJob& job, const SysDev* __restrict__ sys,
                                            int64_t tick_arg, const int64_t* __restrict__ tick_dev)
{
    __shared__ double red[kBlk];
    const int s = job.sys_list[q];
    const SysDev S = sys[s];
    const int64_t n = tick_of(tick_dev, tick_arg) / S.stride;
    double m[kMaxD];
    system_means<D>(S, job.psumY + (int64_t)(n & 1) * D * job.nblk_tot, job.nblk_tot, D, m, red);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < D; ++k) job.ymean[(int64_t)s * kMaxD + k] = m[k];
}

// n_main blocks of Brownian sums, then job.n blocks of system means.
template <int D, int LP, bool F32>
__global__ __launch_bounds__(kBlk) void k_brownian_sum(int n_main, const BlkItem* __restrict__ items,
                                                       const SysDev* __restrict__ sys, Coef cf,
                                                       int64_t P, int64_t tick_arg,
                                                       const int64_t* __restrict__ tick_dev,
                                                       const double* __restrict__ win, double* __restrict__ dW,
                                                       YMeanJob job)
{
    if ((int)blockIdx.x < n_main)
        brownian_block<D, LP, F32>(blockIdx.x, items, sys, cf, P, tick_arg, tick_dev, win, dW);
    else
        ymean_block<D>(blockIdx.x - n_main, job, sys, tick_arg, tick_dev);
}

// k_bm_window: the window of a path group, drawn at its first tick t0
// (*tick_dev or tick_arg): win[win_off + (p D + k) N + i] = sum of particle
// i's normals of component k over the fine steps of tick t0 + p, that is
// stream normals [((t0 + p) r_min + m) d + k, m < r_min] with r_min fine
// steps per tick.  Items are the blocks of one member system per group;
// blockIdx.y = p; LP lanes per particle as in k_brownian_sum.
template <int D, int LP, bool F32>
__global__ __launch_bounds__(kBlk) void k_bm_window(const BlkItem* __restrict__ items,
                                                    const SysDev* __restrict__ sys, Coef cf, int64_t r_min,
                                                    int64_t tick_arg, const int64_t* __restrict__ tick_dev,
                                                    double* __restrict__ win)
{
    const BlkItem it = items[blockIdx.x / LP];
    const int sub = blockIdx.x % LP;
    const int p = blockIdx.y;
    const SysDev S = sys[it.sys];
    const int q = threadIdx.x % LP;
    const int i = it.blk * kBlk + sub * (kBlk / LP) + threadIdx.x / LP;
    const int64_t t = tick_of(tick_dev, tick_arg) + p;
    double zs[kMaxD] = {0.0, 0.0, 0.0, 0.0};
    if (i < S.N) {
        const uint64_t q0 = (uint64_t)t * (uint64_t)r_min * D;
        const uint64_t q1 = q0 + (uint64_t)r_min * D;
        stream_sum<D, F32>(cf.seed, (uint64_t)i, (uint64_t)S.ens, q0, q1, q0 / 4 + q, LP, zs);
    }
    lane_butterfly<LP, D>(zs);
    if (q == 0 && i < S.N) {
#pragma unroll
        for (int k = 0; k < D; ++k) win[S.win_off + ((int64_t)p * D + k) * S.N + i] = zs[k];
    }
}

// k_prep: the combine (first n_combine blocks), the Brownian sums (up to
// n_main) and the system means (job.n blocks) of an exact tick in one launch;
// the parts are independent, so the HBM-bound combine runs beside the
// FP64-bound Philox/Box-Muller work.
template <typename PT, int D, int LP>
__global__ __launch_bounds__(kBlk) void k_prep(int n_combine, int n_main, const BlkItem* __restrict__ items,
                                               const SysDev* __restrict__ sys, Coef cf, int64_t P,
                                               const PT* __restrict__ Bp, const PT* __restrict__ Bpj,
                                               const double* __restrict__ jtot,
                                               double* __restrict__ pairsum, int64_t tick_arg,
                                               const int64_t* __restrict__ tick_dev, const double* __restrict__ win,
                                               double* __restrict__ dW, YMeanJob job)
{
    static_assert(64 * kCombineWaves == kBlk, "one block shape for both parts");
    __shared__ double part[kCombineWaves][D][64];
    if ((int)blockIdx.x < n_combine)
        combine_block<PT, D>(blockIdx.x, items, sys, P, Bp, Bpj, jtot, pairsum, part);
    else if ((int)blockIdx.x < n_main)
        brownian_block<D, LP, (sizeof(PT) == 4)>(blockIdx.x - n_combine, items, sys, cf, P, tick_arg, tick_dev, win, dW);
    else
        ymean_block<D>(blockIdx.x - n_main, job, sys, tick_arg, tick_dev);
}

// Advance the context's device tick counter (last launch of every tick).
__global__ void k_tick_advance(int64_t* tick_dev)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *tick_dev += 1;
}

// ---------------------------------------------------------------------------
// k_pair: one wavefront per work item.  Lane l holds R targets
// i = tgt0 + l + 64 r; the wavefront sweeps the item's sources j, which are
// wave-uniform (scalar loads), and accumulates
//   acc_k(i) += (Ys_k^j - Ys_k^i) * exp2(-|Ys^j - Ys^i|^2)
// in T.  KAHAN: plain sums over chunks of kKahanChunk sources, each chunk
// total added into a (hi, lo) pair with Neumaier's compensated summation.
// Writes Bp[split][k][slot] (in T).
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

// ---------------------------------------------------------------------------
// Symmetric work item: each unordered pair (i, j), i in the wavefront's
// target block and j in the item's source range, is evaluated once; +q goes to
// i and -q to j (q = (s_j - s_i) exp2(-|s_j - s_i|^2) is odd in (i, j)).
// Sources come in chunks of 16, one per lane of each 16-lane row (the four
// rows see the same chunk).  At step k lane p reads the source of lane
// (p + k) % 16 with DPP row_ror:(16 - k), so no source moves; its q's go to
// the i-side accumulators and to a per-step j-side accumulator, and after the
// 16 steps the per-step accumulators are sent to their owners with
// row_ror:k and summed over the rows.
// Out-of-range targets and sources sit at +-1e15: their terms are exactly 0.
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ float dpp_ror(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x120 + N, 0xF, 0xF, false));
}

// A double through the same rotation: its two 32-bit halves move alike.
template <int N>
__device__ __forceinline__ double dpp_ror(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x120 + N, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x120 + N, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return fma(a, b, c); }

// LDS j-side row of the symmetric kernel in elements of T (FP64 rows carry
// no dummy tail: their stores take the branch).
template <typename T, int D>
__host__ __device__ constexpr int sym_lds_t() { return sym_lds_for(sizeof(T) == 8, D); }
template <typename T, int D>
__host__ __device__ constexpr int sym_row_t() { return sizeof(T) == 8 ? sym_lds_f64(D) : sym_row(D); }

template <typename T, int D, int R, int K, bool JSIDE>
__device__ __forceinline__ void sym_step(const T (&s)[D], const T (&yi)[R][D], T (&acc)[R][D],
                                         T (&accj)[16][D])
{
    T sk[D];
#pragma unroll
    for (int c = 0; c < D; ++c) sk[c] = (K == 0) ? s[c] : dpp_ror<(16 - K) & 15>(s[c]);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        T z[D];
        T t = (T)0;
#pragma unroll
        for (int c = 0; c < D; ++c) {
            z[c] = sk[c] - yi[r][c];
            t = (c == 0) ? z[c] * z[c] : fma_t(z[c], z[c], t);
        }
        const T e = exp2_fast<T>(-t);
#pragma unroll
        for (int c = 0; c < D; ++c) {
            acc[r][c] = fma_t(z[c], e, acc[r][c]);
            if constexpr (JSIDE) accj[K][c] = fma_t(z[c], e, accj[K][c]);
        }
    }
}

// One step of the FP64 form: the same pair terms as sym_step against the
// lane's current source sk, with one j-side accumulator that travels with it.
template <typename T, int D, int R, bool JSIDE>
__device__ __forceinline__ void sym_eval(const T (&sk)[D], const T (&yi)[R][D], T (&acc)[R][D], T (&aj)[D])
{
#pragma unroll
    for (int r = 0; r < R; ++r) {
        T z[D];
        T t = (T)0;
#pragma unroll
        for (int c = 0; c < D; ++c) {
            z[c] = sk[c] - yi[r][c];
            t = (c == 0) ? z[c] * z[c] : fma_t(z[c], z[c], t);
        }
        const T e = exp2_fast<T>(-t);
#pragma unroll
        for (int c = 0; c < D; ++c) {
            acc[r][c] = fma_t(z[c], e, acc[r][c]);
            if constexpr (JSIDE) aj[c] = fma_t(z[c], e, aj[c]);
        }
    }
}

template <typename T, int D, int K>
__device__ __forceinline__ void sym_route(const T (&accj)[16][D], T (&tot)[D])
{
#pragma unroll
    for (int c = 0; c < D; ++c) tot[c] += dpp_ror<K>(accj[K][c]);
}

// The chunk's j-side sums (before the sign flip) go to out[c * (sym_lds_t<T, D>() / D) + j + jshift]
// for the chunk's valid sources j when write_j holds.  JSIDE = false drops
// the j-side arithmetic at compile time.
template <typename T, int D, int R, bool JSIDE = true>
__device__ __forceinline__ void sym_chunk(const T* __restrict__ base, int64_t P, int c0, int c_end,
                                          const T (&yi)[R][D], T (&acc)[R][D], T* __restrict__ out,
                                          int64_t jshift, bool write_j = true)
{
    const int lane = threadIdx.x & 63;
    const int p = lane & 15;
    const int j = c0 + p;
    const bool vj = j < c_end;
    T s[D];
#pragma unroll
    for (int c = 0; c < D; ++c) s[c] = vj ? base[c * P + j] : (T)1e15;
    T tot[D];
    if constexpr (sizeof(T) == 8) {
        // FP64: one j-side accumulator per component travels with its source
        // (both move one lane per step; the 16th move brings both home) in
        // place of 16 per-step accumulators and the route.  The steps stay a
        // loop: unrolled measured slower (d = 3, R = 2, N = 2^18: 46.3 against
        // 35.5 ms per launch; d = 1, R = 4, N = 2^16: 1.60 against 1.29 ms).
#pragma unroll
        for (int c = 0; c < D; ++c) tot[c] = (T)0;
#pragma unroll 1
        for (int k = 0; k < 16; ++k) {
            sym_eval<T, D, R, JSIDE>(s, yi, acc, tot);
#pragma unroll
            for (int c = 0; c < D; ++c) {
                s[c] = dpp_ror<15>(s[c]);
                if constexpr (JSIDE) tot[c] = dpp_ror<15>(tot[c]);
            }
        }
        if constexpr (!JSIDE) return;
    } else {
        T accj[16][D];
#pragma unroll
        for (int k = 0; k < 16; ++k)
#pragma unroll
            for (int c = 0; c < D; ++c) accj[k][c] = (T)0;
        sym_step<T, D, R, 0, JSIDE>(s, yi, acc, accj);
        sym_step<T, D, R, 1, JSIDE>(s, yi, acc, accj);
        sym_step<T, D, R, 2, JSIDE>(s, yi, acc, accj);
        sym_step<T, D, R, 3, JSIDE>(s, yi, acc, accj);
        sym_step<T, D, R, 4, JSIDE>(s, yi, acc, accj);
        sym_step<T, D, R, 5, JSIDE>(s, yi, acc, accj);
        sym_step<T, D, R, 6, JSIDE>(s, yi, acc, accj);
        sym_step<T, D, R, 7, JSIDE>(s, yi, acc, accj);
        sym_step<T, D, R, 8, JSIDE>(s, yi, acc, accj);
        sym_step<T, D, R, 9, JSIDE>(s, yi, acc, accj);
        sym_step<T, D, R, 10, JSIDE>(s, yi, acc, accj);
        sym_step<T, D, R, 11, JSIDE>(s, yi, acc, accj);
        sym_step<T, D, R, 12, JSIDE>(s, yi, acc, accj);
        sym_step<T, D, R, 13, JSIDE>(s, yi, acc, accj);
        sym_step<T, D, R, 14, JSIDE>(s, yi, acc, accj);
        sym_step<T, D, R, 15, JSIDE>(s, yi, acc, accj);
        if constexpr (!JSIDE) return;
#pragma unroll
        for (int c = 0; c < D; ++c) tot[c] = accj[0][c];
        sym_route<T, D, 1>(accj, tot);
        sym_route<T, D, 2>(accj, tot);
        sym_route<T, D, 3>(accj, tot);
        sym_route<T, D, 4>(accj, tot);
        sym_route<T, D, 5>(accj, tot);
        sym_route<T, D, 6>(accj, tot);
        sym_route<T, D, 7>(accj, tot);
        sym_route<T, D, 8>(accj, tot);
        sym_route<T, D, 9>(accj, tot);
        sym_route<T, D, 10>(accj, tot);
        sym_route<T, D, 11>(accj, tot);
        sym_route<T, D, 12>(accj, tot);
        sym_route<T, D, 13>(accj, tot);
        sym_route<T, D, 14>(accj, tot);
        sym_route<T, D, 15>(accj, tot);
    }
#pragma unroll
    for (int c = 0; c < D; ++c) {
        // across the rows through the LDS crossbar (ds_bpermute runs beside the
        // VALU work; the gfx950 row-swap instructions measured slower here)
        tot[c] += __shfl_xor(tot[c], 16, 64);
        tot[c] += __shfl_xor(tot[c], 32, 64);
    }
    if constexpr (D == 3 && sizeof(T) == 4) {
        const bool wr = write_j && lane < 16 && vj;
#pragma unroll
        for (int c = 0; c < D; ++c) out[wr ? (int)(c * (sym_lds(D) / D) + j + jshift) : sym_lds(D) + lane] = tot[c];
    } else if (write_j && lane < 16 && vj) {
#pragma unroll
        for (int c = 0; c < D; ++c) out[c * (sym_lds_t<T, D>() / D) + j + jshift] = tot[c];
    }
}

// One workgroup of kWaves wavefronts per symmetric work item.  The item
// covers a target group of kWaves blocks of 64 R particles (wavefront w takes
// block w) and either
//  - the group itself (jrow < 0, "diagonal"): wavefront w takes the ordered
//    pairs of its own block (i-side only) and the unordered pairs with the
//    later blocks of the group; i-side partial 0, and
//    the j-side sums of the group's particles form row a of the j-side
//    partials (zero for block 0); or
//  - a later source range (jrow = a): unordered pairs with every block of
//    the group; i-side partial `split`, j-side row a.
// j-side sums pass through LDS (sym_lds(d) / d sources at a time) and are added
// over the wavefronts in a fixed order before they are written.  With banded
// j-side rows (k_jfold) the launch covers the groups of one band and row a
// is stored at a - jrow_base.
template <typename T, int D, int R, bool KAHAN>
__device__ __forceinline__ void kahan_fold(T (&acc)[R][D], T (&hi)[R][D], T (&lo)[R][D])
{
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const T a = acc[r][c];
            const T sm = hi[r][c] + a;
            lo[r][c] += (fabs(hi[r][c]) >= fabs(a)) ? (hi[r][c] - sm) + a : (a - sm) + hi[r][c];
            hi[r][c] = sm;
            acc[r][c] = (T)0;
        }
}

// Sum the wavefronts' LDS j-side sums for sources [j0, j0 + n) (LDS index
// j - lds0) and store them, negated, in row `row` of the j-side partials.
template <typename T, int D>
__device__ __forceinline__ void jside_flush(T (*jred)[(sym_row_t<T, D>())], T* __restrict__ Bpj, int64_t row,
                                            int64_t P, int64_t off, int j0, int n, int lds0)
{
    constexpr int stride = sym_lds_t<T, D>() / D;
    T* Bpj_row = Bpj + row * D * P;
#pragma unroll
    for (int c = 0; c < D; ++c)
        for (int jj = threadIdx.x; jj < n; jj += 64 * kWaves) {
            const int li = c * stride + (j0 + jj - lds0);
            T v = jred[0][li];
#pragma unroll
            for (int w = 1; w < kWaves; ++w) v += jred[w][li];
            Bpj_row[c * P + off + j0 + jj] = -v;
        }
}

template <typename T, int D, int R, bool KAHAN>
__global__ __launch_bounds__(64 * kWaves) void k_pair_sym(const PairItem* __restrict__ items,
                                                          const SysDev* __restrict__ sys,
                                                          const T* __restrict__ Ys, int64_t P,
                                                          T* __restrict__ Bp, T* __restrict__ Bpj, int jrow_base)
{
    constexpr int stride = sym_lds_t<T, D>() / D;  // LDS j-side capacity (sources) per component
    __shared__ T jred[kWaves][(sym_row_t<T, D>())];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const PairItem it = items[blockIdx.x];
    const SysDev S = sys[it.sys];
    const T* __restrict__ base = Ys + S.off;
    const int blk = 64 * R;
    const int tb0 = it.tgt0 + wave * blk;  // this wavefront's target block

    T yi[R][D], acc[R][D], hi[R][D], lo[R][D];
    bool valid[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = tb0 + lane + 64 * r;
        valid[r] = i < S.N;
#pragma unroll
        for (int c = 0; c < D; ++c) {
            yi[r][c] = valid[r] ? base[c * P + i] : (T)-1e15;
            acc[r][c] = hi[r][c] = lo[r][c] = (T)0;
        }
    }

    // One loop for both kinds of item (a single inlined copy of the chunk
    // routine keeps the register count down):
    //  - group itself: wavefront w sweeps [own block start, group end); the
    //    chunks of its own block skip the j-side store (a block against
    //    itself gives each target its full ordered sum; its j-side would
    //    count the pairs twice); one j-side flush at the end;
    //  - later range: all wavefronts sweep the range, flushing the j-side
    //    every `stride` sources (uniform trip counts around the barriers).
    const bool diag = it.jrow < 0;
    const int g_end = it.tgt0 + it.nsrc;
    const int own_end = min(tb0 + blk, g_end);
    const int start = diag ? tb0 : it.src0;
    const int end = diag ? g_end : it.src0 + it.nsrc;
    const int piece = diag ? sym_lds_t<T, D>() : stride;  // group x d <= the row: one piece
    if (diag) {
        for (int q = lane; q < sym_lds_t<T, D>(); q += 64) jred[wave][q] = (T)0;
    }
    int chunks = 0;
    for (int u0 = start; u0 < end; u0 += piece) {
        const int u1 = min(u0 + piece, end);
        const int64_t jshift = diag ? -(int64_t)it.tgt0 : -(int64_t)u0;
        for (int c0 = u0; c0 < u1; c0 += 16) {
            const int ce = (diag && c0 < own_end) ? own_end : u1;
            sym_chunk<T, D, R>(base, P, c0, ce, yi, acc, &jred[wave][0], jshift, !(diag && c0 < own_end));
            if constexpr (KAHAN) {
                if (++chunks == kKahanChunk / 16) {
                    chunks = 0;
                    kahan_fold<T, D, R, KAHAN>(acc, hi, lo);
                }
            }
        }
        if (!diag) {
            __syncthreads();
            jside_flush<T, D>(jred, Bpj, (int64_t)(it.jrow - jrow_base), P, S.off, u0, u1 - u0, u0);
            if (u1 < end) __syncthreads();  // the next piece reuses the LDS
        }
    }
    if constexpr (KAHAN) kahan_fold<T, D, R, KAHAN>(acc, hi, lo);
    if (diag) {
        __syncthreads();
        jside_flush<T, D>(jred, Bpj, (int64_t)(it.tgt0 / (blk * kWaves) - jrow_base), P, S.off, it.tgt0, it.nsrc,
                          it.tgt0);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = tb0 + lane + 64 * r;
        if (!valid[r]) continue;
#pragma unroll
        for (int c = 0; c < D; ++c) {
            // the compensated sum hi + lo, rounded once
            const T v = KAHAN ? (T)((double)hi[r][c] + (double)lo[r][c]) : acc[r][c];
            Bp[((int64_t)it.split * D + c) * P + S.off + i] = v;
        }
    }
}

template <typename T, int D, int R, bool KAHAN>
__global__ __launch_bounds__(64 * kWaves) void k_pair(const PairItem* __restrict__ items,
                                                      int n_items,
                                                      const SysDev* __restrict__ sys,
                                                      const T* __restrict__ Ys, int64_t P,
                                                      T* __restrict__ Bp)
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
        // hi + lo is added in double and rounded once to T at the store below
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = it.tgt0 + lane + 64 * r;
            if (!valid[r]) continue;
#pragma unroll
            for (int k = 0; k < D; ++k)
                Bp[((int64_t)it.split * D + k) * P + S.off + i] = (T)((double)hi[r][k] + (double)lo[r][k]);
        }
        return;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = it.tgt0 + lane + 64 * r;
        if (!valid[r]) continue;
#pragma unroll
        for (int k = 0; k < D; ++k) Bp[((int64_t)it.split * D + k) * P + S.off + i] = acc[r][k];
    }
}

// FP32 study variant of the ordered kernel: every pair's term is added into
// the target's (hi, lo) pair by Neumaier's method (no plain partial sums), so
// the pair sums carry no FP32 accumulation error beyond each term's own
// rounding.  Same items and partial layout as k_pair; hi + lo is rounded once
// to float per item.
template <int D, int R>
__global__ __launch_bounds__(64 * kWaves) void k_pair_kpair(const PairItem* __restrict__ items, int n_items,
                                                            const SysDev* __restrict__ sys,
                                                            const float* __restrict__ Ys, int64_t P,
                                                            float* __restrict__ Bp)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int idx = blockIdx.x * kWaves + wave;
    if (idx >= n_items) return;
    const PairItem it = items[idx];
    const SysDev S = sys[it.sys];
    const float* __restrict__ base = Ys + S.off;
    float yi[R][D], hi[R][D], lo[R][D];
    bool valid[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = it.tgt0 + lane + 64 * r;
        valid[r] = i < S.N;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            yi[r][k] = valid[r] ? base[k * P + i] : 0.0f;
            hi[r][k] = lo[r][k] = 0.0f;
        }
    }
    for (int j = it.src0; j < it.src0 + it.nsrc; ++j) {
        float s[D];
#pragma unroll
        for (int k = 0; k < D; ++k) s[k] = base[k * P + j];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            float z[D];
            float t = 0.0f;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                z[k] = s[k] - yi[r][k];
                t = (k == 0) ? z[k] * z[k] : fmaf(z[k], z[k], t);
            }
            const float e = exp2_fast<float>(-t);
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const float a = z[k] * e;
                const float sm = hi[r][k] + a;
                lo[r][k] += (fabsf(hi[r][k]) >= fabsf(a)) ? (hi[r][k] - sm) + a : (a - sm) + hi[r][k];
                hi[r][k] = sm;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = it.tgt0 + lane + 64 * r;
        if (!valid[r]) continue;
#pragma unroll
        for (int k = 0; k < D; ++k)
            Bp[((int64_t)it.split * D + k) * P + S.off + i] = (float)((double)hi[r][k] + (double)lo[r][k]);
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

__global__ void k_brownian(int d, int64_t N, uint64_t seed, int32_t ens, int64_t n0, int32_t r,
                           double sqrt_hf, double* __restrict__ dW);

__global__ void k_philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                         uint64_t k1, int64_t count, uint64_t* __restrict__ out);

}  // namespace ssm
