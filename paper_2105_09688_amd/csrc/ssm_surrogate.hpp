// ssm_surrogate.hpp -- learned surrogate of the interaction drift (not in the
// paper): random-Fourier-feature moments of mu^Y and a small MLP
//   [hi(y) (d), lo(y) (d), C_1..C_K, S_1..S_K] -> 64 -> 64 -> 64 -> d,
// SiLU hidden layers, where hi(y) = bf16(y) and lo(y) = bf16(y - hi(y)) carry
// the position to about 16 significant bits through the BF16 input layer,
// BF16 operands with FP32 accumulation on the matrix cores (MFMA), trained
// on (y, moments, exact pair term) samples by hand-written kernels with Adam.
//
// Matrix-core tiles: v_mfma_f32_16x16x32_bf16.  For one wavefront (lane l):
//   A (16 x 32): lane holds A[l % 16][8 (l / 16) + 0..7]
//   B (32 x 16): lane holds B[8 (l / 16) + 0..7][l % 16]
//   D (16 x 16): lane holds D[4 (l / 16) + 0..3][l % 16]
// A wavefront always works on 16 samples (rows); features are columns.
#pragma once

#include "ssm_kernels.hpp"

namespace ssm {

constexpr int kRff = 16;         // frequencies; 2 kRff moments
constexpr int kHid = 64;         // hidden width
constexpr int kKpad = 64;        // input features padded: 2 d + 2 kRff <= 40 -> 64
constexpr int kOutPad = 16;      // outputs padded to one 16-column tile
constexpr int kStride = 72;      // LDS/global row stride (bf16) of 64-wide rows (bank spread)
constexpr int kStrideT4 = 40;    // row stride of the transposed output layer (32 used)
constexpr int kRffWaves = 4;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Inference layout (k_mlp_infer, k_mlp_apply).  The products run transposed,
// D = W (16 outputs x K) * act^T (K x 16 samples): each lane then holds, for
// its sample l % 16, the outputs 16 nt + 4 (l / 16) + i of every output tile
// nt, which are exactly the eight K entries it must supply to the next layer's
// B operand once the next layer's input columns are taken in the order
//   K slice ks, entry k (0..31)  <->  input feature (2 ks + (k % 8) / 4) 16 + 4 (k / 8) + k % 4.
// So an activation never leaves its lane; the permutation is applied to the
// weights once, when they are packed, and every A operand is stored in lane
// order (lane l's 8 BF16 at [l]), one conflict-free 16-byte LDS read each.
// Layer 1 takes only the position columns [hi(y), lo(y)] on the matrix cores;
// the moment columns act on per-system constants, so their product with the
// moments is a per-system bias computed in FP32 (W1m below).
struct MlpInfer {
    bf16x8 W1[4][64];         // [out tile][lane]: W1[16 nt + l % 16][k], k = 8 (l / 16) + j < 2 d, else 0
    bf16x8 W2[4][2][64];      // [out tile][K slice][lane], permuted input columns
    bf16x8 W3[4][2][64];
    bf16x8 W4[2][64];         // [K slice][lane]: rows l % 16 < d
    float W1m[kHid][2 * kRff];  // moment columns of W1 (BF16 values) as float
};

// Packed device weights: BF16 row-major [out][in] rows padded to kStride, and
// the transposes needed by the backward pass; FP32 biases; the inference layout.
struct MlpPacked {
    __bf16 W1[kHid * kStride];      // [64 out][64 in (d + 2K used)]
    __bf16 W2[kHid * kStride];
    __bf16 W3[kHid * kStride];
    __bf16 W4[kOutPad * kStride];   // [16 out (d used)][64 in]
    __bf16 W2t[kHid * kStride];     // [64 in][64 out]
    __bf16 W3t[kHid * kStride];
    __bf16 W4t[kHid * kStrideT4];   // [64 in][32 out (d used)]
    float b1[kHid], b2[kHid], b3[kHid], b4[kOutPad];
    MlpInfer inf;
};

// Flat master layout (FP32), as the oracle's: W1[64][in] b1[64] W2[64][64] b2
// W3[64][64] b3 W4[d][64] b4[d], in = 2 d + 2 kRff network inputs.  Sample
// rows handed to the library are "raw": [y (d), moments (2 kRff)].
__host__ __device__ constexpr int mlp_in(int d) { return 2 * d + 2 * kRff; }
__host__ __device__ constexpr int raw_in(int d) { return d + 2 * kRff; }

__device__ __forceinline__ __bf16 bf_hi(float y) { return (__bf16)y; }
__device__ __forceinline__ __bf16 bf_lo(float y) { return (__bf16)(y - (float)(__bf16)y); }
__host__ __device__ constexpr int64_t mlp_params(int d)
{
    return (int64_t)kHid * mlp_in(d) + kHid + 2 * ((int64_t)kHid * kHid + kHid) + (int64_t)d * kHid + d;
}

struct MlpOffsets {
    int64_t W1, b1, W2, b2, W3, b3, W4, b4;
};

__host__ __device__ inline MlpOffsets mlp_offsets(int d)
{
    MlpOffsets o{};
    const int in = mlp_in(d);
    o.W1 = 0;
    o.b1 = o.W1 + (int64_t)kHid * in;
    o.W2 = o.b1 + kHid;
    o.b2 = o.W2 + kHid * kHid;
    o.W3 = o.b2 + kHid;
    o.b3 = o.W3 + kHid * kHid;
    o.W4 = o.b3 + kHid;
    o.b4 = o.W4 + (int64_t)d * kHid;
    return o;
}

__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// sigma(z) = 1 / (1 + e^-z) with the hardware reciprocal (v_rcp_f32, 1 ulp)
// instead of a correctly rounded division: the network's activations carry
// about 16 significant bits, and the division was most of SiLU's cost.  For
// z -> -inf, e^-z -> inf and the reciprocal gives 0.
__device__ __forceinline__ float sigmoid_f(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

__device__ __forceinline__ float silu_f(float z) { return z * sigmoid_f(z); }

__device__ __forceinline__ float silu_prime_f(float z)
{
    const float s = sigmoid_f(z);
    return s * (1.0f + z * (1.0f - s));
}

// ---------------------------------------------------------------------------
// Fresh master weights: each weight matrix uniform on +-sqrt(6 / (fan_in +
// fan_out)), biases zero.  Parameter p takes word p % 4 of the Philox block
// with counter (p / 4, 0, 0, 5 * 2^32) under key (seed, 0) (stream tag 5).
// ---------------------------------------------------------------------------
__global__ void k_mlp_init(uint64_t seed, int d, float* __restrict__ master)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const MlpOffsets o = mlp_offsets(d);
    if (p >= mlp_params(d)) return;
    int fan_in = 0, fan_out = 0;
    if (p < o.b1) { fan_in = mlp_in(d); fan_out = kHid; }
    else if (p >= o.W2 && p < o.b2) { fan_in = kHid; fan_out = kHid; }
    else if (p >= o.W3 && p < o.b3) { fan_in = kHid; fan_out = kHid; }
    else if (p >= o.W4 && p < o.b4) { fan_in = kHid; fan_out = d; }
    float v = 0.0f;
    if (fan_in > 0) {
        const Block4 b = philox4x64_10((uint64_t)(p / 4), 0ull, 0ull, (uint64_t)5 << 32, seed, 0ull);
        const double u = unit_open(b.w[p % 4]);
        v = (float)(sqrt(6.0 / (double)(fan_in + fan_out)) * (2.0 * u - 1.0));
    }
    master[p] = v;
}

// ---------------------------------------------------------------------------
// master (flat FP32) -> packed BF16 (+ transposes), zero padding
// ---------------------------------------------------------------------------
__global__ void k_mlp_pack(const float* __restrict__ master, int d, MlpPacked* __restrict__ P)
{
    const MlpOffsets o = mlp_offsets(d);
    const int in = mlp_in(d);
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    // t indexes a (row, col) of a 64 x 72 grid, reused for every matrix
    if (t >= kHid * kStride) return;
    const int r = t / kStride, c = t % kStride;
    auto bf = [](float x) { return (__bf16)x; };
    P->W1[t] = bf((c < in) ? master[o.W1 + (int64_t)r * in + c] : 0.0f);
    P->W2[t] = bf((c < kHid) ? master[o.W2 + (int64_t)r * kHid + c] : 0.0f);
    P->W3[t] = bf((c < kHid) ? master[o.W3 + (int64_t)r * kHid + c] : 0.0f);
    P->W2t[t] = bf((c < kHid) ? master[o.W2 + (int64_t)c * kHid + r] : 0.0f);  // [in r][out c]
    P->W3t[t] = bf((c < kHid) ? master[o.W3 + (int64_t)c * kHid + r] : 0.0f);
    if (r < kOutPad) P->W4[t] = bf((r < d && c < kHid) ? master[o.W4 + (int64_t)r * kHid + c] : 0.0f);
    if (c < kStrideT4) P->W4t[r * kStrideT4 + c] = bf((c < d) ? master[o.W4 + (int64_t)c * kHid + r] : 0.0f);
    if (c == 0) {
        P->b1[r] = master[o.b1 + r];
        P->b2[r] = master[o.b2 + r];
        P->b3[r] = master[o.b3 + r];
        if (r < kOutPad) P->b4[r] = (r < d) ? master[o.b4 + r] : 0.0f;
    }
}

// The inference layout of master (flat FP32) weights: A operands in lane
// order with the permuted input columns of layers 2-4, and the moment columns
// of W1 as float (of their BF16 values).
__host__ __device__ constexpr int infer_feature(int ks, int k) { return (2 * ks + (k % 8) / 4) * 16 + 4 * (k / 8) + k % 4; }

__global__ void k_mlp_pack_infer(const float* __restrict__ master, int d, MlpInfer* __restrict__ P)
{
    const MlpOffsets o = mlp_offsets(d);
    const int in = mlp_in(d);
    const int nW1 = 4 * 64 * 8, nW2 = 4 * 2 * 64 * 8, nW4 = 2 * 64 * 8, nM = kHid * 2 * kRff;
    const int total = nW1 + 2 * nW2 + nW4 + nM;
    // element stores through scalar pointers (flat index = the array's own
    // [..][lane][j] order): one thread per BF16 value, no shared 16-byte word
    __bf16* w1 = (__bf16*)P->W1;
    __bf16* w2 = (__bf16*)P->W2;
    __bf16* w3 = (__bf16*)P->W3;
    __bf16* w4 = (__bf16*)P->W4;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        int q = e;
        if (q < nW1) {
            const int nt = q / 512, l = (q / 8) % 64, j = q % 8, k = 8 * (l / 16) + j;
            w1[q] = (__bf16)((k < 2 * d) ? master[o.W1 + (int64_t)(16 * nt + l % 16) * in + k] : 0.0f);
            continue;
        }
        q -= nW1;
        if (q < 2 * nW2) {
            const int layer = q / nW2;
            q %= nW2;
            const int nt = q / 1024, ks = (q / 512) % 2, l = (q / 8) % 64, j = q % 8;
            const int f = infer_feature(ks, 8 * (l / 16) + j);
            const int64_t base = layer == 0 ? o.W2 : o.W3;
            (layer == 0 ? w2 : w3)[q] = (__bf16)master[base + (int64_t)(16 * nt + l % 16) * kHid + f];
            continue;
        }
        q -= 2 * nW2;
        if (q < nW4) {
            const int ks = q / 512, l = (q / 8) % 64, j = q % 8, m = l % 16;
            const int f = infer_feature(ks, 8 * (l / 16) + j);
            w4[q] = (__bf16)((m < d) ? master[o.W4 + (int64_t)m * kHid + f] : 0.0f);
            continue;
        }
        q -= nW4;
        const int r = q / (2 * kRff), c = q % (2 * kRff);
        P->W1m[r][c] = (float)(__bf16)master[o.W1 + (int64_t)r * in + 2 * d + c];
    }
}

// Copy the forward weights (W1..W4, biases) into LDS.
__device__ __forceinline__ void load_fwd_weights(const MlpPacked* __restrict__ P, __bf16* sW1, __bf16* sW2,
                                                 __bf16* sW3, __bf16* sW4, float* sb)
{
    const int nt = blockDim.x;
    const uint4* g1 = (const uint4*)P->W1;
    const uint4* g2 = (const uint4*)P->W2;
    const uint4* g3 = (const uint4*)P->W3;
    const uint4* g4 = (const uint4*)P->W4;
    const int n64 = kHid * kStride * 2 / 16;
    const int n16 = kOutPad * kStride * 2 / 16;
    for (int q = threadIdx.x; q < n64; q += nt) {
        ((uint4*)sW1)[q] = g1[q];
        ((uint4*)sW2)[q] = g2[q];
        ((uint4*)sW3)[q] = g3[q];
    }
    for (int q = threadIdx.x; q < n16; q += nt) ((uint4*)sW4)[q] = g4[q];
    for (int q = threadIdx.x; q < 3 * kHid + kOutPad; q += nt) {
        float v;
        if (q < kHid) v = P->b1[q];
        else if (q < 2 * kHid) v = P->b2[q - kHid];
        else if (q < 3 * kHid) v = P->b3[q - 2 * kHid];
        else v = P->b4[q - 3 * kHid];
        sb[q] = v;
    }
}

// One dense layer for the wavefront's 16 samples: acc[nt] = A (16 x 64) * W^T
// for NT column tiles; W is LDS [NT*16][kStride] (row = output feature).
template <int NT>
__device__ __forceinline__ void dense_tiles(const __bf16* W, const bf16x8 a[2], f32x4 acc[NT])
{
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        f32x4 c = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const bf16x8 b = *(const bf16x8*)&W[(nt * 16 + (l & 15)) * kStride + ks * 32 + 8 * (l >> 4)];
            c = mfma_bf16(a[ks], b, c);
        }
        acc[nt] = c;
    }
}

// Write 16 x (16 NT) values held in D layout into an LDS tile [16][kStride]
// as BF16, then read them back in A layout (two K slices of 32).
template <int NT>
__device__ __forceinline__ void d_to_a(const f32x4 v[NT], __bf16* tile, bf16x8 a[2])
{
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) tile[(4 * (l >> 4) + i) * kStride + nt * 16 + (l & 15)] = (__bf16)v[nt][i];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) a[ks] = *(const bf16x8*)&tile[(l & 15) * kStride + ks * 32 + 8 * (l >> 4)];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Input features of one sample in A layout (training): lane l holds features
// k = 32 ks + 8 (l / 16) + 0..7 of sample l % 16:  u = [hi(y), lo(y), m_0..m_{2K-1}, 0...],
// from a raw row r = [y (d), m (2K)] in global memory (r may be null: zeros).
__device__ __forceinline__ void build_input_row(const float* r, int d, bf16x8 a[2])
{
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = ks * 32 + 8 * (l >> 4) + i;
            __bf16 v = (__bf16)0.0f;
            if (r) {
                if (k < d) v = bf_hi(r[k]);
                else if (k < 2 * d) v = bf_lo(r[k - d]);
                else if (k < 2 * d + 2 * kRff) v = (__bf16)r[k - d];
            }
            a[ks][i] = v;
        }
}

// Forward pass of the wavefront's 16 samples.  Returns the output tile
// (D layout, columns 0..d-1 valid, bias added) and optionally the
// pre-activations z1..z3 (D layout) for the backward pass.
__device__ __forceinline__ void mlp_forward16(const __bf16* sW1, const __bf16* sW2, const __bf16* sW3,
                                              const __bf16* sW4, const float* sb, bf16x8 a[2],
                                              __bf16* tile, f32x4 z[3][4], f32x4& out, bf16x8 act[3][2])
{
    const int l = threadIdx.x & 63;
    const __bf16* Ws[3] = {sW1, sW2, sW3};
#pragma unroll
    for (int layer = 0; layer < 3; ++layer) {
        f32x4 acc[4];
        dense_tiles<4>(Ws[layer], a, acc);
        f32x4 h[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const float bias = sb[layer * kHid + nt * 16 + (l & 15)];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float zz = acc[nt][i] + bias;
                z[layer][nt][i] = zz;
                h[nt][i] = silu_f(zz);
            }
        }
        d_to_a<4>(h, tile, a);
        act[layer][0] = a[0];
        act[layer][1] = a[1];
    }
    f32x4 o[1];
    dense_tiles<1>(sW4, a, o);
    const float b4 = sb[3 * kHid + (l & 15)];
#pragma unroll
    for (int i = 0; i < 4; ++i) out[i] = o[0][i] + b4;
}

// ---------------------------------------------------------------------------
// RFF moments: per-block sums of cos / sin(omega_k . y) (FP32 within a block,
// FP64 partials), then one block per system reduces its partials in order.
// ---------------------------------------------------------------------------
struct RffFreq {
    float w[kRff][kMaxD];  // omega_k (already divided by ell)
};

template <typename T, int D>
__global__ __launch_bounds__(kBlk) void k_rff_partial(const BlkItem* __restrict__ items,
                                                      const SysDev* __restrict__ sys, int64_t P,
                                                      const T* __restrict__ Y, RffFreq fq,
                                                      double* __restrict__ part /*[nblk_tot][2K]*/)
{
    __shared__ float red[2 * kRff][kBlk + 1];
    const BlkItem it = items[blockIdx.x];
    const SysDev S = sys[it.sys];
    const int i = it.blk * kBlk + threadIdx.x;
    const bool valid = i < S.N;
    float y[D];
#pragma unroll
    for (int k = 0; k < D; ++k) y[k] = valid ? (float)Y[k * P + S.off + i] : 0.0f;
#pragma unroll
    for (int q = 0; q < kRff; ++q) {
        float ph = 0.0f;
#pragma unroll
        for (int k = 0; k < D; ++k) ph = fmaf(fq.w[q][k], y[k], ph);
        float sn, cs;
        __sincosf(ph, &sn, &cs);
        red[q][threadIdx.x] = valid ? cs : 0.0f;
        red[kRff + q][threadIdx.x] = valid ? sn : 0.0f;
    }
    __syncthreads();
    if (threadIdx.x < 2 * kRff) {
        double s = 0.0;
        for (int t = 0; t < kBlk; ++t) s += (double)red[threadIdx.x][t];
        part[(int64_t)(S.blk0 + it.blk) * (2 * kRff) + threadIdx.x] = s;
    }
}

// Sum over a system's block partials part[(blk0 + b) * stride + q], b < nblk:
// thread t adds b = t, t + kBlk, ... in order, then a fixed-order tree over
// the block.  All threads of the block must call it.
__device__ __forceinline__ double sum_block_partials(const double* __restrict__ part, int64_t blk0, int64_t nblk,
                                                     int stride, int q, double* red)
{
    double acc = 0.0;
    for (int64_t b = threadIdx.x; b < nblk; b += kBlk) acc += part[(blk0 + b) * stride + q];
    return block_sum(acc, red);
}

// grid (listed systems, 2K), kBlk threads: mom[sys][q] = (1/N) sum of its block partials
__global__ __launch_bounds__(kBlk) void k_rff_final(const int32_t* __restrict__ sys_list,
                                                    const SysDev* __restrict__ sys,
                                                    const double* __restrict__ part, float* __restrict__ mom)
{
    __shared__ double red[kBlk];
    const int s = sys_list[blockIdx.x];
    const SysDev S = sys[s];
    const int q = blockIdx.y;
    const double t = sum_block_partials(part, S.blk0, S.nblk, 2 * kRff, q, red);
    if (threadIdx.x == 0) mom[(int64_t)s * (2 * kRff) + q] = (float)(t / (double)S.N);
}

// ---------------------------------------------------------------------------
// Inference (split precision).  Every activation enters the matrix cores as
// hi + lo with hi = bf16(v) and lo = bf16(v - hi) (about 16 significant bits),
// each product as W hi + W lo; the weights stay BF16 (the network is trained
// with them), so the network stays a smooth function of its inputs (plain
// BF16 activations add rounding noise of order 1e-3 relative that changes
// from one step to the next).  A wavefront runs two 16-sample tiles at a
// time in the transposed layout of MlpInfer.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Two floats -> packed BF16 (one v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint32_t pk_bf16(float a, float b)
{
    const f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}

// hi / lo B operands of 8 values (4 from each of two output tiles).
__device__ __forceinline__ void split8(const f32x4& a, const f32x4& b, bf16x8& hi, bf16x8& lo)
{
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    u32x4 h, l;
    const float v[8] = {a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t hp = pk_bf16(v[2 * q], v[2 * q + 1]);
        h[q] = hp;
        l[q] = pk_bf16(v[2 * q] - __uint_as_float(hp << 16), v[2 * q + 1] - __uint_as_float(hp & 0xffff0000u));
    }
    hi = __builtin_bit_cast(bf16x8, h);
    lo = __builtin_bit_cast(bf16x8, l);
}

// The hidden layers run on scaled values u = -log2(e) z (pre-activations)
// and a~ = -log2(e) a (activations): every hidden layer's input and bias
// carry the factor, so its output is u directly (the product is linear), and
//   a~ = -log2(e) z sigma(z) = u / (1 + 2^u)
// with the hardware exp2 and reciprocal (sigma(z) = 1 / (1 + e^-z)).  The
// factor enters before the hi / lo split, so it costs no precision.  Layer 1
// scales its output (its inputs hi(y), lo(y) are features of their own, with
// their own weights, and are taken as they are); the output layer undoes the
// factor once.
constexpr float kNegLog2e = -1.4426950408889634f;
constexpr float kNegLn2 = -0.6931471805599453f;

__device__ __forceinline__ float silu_scaled(float u) { return u * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(u)); }

// SiLU of a layer's four output tiles (scaled), split into the next layer's
// operands (K slice 0: tiles 0, 1; slice 1: tiles 2, 3).
__device__ __forceinline__ void act_split(f32x4 (&acc)[4], bf16x8 (&hi)[2], bf16x8 (&lo)[2])
{
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[nt][i] = silu_scaled(acc[nt][i]);
    split8(acc[0], acc[1], hi[0], lo[0]);
    split8(acc[2], acc[3], hi[1], lo[1]);
}

// LDS copy of the inference weights and biases (-log2(e) b2, -log2(e) b3, -log2(e) b4).
struct InferLds {
    bf16x8 W1[4][64];
    bf16x8 W2[4][2][64];
    bf16x8 W3[4][2][64];
    bf16x8 W4[2][64];
    float b[2 * kHid + kOutPad];
};

__device__ __forceinline__ void load_infer(const MlpPacked* __restrict__ P, InferLds& L)
{
    const uint4* src[4] = {(const uint4*)P->inf.W1, (const uint4*)P->inf.W2, (const uint4*)P->inf.W3,
                           (const uint4*)P->inf.W4};
    uint4* dst[4] = {(uint4*)L.W1, (uint4*)L.W2, (uint4*)L.W3, (uint4*)L.W4};
    const int n[4] = {4 * 64, 8 * 64, 8 * 64, 2 * 64};
#pragma unroll
    for (int m = 0; m < 4; ++m)
        for (int q = threadIdx.x; q < n[m]; q += blockDim.x) dst[m][q] = src[m][q];
    for (int q = threadIdx.x; q < 2 * kHid + kOutPad; q += blockDim.x)
        L.b[q] = kNegLog2e * (q < kHid ? P->b2[q] : q < 2 * kHid ? P->b3[q - kHid] : P->b4[q - 2 * kHid]);
}

// acc[nt][i] = v[16 nt + 4 (l / 16) + i]: a bias vector in the D layout.
__device__ __forceinline__ void bias_tiles(const float* v, f32x4 (&acc)[4])
{
    const int g = (threadIdx.x & 63) >> 4;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = *(const f32x4*)&v[16 * nt + 4 * g];
}

// One hidden layer (64 -> 64) for two tiles; acc in: bias, out: pre-activation.
__device__ __forceinline__ void hidden_layer2(const bf16x8 (*W)[2][64], const bf16x8 (&h0)[2], const bf16x8 (&l0)[2],
                                              const bf16x8 (&h1)[2], const bf16x8 (&l1)[2], f32x4 (&a0)[4],
                                              f32x4 (&a1)[4])
{
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const bf16x8 w = W[nt][ks][l];
            a0[nt] = mfma_bf16(w, l0[ks], a0[nt]);
            a1[nt] = mfma_bf16(w, l1[ks], a1[nt]);
            a0[nt] = mfma_bf16(w, h0[ks], a0[nt]);
            a1[nt] = mfma_bf16(w, h1[ks], a1[nt]);
        }
}

// The network for two tiles of 16 samples.  yin[t][c]: coordinate c of the
// lane's sample l % 16 in tile t; c1[t]: layer 1's bias plus its moment part
// for tile t, in the D layout.  out[t]: D layout of the output tile (lane l,
// l < 16: components 0..3 of sample l; bias added).
template <int D>
__device__ __forceinline__ void mlp_infer_pair(const InferLds& L, const float (&yin)[2][kMaxD], f32x4 (&c1)[2][4],
                                               f32x4 (&out)[2])
{
    const int l = threadIdx.x & 63;
    const int g = l >> 4;
    // layer 1: K slice [hi(y), lo(y), 0 ...]; lanes of group 0 hold the entries
    bf16x8 x[2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            __bf16 v = (__bf16)0.0f;
            if (g == 0 && j < 2 * D) {
                const float y = yin[t][j < D ? j : j - D];
                v = j < D ? (__bf16)y : (__bf16)(y - (float)(__bf16)y);
            }
            x[t][j] = v;
        }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const bf16x8 w = L.W1[nt][l];
        c1[0][nt] = mfma_bf16(w, x[0], c1[0][nt]);
        c1[1][nt] = mfma_bf16(w, x[1], c1[1][nt]);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) c1[t][nt][i] *= kNegLog2e;
    bf16x8 h0[2], l0[2], h1[2], l1[2];
    act_split(c1[0], h0, l0);
    act_split(c1[1], h1, l1);
    f32x4 a0[4], a1[4];
    bias_tiles(&L.b[0], a0);
    bias_tiles(&L.b[0], a1);
    hidden_layer2(L.W2, h0, l0, h1, l1, a0, a1);
    act_split(a0, h0, l0);
    act_split(a1, h1, l1);
    bias_tiles(&L.b[kHid], a0);
    bias_tiles(&L.b[kHid], a1);
    hidden_layer2(L.W3, h0, l0, h1, l1, a0, a1);
    act_split(a0, h0, l0);
    act_split(a1, h1, l1);
    out[0] = out[1] = *(const f32x4*)&L.b[2 * kHid + 4 * g];
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
        const bf16x8 w = L.W4[ks][l];
        out[0] = mfma_bf16(w, l0[ks], out[0]);
        out[1] = mfma_bf16(w, l1[ks], out[1]);
        out[0] = mfma_bf16(w, h0[ks], out[0]);
        out[1] = mfma_bf16(w, h1[ks], out[1]);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) out[t][i] *= kNegLn2;
}

// Layer 1's bias plus its moment columns times the moments m (FP32, ascending
// moment index), for output feature o.
__device__ __forceinline__ float layer1_const(const MlpPacked* __restrict__ P, int o, const float* m)
{
    float a = P->b1[o];
#pragma unroll 8
    for (int q = 0; q < 2 * kRff; ++q) a = fmaf(P->inf.W1m[o][q], m[q], a);
    return a;
}

// ---------------------------------------------------------------------------
// k_mlp_infer: surrogate pair term for every particle of the listed blocks
// (256 particles each): surr[k][slot] (FP32) for k < d.  Wavefront w takes
// the tiles 4 w .. 4 w + 3 of a block, two at a time.
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ __launch_bounds__(256) void k_mlp_infer(const BlkItem* __restrict__ items, int n_items,
                                                   const SysDev* __restrict__ sys, int64_t P,
                                                   const T* __restrict__ Y, const float* __restrict__ mom,
                                                   const MlpPacked* __restrict__ W, float* __restrict__ surr)
{
    __shared__ InferLds L;
    __shared__ __align__(16) float c1s[kHid];
    load_infer(W, L);
    const int wave = threadIdx.x >> 6;
    const int l = threadIdx.x & 63;
    int cur_sys = -1;
    for (int itx = blockIdx.x; itx < n_items; itx += gridDim.x) {
        const BlkItem it = items[itx];
        const SysDev S = sys[it.sys];
        if (it.sys != cur_sys) {  // block-uniform
            __syncthreads();
            if (threadIdx.x < kHid) c1s[threadIdx.x] = layer1_const(W, threadIdx.x, mom + (int64_t)it.sys * (2 * kRff));
            cur_sys = it.sys;
        }
        __syncthreads();
#pragma unroll 1
        for (int tp = 0; tp < 2; ++tp) {
            const int i0 = it.blk * kBlk + (4 * wave + 2 * tp) * 16;
            if (i0 >= S.N) break;  // wave-uniform
            float yin[2][kMaxD] = {{0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int i = i0 + 16 * t + (l & 15);
#pragma unroll
                for (int k = 0; k < D; ++k) yin[t][k] = (i < S.N) ? (float)Y[k * P + S.off + i] : 0.0f;
            }
            f32x4 c1[2][4], out[2];
            bias_tiles(c1s, c1[0]);
            bias_tiles(c1s, c1[1]);
            mlp_infer_pair<D>(L, yin, c1, out);
            if (l < 16) {
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const int i = i0 + 16 * t + l;
                    if (i < S.N)
#pragma unroll
                        for (int k = 0; k < D; ++k) surr[(int64_t)k * P + S.off + i] = out[t][k];
                }
            }
        }
    }
}

// Inference on explicit raw rows U [n][d + 2K] -> out [n][d]: the same
// network, with layer 1's moment part computed per row (each lane for its
// sample and its 16 output features).
template <int D>
__global__ __launch_bounds__(256) void k_mlp_apply(const float* __restrict__ U, int64_t n,
                                                   const MlpPacked* __restrict__ W, float* __restrict__ out)
{
    __shared__ InferLds L;
    load_infer(W, L);
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    const int l = threadIdx.x & 63;
    const int g = l >> 4;
    constexpr int in = raw_in(D);
    for (int64_t r0 = ((int64_t)blockIdx.x * 4 + wave) * 32; r0 < n; r0 += (int64_t)gridDim.x * 128) {
        float yin[2][kMaxD] = {{0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
        f32x4 c1[2][4];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int64_t row = r0 + 16 * t + (l & 15);
            float m[2 * kRff];
#pragma unroll
            for (int q = 0; q < 2 * kRff; ++q) m[q] = row < n ? U[row * in + D + q] : 0.0f;
#pragma unroll
            for (int k = 0; k < D; ++k) yin[t][k] = row < n ? U[row * in + k] : 0.0f;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int i = 0; i < 4; ++i) c1[t][nt][i] = layer1_const(W, 16 * nt + 4 * g + i, m);
        }
        f32x4 o[2];
        mlp_infer_pair<D>(L, yin, c1, o);
        if (l < 16) {
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int64_t row = r0 + 16 * t + l;
                if (row < n)
#pragma unroll
                    for (int k = 0; k < D; ++k) out[row * D + k] = o[t][k];
            }
        }
    }
}

// Sampled training pairs of one system: u = [y_i, moments], t = exact pair term
// at particle i, for n draws of i (Philox tag 4, counter (q, 0, 1)).
template <typename T, int D>
__global__ void k_gather_samples(const SysDev* __restrict__ sys, int s, int64_t P, const T* __restrict__ Y,
                                 const double* __restrict__ pairsum, const float* __restrict__ mom, int64_t n,
                                 uint64_t seed, float* __restrict__ U, float* __restrict__ Tt)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const SysDev S = sys[s];
    const Block4 rb = philox4x64_10((uint64_t)q, 0ull, 1ull, 4ull << 32, seed, 0ull);
    const int64_t i = (int64_t)(rb.w[0] % (uint64_t)S.N);
    const int64_t slot = S.off + i;
    const int in = raw_in(D);
#pragma unroll
    for (int k = 0; k < D; ++k) {
        U[q * in + k] = (float)Y[k * P + slot];
        Tt[q * D + k] = (float)pairsum[k * P + slot];
    }
    for (int m = 0; m < 2 * kRff; ++m) U[q * in + D + m] = mom[(int64_t)s * (2 * kRff) + m];
}

// ---------------------------------------------------------------------------
// Training.  k_train_fwdbwd: 64 samples per block (16 per wavefront), drawn
// with replacement by Philox (tag 4) from the sample set; forward, loss and
// back-propagated deltas; activations and deltas stored feature-major
// ([feature][batch], BF16) for the weight-gradient kernel.
// ---------------------------------------------------------------------------
// Row `row` of minibatch `step`: a uniform draw (with replacement) from the
// sample set, Philox stream tag 4; or row itself for sequential batches.
__device__ __forceinline__ int64_t sample_index(int row, int64_t step, uint64_t seed, int64_t n, int sequential)
{
    if (sequential) return (int64_t)row % n;
    const Block4 rb = philox4x64_10((uint64_t)row, (uint64_t)step, 0ull, 4ull << 32, seed, 0ull);
    return (int64_t)(rb.w[0] % (uint64_t)n);
}

struct TrainBufs {
    __bf16* act[4];    // act[0]: inputs [64][B]; act[1..3]: SiLU outputs [64][B]
    __bf16* delta[4];  // delta[0..2]: dL/dz of hidden layers 1..3 [64][B]; delta[3]: dL/dy [16][B]
    float* loss_part;  // [B / 64]
};

__global__ __launch_bounds__(256) void k_train_fwdbwd(const MlpPacked* __restrict__ W, const float* __restrict__ U,
                                                      const float* __restrict__ Tg, int64_t n_samples, int d,
                                                      int B, uint64_t seed, int64_t step, int sequential,
                                                      TrainBufs tb)
{
    __shared__ __align__(16) __bf16 sW1[kHid * kStride];
    __shared__ __align__(16) __bf16 sW2[kHid * kStride];
    __shared__ __align__(16) __bf16 sW3[kHid * kStride];
    __shared__ __align__(16) __bf16 sW4[kOutPad * kStride];
    __shared__ __align__(16) __bf16 sW2t[kHid * kStride];
    __shared__ __align__(16) __bf16 sW3t[kHid * kStride];
    __shared__ __align__(16) __bf16 sW4t[kHid * kStrideT4];
    __shared__ float sb[3 * kHid + kOutPad];
    __shared__ __align__(16) __bf16 tiles[4][16 * kStride];
    __shared__ float lossw[4];
    load_fwd_weights(W, sW1, sW2, sW3, sW4, sb);
    {
        const int n64 = kHid * kStride * 2 / 16;
        const int n4 = kHid * kStrideT4 * 2 / 16;
        for (int q = threadIdx.x; q < n64; q += blockDim.x) {
            ((uint4*)sW2t)[q] = ((const uint4*)W->W2t)[q];
            ((uint4*)sW3t)[q] = ((const uint4*)W->W3t)[q];
        }
        for (int q = threadIdx.x; q < n4; q += blockDim.x) ((uint4*)sW4t)[q] = ((const uint4*)W->W4t)[q];
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    const int l = threadIdx.x & 63;
    const int in = raw_in(d);
    const int b0 = blockIdx.x * 64 + wave * 16;  // first batch row of this wavefront
    // this lane's sample (A layout row l % 16)
    const int brow = b0 + (l & 15);
    const int64_t sidx = sample_index(brow, step, seed, n_samples, sequential);
    bf16x8 a[2];
    build_input_row(U + sidx * in, d, a);
    // inputs, feature-major
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int i = 0; i < 8; ++i) tb.act[0][(int64_t)(ks * 32 + 8 * (l >> 4) + i) * B + brow] = a[ks][i];

    f32x4 z[3][4];
    bf16x8 act[3][2];
    f32x4 out;
    mlp_forward16(sW1, sW2, sW3, sW4, sb, a, tiles[wave], z, out, act);

    // dL/dy in D layout: rows = samples 4 (l/16) + r, column = output l % 16
    const int comp = l & 15;
    f32x4 dy;
    float lsum = 0.0f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = b0 + 4 * (l >> 4) + r;
        float g = 0.0f;
        if (comp < d) {
            const int64_t si = sample_index(row, step, seed, n_samples, sequential);
            const float res = out[r] - Tg[si * d + comp];
            lsum += res * res;
            g = 2.0f * res / (float)B;
        }
        dy[r] = g;
        tb.delta[3][(int64_t)comp * B + row] = (__bf16)g;
    }
    // activations of the hidden layers, feature-major, from the D-layout values
    // (recomputed SiLU of z, rounded to BF16 exactly as the forward pass fed them)
#pragma unroll
    for (int layer = 0; layer < 3; ++layer)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                tb.act[layer + 1][(int64_t)(nt * 16 + (l & 15)) * B + b0 + 4 * (l >> 4) + r] =
                    (__bf16)silu_f(z[layer][nt][r]);

    // back-propagation: delta_3 = (dy W4) * silu'(z3) ...
    bf16x8 ga[2];
    {
        // dy (16 x 16, D layout) -> A layout with K = 32 (outputs 16..31 zero)
        f32x4 v[1] = {dy};
        __bf16* tile = tiles[wave];
#pragma unroll
        for (int i = 0; i < 4; ++i) tile[(4 * (l >> 4) + i) * kStride + (l & 15)] = (__bf16)v[0][i];
#pragma unroll
        for (int i = 0; i < 4; ++i) tile[(4 * (l >> 4) + i) * kStride + 16 + (l & 15)] = (__bf16)0.0f;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        ga[0] = *(const bf16x8*)&tile[(l & 15) * kStride + 8 * (l >> 4)];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    f32x4 g[4];
    // layer 4 backward: K = 32 (padded outputs), B operand from W4t [in][out]
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        f32x4 c = {0.0f, 0.0f, 0.0f, 0.0f};
        const bf16x8 b = *(const bf16x8*)&sW4t[(nt * 16 + (l & 15)) * kStrideT4 + 8 * (l >> 4)];
        c = mfma_bf16(ga[0], b, c);
        g[nt] = c;
    }
    const __bf16* Wt[2] = {sW3t, sW2t};
#pragma unroll
    for (int layer = 2; layer >= 0; --layer) {
        // delta of hidden layer (layer+1) = g * silu'(z)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r) g[nt][r] *= silu_prime_f(z[layer][nt][r]);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                tb.delta[layer][(int64_t)(nt * 16 + (l & 15)) * B + b0 + 4 * (l >> 4) + r] = (__bf16)g[nt][r];
        if (layer == 0) break;
        d_to_a<4>(g, tiles[wave], ga);
        f32x4 nxt[4];
        dense_tiles<4>(Wt[2 - layer], ga, nxt);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) g[nt] = nxt[nt];
    }
    // loss partial of this block, fixed order
    float ls = lsum;
    for (int off = 32; off > 0; off >>= 1) ls += __shfl_down(ls, off, 64);
    if (l == 0) lossw[wave] = ls;
    __syncthreads();
    if (threadIdx.x == 0) tb.loss_part[blockIdx.x] = (lossw[0] + lossw[1]) + (lossw[2] + lossw[3]);
}

// Weight gradients: one wavefront per 16 x 16 tile of a layer's weight matrix,
// summing over the batch with K = 32 samples per MFMA (fixed order); the
// tiles of input-column block 0 also produce the bias gradients.
// Tiles: layer 1: 4 x 4, layers 2 and 3: 4 x 4, layer 4: 1 x 4  -> 52.
__global__ __launch_bounds__(64) void k_train_wgrad(TrainBufs tb, int d, int B, float* __restrict__ grad)
{
    int t = blockIdx.x;
    int layer, ot, it;
    if (t < 48) {
        layer = t / 16;
        ot = (t % 16) / 4;
        it = t % 4;
    } else {
        layer = 3;
        ot = 0;
        it = t - 48;
    }
    const int l = threadIdx.x & 63;
    const __bf16* dl = tb.delta[layer];  // [out][B]
    const __bf16* al = tb.act[layer];    // [in][B]
    const int nout = layer < 3 ? kHid : d;
    const int nin = layer == 0 ? mlp_in(d) : kHid;
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    f32x4 bacc = {0.0f, 0.0f, 0.0f, 0.0f};
    bf16x8 ones;
#pragma unroll
    for (int i = 0; i < 8; ++i) ones[i] = (__bf16)1.0f;
    const int orow = ot * 16 + (l & 15);
    const int icol = it * 16 + (l & 15);
    for (int k0 = 0; k0 < B; k0 += 32) {
        bf16x8 a, b;
        const int kk = k0 + 8 * (l >> 4);
        if (layer == 3 && orow >= kOutPad) {
#pragma unroll
            for (int i = 0; i < 8; ++i) a[i] = (__bf16)0.0f;
        } else {
            a = *(const bf16x8*)&dl[(int64_t)orow * B + kk];
        }
        b = *(const bf16x8*)&al[(int64_t)icol * B + kk];
        acc = mfma_bf16(a, b, acc);
        if (it == 0) bacc = mfma_bf16(a, ones, bacc);
    }
    const MlpOffsets o = mlp_offsets(d);
    const int64_t wo[4] = {o.W1, o.W2, o.W3, o.W4};
    const int64_t bo[4] = {o.b1, o.b2, o.b3, o.b4};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int orr = ot * 16 + 4 * (l >> 4) + r;  // D row = output feature
        const int ic = it * 16 + (l & 15);          // D column = input feature
        if (orr < nout && ic < nin) grad[wo[layer] + (int64_t)orr * nin + ic] = acc[r];
        if (it == 0 && (l & 15) == 0 && orr < nout) grad[bo[layer] + orr] = bacc[r];
    }
}

// Adam on the flat FP32 master weights (Kingma & Ba), bias-corrected.
__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const float gg = g[q];
    const float mm = b1 * m[q] + (1.0f - b1) * gg;
    const float vv = b2 * v[q] + (1.0f - b2) * gg * gg;
    m[q] = mm;
    v[q] = vv;
    w[q] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// The exact pair term has zero net force (odd kernel: sum_i K^i = 0).  The
// surrogate is projected onto that constraint: block sums of its outputs,
// then per-system means that k_update / k_surr_err subtract.
template <int D>
__global__ __launch_bounds__(kBlk) void k_surr_partial(const BlkItem* __restrict__ items,
                                                       const SysDev* __restrict__ sys, int64_t P,
                                                       const float* __restrict__ surr,
                                                       double* __restrict__ part /*[nblk_tot][kMaxD]*/)
{
    __shared__ double red[kBlk];
    const BlkItem it = items[blockIdx.x];
    const SysDev S = sys[it.sys];
    const int i = it.blk * kBlk + threadIdx.x;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double v = (i < S.N) ? (double)surr[k * P + S.off + i] : 0.0;
        const double t = block_sum(v, red);
        if (threadIdx.x == 0) part[(int64_t)(S.blk0 + it.blk) * kMaxD + k] = t;
    }
}

// grid (listed systems, d), kBlk threads
__global__ __launch_bounds__(kBlk) void k_surr_final(const int32_t* __restrict__ sys_list,
                                                     const SysDev* __restrict__ sys,
                                                     const double* __restrict__ part,
                                                     float* __restrict__ mean /*[n_sys][kMaxD]*/)
{
    __shared__ double red[kBlk];
    const int s = sys_list[blockIdx.x];
    const SysDev S = sys[s];
    const int k = blockIdx.y;
    const double t = sum_block_partials(part, S.blk0, S.nblk, kMaxD, k, red);
    if (threadIdx.x == 0) mean[(int64_t)s * kMaxD + k] = (float)(t / (double)S.N);
}

// Check statistics per update block (fixed-order block sums), for the listed
// blocks, with s = surrogate minus its system mean, p = exact pair term and
// q = s + r the prediction (r = the stored residual when res_read, else 0):
//   [0] sum |q - p|^2, [1] sum |p|^2, then per component k:
//   [2 + 2k] sum p_k s_k, [3 + 2k] sum s_k^2, and [2 + 2 kMaxD] sum |s - p|^2.
// With res_write the residuals p - s replace the stored ones (each thread
// reads its own slots before it writes them).
constexpr int kErrStats = 3 + 2 * kMaxD;

template <typename T, int D>
__global__ __launch_bounds__(kBlk) void k_surr_err(const BlkItem* __restrict__ items,
                                                   const SysDev* __restrict__ sys, int64_t P,
                                                   const double* __restrict__ pairsum,
                                                   const float* __restrict__ surr,
                                                   const float* __restrict__ surr_mean,
                                                   float* res, int res_read, int res_write,
                                                   double* __restrict__ err_part /*[nblk][kErrStats]*/)
{
    __shared__ double red[kBlk];
    const BlkItem it = items[blockIdx.x];
    const SysDev S = sys[it.sys];
    const int i = it.blk * kBlk + threadIdx.x;
    double e2 = 0.0, b2 = 0.0, r2 = 0.0, ps[kMaxD] = {0.0, 0.0, 0.0, 0.0}, ss[kMaxD] = {0.0, 0.0, 0.0, 0.0};
    if (i < S.N) {
        const int64_t slot = S.off + i;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double pair = pairsum[k * P + slot];
            const double sv = (double)surr[k * P + slot] - (double)surr_mean[(int64_t)it.sys * kMaxD + k];
            const double q = res_read ? sv + (double)res[k * P + slot] : sv;
            if (res_write) res[k * P + slot] = (float)(pair - sv);
            e2 += (q - pair) * (q - pair);
            r2 += (sv - pair) * (sv - pair);
            b2 += pair * pair;
            ps[k] = pair * sv;
            ss[k] = sv * sv;
        }
    }
    double* out = err_part + (int64_t)blockIdx.x * kErrStats;
    const double t0 = block_sum(e2, red);
    const double t1 = block_sum(b2, red);
    const double t2 = block_sum(r2, red);
    if (threadIdx.x == 0) {
        out[0] = t0;
        out[1] = t1;
        out[2 + 2 * kMaxD] = t2;
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double a = block_sum(ps[k], red);
        const double b = block_sum(ss[k], red);
        if (threadIdx.x == 0) {
            out[2 + 2 * k] = a;
            out[3 + 2 * k] = b;
        }
    }
}

}  // namespace ssm
