// ssm_device.hpp -- device helpers of libssm (gfx950): counter-based normals
// and the per-particle implicit solve.  Included by ssm.hip only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssm {

constexpr int kMaxD = 4;

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Each round multiplies
// words 0 and 2 by two fixed odd 64-bit constants into 128-bit products and
// mixes the high halves with words 1, 3 and the round key; the key advances
// by two Weyl increments per round.
// ---------------------------------------------------------------------------
struct Block4 {
    uint64_t w[4];
};

// The 128-bit product a b from four 32 x 32 + 64 multiply-adds
// (v_mad_u64_u32), both halves from the same partial products.  No sum
// overflows: (2^32 - 1)^2 + 2 (2^32 - 1) < 2^64.
__device__ __forceinline__ void mulhilo64(uint64_t a, uint64_t b, uint64_t* lo, uint64_t* hi)
{
    const uint64_t a0 = (uint32_t)a, a1 = a >> 32, b0 = (uint32_t)b, b1 = b >> 32;
    const uint64_t t = a0 * b0;
    const uint64_t u = a1 * b0 + (t >> 32);
    const uint64_t v = a0 * b1 + (uint32_t)u;
    const uint64_t w = a1 * b1 + (u >> 32);
    *hi = w + (v >> 32);
    *lo = (v << 32) | (uint32_t)t;
}

__device__ __forceinline__ Block4 philox4x64_10(uint64_t x0, uint64_t x1, uint64_t x2, uint64_t x3,
                                                uint64_t k0, uint64_t k1)
{
    constexpr uint64_t kMulA = 0xD2E7470EE14C6C93ull;
    constexpr uint64_t kMulB = 0xCA5A826395121157ull;
    constexpr uint64_t kWeylA = 0x9E3779B97F4A7C15ull;
    constexpr uint64_t kWeylB = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        uint64_t a_lo, a_hi, b_lo, b_hi;
        mulhilo64(kMulA, x0, &a_lo, &a_hi);
        mulhilo64(kMulB, x2, &b_lo, &b_hi);
        const uint64_t n0 = b_hi ^ x1 ^ k0;
        const uint64_t n2 = a_hi ^ x3 ^ k1;
        x0 = n0;
        x1 = b_lo;
        x2 = n2;
        x3 = a_lo;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    Block4 r;
    r.w[0] = x0;
    r.w[1] = x1;
    r.w[2] = x2;
    r.w[3] = x3;
    return r;
}

// 53 high bits of a word, centred in their cell: a double in (0, 1).
__device__ __forceinline__ double unit_open(uint64_t w)
{
    return ((double)(w >> 11) + 0.5) * 0x1.0p-53;
}

// log u for u in (0, 1) (the Box-Muller radius; unit_open's range): u = m 2^e
// with m in [sqrt(1/2), sqrt(2)); log m = 2 atanh(s), s = (m - 1) / (m + 1),
// |s| <= 0.1716, by the atanh series to s^23 (the first term left out is
// below 1e-20 relative); e ln 2 in two parts, the first with 33 significant
// bits so that e ln2_hi is exact.  No range tests: u is never 0, negative,
// subnormal or infinite here.  Worst case seen 1.30 ulp (the rounded quotient
// and the final sums), against 60-digit values on the CPU.
__device__ __forceinline__ double log_unit(double u)
{
    constexpr double inv_odd[11] = {0x1.5555555555555p-2, 0x1.999999999999ap-3, 0x1.2492492492492p-3,
                                    0x1.c71c71c71c71cp-4, 0x1.745d1745d1746p-4, 0x1.3b13b13b13b14p-4,
                                    0x1.1111111111111p-4, 0x1.e1e1e1e1e1e1ep-5, 0x1.af286bca1af28p-5,
                                    0x1.8618618618618p-5, 0x1.642c8590b2164p-5};  // 1/3, 1/5, ..., 1/23
    constexpr double ln2_hi = 0x1.62e42fef00000p-1, ln2_lo = 0x1.473de6af278edp-34;
    int e;
    double m = frexp(u, &e);  // m in [1/2, 1)
    if (m < 0x1.6a09e667f3bcdp-1) {
        m *= 2.0;
        e -= 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double s2 = s * s;
    double p = inv_odd[10];
#pragma unroll
    for (int k = 9; k >= 0; --k) p = fma(p, s2, inv_odd[k]);
    const double at = fma(s * s2, p, s);  // atanh(s)
    const double de = (double)e;
    return fma(de, ln2_hi, fma(de, ln2_lo, 2.0 * at));
}

// sin x and cos x for x in [0, 2 pi] (the Box-Muller angle): x = k pi/2 + r,
// k = rint(2x/pi) in 0..4, |r| <= pi/4, reduced by fused multiply-adds
// against pi/2 in three parts (159 bits); sin r by its Taylor series to r^19,
// cos r to r^18 (the first terms left out are below 1e-19 relative); the
// quadrant k mod 4 picks and signs the pair.  Worst case seen 1.19 ulp.
__device__ __forceinline__ void sincos_angle(double x, double* sn, double* cs)
{
    constexpr double sin_c[9] = {-0x1.5555555555555p-3, 0x1.1111111111111p-7, -0x1.a01a01a01a01ap-13,
                                 0x1.71de3a556c734p-19, -0x1.ae64567f544e4p-26, 0x1.6124613a86d09p-33,
                                 -0x1.ae7f3e733b81fp-41, 0x1.952c77030ad4ap-49, -0x1.2f49b46814157p-57};
    constexpr double cos_c[9] = {-0x1.0000000000000p-1, 0x1.5555555555555p-5, -0x1.6c16c16c16c17p-10,
                                 0x1.a01a01a01a01ap-16, -0x1.27e4fb7789f5cp-22, 0x1.1eed8eff8d898p-29,
                                 -0x1.93974a8c07c9dp-37, 0x1.ae7f3e733b81fp-45, -0x1.6827863b97d97p-53};
    constexpr double pio2_a = 0x1.921fb54442d18p+0, pio2_b = 0x1.1a62633145c07p-54, pio2_c = -0x1.f1976b7ed8fbcp-110;
    const double k = rint(x * 0x1.45f306dc9c883p-1);
    double r = fma(-k, pio2_a, x);
    r = fma(-k, pio2_b, r);
    r = fma(-k, pio2_c, r);
    const double r2 = r * r;
    double ps = sin_c[8], pc = cos_c[8];
#pragma unroll
    for (int j = 7; j >= 0; --j) {
        ps = fma(ps, r2, sin_c[j]);
        pc = fma(pc, r2, cos_c[j]);
    }
    const double sr = fma(r * r2, ps, r);
    const double cr = fma(r2, pc, 1.0);
    const int q = (int)k & 3;
    const double a = (q & 1) ? cr : sr;
    const double b = (q & 1) ? sr : cr;
    *sn = (q & 2) ? -a : a;
    *cs = ((q + 1) & 2) ? -b : b;
}

// The first `count` (1..4) standard normals of stream `tag` for particle i,
// grid index n, ensemble e (Box-Muller on word pairs (0,1) and (2,3)).
__device__ __forceinline__ void normals(uint64_t seed, uint32_t tag, uint64_t i, uint64_t n,
                                        uint64_t e, int count, double z[kMaxD])
{
    const Block4 b = philox4x64_10(i, n, e, (uint64_t)tag << 32, seed, 0ull);
    const double two_pi = 6.283185307179586476925286766559;
    // The angle 2 pi u is rounded to double first, as in the plain formula;
    // one reduction serves its sine and cosine.
    {
        const double rad = sqrt(-2.0 * log_unit(unit_open(b.w[0])));
        const double ang = two_pi * unit_open(b.w[1]);
        double sn, cs;
        sincos_angle(ang, &sn, &cs);
        z[0] = rad * cs;
        if (count >= 2) z[1] = rad * sn;
    }
    if (count >= 3) {
        const double rad = sqrt(-2.0 * log_unit(unit_open(b.w[2])));
        const double ang = two_pi * unit_open(b.w[3]);
        double sn, cs;
        sincos_angle(ang, &sn, &cs);
        z[2] = rad * cs;
        z[3] = rad * sn;
    }
}

// The same four normals with the transform in FP32, for the FP32 precision
// modes (whose state carries 24 bits): u from the same 53 bits, rounded once
// to float (both halves of the word enter, so a small u keeps its relative
// precision and log u stays accurate); the hardware log2, square root, sine
// and cosine (the last two take the angle in turns, so 2 pi u needs no
// multiplication).  About 12 instructions per pair against about 70 for the
// FP64 transform; the normals agree with the FP64 ones to about 1e-6.
__device__ __forceinline__ float unit_open_f32(uint64_t w)
{
    const float a = (float)(uint32_t)(w >> 32) * 0x1.0p-32f;
    const float b = (float)((uint32_t)w >> 11) + 0.5f;  // exact
    return fmaf(b, 0x1.0p-53f, a);                      // ((w >> 11) + 0.5) 2^-53, rounded once
}

__device__ __forceinline__ void normals4_f32(uint64_t seed, uint32_t tag, uint64_t i, uint64_t n, uint64_t e,
                                             float z[4])
{
    const Block4 b = philox4x64_10(i, n, e, (uint64_t)tag << 32, seed, 0ull);
    constexpr float kNeg2Ln2 = -1.3862943611198906f;  // -2 ln 2: -2 ln u = -2 ln 2 log2 u
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const float u0 = unit_open_f32(b.w[2 * p]), u1 = unit_open_f32(b.w[2 * p + 1]);
        const float rad = __builtin_amdgcn_sqrtf(kNeg2Ln2 * __builtin_amdgcn_logf(u0));
        z[2 * p] = rad * __builtin_amdgcn_cosf(u1);
        z[2 * p + 1] = rad * __builtin_amdgcn_sinf(u1);
    }
}

// ---------------------------------------------------------------------------
// Implicit step (2.3) for one particle, Lemma 4.1.  For
//   v(c) = (rho - kappa m2) c - a |c|^2 c + lam xbar
// the equation c = x + h v(c) is c (alpha + h a |c|^2) = w with
// alpha = 1 - h (rho - kappa m2), w = x + h lam xbar.  The factor is positive
// for alpha > 0, a >= 0, so c = (s / |w|) w with s >= 0 the root of the
// increasing convex cubic q(s) = h a s^3 + alpha s - |w|.
//
// Both |w| / alpha and cbrt(|w| / (h a)) are upper bounds of the root (q >= 0
// there); Newton started at their minimum decreases monotonically onto the
// root (q convex and increasing).  The bracket [lo, hi] is kept anyway: an
// iterate that leaves it (possible only through rounding) is replaced by the
// midpoint.  Iteration stops once a Newton correction is a few ulp.
// Returns the iteration count, -1 if max_iter is exhausted, or -2 (y = w) if
// w is not finite (a corrupted particle: there is no root to find).
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ int implicit_radial(const double w[D], double alpha, double ha,
                                               int max_iter, double y[D])
{
    double nw2 = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) nw2 = fma(w[k], w[k], nw2);
    if (!isfinite(nw2)) {
        // NaN or infinite coordinates (an overflowing |w|^2 of finite ones is
        // far outside any state the scheme reaches): passed through, flagged
#pragma unroll
        for (int k = 0; k < D; ++k) y[k] = w[k];
        return -2;
    }
    const double nw = sqrt(nw2);
    if (nw == 0.0) {
#pragma unroll
        for (int k = 0; k < D; ++k) y[k] = 0.0;
        return 0;
    }
    double s;
    int iters = 0;
    if (ha == 0.0) {
        s = nw / alpha;
    } else {
        double hi = fmin(nw / alpha, cbrt(nw / ha));
        double lo = 0.0;
        s = hi;
        bool done = false;
        for (iters = 1; iters <= max_iter; ++iters) {
            const double s2 = s * s;
            const double q = fma(ha * s2, s, fma(alpha, s, -nw));
            if (q == 0.0) {
                done = true;
                break;
            }
            if (q > 0.0) hi = s; else lo = s;
            const double dq = fma(3.0 * ha, s2, alpha);
            const double corr = q / dq;
            if (fabs(corr) <= 0x1.0p-50 * s) {
                s -= corr;
                done = true;
                break;
            }
            double sn = s - corr;
            if (!(sn > lo && sn < hi)) sn = 0.5 * (lo + hi);
            s = sn;
            if (hi - lo <= 0x1.0p-52 * hi) {
                done = true;
                break;
            }
        }
        if (!done) iters = -1;
    }
    const double scale = s / nw;
#pragma unroll
    for (int k = 0; k < D; ++k) y[k] = w[k] * scale;
    return iters;
}

}  // namespace ssm
