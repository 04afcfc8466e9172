/*
 * ssm_oracle.c -- plain FP64 CPU oracle of the split-step method (SSM),
 * arXiv:2105.09688, Section 2.2 scheme (2.3)-(2.4).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, by the smoke check and by
 * the CPU-baseline leg of the benchmark, never by the library.  It is
 * compiled with -ffp-contract=off and uses libm exp/log/sin/cos/sqrt.  Sums
 * run over j in ascending order.  The only parallelism is an OpenMP loop over
 * independent particles i, which does not change any result.
 */
#include "ssm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11).  The round multiplies words 0 and 2 by two      */
/* fixed odd constants, producing 128-bit products (hi, lo); the new state   */
/* is (hi(c2*M1) ^ x1 ^ k0, lo(c2*M1), hi(c0*M0) ^ x3 ^ k1, lo(c0*M0)).  The */
/* key is advanced by two Weyl constants between rounds.                     */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2E7470EE14C6C93ULL
#define PHILOX_M1 0xCA5A826395121157ULL
#define PHILOX_W0 0x9E3779B97F4A7C15ULL /* golden ratio */
#define PHILOX_W1 0xBB67AE8584CAA73BULL /* sqrt(3) - 1 */

static void mul128(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void ssmo_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mul128(PHILOX_M0, x0, &hi0, &lo0);
        mul128(PHILOX_M1, x2, &hi1, &lo1);
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static double word_to_unit(uint64_t w)
{
    /* 53 random bits, centred in their cell: strictly inside (0, 1) */
    return ((double)(w >> 11) + 0.5) * 0x1.0p-53;
}

void ssmo_normals4(uint64_t seed, uint32_t tag, uint64_t i, uint64_t n, uint64_t e, double z[4])
{
    const uint64_t ctr[4] = {i, n, e, (uint64_t)tag << 32};
    const uint64_t key[2] = {seed, 0};
    uint64_t w[4];
    ssmo_philox4x64_10(ctr, key, w);
    const double two_pi = 6.283185307179586476925286766559;
    for (int p = 0; p < 2; ++p) {
        double u1 = word_to_unit(w[2 * p]);
        double u2 = word_to_unit(w[2 * p + 1]);
        double rad = sqrt(-2.0 * log(u1));
        z[2 * p] = rad * cos(two_pi * u2);
        z[2 * p + 1] = rad * sin(two_pi * u2);
    }
}

/* Normal number q of the Brownian stream of particle i in ensemble e: the
 * stream is the concatenation of the four normals of blocks b = 0, 1, 2, ...
 * of stream tag 0, so normal q is component q % 4 of block q / 4. */
double ssmo_stream_normal(uint64_t seed, uint64_t i, uint64_t e, uint64_t q)
{
    double z[4];
    ssmo_normals4(seed, 0u, i, q >> 2, e, z);
    return z[q & 3];
}

void ssmo_brownian(uint64_t seed, int d, uint64_t i, uint64_t e, uint64_t n0, int64_t r, double h_fine,
                   double *dW)
{
    double zsum[SSMO_MAX_D] = {0, 0, 0, 0};
    const uint64_t q0 = n0 * (uint64_t)d;
    const uint64_t q1 = q0 + (uint64_t)r * (uint64_t)d;
    uint64_t cached = ~(uint64_t)0;
    double z[4] = {0, 0, 0, 0};
    for (uint64_t q = q0; q < q1; ++q) {
        if ((q >> 2) != cached) {
            cached = q >> 2;
            ssmo_normals4(seed, 0u, i, cached, e, z);
        }
        zsum[(q - q0) % (uint64_t)d] += z[q & 3];
    }
    const double sq = sqrt(h_fine);
    for (int k = 0; k < d; ++k) dW[k] = sq * zsum[k];
}

/* ------------------------------------------------------------------------ */
/* Implicit step (2.3), Lemma 4.1.                                          */
/*                                                                          */
/* For v(c, mu) = (rho - kappa m2) c - a |c|^2 c + lam xbar the equation    */
/* c = x + h v(c, mu) reads c (alpha + h a |c|^2) = w with                  */
/* alpha = 1 - h (rho - kappa m2) and w = x + h lam xbar.  For a >= 0 and   */
/* alpha > 0 the factor is positive, so c is a non-negative multiple of w:  */
/* c = (r / |w|) w where r >= 0 is the unique root of the strictly          */
/* increasing cubic p(r) = h a r^3 + alpha r - |w|, which lies in           */
/* [0, |w| / alpha].  The root is found by Newton's method, with a          */
/* bisection step whenever a Newton iterate leaves the current bracket.     */
/* ------------------------------------------------------------------------ */
int ssmo_implicit(int d, const double *x, double h, double v_rho, double v_a,
                  double v_kappa, double v_lam, const double *xbar, double m2,
                  int max_iter, double *y)
{
    if (d < 1 || d > SSMO_MAX_D || !(v_a >= 0.0)) return SSMO_ERR_INVALID;
    if (max_iter <= 0) max_iter = 64;
    const double alpha = 1.0 - h * (v_rho - v_kappa * m2);
    if (!(alpha > 0.0)) return SSMO_ERR_INVALID;

    double w[SSMO_MAX_D];
    double nw2 = 0.0;
    for (int k = 0; k < d; ++k) {
        w[k] = x[k] + h * v_lam * (xbar ? xbar[k] : 0.0);
        nw2 += w[k] * w[k];
    }
    const double nw = sqrt(nw2);
    if (nw == 0.0) {
        for (int k = 0; k < d; ++k) y[k] = 0.0;
        return 0;
    }
    const double ha = h * v_a;
    double r;
    int it = 0;
    if (ha == 0.0) {
        r = nw / alpha; /* linear v: c = w / (1 - h rho), Remark 4.3 */
    } else {
        double lo = 0.0, hi = nw / alpha;
        r = nw / (alpha + ha * nw * nw);
        int converged = 0;
        for (it = 1; it <= max_iter; ++it) {
            double p = ha * r * r * r + alpha * r - nw;
            if (p == 0.0) { converged = 1; break; }
            if (p > 0.0) hi = r; else lo = r;
            double dp = 3.0 * ha * r * r + alpha;
            double delta = p / dp;
            /* a Newton correction of a few ulp: the corrected iterate is the
             * root up to rounding (quadratic convergence) */
            if (fabs(delta) <= 0x1.0p-50 * r) { r -= delta; converged = 1; break; }
            double rn = r - delta;
            if (!(rn > lo && rn < hi)) rn = 0.5 * (lo + hi);
            r = rn;
            if (hi - lo <= 0x1.0p-52 * hi) { converged = 1; break; }
        }
        if (!converged) return SSMO_ERR_NEWTON;
    }
    const double scale = r / nw;
    for (int k = 0; k < d; ++k) y[k] = w[k] * scale;
    return it;
}

/* ------------------------------------------------------------------------ */
/* Measure terms of (2.4), evaluated at the empirical measure of Y*.        */
/* ------------------------------------------------------------------------ */
void ssmo_pair_sum(int d, int64_t N, const double *Y, double ell, double *K)
{
    const double inv2l2 = 1.0 / (2.0 * ell * ell);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double acc[SSMO_MAX_D] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t j = 0; j < N; ++j) {
            double diff[SSMO_MAX_D];
            double dist2 = 0.0;
            for (int k = 0; k < d; ++k) {
                diff[k] = Y[(int64_t)k * N + j] - Y[(int64_t)k * N + i];
                dist2 += diff[k] * diff[k];
            }
            double kern = exp(-dist2 * inv2l2);
            for (int k = 0; k < d; ++k) acc[k] += diff[k] * kern;
        }
        for (int k = 0; k < d; ++k) K[(int64_t)k * N + i] = acc[k] / (double)N;
    }
}

void ssmo_pair_sum_at(int d, int64_t N, const double *Y, double ell, int64_t n_idx,
                      const int64_t *idx, double *K)
{
    const double inv2l2 = 1.0 / (2.0 * ell * ell);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n_idx; ++q) {
        const int64_t i = idx[q];
        double acc[SSMO_MAX_D] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t j = 0; j < N; ++j) {
            double diff[SSMO_MAX_D];
            double dist2 = 0.0;
            for (int k = 0; k < d; ++k) {
                diff[k] = Y[(int64_t)k * N + j] - Y[(int64_t)k * N + i];
                dist2 += diff[k] * diff[k];
            }
            double kern = exp(-dist2 * inv2l2);
            for (int k = 0; k < d; ++k) acc[k] += diff[k] * kern;
        }
        for (int k = 0; k < d; ++k) K[(int64_t)k * n_idx + q] = acc[k] / (double)N;
    }
}

static void mean_of(int d, int64_t N, const double *X, double *mean)
{
    for (int k = 0; k < d; ++k) {
        double s = 0.0;
        for (int64_t j = 0; j < N; ++j) s += X[(int64_t)k * N + j];
        mean[k] = s / (double)N;
    }
}

void ssmo_drift(int d, int64_t N, const double *Y, double b_c0, double b_lam,
                double b_g, double b_ell, double *B)
{
    double ybar[SSMO_MAX_D];
    mean_of(d, N, Y, ybar);
    if (b_g != 0.0) {
        ssmo_pair_sum(d, N, Y, b_ell, B);
    } else {
        for (int64_t q = 0; q < (int64_t)d * N; ++q) B[q] = 0.0;
    }
    for (int k = 0; k < d; ++k)
        for (int64_t i = 0; i < N; ++i) {
            int64_t q = (int64_t)k * N + i;
            B[q] = b_c0 * Y[q] + b_lam * ybar[k] + b_g * B[q];
        }
}

/* ------------------------------------------------------------------------ */
/* One step of (2.3)-(2.4).                                                  */
/* ------------------------------------------------------------------------ */
static int steps_per_increment(double h, double h_fine, int64_t *r)
{
    double q = h / h_fine;
    double rq = nearbyint(q);
    if (!(rq >= 1.0) || fabs(q - rq) > 1e-9 * rq) return SSMO_ERR_INVALID;
    *r = (int64_t)rq;
    return SSMO_OK;
}

/* (2.3) for every particle: Y*_n^i = X_n^i + h v(t_n, Y*_n^i, mu^X_n). */
static int implicit_all(const ssmo_cfg *cfg, int64_t N, double h, const double *X, double *Y)
{
    const int d = cfg->d;
    double xbar[SSMO_MAX_D] = {0, 0, 0, 0};
    double m2 = 0.0;
    if (cfg->v_lam != 0.0) mean_of(d, N, X, xbar);
    if (cfg->v_kappa != 0.0) {
        for (int64_t j = 0; j < N; ++j) {
            double s = 0.0;
            for (int k = 0; k < d; ++k) s += X[(int64_t)k * N + j] * X[(int64_t)k * N + j];
            m2 += s;
        }
        m2 /= (double)N;
    }
    int status = SSMO_OK;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double xi[SSMO_MAX_D], yi[SSMO_MAX_D];
        for (int k = 0; k < d; ++k) xi[k] = X[(int64_t)k * N + i];
        int it = 0;
        if (cfg->v_componentwise) {
            /* v_k = (rho - kappa m2) y_k - a_k y_k^3 + lam xbar_k: one scalar cubic per component */
            for (int k = 0; k < d && it >= 0; ++k)
                it = ssmo_implicit(1, &xi[k], h, cfg->v_rho, cfg->v_ak[k], cfg->v_kappa, cfg->v_lam,
                                   &xbar[k], m2, cfg->newton_max_iter, &yi[k]);
        } else {
            it = ssmo_implicit(d, xi, h, cfg->v_rho, cfg->v_a, cfg->v_kappa, cfg->v_lam,
                               xbar, m2, cfg->newton_max_iter, yi);
        }
        if (it < 0) {
#pragma omp critical
            status = it;
        }
        for (int k = 0; k < d; ++k) Y[(int64_t)k * N + i] = yi[k];
    }
    return status;
}

/* (2.4) for particle i, component k, given its drift term b (the O(N^2)
 * part and b_c0 y + b_lam ybar already in it). */
static double update_one(const ssmo_cfg *cfg, int64_t N, double h, const double *Y, const double *ybar,
                         int64_t i, int k, double b, const double *dW)
{
    const int d = cfg->d;
    const int64_t q = (int64_t)k * N + i;
    /* the linear extension b_const + b_mat y + b_mean o ybar, terms in ascending l */
    b += cfg->b_const[k];
    for (int l = 0; l < d; ++l) b += cfg->b_mat[k * SSMO_MAX_D + l] * Y[(int64_t)l * N + i];
    b += cfg->b_mean[k] * ybar[k];
    double sig = cfg->s0[k] + cfg->s1[k] * Y[q] + cfg->s2[k] * ybar[k];
    return (Y[q] + h * b) + sig * dW[k];
}

int ssmo_step(const ssmo_cfg *cfg, int32_t ens, int64_t N, double h, int64_t n,
              double *X, double *Y_out)
{
    const int d = cfg->d;
    int64_t r;
    if (steps_per_increment(h, cfg->h_fine, &r) != SSMO_OK) return SSMO_ERR_INVALID;
    double *Y = (double *)malloc(sizeof(double) * (size_t)d * (size_t)N);
    double *B = (double *)malloc(sizeof(double) * (size_t)d * (size_t)N);
    if (!Y || !B) { free(Y); free(B); return SSMO_ERR_INVALID; }

    int status = implicit_all(cfg, N, h, X, Y);
    if (status != SSMO_OK) { free(Y); free(B); return status; }

    /* drift and diffusion at mu^Y_n */
    ssmo_drift(d, N, Y, cfg->b_c0, cfg->b_lam, cfg->b_g, cfg->b_ell, B);
    double ybar[SSMO_MAX_D];
    mean_of(d, N, Y, ybar);

    /* (2.4): X_{n+1}^i = Y*^i + b h + sigma dW */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double dW[SSMO_MAX_D];
        ssmo_brownian(cfg->seed, d, (uint64_t)i, (uint64_t)ens, (uint64_t)(n * r), r, cfg->h_fine, dW);
        for (int k = 0; k < d; ++k) X[(int64_t)k * N + i] = update_one(cfg, N, h, Y, ybar, i, k, B[(int64_t)k * N + i], dW);
    }
    for (int64_t q = 0; q < (int64_t)d * N; ++q)
        if (!isfinite(X[q])) status = SSMO_ERR_NONFINITE;
    if (Y_out) memcpy(Y_out, Y, sizeof(double) * (size_t)d * (size_t)N);
    free(Y);
    free(B);
    return status;
}

int ssmo_step_at(const ssmo_cfg *cfg, int32_t ens, int64_t N, double h, int64_t n, const double *X,
                 int64_t n_idx, const int64_t *idx, double *X_at)
{
    const int d = cfg->d;
    int64_t r;
    if (steps_per_increment(h, cfg->h_fine, &r) != SSMO_OK) return SSMO_ERR_INVALID;
    for (int64_t q = 0; q < n_idx; ++q)
        if (idx[q] < 0 || idx[q] >= N) return SSMO_ERR_INVALID;
    double *Y = (double *)malloc(sizeof(double) * (size_t)d * (size_t)N);
    double *K = (double *)malloc(sizeof(double) * (size_t)d * (size_t)(n_idx > 0 ? n_idx : 1));
    if (!Y || !K) { free(Y); free(K); return SSMO_ERR_INVALID; }
    int status = implicit_all(cfg, N, h, X, Y);
    if (status != SSMO_OK) { free(Y); free(K); return status; }
    double ybar[SSMO_MAX_D];
    mean_of(d, N, Y, ybar);
    if (cfg->b_g != 0.0) {
        ssmo_pair_sum_at(d, N, Y, cfg->b_ell, n_idx, idx, K);
    } else {
        for (int64_t q = 0; q < (int64_t)d * n_idx; ++q) K[q] = 0.0;
    }
    for (int64_t q = 0; q < n_idx; ++q) {
        const int64_t i = idx[q];
        double dW[SSMO_MAX_D];
        ssmo_brownian(cfg->seed, d, (uint64_t)i, (uint64_t)ens, (uint64_t)(n * r), r, cfg->h_fine, dW);
        for (int k = 0; k < d; ++k) {
            /* the drift as ssmo_drift forms it: b_c0 y + b_lam ybar + b_g (pair term) */
            const double b = cfg->b_c0 * Y[(int64_t)k * N + i] + cfg->b_lam * ybar[k] + cfg->b_g * K[(int64_t)k * n_idx + q];
            X_at[(int64_t)k * n_idx + q] = update_one(cfg, N, h, Y, ybar, i, k, b, dW);
            if (!isfinite(X_at[(int64_t)k * n_idx + q])) status = SSMO_ERR_NONFINITE;
        }
    }
    free(Y);
    free(K);
    return status;
}

void ssmo_init_state(const ssmo_cfg *cfg, int32_t ens, int64_t N, double *X)
{
    const int d = cfg->d;
    for (int64_t i = 0; i < N; ++i) {
        double z[4];
        ssmo_normals4(cfg->seed, 1u, (uint64_t)i, 0u, (uint64_t)ens, z);
        for (int k = 0; k < d; ++k) X[(int64_t)k * N + i] = cfg->x0_mean[k] + cfg->x0_std[k] * z[k];
    }
}

static int check_cfg(const ssmo_cfg *cfg)
{
    if (cfg->d < 1 || cfg->d > SSMO_MAX_D || cfg->n_sys < 1) return SSMO_ERR_INVALID;
    if (!(cfg->T > 0.0) || !(cfg->h_fine > 0.0) || !(cfg->v_a >= 0.0) || !(cfg->v_kappa >= 0.0))
        return SSMO_ERR_INVALID;
    for (int k = 0; k < cfg->d; ++k)
        if (!(cfg->v_ak[k] >= 0.0)) return SSMO_ERR_INVALID;
    if (cfg->b_g != 0.0 && !(cfg->b_ell > 0.0)) return SSMO_ERR_INVALID;
    for (int s = 0; s < cfg->n_sys; ++s) {
        double h = cfg->h[s];
        if (!(h > 0.0) || cfg->N[s] < 1) return SSMO_ERR_INVALID;
        double m = cfg->T / h;
        if (fabs(m - nearbyint(m)) > 1e-9 * m) return SSMO_ERR_INVALID;
        int64_t r;
        if (steps_per_increment(h, cfg->h_fine, &r) != SSMO_OK) return SSMO_ERR_INVALID;
        /* Theorem 2.6 / Lemma 4.1: 1 - h (2 L_v + 1) > 0, with L_v = v_rho */
        if (!cfg->allow_unstable_h && !(1.0 - h * (2.0 * cfg->v_rho + 1.0) > 0.0))
            return SSMO_ERR_INVALID;
        if (!(1.0 - h * cfg->v_rho > 0.0)) return SSMO_ERR_INVALID;
    }
    return SSMO_OK;
}

int ssmo_run(const ssmo_cfg *cfg, int64_t stop_after, double *X_out, int64_t *steps_out)
{
    int st = check_cfg(cfg);
    if (st != SSMO_OK) return st;
    int64_t off = 0;
    for (int s = 0; s < cfg->n_sys; ++s) {
        const int64_t N = cfg->N[s];
        const double h = cfg->h[s];
        const int64_t M = (int64_t)nearbyint(cfg->T / h);
        double *X = X_out + off;
        ssmo_init_state(cfg, cfg->ens[s], N, X);
        int64_t n = 0;
        for (; n < M; ++n) {
            if (stop_after > 0 && n >= stop_after) break;
            st = ssmo_step(cfg, cfg->ens[s], N, h, n, X, NULL);
            if (st != SSMO_OK) return st;
        }
        if (steps_out) steps_out[s] = n;
        off += (int64_t)cfg->d * N;
    }
    return SSMO_OK;
}

void ssmo_moments(int d, int64_t N, const double *X, double *mean, double *var)
{
    mean_of(d, N, X, mean);
    for (int k = 0; k < d; ++k) {
        double s = 0.0;
        for (int64_t j = 0; j < N; ++j) {
            double c = X[(int64_t)k * N + j] - mean[k];
            s += c * c;
        }
        var[k] = s / (double)N;
    }
}

/* ------------------------------------------------------------------------ */
/* Learned-surrogate support: random Fourier feature moments and an MLP.     */
/* Not part of the paper; plain definitions for checking the GPU kernels.   */
/* ------------------------------------------------------------------------ */
void ssmo_rff_omegas(uint64_t seed, int d, int K, double ell, double *omega)
{
    for (int k = 0; k < K; ++k) {
        double z[4];
        ssmo_normals4(seed, 3u, (uint64_t)k, 0u, 0u, z);
        for (int c = 0; c < d; ++c) omega[k * d + c] = z[c] / ell;
    }
}

void ssmo_rff_moments(int d, int64_t N, const double *Y, int K, const double *omega, double *m)
{
    for (int k = 0; k < K; ++k) {
        double sc = 0.0, ss = 0.0;
        for (int64_t j = 0; j < N; ++j) {
            double ph = 0.0;
            for (int c = 0; c < d; ++c) ph += omega[k * d + c] * Y[(int64_t)c * N + j];
            sc += cos(ph);
            ss += sin(ph);
        }
        m[k] = sc / (double)N;
        m[K + k] = ss / (double)N;
    }
}

int64_t ssmo_mlp_num_params(int in, int H, int out)
{
    return (int64_t)H * in + H + 2 * ((int64_t)H * H + H) + (int64_t)out * H + out;
}

static double silu(double z) { return z / (1.0 + exp(-z)); }

/* derivative of z / (1 + e^-z): s(z) (1 + z (1 - s(z))) with s the logistic function */
static double silu_prime(double z)
{
    double sg = 1.0 / (1.0 + exp(-z));
    return sg * (1.0 + z * (1.0 - sg));
}

/* y[o] = b[o] + sum_i W[o][i] x[i] */
static void dense(int nin, int nout, const double *W, const double *b, const double *x, double *y)
{
    for (int o = 0; o < nout; ++o) {
        double acc = b[o];
        for (int i = 0; i < nin; ++i) acc += W[(int64_t)o * nin + i] * x[i];
        y[o] = acc;
    }
}

typedef struct {
    const double *W[4];
    const double *b[4];
} mlp_view;

static mlp_view mlp_split(int in, int H, int out, const double *p)
{
    mlp_view v;
    v.W[0] = p; p += (int64_t)H * in;
    v.b[0] = p; p += H;
    v.W[1] = p; p += (int64_t)H * H;
    v.b[1] = p; p += H;
    v.W[2] = p; p += (int64_t)H * H;
    v.b[2] = p; p += H;
    v.W[3] = p; p += (int64_t)out * H;
    v.b[3] = p;
    (void)out;
    return v;
}

void ssmo_mlp_forward(int in, int H, int out, const double *params, int64_t B, const double *X,
                      double *Y)
{
    const mlp_view v = mlp_split(in, H, out, params);
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < B; ++b) {
        double z[256], a[256], a2[256];
        dense(in, H, v.W[0], v.b[0], X + b * in, z);
        for (int h = 0; h < H; ++h) a[h] = silu(z[h]);
        dense(H, H, v.W[1], v.b[1], a, z);
        for (int h = 0; h < H; ++h) a2[h] = silu(z[h]);
        dense(H, H, v.W[2], v.b[2], a2, z);
        for (int h = 0; h < H; ++h) a[h] = silu(z[h]);
        dense(H, out, v.W[3], v.b[3], a, Y + b * out);
    }
}

double ssmo_mlp_loss_grad(int in, int H, int out, const double *params, int64_t B,
                          const double *X, const double *T, double *grad)
{
    const mlp_view v = mlp_split(in, H, out, params);
    const int64_t P = ssmo_mlp_num_params(in, H, out);
    for (int64_t q = 0; q < P; ++q) grad[q] = 0.0;
    double *gW[4], *gb[4];
    {
        double *g = grad;
        gW[0] = g; g += (int64_t)H * in; gb[0] = g; g += H;
        gW[1] = g; g += (int64_t)H * H; gb[1] = g; g += H;
        gW[2] = g; g += (int64_t)H * H; gb[2] = g; g += H;
        gW[3] = g; g += (int64_t)out * H; gb[3] = g;
    }
    double loss = 0.0;
    /* sequential over samples: gradients accumulate in sample order */
    for (int64_t b = 0; b < B; ++b) {
        const double *x0 = X + b * in;
        double z1[256], a1[256], z2[256], a2[256], z3[256], a3[256], y[16];
        dense(in, H, v.W[0], v.b[0], x0, z1);
        for (int h = 0; h < H; ++h) a1[h] = silu(z1[h]);
        dense(H, H, v.W[1], v.b[1], a1, z2);
        for (int h = 0; h < H; ++h) a2[h] = silu(z2[h]);
        dense(H, H, v.W[2], v.b[2], a2, z3);
        for (int h = 0; h < H; ++h) a3[h] = silu(z3[h]);
        dense(H, out, v.W[3], v.b[3], a3, y);
        /* dL/dy */
        double gy[16];
        for (int o = 0; o < out; ++o) {
            double r = y[o] - T[b * out + o];
            loss += r * r;
            gy[o] = 2.0 * r / (double)B;
        }
        /* output layer */
        double g3[256], g2[256], g1[256];
        for (int o = 0; o < out; ++o) {
            gb[3][o] += gy[o];
            for (int h = 0; h < H; ++h) gW[3][(int64_t)o * H + h] += gy[o] * a3[h];
        }
        for (int h = 0; h < H; ++h) {
            double s = 0.0;
            for (int o = 0; o < out; ++o) s += v.W[3][(int64_t)o * H + h] * gy[o];
            g3[h] = s * silu_prime(z3[h]);
        }
        /* third hidden layer */
        for (int o = 0; o < H; ++o) {
            gb[2][o] += g3[o];
            for (int h = 0; h < H; ++h) gW[2][(int64_t)o * H + h] += g3[o] * a2[h];
        }
        for (int h = 0; h < H; ++h) {
            double s = 0.0;
            for (int o = 0; o < H; ++o) s += v.W[2][(int64_t)o * H + h] * g3[o];
            g2[h] = s * silu_prime(z2[h]);
        }
        /* second hidden layer */
        for (int o = 0; o < H; ++o) {
            gb[1][o] += g2[o];
            for (int h = 0; h < H; ++h) gW[1][(int64_t)o * H + h] += g2[o] * a1[h];
        }
        for (int h = 0; h < H; ++h) {
            double s = 0.0;
            for (int o = 0; o < H; ++o) s += v.W[1][(int64_t)o * H + h] * g2[o];
            g1[h] = s * silu_prime(z1[h]);
        }
        /* first layer */
        for (int o = 0; o < H; ++o) {
            gb[0][o] += g1[o];
            for (int i = 0; i < in; ++i) gW[0][(int64_t)o * in + i] += g1[o] * x0[i];
        }
    }
    return loss / (double)B;
}

int ssmo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void ssmo_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
