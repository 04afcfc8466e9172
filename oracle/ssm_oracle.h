/*
 * ssm_oracle.h -- plain FP64 CPU oracle for the split-step method (SSM) of
 * Chen & dos Reis, "A flexible split-step scheme for solving McKean-Vlasov
 * stochastic differential equations" (arXiv:2105.09688).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the HIP library
 * against a slow, obviously correct implementation.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no code, header, table or helper with the HIP library.
 *
 * Everything here is double precision, evaluated in the order the paper
 * writes it, with plain ascending sums and no blocking or reordering.
 */
#ifndef SSM_ORACLE_H
#define SSM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SSMO_MAX_D 4

/* Coefficients of one McKean-Vlasov system, eq. (1.1)/(1.2), in the split
 * v + b of Section 2 (Remark 2.7 lets the caller move a linear term gamma*x
 * between v and b through v_rho and b_c0).
 *
 *   v(y, mu_X)   = (v_rho - v_kappa * m2(mu_X)) y - v_a |y|^2 y + v_lam * mean(mu_X)
 *   b(y, mu_Y)   = b_c0 y + b_lam mean(mu_Y)
 *                  + b_g * int (z - y) exp(-|y - z|^2 / (2 b_ell^2)) mu_Y(dz)
 *   sigma(y,mu_Y) = diag_k( s0[k] + s1[k] y_k + s2[k] mean_k(mu_Y) )
 *
 * m2(mu) = int |z|^2 mu(dz).  With mu the empirical measure of N particles
 * the integrals are (1/N) sums over all particles, self included (eq. (1.2)).
 */
typedef struct {
    int32_t d;              /* state dimension, 1..4 */
    int32_t n_sys;          /* number of independent particle systems */
    const int64_t *N;       /* [n_sys] particles per system */
    const int32_t *ens;     /* [n_sys] ensemble id: Brownian paths depend on (ens, i) only */
    const double *h;        /* [n_sys] time step of each system */
    double T;               /* horizon; T/h[s] must be an integer */
    double h_fine;          /* Brownian increments are sums over a grid of step h_fine */
    uint64_t seed;          /* Philox key word 0 */
    double v_rho, v_a, v_kappa, v_lam;
    double b_c0, b_lam, b_g, b_ell;
    double s0[SSMO_MAX_D], s1[SSMO_MAX_D], s2[SSMO_MAX_D];
    double x0_mean[SSMO_MAX_D], x0_std[SSMO_MAX_D];
    int32_t newton_max_iter;   /* 0 -> 64 */
    int32_t allow_unstable_h;  /* skip the Theorem 2.6 step-size check (stability studies) */
    /* Extensions for coefficient sets outside the radial/isotropic family
     * (the two-dimensional Cucker-Smale model of Section 3.4.3):
     *   v_componentwise: the cubic part of v is -v_ak[k] y_k^3 per component
     *                    (v_a unused), so (2.3) is d scalar cubics;
     *   b += b_const + b_mat y + b_mean o mean(mu_Y)  (b_mat row-major [k][l]). */
    int32_t v_componentwise;
    int32_t pad;
    double v_ak[SSMO_MAX_D];
    double b_const[SSMO_MAX_D];
    double b_mat[SSMO_MAX_D * SSMO_MAX_D];
    double b_mean[SSMO_MAX_D];
} ssmo_cfg;

/* Status codes */
#define SSMO_OK 0
#define SSMO_ERR_INVALID (-1)
#define SSMO_ERR_NEWTON (-2)
#define SSMO_ERR_NONFINITE (-3)

/* Philox4x64-10 block cipher of Salmon, Moraes, Dror & Shaw (SC'11):
 * ten rounds of the Philox S-box on a 4x64-bit counter under a 2x64-bit key. */
void ssmo_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Four independent standard normals for (tag, i, n, e):
 * counter = (i, n, e, tag << 32), key = (seed, 0); each 64-bit word w gives
 * u = ((w >> 11) + 0.5) 2^-53 in (0,1); Box-Muller on (u0,u1) and (u2,u3). */
void ssmo_normals4(uint64_t seed, uint32_t tag, uint64_t i, uint64_t n, uint64_t e, double z[4]);

/* Brownian stream of particle i, ensemble e: normal q is component q % 4 of
 * block q / 4 of stream tag 0 (ssmo_normals4(seed, 0, i, q / 4, e)). */
double ssmo_stream_normal(uint64_t seed, uint64_t i, uint64_t e, uint64_t q);

/* Increment over fine steps n0 .. n0 + r - 1 (grid step h_fine):
 * dW[k] = sqrt(h_fine) sum_{m < r} stream normal (n0 + m) d + k, summed in
 * ascending order. */
void ssmo_brownian(uint64_t seed, int d, uint64_t i, uint64_t e, uint64_t n0, int64_t r, double h_fine,
                   double *dW);

/* Implicit step (2.3) for one particle: the unique c with c = x + h v(c, mu_X)
 * (Lemma 4.1), by safeguarded Newton on the radial cubic.  x, y are [d].
 * Returns the number of Newton iterations, or SSMO_ERR_NEWTON / SSMO_ERR_INVALID. */
int ssmo_implicit(int d, const double *x, double h, double v_rho, double v_a,
                  double v_kappa, double v_lam, const double *xbar, double m2,
                  int max_iter, double *y);

/* The pairwise part at selected targets only: K[k][q] for i = idx[q]. */
void ssmo_pair_sum_at(int d, int64_t N, const double *Y, double ell, int64_t n_idx,
                      const int64_t *idx, double *K);

/* Interaction drift b at mu_Y for every particle (eq. (2.4) drift term).
 * Y, B are component-major [d][N]. */
void ssmo_drift(int d, int64_t N, const double *Y, double b_c0, double b_lam,
                double b_g, double b_ell, double *B);

/* Only the pairwise part: K[k][i] = (1/N) sum_j (Y_k^j - Y_k^i) exp(-|Y^i-Y^j|^2/(2 ell^2)). */
void ssmo_pair_sum(int d, int64_t N, const double *Y, double ell, double *K);

/* One SSM step (2.3)-(2.4) of one system in place.  X is [d][N].  n is the
 * step index (t_n = n h); the Brownian increment of particle i is
 * ssmo_brownian(seed, d, i, ens, n r, r, h_fine) with r = h / h_fine.
 * If Y_out is non-NULL it receives Y*_n.  Returns SSMO_OK or an error. */
int ssmo_step(const ssmo_cfg *cfg, int32_t ens, int64_t N, double h, int64_t n,
              double *X, double *Y_out);

/* The same step at a sample of particles only: X_at[k][q] = X_{n+1}^{idx[q]}
 * component k ([d][n_idx]) from X ([d][N], not modified).  Y* is solved for
 * every particle (the measures need the whole cloud) and the O(N^2) term
 * only at the sampled targets, with the same operations in the same order
 * as ssmo_step. */
int ssmo_step_at(const ssmo_cfg *cfg, int32_t ens, int64_t N, double h, int64_t n, const double *X,
                 int64_t n_idx, const int64_t *idx, double *X_at);

/* Initial condition X0^i_k = x0_mean[k] + x0_std[k] Z(1, i, 0, ens)_k. */
void ssmo_init_state(const ssmo_cfg *cfg, int32_t ens, int64_t N, double *X);

/* Run every system from t = 0 to T.  X_out holds the systems back to back,
 * each [d][N_s].  steps_out[s] receives the number of steps taken.
 * stop_after (if > 0) stops each system after that many steps (partial runs). */
int ssmo_run(const ssmo_cfg *cfg, int64_t stop_after, double *X_out, int64_t *steps_out);

/* mean_k and var_k = (1/N) sum (X_k - mean_k)^2, two passes, for [d][N]. */
void ssmo_moments(int d, int64_t N, const double *X, double *mean, double *var);

/* ---- learned-surrogate support (not in the paper; test infrastructure) ----
 * The oracle evaluates and differentiates a network at given weights; it
 * never trains one.  Trained weights are parity unpinned: they have no closed
 * form, and only the exact check at run time and the strong-error comparison
 * with the exact method assess a trained network.
 * Random Fourier feature frequencies: omega_k = Z(3, k, 0, 0)[0..d) / ell,
 * i.e. omega_k ~ N(0, I / ell^2), for which E cos(omega.(x - z)) =
 * exp(-|x - z|^2 / (2 ell^2)).  omega: [K][d]. */
void ssmo_rff_omegas(uint64_t seed, int d, int K, double ell, double *omega);

/* Moments of the empirical measure of Y ([d][N]) at the K frequencies:
 * m[k] = (1/N) sum_j cos(omega_k . Y^j), m[K + k] = (1/N) sum_j sin(omega_k . Y^j). */
void ssmo_rff_moments(int d, int64_t N, const double *Y, int K, const double *omega, double *m);

/* Multilayer perceptron in -> H -> H -> H -> out, SiLU (s(z) = z / (1 + e^-z))
 * after each hidden layer, linear output.  params (flat, row-major):
 * W1[H][in], b1[H], W2[H][H], b2[H], W3[H][H], b3[H], W4[out][H], b4[out].
 * X: [B][in], Y: [B][out]. */
int64_t ssmo_mlp_num_params(int in, int H, int out);
void ssmo_mlp_forward(int in, int H, int out, const double *params, int64_t B, const double *X,
                      double *Y);

/* Loss L = (1/B) sum_b sum_o (Y_bo - T_bo)^2 and its gradient dL/dparams
 * (same layout as params) by reverse-mode differentiation written out layer by
 * layer.  Returns L. */
double ssmo_mlp_loss_grad(int in, int H, int out, const double *params, int64_t B,
                          const double *X, const double *T, double *grad);

/* Threads OpenMP will use (1 when built without OpenMP). */
int ssmo_num_threads(void);
void ssmo_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif /* SSM_ORACLE_H */
