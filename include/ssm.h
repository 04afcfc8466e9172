/*
 * ssm.h -- C ABI of libssm, an MI355X (gfx950) implementation of the
 * split-step method (SSM) of Chen & dos Reis, arXiv:2105.09688, for
 * N-particle McKean-Vlasov systems.
 *
 * One time step of the scheme, Section 2.2, eqs. (2.3)-(2.4):
 *   Y*_n^i    = X_n^i + h v(t_n, Y*_n^i, mu^X_n)                       (2.3)
 *   X_{n+1}^i = Y*_n^i + b(t_n, Y*_n^i, mu^Y_n) h
 *               + sigma(t_n, Y*_n^i, mu^Y_n) dW_n^i                    (2.4)
 * with mu^X_n, mu^Y_n the empirical measures of all N particles (self
 * included).  Everything runs in HIP kernels on the device; the host only
 * validates, allocates and launches.
 *
 * Conventions for every entry point:
 *  - Returns ssm_status: SSM_OK (0) or a negative error.  No C++ exception
 *    crosses the ABI.  ssm_last_error() returns a thread-local message for the
 *    last failure on the calling thread.
 *  - "host" pointers are read or written during the call only; the caller
 *    keeps ownership.  "device" pointers are HIP device memory owned by the
 *    caller (for instance torch tensors); the library never frees them.
 *  - Arrays of particle data are component-major (SoA): element (k, i) of a
 *    [d][N] array is at k*N + i.
 *  - "stream" is a hipStream_t passed as void* (NULL = the null stream).
 *    Entry points that take device pointers are asynchronous on that stream;
 *    errors of the kernels themselves (sticky flags) are reported by
 *    ssm_sync()/ssm_run()/ssm_moments()/ssm_get_state() of a context.
 *  - A context is used by one host thread at a time.
 */
#ifndef SSM_H
#define SSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SSM_MAX_D 4

typedef enum {
    SSM_OK = 0,
    SSM_ERR_INVALID = -1,   /* bad argument or configuration */
    SSM_ERR_NEWTON = -2,    /* implicit solve did not converge within newton_max_iter */
    SSM_ERR_NONFINITE = -3, /* a particle became NaN/Inf */
    SSM_ERR_HIP = -4,       /* HIP runtime error */
    SSM_ERR_OOM = -5,       /* device allocation failed */
    SSM_ERR_STATE = -6      /* call not valid in the context's current state (e.g. past T) */
} ssm_status;

typedef enum {
    SSM_FP64 = 0,       /* state and pairwise sums in double precision */
    SSM_FP32 = 1,       /* state in float, pairwise sums accumulated plainly in float */
    SSM_FP32_KAHAN = 2  /* state in float, pairwise sums in float within a tile of
                           sources, compensated (Neumaier) across tiles */
} ssm_precision;

/*
 * Coefficients (the split v + b of Section 2; Remark 2.7 moves a linear term
 * between them through v_rho and b_c0):
 *   v(y, mu_X) = (v_rho - v_kappa m2(mu_X)) y - v_a |y|^2 y + v_lam mean(mu_X)
 *                (v_componentwise: -v_ak[k] y_k^3 in component k in place of
 *                -v_a |y|^2 y, so (2.3) is d scalar cubics)
 *   b(y, mu_Y) = b_c0 y + b_lam mean(mu_Y) + b_const + b_mat y + b_mean o mean(mu_Y)
 *                + b_g (1/N) sum_j (Y^j - y) exp(-|y - Y^j|^2 / (2 b_ell^2))
 *   sigma(y, mu_Y) = diag_k(s0[k] + s1[k] y_k + s2[k] mean_k(mu_Y))  (one Brownian
 *                    motion per component)
 * with m2(mu) = (1/N) sum_j |X^j|^2 (b_mat row-major [k][l], b_mean per component; the two-dimensional
 * Cucker-Smale model of Section 3.4.3 needs the component-wise cubic, the
 * constant and the coupling b_X = V).  Requirements: v_a >= 0, v_ak >= 0, v_kappa >= 0,
 * b_ell > 0 if b_g != 0, and for every system 1 - h v_rho > 0 (Lemma 4.1:
 * unique implicit root) and, unless allow_unstable_h, 1 - h (2 v_rho + 1) > 0
 * (the step-size condition of Theorem 2.6, L_v = v_rho).
 *
 * Systems: n_sys independent particle clouds advanced together.  System s has
 * N[s] particles, time step h[s] and ensemble id ens[s].  Brownian paths depend
 * on (ens, particle index) only, so systems of one ensemble with different h
 * see the same paths (Section 3 compares step sizes on the same paths).
 * Z(tag, i, b, e) denotes four standard normals: Philox4x64-10 (Salmon et al.,
 * SC'11) of counter (i, b, e, tag << 32) under key (seed, 0), each word w
 * mapped to u = ((w >> 11) + 0.5) 2^-53 and Box-Muller applied to (u0, u1) and
 * (u2, u3).  The Brownian stream of particle i is Z(0, i, 0, ens), Z(0, i, 1,
 * ens), ... concatenated (normal q = component q % 4 of block q / 4), and fine
 * step m, component k uses stream normal m d + k.  The increment over a step is
 * the sum of its r = h / h_fine fine increments:
 *   dW_{n,k}^i = sqrt(h_fine) sum_{m < r} (stream normal (n r + m) d + k).
 * X_0^i = x0_mean + x0_std * Z(1, i, 0, ens) (component k uses normal k).
 * The FP64 mode transforms the words in double precision; the FP32 modes take
 * the same u rounded once to float and the hardware log2, square root, sine
 * and cosine (normals within about 1e-6 of the double-precision ones, the
 * precision of their FP32 state); increments are summed in double.
 *
 * Time: every h[s] must divide T and be an integer multiple of h_fine.  Let
 * h_min = min h[s]; a "tick" advances time by h_min, and system s takes a step
 * on every tick t with t % (h[s]/h_min) == 0 (h[s]/h_min must divide the
 * largest such ratio).
 */
typedef struct {
    int32_t d;              /* state dimension, 1..SSM_MAX_D */
    int32_t n_sys;          /* number of systems, >= 1 */
    const int64_t *N;       /* host [n_sys]: particles per system, 1 .. 2^31-1 */
    const int32_t *ens;     /* host [n_sys]: ensemble id (Philox counter word 2) */
    const double *h;        /* host [n_sys]: time step per system */
    double T;               /* horizon */
    double h_fine;          /* Brownian grid step */
    uint64_t seed;          /* Philox key word 0 */
    int32_t precision;      /* ssm_precision */
    double v_rho, v_a, v_kappa, v_lam;
    double b_c0, b_lam, b_g, b_ell;
    double s0[SSM_MAX_D], s1[SSM_MAX_D], s2[SSM_MAX_D];
    double x0_mean[SSM_MAX_D], x0_std[SSM_MAX_D];
    int32_t newton_max_iter;   /* 0 -> 64 */
    int32_t allow_unstable_h;  /* nonzero: skip the Theorem 2.6 check (stability studies) */
    void *stream;              /* hipStream_t the context launches on; NULL -> a stream it owns */
    /* Tiling of the pairwise kernel; 0 = library default.  Results do not
     * depend on these beyond floating-point summation order. */
    int32_t targets_per_lane;  /* 1, 2, 4 or 8 (a target block is 64 x this; the symmetric scheme
                                  takes groups of 4 blocks, whose 256 x this x d j-side sums must
                                  fit 2048 floats (3072 at d = 3) or 1024 doubles (1536 at d = 3)).
                                  0: 4 for d = 1, 2 for d >= 2, halved while one work item would
                                  exceed the average work of a resident workgroup (small runs) and,
                                  in the symmetric scheme, until the group fits */
    int32_t sources_per_item;  /* sources per work item: one wavefront's source range (ordered
                                  scheme, >= 64) or a range against a 4-block target group
                                  (symmetric, rounded up to a multiple of 16) */
    int32_t pair_scheme;       /* 0: default (symmetric where the group fits, else ordered);
                                  1: every ordered pair (i, j) evaluated; 2: symmetric: each unordered
                                  pair evaluated once, +q to i and -q to j (the kernel is odd) */
    int32_t graphs;            /* nonzero: each tick replays a HIP graph captured once per tick
                                  phase (tick % (h_max/h_min)); not used while profiling or with
                                  the surrogate enabled */
    /* Coefficient extensions (zero: off), see "Coefficients" above. */
    int32_t v_componentwise;   /* nonzero: component-wise cubic -v_ak[k] y_k^3 (v_a unused) */
    int32_t kahan_span;        /* SSM_FP32_KAHAN only: 0 -> plain sums over 256 sources between
                                  compensated adds (default); 1 -> every pair term added by
                                  Neumaier's method (a precision-study variant: ordered scheme,
                                  about 2x the pair time at d = 3); other values are rejected */
    double v_ak[SSM_MAX_D];
    double b_const[SSM_MAX_D];
    double b_mat[SSM_MAX_D * SSM_MAX_D];
    double b_mean[SSM_MAX_D];
    /* Symmetric scheme: target groups per band of j-side rows.  0: all groups
     * at once while their rows (one per target group, d x P elements each) fit
     * 40 % of the free device memory, else bands of as many groups as fit
     * 16 GiB (or that 40 %, if less).
     * > 0: bands of this many groups (capped at the group count).  Banded, the
     * pair sums run band by band and after each band every particle adds the
     * band's rows it has to a running total (fixed order: runs stay bitwise
     * reproducible), so the j-side memory is one band's rows; the results
     * differ from unbanded ones by summation order only. */
    int32_t jside_band_groups;
    /* Persistent runs of small systems: one cooperative launch runs every
     * tick of an ssm_step call (up to 4096 ticks per launch).  Each workgroup owns 64 particles of one
     * system, stages the system's positions in LDS, sums the interaction
     * over every ordered pair of its particles, draws their increments and
     * updates them; the workgroups of a system then wait at that system's
     * barrier (one per tick, two when v depends on mu^X; a system steps on
     * its own ticks and draws its own increments).  Needs d x N (rounded up
     * to 4) elements of the precision within 32 KiB per system, the
     * compensated-sum default (kahan_span = 0) and co-resident workgroups for
     * every 64 particles.
     * Ticks with the surrogate enabled, with profiling or with graphs run the
     * multi-launch path.  Every barrier wait is bounded (4 s; the environment
     * variable SSM_PERSISTENT_WAIT_US, read by ssm_init, sets another limit
     * in microseconds): a wait that runs out ends the launch in every
     * workgroup, ssm_sync returns SSM_ERR_HIP and the context refuses
     * further steps.  Persistent launches of several contexts on different
     * streams run side by side only while their workgroups fit the GPU
     * together (one per compute unit for each); a launch whose workgroups
     * cannot all start waits on the others and is aborted if that takes
     * longer than the limit.  Results differ from the multi-launch path by
     * summation order only (ordered pairs, per-tile sums of the measures).
     *   0: on when eligible, the systems total at most one tile of 64
     *      particles per compute unit, a cost estimate of the two paths (from
     *      MI355X measurements) favours it (the multi-launch tick is bound by
     *      launch latency for small systems, while a persistent tile sums its
     *      particles' pairs on one compute unit), and no tiling of the
     *      multi-launch pair kernels (targets_per_lane, sources_per_item,
     *      pair_scheme, jside_band_groups) is given;  1: on whenever
     *      eligible (ssm_init fails if the configuration never is);  -1: off. */
    int32_t persistent;
} ssm_config;

typedef struct {
    int64_t tick;            /* ticks taken */
    int64_t ticks_total;     /* T / h_min */
    int32_t newton_max_seen; /* largest Newton iteration count seen so far */
    int32_t newton_failures; /* particles whose implicit solve failed (sticky) */
    int32_t nonfinite;       /* non-finite particles met by the implicit solve, which follows every
                                update and every ssm_set_state / ssm_state_refresh (sticky) */
    int32_t n_pair_items;    /* work items of the pairwise kernel per tick (phase 0): wavefronts in
                                the ordered scheme, workgroups in the symmetric scheme */
    int32_t targets_per_lane;
    int32_t sources_per_item;
    int32_t symmetric;       /* 1: symmetric pair scheme, 0: ordered pairs */
    int32_t jside_band_groups; /* target groups per band of j-side rows (0: not banded) */
    int64_t device_bytes;    /* device memory the context holds */
    /* Kernel timing (ssm_profile enabled): HIP events recorded on the context's
     * stream around the launches of the sampled ticks since the last ssm_profile. */
    int64_t pair_launches;   /* launches of the pairwise kernel */
    double pair_ms;          /* their summed duration, milliseconds */
    int64_t update_launches; /* launches of the per-particle update (+ implicit solve) kernels */
    double update_ms;
    /* learned surrogate (ssm_surrogate_enable) */
    int64_t surr_checks;         /* check ticks: exact pair term computed and compared */
    int64_t surr_ticks;          /* ticks whose update used the surrogate */
    int64_t surr_fallback_ticks; /* non-check ticks that used the exact term after a failed check */
    double surr_last_err;        /* relative error of the last check's prediction (see ssm_surrogate_enable) */
    double surr_max_err;         /* largest such error seen */
    double surr_last_raw_err;    /* relative error of the last check's bare network output s - mean s */
    double surr_gain[SSM_MAX_D]; /* per-component gain fitted at the last check */
    /* persistent runs of small systems (ssm_config.persistent) */
    int32_t persistent;          /* 1: eligible (ticks without surrogate, profiling or graphs use it) */
    int32_t persistent_tiles;    /* workgroups of a persistent launch (64 particles each) */
    int64_t persistent_launches; /* cooperative launches so far */
    int64_t persistent_ticks;    /* ticks they ran */
    int64_t surr_rechecks;       /* checks made during a fallback (ssm_surrogate_recheck) */
} ssm_info_t;

/* Training settings of ssm_mlp_train (Adam; zeros select the defaults in brackets). */
typedef struct {
    int64_t steps;   /* optimizer steps (>= 1) */
    int32_t batch;   /* samples per step, multiple of 64 */
    float lr;        /* learning rate (> 0) */
    float beta1;     /* [0.9] */
    float beta2;     /* [0.999] */
    float eps;       /* [1e-8] */
    uint64_t seed;   /* minibatch draws: Philox stream tag 4 */
} ssm_train_cfg;

typedef struct ssm_ctx ssm_ctx; /* opaque; owned by the library */

/* Create a context: validate cfg, allocate the device state, draw X_0
 * (Philox stream tag 1) and solve the implicit step (2.3) of the first step.
 * *out receives the context, or NULL on error.  Asynchronous on the stream. */
ssm_status ssm_init(const ssm_config *cfg, ssm_ctx **out);

/* Advance n_ticks ticks (each system steps when its step boundary falls on
 * the tick).  Asynchronous: enqueues kernels on the context's stream and
 * returns.  SSM_ERR_STATE if this would pass T. */
ssm_status ssm_step(ssm_ctx *ctx, int64_t n_ticks);

/* Advance every system to T and synchronize; reports sticky kernel errors. */
ssm_status ssm_run(ssm_ctx *ctx);

/* Wait for the context's stream; return SSM_ERR_NEWTON / SSM_ERR_NONFINITE if
 * a kernel flagged a particle since init (a NaN or infinite coordinate, from
 * the update (2.4) or written by the caller, is passed through unchanged
 * and flagged: the explicit part of the scheme is where the paper locates
 * the risk of corrupted particles; the run continues on the device). */
ssm_status ssm_sync(ssm_ctx *ctx);

/* Empirical moments of system sys (Section 3): mean[k] = (1/N) sum_i X_k^i and
 * var[k] = (1/N) sum_i (X_k^i - mean[k])^2, two passes in double precision on
 * the device.  mean, var: host [d].  Synchronizes. */
ssm_status ssm_moments(ssm_ctx *ctx, int32_t sys, double *mean, double *var);

/* Copy the state of system sys to host memory as double, [d][N].  which = 0:
 * X (current positions); which = 1: Y* = F_h(X), the solution of (2.3) for the
 * current X (valid once computed; the library keeps it one step ahead).
 * *step (may be NULL) receives the number of steps the system has taken.
 * Synchronizes. */
ssm_status ssm_get_state(ssm_ctx *ctx, int32_t sys, int32_t which, double *host, int64_t *step);

/* Overwrite X of system sys with host [d][N] (rounded to the storage
 * precision) and recompute Y* = F_h(X) of (2.3) for it (when v depends on
 * mu^X, from the moments of the new X).
 * step = -1 keeps the context's step count.  step >= 0 declares host to be
 * X after `step` steps of system sys: the context moves to tick
 * t = step * (h / h_min), which must be a step boundary of every system
 * (a multiple of h_max / h_min) and at most T / h_min, and every system's
 * step count becomes ceil(t / (h_s / h_min)).  The next step then draws the
 * Brownian increment dW_step of (2.4), so a state saved with ssm_get_state
 * (which returns the step count) continues on the same Brownian path in a
 * fresh context (Section 3 compares step sizes on the same paths).  Moving
 * the tick recomputes Y* of every system; in a context of several systems the
 * caller restores each of them, each with a step of the same tick.  The
 * surrogate's stored residuals and gains are dropped: ticks up to the next
 * check use the exact pair sums.  Synchronizes. */
ssm_status ssm_set_state(ssm_ctx *ctx, int32_t sys, const double *host, int64_t step);

/* Device layout of the particle state X of a context: one row of *P slots per
 * component (row k starts at element k * *P), system s at slots
 * [offsets[s], offsets[s] + N_s) of every row (offsets: host [n_sys], may be
 * NULL; each a multiple of 256), elements of *elt_bytes bytes (8: double in
 * FP64 mode, 4: float in the FP32 modes; may be NULL).  The other slots are
 * padding. */
ssm_status ssm_state_layout(ssm_ctx *ctx, int64_t *P, int64_t *offsets, int32_t *elt_bytes);

/* Make a caller-owned device buffer (for instance a torch tensor) the
 * context's state X, so the caller reads the particles in place.  bytes >=
 * d * P * elt_bytes (ssm_state_layout); 16-byte aligned.  The current state,
 * padding included, is copied into it and the context's own X is freed.  The
 * caller keeps the buffer alive until ssm_destroy (or until another buffer is
 * bound) and never frees it while the context may use it; the library never
 * frees it.  The kernels write X on the context's stream: read it after
 * ssm_sync or on that stream.  A caller that writes X (padding slots stay
 * finite) calls ssm_state_refresh before the next step, as the library keeps
 * Y* = F_h(X) of (2.3) one step ahead.  Synchronizes. */
ssm_status ssm_bind_state(ssm_ctx *ctx, void *dev, size_t bytes);

/* Recompute Y* = F_h(X) (2.3) and the block sums of X for system sys
 * (sys = -1: every system) after the caller changed X in a bound buffer (when
 * v depends on mu^X, from the moments of the changed X).  The surrogate's
 * stored residuals and gains are dropped, as in ssm_set_state.
 * Synchronizes. */
ssm_status ssm_state_refresh(ssm_ctx *ctx, int32_t sys);

/* Strong error between two contexts with identical system layouts:
 * per_sys[s] = sum_i |X_a^i - X_b^i|^2 over system s (host [n_sys], may be
 * NULL), *rmse = sqrt(sum over all systems / total particles).  This is the
 * epsilon_2 estimator of Section 3 when b holds the proxy solution.
 * Synchronizes both contexts. */
ssm_status ssm_rmse(ssm_ctx *a, ssm_ctx *b, double *per_sys, double *rmse);

/* Sum of squared differences between system sys_a of context a and system
 * sys_b of context b (same d and N): *out = sum_i |X_a^i - X_b^i|^2, double
 * precision on the device.  Lets a batch at several step sizes be compared
 * with a proxy-solution context of another layout (Section 3).  Synchronizes
 * both contexts. */
ssm_status ssm_sqdiff(ssm_ctx *a, int32_t sys_a, ssm_ctx *b, int32_t sys_b, double *out);

/* Per-kernel timing with HIP events on the context's stream: every = 0
 * disables it; every = k >= 1 records one event before and one after the
 * pairwise launch and the update launches of each tick with tick % k == 0
 * (k = 1: every tick).  Enabling resets the accumulated times.  The events
 * are for timing only (created without a system-scope fence; their times are
 * read after the stream is synchronized).  Each event pair costs about 3
 * microseconds of stream time, so a stride k > 1 keeps a timed run close to
 * an untimed one while still averaging over the whole run. */
ssm_status ssm_profile(ssm_ctx *ctx, int32_t every);

/* Counters, tiling and (if enabled) kernel times of a context.  Synchronizes. */
ssm_status ssm_info(ssm_ctx *ctx, ssm_info_t *out);

/* Destroy a context (waits for its stream first).  NULL is a no-op. */
void ssm_destroy(ssm_ctx *ctx);

/* Message of the last failure on this thread ("" if none). */
const char *ssm_last_error(void);

/* ---------------------------------------------------------------------------
 * Kernel-level entry points on caller-owned device memory.  They run the
 * same kernels the context uses, for one system, and exist so that a caller
 * (or a test) can drive a single stage of the step.
 * ------------------------------------------------------------------------- */

/* Pairwise part of b (eq. (2.4) drift, the O(N^2) term):
 *   K[k][i] = (1/N) sum_j (Y_k^j - Y_k^i) exp(-|Y^i - Y^j|^2 / (2 ell^2)),
 * j over all N particles.  Y: device [d][N], double for SSM_FP64 and float for
 * the FP32 modes.  K: device [d][N] double.  workspace: device buffer of at
 * least ssm_pair_workspace_bytes(d, N, precision) bytes (scratch for partial
 * sums; contents on entry ignored).  Synchronizes stream (the work list is
 * uploaded from host memory). */
ssm_status ssm_pair_sum(int32_t d, int64_t N, int32_t precision, const void *Y, double ell,
                        double *K, void *workspace, size_t workspace_bytes, void *stream);

/* Bytes of workspace ssm_pair_sum needs (deterministic function of its args). */
size_t ssm_pair_workspace_bytes(int32_t d, int64_t N, int32_t precision);

/* Implicit step (2.3) for N particles: Y^i = F_h(X^i), the unique c with
 * c = X^i + h v(c, mu_X) for the coefficient family above (Lemma 4.1).  X, Y:
 * device [d][N] double.  xbar: host [d] (mean of mu_X, used if v_lam != 0);
 * m2: second moment of mu_X (used if v_kappa != 0).  iters: device [N] int32
 * (Newton iterations, -1 on failure, -2 where X^i is not finite: Y^i = X^i),
 * may be NULL.  Asynchronous on stream. */
ssm_status ssm_implicit_solve(int32_t d, int64_t N, const double *X, double h, double v_rho,
                              double v_a, double v_kappa, double v_lam, const double *xbar,
                              double m2, int32_t max_iter, double *Y, int32_t *iters, void *stream);

/* Brownian increments over fine steps n0 .. n0 + r - 1 for particles
 * 0..N-1 of ensemble ens: dW[k][i] = sqrt(h_fine) sum_{m < r} (stream normal
 * (n0 + m) d + k of particle i).  dW: device [d][N] double.  Asynchronous on
 * stream. */
ssm_status ssm_brownian(int32_t d, int64_t N, uint64_t seed, int32_t ens, int64_t n0, int32_t r,
                        double h_fine, double *dW, void *stream);

/* Raw Philox4x64-10 blocks: out[4 q + w] = word w of the block of counter
 * (c0 + q, c1, c2, c3) under key (k0, k1), q = 0..count-1.  out: device
 * uint64 [4 count].  Asynchronous on stream. */
ssm_status ssm_philox_blocks(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                             uint64_t k1, int64_t count, uint64_t *out, void *stream);

/* ---------------------------------------------------------------------------
 * Learned surrogate of the pairwise term (an extension; not in the paper).
 *
 * Raw features of particle i: [Y*_i (d values), C_1..C_K, S_1..S_K] with
 * C_k = (1/N) sum_j cos(omega_k . Y*_j), S_k = (1/N) sum_j sin(omega_k . Y*_j),
 * K = 16, omega_k = Z(3, k, 0, 0)[0..d) / b_ell (so E cos(omega.(x - z)) is the
 * Gaussian kernel of the pairwise term).  Network input: [hi(y), lo(y),
 * C, S] (2d + 2K values) with hi(y) = bf16(y), lo(y) = bf16(y - hi(y)), so the
 * position passes the BF16 input layer with about 16 significant bits.
 * Network: input -> 64 -> 64 -> 64 -> d, SiLU after each hidden layer, BF16
 * weights and activations on the matrix cores with FP32 accumulation.
 * Parameters are FP32 "master" weights in the flat layout
 * W1[64][2d+2K] b1[64] W2[64][64] b2[64] W3[64][64] b3[64]
 * W4[d][64] b4[d] (row-major, [out][in]).  The output approximates
 * b_g (1/N) sum_j (Y^j - Y^i) exp(-|Y^i - Y^j|^2 / (2 b_ell^2)); inside a
 * step its mean over the system's particles is subtracted, since the exact
 * term has zero net force (odd kernel).
 * ------------------------------------------------------------------------- */

/* Number of parameters for state dimension d (0 if d is out of range). */
int64_t ssm_mlp_num_params(int32_t d);

/* Load master weights (host [n], n = ssm_mlp_num_params(d)) into a context
 * with a pairwise term.  Synchronizes. */
ssm_status ssm_surrogate_load(ssm_ctx *ctx, const float *master, int64_t n);

/* Prediction modes of ssm_surrogate_enable. */
#define SSM_SURR_GAIN 0     /* g_k (s_k - mean s_k) */
#define SSM_SURR_RESIDUAL 1 /* (s_k - mean s_k) + r_k, r from the last check */

/* Use the loaded surrogate in place of the O(N^2) pairwise sums.  Every
 * check_every-th tick (tick % check_every == 0) the exact sums p are computed
 * as well, the update uses them, and the relative error
 * sqrt(sum_i |q_i - p_i|^2 / sum_i |p_i|^2) of the prediction q over the
 * stepping systems decides whether the following ticks use the prediction
 * (error <= tol) or the exact sums (until the next check).  The network
 * output s enters with its mean over the system removed (the exact term has
 * zero net force), and
 *  - mode SSM_SURR_GAIN: q_k = g_k (s_k - mean s_k), where
 *    g_k = sum p_k s_k / sum s_k^2 is the least-squares gain fitted at the
 *    last check (1 before the first); the error compared with tol is that of
 *    the gain fitted at this check;
 *  - mode SSM_SURR_RESIDUAL: q_k^i = (s_k^i - mean s_k) + r_k^i, where
 *    r^i = p^i - (s^i - mean s) is particle i's residual stored at the last
 *    check (one float per particle and component); the error compared with
 *    tol is that of the residual carried over from the previous check, so it
 *    measures how far the network's error moved in check_every ticks.  The
 *    first check has no earlier residual and is compared without one.  Every
 *    system must step on check ticks: check_every a multiple of the ratio of
 *    the largest to the smallest step of the context.
 * Check ticks synchronize the stream.  check_every = 0 turns the surrogate
 * off.  Enabling (again) forgets the gain and the residuals. */
ssm_status ssm_surrogate_enable(ssm_ctx *ctx, int32_t check_every, double tol, int32_t mode);

/* Rechecks during a fallback (an extension; off by default).  With on = 1,
 * after a failed check every following tick on which all systems step is a
 * check as well: its exact sums are computed anyway (the fallback uses them),
 * so the prediction is compared with them at the cost of one inference, and
 * a passing recheck ends the fallback before the next scheduled check.  The
 * scheduled checks every check_every ticks stay, so no tick uses the
 * prediction more than check_every - 1 ticks after a passing check.  In
 * residual mode a recheck stores the residuals of its tick, so the error it
 * compares is that of one tick's drift.  Rechecks count in surr_checks and in
 * surr_rechecks, and not in surr_fallback_ticks; they synchronize the stream
 * like the other checks.  SSM_ERR_INVALID unless on is 0 or 1. */
ssm_status ssm_surrogate_recheck(ssm_ctx *ctx, int32_t on);

/* The surrogate's raw output at the current Y* of system sys, from the
 * kernels a surrogate tick runs: moments (host float [2K], may be NULL)
 * receives C_1..C_K, S_1..S_K of mu^Y of the system, and out (host double
 * [d][N]) the network output s^i of every particle, before its mean over
 * the system is removed.  Needs loaded weights (SSM_ERR_STATE otherwise).
 * Synchronizes. */
ssm_status ssm_surrogate_predict(ssm_ctx *ctx, int32_t sys, double *out, float *moments);

/* Training pairs from the current state of system sys: n draws (with
 * replacement, Philox stream tag 4 under seed) of a particle i, writing its
 * features to U (device float [n][d + 2K]) and its exact pairwise term to T
 * (device float [n][d]).  Synchronizes. */
ssm_status ssm_surrogate_samples(ssm_ctx *ctx, int32_t sys, int64_t n, uint64_t seed, float *U, float *T);

/* Network output for explicit raw rows: out (device float [n][d]) from U
 * (device float [n][d + 2K]) and master weights (device float).  Synchronizes stream. */
ssm_status ssm_mlp_forward(int32_t d, const float *master, const float *U, int64_t n, float *out,
                           void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * ssm_mlp_forward without any allocation.  The packed weights go to a device
 * buffer of the library (one per GPU, about 85 KB, held until the process
 * ends) in place of memory allocated for the call.  Same arguments and
 * results as ssm_mlp_forward (bitwise); d in 1..4 (the buffer holds a network
 * for d <= 4) and n in 1..2^31, else SSM_ERR_INVALID.  Asynchronous on stream:
 * it does not synchronize, so out is ready once the stream has reached the
 * call.  Every call on one GPU shares that GPU's buffer and it keeps the last
 * call's weights: calls whose kernels overlap on one GPU (other streams,
 * other threads) race; calls in order on one stream do not. */
ssm_status ssm_mlp_forward_noalloc(int32_t d, const float *master, const float *U, int64_t n, float *out,
                                   void *stream);

/* Loss L = (1/n) sum_rows |net(U_r) - T_r|^2 and dL/dparams (device float,
 * flat layout) for the n rows in order (n a multiple of 64), computed with
 * the training kernels.  *loss (host, may be NULL).  Synchronizes stream. */
ssm_status ssm_mlp_loss_grad(int32_t d, const float *master, const float *U, const float *T, int64_t n,
                             float *grad, double *loss, void *stream);

/* Adam training of the master weights (device float, updated in place) on
 * n_samples pairs (U, T) with minibatches drawn with replacement.
 * loss_hist (host float [steps], may be NULL) receives each step's minibatch
 * loss.  Synchronizes stream. */
ssm_status ssm_mlp_train(int32_t d, const float *U, const float *T, int64_t n_samples,
                         const ssm_train_cfg *cfg, float *master, float *loss_hist, void *stream);

/* Settings of ssm_surrogate_train. */
typedef struct {
    int32_t n_ens;       /* training systems: ensembles ens0 .. ens0 + n_ens - 1 (keep them
                            apart from the ensembles the network will be used on) */
    int32_t ens0;
    int64_t N;           /* particles per training system (0: N of the context's system 0) */
    int64_t n_samples;   /* training rows in total, a multiple of n_ens * snapshots */
    int32_t snapshots;   /* states per training run at which rows are drawn: the states after
                            k M / snapshots steps, k = 0 .. snapshots - 1, M = T / h */
    int32_t pad;
    uint64_t seed;       /* row draws and, without initial weights, the fresh weights */
    ssm_train_cfg train; /* Adam settings (ssm_mlp_train) */
} ssm_surrogate_train_cfg;

/* Train the surrogate for this context's workload and load it into the
 * context (an extension; not in the paper).  Runs the exact method on n_ens
 * systems that copy the context's system 0 (coefficients, h, T, precision,
 * seed; ensembles and N from cfg), draws n_samples / (n_ens snapshots) rows
 * (ssm_surrogate_samples) at each snapshot, and trains with ssm_mlp_train
 * from init (host [ssm_mlp_num_params(d)]) or, if init is NULL, from fresh
 * weights: each weight matrix uniform on +-sqrt(6 / (fan_in + fan_out)),
 * biases zero, parameter p from word p % 4 of the Philox block with counter
 * (p / 4, 0, 0, 5 * 2^32) under key (seed, 0).  master_out (host, may be NULL)
 * receives the trained weights, loss_hist (host float [train.steps], may be
 * NULL) the minibatch losses.  The rows live in device memory allocated for
 * the call (n_samples x (2d + 32) floats).  Synchronizes. */
ssm_status ssm_surrogate_train(ssm_ctx *ctx, const ssm_surrogate_train_cfg *cfg, const float *init,
                               float *master_out, float *loss_hist);

#ifdef __cplusplus
}
#endif
#endif /* SSM_H */
