/*
 * gpmppi.h - C ABI of the MI355X (gfx950) GP-augmented chance-constrained MPPI
 * rollout library.
 *
 * Method: Trivedi et al., "Data-Driven Sampling Based Stochastic MPC for
 * Skid-Steer Mobile Robot Navigation" (arXiv 2411.03289).  One controller
 * iteration is Algorithm 1, Step 1: K sampled control sequences are rolled out
 * over T steps through the dynamic unicycle with a GP residual (Eqs. 1-3, 6),
 * the mean and covariance are propagated per sample (Eq. 10), the lane and
 * obstacle chance constraints are tightened by the propagated position
 * covariance (Eqs. 13-16), a stage cost built from Eqs. (11)-(12) is summed
 * (Eq. 5), and the nominal sequence is replaced by the exponentially weighted
 * average of the samples.
 *
 * Conventions for every entry point:
 *  - Functions return a gpmppi_status; GPMPPI_OK is 0, errors are negative.
 *    On error a message is available from gpmppi_last_error() (thread-local,
 *    valid until the next call on the same thread).
 *  - Host arrays (const double *, in init / set_gp) are read during the call
 *    only; the caller keeps ownership.
 *  - Device arrays (float *, uint32_t * with a _d suffix) are caller-owned
 *    device allocations on the context's device, e.g. torch tensors.  Calls
 *    that take a `stream` (a hipStream_t, NULL = the default stream) only
 *    enqueue work: results are ready when that stream has reached them.
 *  - All arguments are validated on the host before any device work is
 *    enqueued; an invalid argument enqueues nothing.
 *  - Results are deterministic: the same inputs and seed give bitwise
 *    identical outputs (fixed-order reductions, no floating-point atomics).
 *  - A context may be used from one host thread at a time; calls that share
 *    a context and overlap on different streams race on its work buffers.
 */
#ifndef GPMPPI_H
#define GPMPPI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GPMPPI_OK = 0,
    GPMPPI_E_INVALID = -1,      /* bad size, pointer or parameter value */
    GPMPPI_E_NOT_PD = -2,       /* K(Z,Z) + sn^2 I is not positive definite (no jitter is added) */
    GPMPPI_E_HIP = -3,          /* a HIP runtime call failed */
    GPMPPI_E_NOMEM = -4,        /* device allocation failed */
    GPMPPI_E_NONFINITE = -5,    /* a host input holds NaN or Inf */
    GPMPPI_E_UNSUPPORTED = -6   /* a size beyond the supported maximum (e.g. M > 1024) */
} gpmppi_status;

/* Arithmetic of the GP variance contraction k^T (K + sn^2 I)^-1 k, computed as
 * ||W k||^2 with W = L^-1 on the matrix cores.  Kernel vectors, the GP mean,
 * the dynamics, constraints and costs are FP32 in every form. */
typedef enum {
    GPMPPI_FP32 = 0,            /* FP32 operands, FP32 accumulation */
    GPMPPI_BF16 = 1,            /* BF16 W and k, FP32 accumulation */
    GPMPPI_BF16X3 = 2           /* hi+lo BF16 splits, three products, FP32 accumulation */
} gpmppi_precision;

typedef struct gpmppi_ctx gpmppi_ctx;   /* opaque; owns every device buffer it allocates */

/* One residual GP (Sec. III-A: one GP per velocity output; Sec. V-A: input
 * (v, w, v_cmd, w_cmd)).  Squared-exponential ARD covariance
 * k(a,b) = exp(2 log_sf) exp(-1/2 sum_d (a_d-b_d)^2 exp(-2 log_ell[d])),
 * observation noise variance exp(2 log_sn). */
typedef struct {
    int32_t M;                  /* training / inducing points, 1 <= M <= 1024 */
    const double *Z;            /* [M][4] row-major host array */
    const double *y;            /* [M] host array of residual targets */
    double log_ell[4];
    double log_sf;
    double log_sn;
} gpmppi_gp;

/* Circular obstacles (Sec. IV-C: obstacles are approximated by circles). */
typedef struct {
    int32_t n;                  /* 0 <= n <= 4096 */
    const double *xyr;          /* [n][3] (centre x, centre y, radius > 0), host; may be NULL if n == 0 */
} gpmppi_obstacles;

/* Lane centreline (Eq. 13): kind 0 = circle (cx, cy, R), kind 1 = closed
 * polyline through P vertices (the last vertex joins the first). */
typedef struct {
    int32_t kind;
    double cx, cy, R;           /* kind 0 */
    int32_t P;                  /* kind 1: 3 <= P <= 65536 */
    const double *pts;          /* kind 1: [P][2] host array */
    double half_width;          /* r in Eq. (13), > 0 */
} gpmppi_path;

/* Controller parameters (Alg. 1 inputs; Eqs. 8, 11, 12, 16). */
typedef struct {
    int32_t K;                  /* samples, >= 1 */
    int32_t T;                  /* horizon steps, 1 <= T <= 4096 */
    double dt;                  /* step length [s] */
    double tau_v, tau_w;        /* first-order lags of the nominal velocity model */
    double sig_v, sig_w;        /* Sigma_sim = diag(sig_v^2, sig_w^2), >= 0 */
    double u_min[2], u_max[2];  /* control box (Eq. 8), u_min < u_max */
    double lambda;              /* MPPI temperature, > 0 */
    double p_x;                 /* chance-constraint level (Eq. 7), 0 < p_x < 1 */
    double w_var, w_dev, w_lane, w_speed, w_obs;   /* stage-cost weights */
    double v_des;               /* desired speed of the speed term */
    double discount;            /* lane-exit discount base (0.9 in Eq. 11) */
    int32_t precision;          /* gpmppi_precision */
    int32_t problem_id;         /* Philox counter word 2 */
    /* goal terms of the avoidance cost (Eq. 12): w_goal |p_{k+1} - goal| every step, and w_term once
       when no step of the rollout comes within goal_tol of the goal (both >= 0; 0 disables) */
    double w_goal, w_term;
    double goal[2];
    double goal_tol;            /* > 0 */
    int32_t tighten;            /* 0: each sample's constraints use its own propagated Sigma_XY;
                                   1: Sigma_XY propagated once along the nominal sequence clip(U) with
                                   the GP mean and variance (Alg. 1 Step 2), shared by all samples */
} gpmppi_params;

/* Optional per-step outputs of a rollout, all SoA with the sample index
 * innermost.  Any pointer may be NULL (not written). */
typedef struct {
    float *x_d;                 /* [T+1][5][K] states (X, Y, theta, v, w), step 0 = x0 */
    float *sxy_d;               /* [T+1][3][K] (Sigma_XX, Sigma_XY, Sigma_YY) */
    float *gp_mean_d;           /* [T][2][K] GP means (v, w) of query k */
    float *gp_var_d;            /* [T][2][K] predictive GP variances */
    float *d_lane_d;            /* [T][K] distance to the centreline at step k+1 */
    float *lane_margin_d;       /* [T][K] r_bar - d_lane (lane exit iff < 0), Eq. (14) */
    float *obs_margin_d;        /* [T][K] min_j d_bar_j (collision iff <= 0; +inf without obstacles), Eq. (16) */
    float *u_d;                 /* [T][2][K] sampled, clipped controls */
} gpmppi_trace;

/* Creates a context on the current HIP device.  Copies every host array,
 * builds both GPs on the GPU in FP64 (Cholesky of K(Z,Z) + sn^2 I, alpha,
 * W = L^-1; Rasmussen & Williams Alg. 2.1) and packs them for the rollout.
 * Synchronises the device.  *out is set only on success. */
gpmppi_status gpmppi_init(const gpmppi_params *params, const gpmppi_gp gp[2],
                          const gpmppi_obstacles *obstacles, const gpmppi_path *path,
                          gpmppi_ctx **out);

/* Rebuilds both GPs (same M as at init) - once per GP update, off the hot path.  Synchronises. */
gpmppi_status gpmppi_set_gp(gpmppi_ctx *ctx, const gpmppi_gp gp[2]);

/* Terrain ensemble (Sec. III-A, Eq. 3): n_terr target sets on the context's
 * GP inputs and hyperparameters (one GP per terrain and output, as a batch GP
 * with shared inputs).  The rollout then uses mean sum_i w_i m_i and variance
 * sum_i w_i^2 C_i; with shared inputs and hyperparameters every C_i is the
 * same, so this is alpha_bar = sum_i w_i alpha_i and a variance factor
 * sum_i w_i^2.  y [n_terr][2][M] host (row i: terrain i; [o][M] per output),
 * w [n_terr] host, 1 <= n_terr <= 8.  Synchronises. */
gpmppi_status gpmppi_set_terrains(gpmppi_ctx *ctx, int32_t n_terr, const double *y, const double *w);

/* New ensemble weights for the terrains already set (e.g. from the weight
 * estimate of Eq. 4); cheap (no refactorisation).  w [n_terr] host.  Synchronises. */
gpmppi_status gpmppi_set_terrain_weights(gpmppi_ctx *ctx, const double *w);

/* Each terrain's GP means at n queries q = (v, w, v_cmd, w_cmd): the rows
 * F[h][i] of Eq. (4).  q_d [n][4] device; out_d [n][n_terr][2] device
 * (output o = 0 linear, 1 angular).  Needs terrains (gpmppi_set_terrains). */
gpmppi_status gpmppi_terrain_means(gpmppi_ctx *ctx, const float *q_d, int32_t n, float *out_d, void *stream);

/* Terrain-weight estimate (Eq. 4, Alg. 1 Step 3), host-only (needs no device):
 * minimises ||Yv - Fv w||^2 + ||Yw - Fw w||^2 + gamma ||w - w_prev||_1 subject to
 * 0 <= w_i <= 1 and sum_i w_i = 1.  Yv, Yw [H] measured residuals of the last H
 * steps; Fv, Fw [H][n] row-major, terrain i's GP mean at step h; w_prev, w_out
 * [n] host arrays; 1 <= n <= 8, H >= 1, gamma >= 0.  Exact pairwise descent:
 * every move minimises the convex piecewise-quadratic objective along
 * e_i - e_j in closed form; it stops when no move exceeds 1e-15. */
gpmppi_status gpmppi_terrain_weights(int32_t H, int32_t n, const double *Yv, const double *Yw, const double *Fv,
                                     const double *Fw, const double *w_prev, double gamma, double *w_out);

/* One MPPI iteration (Alg. 1, Step 1): rollout of K samples over T steps
 * from x0, then weights w^s = exp(-(S^s - min S)/lambda) / sum and
 * U'_k = sum_s w^s clip(U_k + eps_k^s).
 *   x0_d      [5] device, initial state
 *   U_d       [T][2] device, nominal controls
 *   seed      64-bit Philox key of the control noise (counter (k, s, problem_id, 0))
 *   U_out_d   [T][2] device, new controls; may alias U_d
 *   costs_d   [K] device, per-sample costs S^s
 *   weights_d [K] device, per-sample weights (may be NULL) */
gpmppi_status gpmppi_step(gpmppi_ctx *ctx, const float *x0_d, const float *U_d, uint64_t seed,
                          float *U_out_d, float *costs_d, float *weights_d, void *stream);

/* The rollout alone (noise, GP, dynamics, covariance, constraints,
 * costs), optionally writing the per-step trace.  trace may be NULL. */
gpmppi_status gpmppi_rollout(gpmppi_ctx *ctx, const float *x0_d, const float *U_d, uint64_t seed,
                             float *costs_d, const gpmppi_trace *trace, void *stream);

/* The weighting and control update alone for given costs:
 * regenerates the sampled controls from (U_d, seed).  U_out_d may alias U_d. */
gpmppi_status gpmppi_weights_update(gpmppi_ctx *ctx, const float *costs_d, const float *U_d,
                                    uint64_t seed, float *U_out_d, float *weights_d, void *stream);

/* Evaluates both GPs at n query points q = (v, w, v_cmd, w_cmd), with the same
 * device arithmetic and precision form as the rollout (Eq. 3, one terrain).
 *   q_d [n][4] device; mean_d [2][n], var_d [2][n] device (predictive variance). */
gpmppi_status gpmppi_gp_predict(gpmppi_ctx *ctx, const float *q_d, int32_t n,
                                float *mean_d, float *var_d, void *stream);

/* Closed loop (the receding-horizon loop of Alg. 1): applies U_d[0] to the synthetic
 * plant x+ = Euler(x, u) + dt * amplitude * sin(v w) on (v, w), writing x_out_d
 * (may alias x_d), and shifts U_d in place to [U_1 .. U_{T-1}, U_{T-1}]. */
gpmppi_status gpmppi_plant_shift(gpmppi_ctx *ctx, const float *x_d, float *x_out_d, float *U_d,
                                 double amplitude, void *stream);

/* n control steps of the closed loop, all on device: for t < n,
 * step(x, U, seed0 + t) -> U', plant(U'_0), shift.  x_d [5] and U_d [T][2] are
 * updated in place; x_hist_d [n+1][5] (may be NULL) receives the states, and
 * U0_hist_d [n][2] (may be NULL) the applied controls.  use_graph != 0
 * captures one control step in a HIP graph and replays it n times. */
gpmppi_status gpmppi_closed_loop(gpmppi_ctx *ctx, float *x_d, float *U_d, uint64_t seed0, int32_t n,
                                 double amplitude, float *x_hist_d, float *U0_hist_d,
                                 int32_t use_graph, void *stream);

/* ------------------------------------------------------------------ differentiation form
 * Gradient of the smoothed expected cost
 *     J(U, log_ell, log_sf) = (1/K) sum_s S~^s,
 * S~ being the rollout cost of gpmppi_rollout (Alg. 1 Step 1, Eqs. 1-3 and
 * 10-16, Eq. 5's sum) with the lane-exit indicator replaced by
 * sigmoid((d_lane - r_bar) / tau) and the collision indicator by
 * sigmoid(-min_j d_bar_j / tau) (tau in metres), with respect to the nominal
 * controls U, the log length-scales [2][4] and the log signal deviations [2] of
 * the two GPs.  The noise is fixed by the seed (common random numbers); the
 * derivative of clip(U + eps) is 1 strictly inside the box and 0 outside; the
 * hyperparameter derivative is total (through the kernel vectors, alpha and
 * (K(Z, Z) + sn^2 I)^-1).  The adjoint rollout stores the state every
 * checkpoint_every steps (in [1, T]) and recomputes each segment before
 * reversing it; results do not depend on checkpoint_every.
 * FP32 on the GPU, whatever the context's precision.  Needs M <= 512, no
 * terrain ensemble, no goal terms and no Step-2 tightening
 * (GPMPPI_E_UNSUPPORTED otherwise).
 * x0_d [5], U_d [T][2] device; outputs (device): J_d [1], dU_d [T][2],
 * dlog_ell_d [2][4], dlog_sf_d [2], costs_d [K] the smoothed per-sample costs
 * (may be NULL).  A workspace of about 8 T K Mpad bytes (the r = A^-1 k rows of
 * every sample and step) is allocated on first use and kept by the context
 * (GPMPPI_E_NOMEM if that fails).  Enqueued on stream. */
gpmppi_status gpmppi_grad(gpmppi_ctx *ctx, const float *x0_d, const float *U_d, uint64_t seed, double tau,
                          int32_t checkpoint_every, float *J_d, float *dU_d, float *dlog_ell_d, float *dlog_sf_d,
                          float *costs_d, void *stream);

/* The gradient's launch shape: split = 1 (the default) runs each 32-sample
 * block's two GP outputs on two workgroups that exchange, per step, their
 * output's mean and variance (forward) and their share of the GP inputs'
 * adjoint (backward), wherever the doubled grid fits the device at once
 * (K <= 4096 at M <= 512 on MI355X); 0 keeps one workgroup per block.  The
 * results do not depend on it (bit for bit).  Exchange waits are bounded as
 * for the rollout (gpmppi_set_exchange_spin); a block whose wait gives up is
 * recomputed by a repair launch and GPMPPI_FLAG_EXCHANGE_TIMEOUT is set. */
gpmppi_status gpmppi_set_grad_split(gpmppi_ctx *ctx, int32_t split);

/* Allocation-free gpmppi_grad, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same arguments, computation and results, with the
 * workspace taken from a fixed scratch array of GPMPPI_GRAD_SCRATCH_BYTES that
 * the library keeps on each GPU it runs on until the process ends, instead of
 * the context's own workspace.  Calls no allocating routine.  A problem whose
 * workspace exceeds the array (about 8 T K M_pad bytes plus per-sample
 * checkpoints) fails with GPMPPI_E_NOMEM and enqueues nothing.  Every call on
 * a GPU shares that GPU's array and leaves its contents behind (no part of it
 * needs to start at zero): calls that overlap on one GPU (other streams, other
 * threads) race and must be serialised by the caller. */
#define GPMPPI_GRAD_SCRATCH_BYTES (128u << 20)
gpmppi_status gpmppi_grad_noalloc(gpmppi_ctx *ctx, const float *x0_d, const float *U_d, uint64_t seed, double tau,
                                  int32_t checkpoint_every, float *J_d, float *dU_d, float *dlog_ell_d,
                                  float *dlog_sf_d, float *costs_d, void *stream);

/* ------------------------------------------------------------------ launch shapes
 * The rollout's launch shape, chosen per context (or batch) by measurement.
 * None of these changes what is computed; they change the grouping of the
 * variance contraction's partial sums, so results differ between shapes only
 * by FP32 rounding.  Defaults: the largest group count that fits LDS,
 * rotate = 1, 4 waves, no output split, one workgroup per compute unit per
 * 80 KB of LDS (at most 2), longest items first. */
typedef struct {
    int32_t groups;      /* sample groups of 32 lanes per workgroup: 1 or 2 (2 only where the k operand fits LDS) */
    int32_t rotate;      /* 1: each workgroup starts its walk over W at a block-dependent row-pair; 0: at pair 0 */
    int32_t wg_per_cu;   /* batches: persistent workgroups per compute unit, 1 or 2 (LDS permitting) */
    int32_t order;       /* batches: 0 = items longest first, 1 = problem order */
    int32_t waves;       /* wave64s per rollout workgroup: 4 or 8, or 12 for the wave-specialised
                          * rollout of the BF16 forms at M_pad = 1024 (contexts, groups = the largest
                          * that fits: eight waves stream W through the matrix cores while four
                          * generate the next kernel vectors on the VALU and carry the sample state,
                          * handing the k operand over column tile by column tile in LDS) */
    int32_t split;       /* contexts: 1 runs the two GP outputs of each 32-sample block on two workgroups
                          * that exchange means and variances every step (groups = 1, and only where the
                          * doubled grid fits the device at once; results equal those of split = 0);
                          * batches: 0 */
    double ms;           /* tune: mean rollout time of this shape in ms; ignored by set */
} gpmppi_tuning;

/* Autotuner: times every admissible shape (groups x rotate x waves x split) with HIP events on `stream`
 * (1 warm-up + reps rollouts each, reps in [1, 100], into internal scratch
 * costs; x0_d [5] and U_d [T][2] as for gpmppi_rollout), installs the fastest
 * and writes it, with its time, to *chosen (may be NULL).  Synchronises. */
gpmppi_status gpmppi_tune(gpmppi_ctx *ctx, const float *x0_d, const float *U_d, uint64_t seed, int32_t reps,
                          gpmppi_tuning *chosen, void *stream);
/* Output split: the number of polls each exchange wait makes before it gives
 * up (the wave-specialised rollout's hand-over waits take the same bound, see
 * GPMPPI_FLAG_PIPELINE_STALL).  A workgroup whose wait gives up (its partner is not running, for
 * instance because other work holds the device) abandons the exchange,
 * computes its sample block alone from step 0 by the unsplit rollout's code
 * (the same results bit for bit, at about twice that workgroup's time) and
 * sets GPMPPI_FLAG_EXCHANGE_TIMEOUT.  0 restores the default (2^18 polls,
 * about 0.3 s); a negative value makes every wait give up at once, so every
 * block of a split launch runs alone: a hook for tests of that path.  Takes
 * effect from the next launch. */
gpmppi_status gpmppi_set_exchange_spin(gpmppi_ctx *ctx, int32_t polls);
/* Installs a shape (wg_per_cu and order are ignored for a context). */
gpmppi_status gpmppi_set_tuning(gpmppi_ctx *ctx, const gpmppi_tuning *t);
gpmppi_status gpmppi_get_tuning(const gpmppi_ctx *ctx, gpmppi_tuning *t);

/* ------------------------------------------------------------------ batches
 * Many independent problems (uneven K, T, M, obstacle count and track) run
 * together: one persistent rollout launch whose workgroups take (problem,
 * sample block) items, longest first, from a device counter, then one update
 * launch with a workgroup per (problem, horizon step).  Results of a problem
 * do not depend on the schedule.  All problems share one precision form and
 * use per-sample tightening (tighten = 0). */
typedef struct gpmppi_batch gpmppi_batch;

/* Creates n problems on the current device, each exactly as gpmppi_init would
 * (arrays: params[n], gp[2n] (problem p: gp[2p], gp[2p+1]), obstacles[n],
 * paths[n]).  Synchronises. */
gpmppi_status gpmppi_batch_init(int32_t n, const gpmppi_params params[], const gpmppi_gp gp[],
                                const gpmppi_obstacles obstacles[], const gpmppi_path paths[],
                                gpmppi_batch **out);

/* Packed layouts of the batched device arrays: problem p owns the floats
 * U[U_off[p] .. U_off[p+1]) ([T_p][2]) and costs/weights [K_off[p] .. K_off[p+1]).
 * Writes n + 1 entries to each non-NULL array. */
gpmppi_status gpmppi_batch_layout(const gpmppi_batch *b, int64_t *U_off, int64_t *K_off);

/* One MPPI iteration of every problem (as gpmppi_step per problem, with
 * Philox counter word 2 = that problem's problem_id).  x0_d [n][5], U_d and
 * U_out_d packed controls (U_out_d may alias U_d), costs_d and weights_d
 * (may be NULL) packed per-sample arrays. */
gpmppi_status gpmppi_batch_step(gpmppi_batch *b, const float *x0_d, const float *U_d, uint64_t seed,
                                float *U_out_d, float *costs_d, float *weights_d, void *stream);

/* n_steps closed-loop steps of every problem, all on device: iteration keyed
 * by seed0 + t, plant step with U'_0, warm-start shift.  x_d [n][5] and U_d
 * (packed) are updated in place; x_hist_d [n_steps + 1][n][5] may be NULL.
 * use_graph != 0 captures one step in a HIP graph and replays it. */
gpmppi_status gpmppi_batch_closed_loop(gpmppi_batch *b, float *x_d, float *U_d, uint64_t seed0, int32_t n_steps,
                                       double amplitude, float *x_hist_d, int32_t use_graph, void *stream);

/* Batch autotuner: as gpmppi_tune over the batch's persistent rollout
 * (groups x rotate x wg_per_cu x order x waves), with x0_d [n][5] and packed U_d. */
gpmppi_status gpmppi_batch_tune(gpmppi_batch *b, const float *x0_d, const float *U_d, uint64_t seed, int32_t reps,
                                gpmppi_tuning *chosen, void *stream);
gpmppi_status gpmppi_batch_set_tuning(gpmppi_batch *b, const gpmppi_tuning *t);
gpmppi_status gpmppi_batch_get_tuning(const gpmppi_batch *b, gpmppi_tuning *t);

/* Frees the batch (NULL is accepted). */
void gpmppi_batch_destroy(gpmppi_batch *b);

/* Philox4x32-10 (Salmon et al., SC'11) raw output for n counters:
 * ctr_d [n][4] device (words), out_d [n][4] device; key = (seed lo, seed hi). */
gpmppi_status gpmppi_philox(uint64_t seed, const uint32_t *ctr_d, int32_t n, uint32_t *out_d,
                            void *stream);

/* Reads and clears the context's device status bits:
 *   GPMPPI_FLAG_NONFINITE         a weights/update call saw a non-finite cost;
 *   GPMPPI_FLAG_EXCHANGE_TIMEOUT  an exchange wait of an output-split rollout
 *                                 gave up and its workgroup computed its block
 *                                 alone (results unchanged, time lost);
 *   GPMPPI_FLAG_PIPELINE_STALL    a hand-over wait inside a wave-specialised
 *                                 rollout workgroup (waves = 12) gave up: that
 *                                 workgroup's costs are NaN.  With the default
 *                                 spin only a defect can cause it (the waits
 *                                 depend on nothing outside the workgroup);
 *                                 gpmppi_set_exchange_spin(ctx, -1) forces it.
 * Synchronises the device. */
#define GPMPPI_FLAG_NONFINITE 1u
#define GPMPPI_FLAG_EXCHANGE_TIMEOUT 2u
#define GPMPPI_FLAG_PIPELINE_STALL 4u
gpmppi_status gpmppi_status_flags(gpmppi_ctx *ctx, uint32_t *flags);

/* Derived scalars of a context: M_pad (M rounded up to a multiple of 64),
 * z = Phi^-1(p_x) (Eq. 16) and c = sqrt(chi2_2(p_x)) (Eq. 14). */
gpmppi_status gpmppi_info(const gpmppi_ctx *ctx, int32_t *M_pad, double *z_p, double *c_p);

/* Phi^-1(p), the standard normal quantile used to tighten obstacle margins
 * (Eq. 16); host-only, needs no device.  Returns NaN outside (0, 1). */
double gpmppi_norm_quantile(double p);

/* Frees every device buffer of the context (NULL is accepted). */
void gpmppi_destroy(gpmppi_ctx *ctx);

/* Message of the last error on the calling thread ("" if none). */
const char *gpmppi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GPMPPI_H */
