/*
 * hawkes.h -- C ABI of the MI355X (gfx950) library for the spatiotemporal
 * Hawkes log-likelihood with per-event rates, its gradient, its Hessian
 * diagonal, and a Hamiltonian Monte Carlo step on the log-rates
 * (Holbrook, Ji & Suchard, arXiv 2103.03348).
 *
 * Model (Sec. 2.1, D = 2).  Events (x_n, t_n), n = 1..N; window [T0, T1] with
 * T1 = max_n t_n; hyperparameters (mu0, tau_x, tau_t, theta0, omega, h); rates
 * theta_n >= 0.
 *   lambda_i = mu0 (2 pi)^{-3/2} tau_x^{-2} tau_t^{-1} sum_{j != i} exp(-r_ij^2/(2 tau_x^2) - dt_ij^2/(2 tau_t^2))
 *            + theta0 omega (2 pi h^2)^{-1} sum_{t_j < t_i} theta_j exp(-omega dt_ij - r_ij^2/(2 h^2))
 *   Lambda   = mu0 sum_n [Phi((T1-t_n)/tau_t) - Phi((T0-t_n)/tau_t)]
 *            + theta0 sum_n theta_n (1 - exp(-omega (T1 - t_n)))          (App. A)
 *   loglik   = sum_i log lambda_i - Lambda                                  (Eq. 1)
 *   d loglik/d theta_j = sum_{t_i > t_j} c_e E_ij / lambda_i - theta0 (1 - exp(-omega (T1 - t_j)))  (Eq. 4)
 *   -d2 loglik/d theta_j^2 = sum_{t_i > t_j} (c_e E_ij / lambda_i)^2                              (Eq. 5)
 * The paper's background is spatial only; the Gaussian-in-time factor is this
 * library's extension.  Its integral is the exact integral of the stated
 * background.  The self-exclusion indicator is j != i; the excitation is
 * strictly causal (events tied in time do not excite each other).
 *
 * Conventions for every call below:
 *  - d_* arguments are DEVICE pointers (any allocator, e.g. PyTorch's caching
 *    allocator); the caller owns them.  Plain pointers without d_ are HOST.
 *  - Every call is ordered on the HIP stream `stream` and returns without
 *    synchronising, except hawkes_plan_create and hawkes_plan_status.
 *  - Inputs and outputs are in the CALLER's event order; the library sorts by
 *    time internally (stable: ties keep the caller's order).
 *  - Return value: argument errors are detected on the host and returned at
 *    once, with nothing enqueued.  Data-dependent conditions found on the
 *    device (a zero intensity, a non-finite value) are recorded in a sticky
 *    status word that hawkes_plan_status returns and clears.
 *  - A plan is not thread-safe; calls on one plan must be ordered by the
 *    caller (one stream, or explicit events).  Separate plans are independent.
 *  - Precision: inputs and outputs are FP64.  The O(N^2) pair terms are FP32
 *    (their exponents formed in FP64 and rounded once where that decides the
 *    accuracy); the sums that build lambda accumulate every term in FP64, the
 *    derivative moments in FP32 per 64-term chunk and FP64 beyond.
 *    Log-intensities, the integral term, the final reductions (in a fixed
 *    order, so results are bit-reproducible) and the HMC energy run in FP64.
 */
#ifndef HAWKES_H_
#define HAWKES_H_

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hawkes_plan_s *hawkes_plan;

typedef enum {
    HAWKES_OK = 0,
    HAWKES_E_INVALID = 1,        /* bad argument: n < 1, NULL required pointer, non-positive
                                    tau_x/tau_t/omega/h, negative mu0/theta0, t_start > min t,
                                    non-finite t/x/y, or (device-detected) a negative or
                                    non-finite theta                                          */
    HAWKES_E_ZERO_INTENSITY = 2, /* some lambda_i == 0 (e.g. a single event): loglik = -inf   */
    HAWKES_E_NONFINITE = 3,      /* a NaN/Inf appeared in a device result                      */
    HAWKES_E_DEVICE = 4,         /* a HIP runtime call failed                                  */
    HAWKES_E_NOMEM = 5,          /* device allocation failed                                   */
    HAWKES_E_UNSUPPORTED = 6,    /* the call needs state that is not set (e.g. no subset)     */
    HAWKES_E_STALE = 7,          /* the plan's intensities are not those the call refers to
                                    (see hawkes_grad_theta_from_last); nothing was enqueued   */
    HAWKES_E_CAPACITY = 8        /* a size exceeds the fixed capacity of an allocation-free
                                    entry point; nothing was enqueued                         */
} hawkes_status;

/* Hyperparameters, in the order (mu0, tau_x, tau_t, theta0, omega, h) used for
 * the 6-vectors d_grad_hyper / d_negH_hyper below.  mu0 and theta0 are the
 * background and self-excitatory weights; tau_x, tau_t the background space and
 * time lengthscales; 1/omega the excitation time lengthscale; h its spatial
 * lengthscale (Sec. 2.1). */
typedef struct {
    double mu0, tau_x, tau_t, theta0, omega, h;
} hawkes_hyper;

/* Build a plan for one event set (Sec. 2.1's data (x_n, t_n)).
 *   n        number of events, >= 1
 *   d_t      [n] event times (device, FP64)
 *   d_xy     [n][2] event locations, row-major x0 y0 x1 y1 ... (device, FP64)
 *   t_start  window start T0 (the paper uses 0); must be <= min t
 * Sorts the events by time on the device, stores the locations in FP64
 * relative to the bounding-box centre, builds the tile tables and allocates
 * all scratch.  Synchronises `stream`.
 * On success *out owns device memory until hawkes_plan_destroy. */
hawkes_status hawkes_plan_create(hawkes_plan *out, int64_t n, const double *d_t, const double *d_xy,
                                 double t_start, hipStream_t stream);

/* Free a plan and everything it owns.  Synchronises the device first. */
hawkes_status hawkes_plan_destroy(hawkes_plan p);

/* Number of events of the plan, or -1 for NULL. */
int64_t hawkes_plan_size(hawkes_plan p);

/* Core evaluation (Eq. 1, Eq. 4, Eq. 5 and the hyperparameter derivatives).
 *   d_theta       [n] rates theta_n >= 0, caller order (device, FP64)
 *   d_loglik      [1] loglik (Eq. 1)                           -- may be NULL
 *   d_grad_theta  [n] d loglik / d theta_j (Eq. 4)            -- may be NULL
 *   d_grad_hyper  [6] d loglik / d (mu0,tau_x,tau_t,theta0,omega,h) -- may be NULL
 *   d_negH_theta  [n] -d2 loglik / d theta_j^2 (Eq. 5)        -- may be NULL
 *   d_negH_hyper  [6] -d2 loglik / d p^2 for the six hyperparameters -- may be NULL
 * One row pass over the causal pairs always runs (it gives lambda); a column
 * pass runs iff d_grad_theta or d_negH_theta is non-NULL.  The pair terms are
 * FP32; an event whose intensity from them falls below (c_b + c_e) n 2^-96
 * (all its terms near or below FP32's range: an event far from every other
 * one) has its lambda_i and derivative sums recomputed from the definitions in
 * FP64, so lambda_i keeps FP64's range.  When some lambda_i is zero in FP64,
 * loglik is -inf and the sticky status becomes HAWKES_E_ZERO_INTENSITY. */
hawkes_status hawkes_eval(hawkes_plan p, const hawkes_hyper *hyper, const double *d_theta,
                          double *d_loglik, double *d_grad_theta, double *d_grad_hyper,
                          double *d_negH_theta, double *d_negH_hyper, hipStream_t stream);

/* Thin wrappers of hawkes_eval (same argument meaning). */
hawkes_status hawkes_loglik(hawkes_plan p, const hawkes_hyper *hyper, const double *d_theta,
                            double *d_loglik, hipStream_t stream);
hawkes_status hawkes_grad(hawkes_plan p, const hawkes_hyper *hyper, const double *d_theta,
                          double *d_loglik, double *d_grad_theta, double *d_grad_hyper,
                          hipStream_t stream);
hawkes_status hawkes_hessdiag(hawkes_plan p, const hawkes_hyper *hyper, const double *d_theta,
                              double *d_negH_theta, double *d_negH_hyper, hipStream_t stream);

/* Synchronise the plan's last stream, return the sticky device status and
 * clear it. */
hawkes_status hawkes_plan_status(hawkes_plan p);

/* Underflow cutoff (off by default).  When enabled, the pair passes skip a
 * (row wavefront, column chunk) block whose time gap alone puts every term's
 * exponent below -160 in log2 units -- exp(-omega dt) and
 * exp(-dt^2/(2 tau_t^2)) under 2^-160 -- terms that are exactly zero in the
 * FP32 background and below 1e-48 of a unit term in the excitation.  This is
 * not part of the paper's method, which sums all pairs (Sec. 3.1); throughput
 * with the cutoff is therefore reported apart from pair-evaluations.  Applies
 * to hawkes_eval and the calls built on it. */
hawkes_status hawkes_plan_set_cutoff(hawkes_plan p, int enabled);

/* Number of intensity evaluations the plan has run so far: every hawkes_eval
 * (and every subset evaluation of the HMC path) increments it.  Host-side,
 * no synchronisation. */
int64_t hawkes_plan_epoch(hawkes_plan p);

/* The backward half of an evaluation (Eq. 4, and Eq. 5 when d_negH_theta is
 * not NULL): only the column pass runs, on the intensities lambda_i and the
 * integral terms left by the plan's most recent hawkes_eval.  The call pairs
 * with that evaluation: `epoch` must be the value hawkes_plan_epoch returned
 * right after it and *hyper must equal the hyperparameters it used.  If either
 * differs -- the plan has evaluated something else since -- nothing is
 * enqueued and HAWKES_E_STALE is returned; the caller then runs hawkes_grad.
 * Outputs as in hawkes_eval (caller order, FP64, device). */
hawkes_status hawkes_grad_theta_from_last(hawkes_plan p, const hawkes_hyper *hyper, int64_t epoch,
                                          double *d_grad_theta, double *d_negH_theta, hipStream_t stream);

/* Per-event intermediate results of the last hawkes_eval, caller order:
 * d_lambda [n] the intensities lambda_i (FP64).  Enqueued on `stream`. */
hawkes_status hawkes_copy_lambda(hawkes_plan p, double *d_lambda, hipStream_t stream);

/* ---- Free rates and Hamiltonian Monte Carlo (Sec. 2.2, Sec. 2.3.2) ----
 *
 * The paper samples the log-rates z of the M sequenced events (theta_k =
 * exp(z_k) for k in the subset, every other rate fixed) by HMC with a diagonal
 * mass matrix.  Because only the subset rates move along a trajectory, the
 * library caches the part of every lambda_i that does not depend on them (the
 * background, and the excitation by fixed-rate events) once per
 * hyperparameter setting; each gradient then costs O(N M) pair terms.  As in
 * hawkes_eval, an intensity below (c_b + c_e) n 2^-96 is recomputed from the
 * definitions in FP64 (its static part once, its subset excitation at each
 * evaluation), so the subset path keeps FP64's range of lambda_i. */

/* Declare the free-rate subset of a plan.
 *   m      subset size, 1 <= m <= n
 *   d_idx  [m] distinct caller event indices (device, int64); slot k of the
 *          subset is event d_idx[k].  The array is copied.
 * Invalidates the cached static part.  Synchronises `stream`.  Returns
 * HAWKES_E_INVALID for an index out of range or repeated. */
hawkes_status hawkes_plan_set_subset(hawkes_plan p, int64_t m, const int64_t *d_idx, hipStream_t stream);

/* Eq. 1, Eq. 4 and Eq. 5 restricted to the subset, by the O(N M) path.
 *   d_theta        [n] full rate vector, caller order (device, read only)
 *   refresh_static non-zero: recompute the cached static part (needed when the
 *                  rates OFF the subset changed; a change of hyperparameters is
 *                  detected by the library)
 *   d_loglik       [1] loglik (Eq. 1) -- may be NULL
 *   d_grad_sub     [m] d loglik / d theta_{idx[k]} (Eq. 4) -- may be NULL
 *   d_negH_sub     [m] -d2 loglik / d theta_{idx[k]}^2 (Eq. 5) -- may be NULL
 * Needs hawkes_plan_set_subset first (else HAWKES_E_UNSUPPORTED). */
hawkes_status hawkes_subset_grad(hawkes_plan p, const hawkes_hyper *hyper, const double *d_theta,
                                 int refresh_static, double *d_loglik, double *d_grad_sub, double *d_negH_sub,
                                 hipStream_t stream);

/* Eq. 1 and its gradients in the log-rates z and the temporal-trend
 * coefficient beta of Sec. 2.2, where the subset rates are
 * theta_k = exp(z_k + beta t_k) (f(t) = t) and every other rate is fixed:
 *   d loglik / d z_k  = theta_k (Eq. 4)_k
 *   d loglik / d beta = sum_k t_k theta_k (Eq. 4)_k          -- O(M) after Eq. 4
 *   d_z        [m] log-rates, slot order (device, read)
 *   beta       trend coefficient (finite; 0 = no trend)
 *   d_theta    [n] full rates, caller order: read off the subset (fixed rates),
 *              written on the subset with exp(z_k + beta t_k)
 *   d_loglik [1], d_grad_z [m] (slot order), d_grad_beta [1]: outputs, each may be NULL
 * Needs hawkes_plan_set_subset first (else HAWKES_E_UNSUPPORTED). */
hawkes_status hawkes_subset_trend_grad(hawkes_plan p, const hawkes_hyper *hyper, const double *d_z, double beta,
                                       double *d_theta, double *d_loglik, double *d_grad_z, double *d_grad_beta,
                                       hipStream_t stream);

/* The log-rates of the subset from a full rate vector, slot order:
 * d_z[k] = log d_theta[idx[k]] - beta t_{idx[k]} (Sec. 2.2's theta_k =
 * exp(z_k + beta t_k) solved for z_k).  d_theta [n] caller order, rates > 0. */
hawkes_status hawkes_subset_z(hawkes_plan p, const double *d_theta, double beta, double *d_z, hipStream_t stream);

/* One HMC iteration on z (slot order) with target
 *   log pi(z) = loglik(theta(z)) - sum_k z_k^2 / (2 sigma_z^2),
 *   theta_k = exp(z_k + beta t_k)
 * (the prior of Eq. 2 with V = I; beta is the temporal-trend coefficient of
 * Sec. 2.2, held fixed within the iteration), energy
 * H = -log pi(z) + p^T M^{-1} p / 2, and
 * L leapfrog steps of size eps with dz/dt = M^{-1} p.  Momenta p_k = sqrt(M_k) *
 * N(0,1) from Philox-4x32-10 (Salmon et al. 2011) with key `seed` and counter
 * (k, 0, counter_lo, counter_hi), standard normals by Box-Muller
 * sqrt(-2 log(1-u1)) cos(2 pi u2) on 53-bit uniforms; the Metropolis uniform
 * uses counter (0, 1, counter_lo, counter_hi).  The caller advances `counter`
 * between iterations.  Everything stays on the device; nothing synchronises. */
typedef struct {
    double *d_z;           /* [m] log-rates, slot order (in: current; out: next state)         */
    double *d_theta;       /* [n] full rates, caller order; entries of the subset are written  */
                           /*     with exp(z + beta t), the others are read as the fixed rates */
    const double *d_mass;  /* [m] diagonal mass matrix M (momentum covariance), slot order     */
    double eps;            /* leapfrog step size > 0                                            */
    int L;                 /* leapfrog steps >= 1                                               */
    double sigma_z;        /* prior standard deviation of z > 0                                 */
    uint64_t seed;         /* Philox key                                                        */
    uint64_t counter;      /* Philox counter of this iteration                                  */
    int refresh_static;    /* non-zero: recompute the cached static part first                  */
    double *d_out;         /* [8] device: accepted (1/0), H1 - H0, loglik and log pi at the
                              returned state, min(1, exp(-(H1-H0))), loglik at the proposal, H0, H1 */
    double beta;           /* temporal-trend coefficient (0: theta_k = exp(z_k))              */
    int prior;             /* 0: z ~ N(0, sigma_z^2 I); 1: the phylogenetic prior of Eq. 2,
                              z ~ N(0, sigma_z^2 V) for the tree set by hawkes_plan_set_tree
                              (its tips must be the subset slots)                          */
    double *d_z_proposal;  /* [m] device, may be NULL: the end of the leapfrog path (slot
                              order), written whether or not the proposal is accepted     */
} hawkes_hmc_args;

hawkes_status hmc_step(hawkes_plan p, const hawkes_hyper *hyper, hawkes_hmc_args *args, hipStream_t stream);

/* ---- Phylogenetic Brownian prior (Sec. 2.2, Eq. 2) ----
 *
 * The log-rates z of the subset are the tips of a bifurcating tree on which a
 * Brownian motion diffuses: root ~ N(0, tau0 sigma^2), child = parent +
 * N(0, w sigma^2) for branch length w.  Then z ~ N(0, sigma^2 V) with
 * V_nm = tau0 + length of the root-to-common-ancestor path of tips n and m.
 * The library evaluates log p(z) and its gradient in O(M) by message passing
 * over the tree, never forming V. */

/* Set the tree (host arrays, copied).
 *   n_nodes   2M - 1 (M tips); nodes 0..M-1 are the tips, node k = subset slot k
 *   parent    [n_nodes] parent of each node, -1 for the root (exactly one)
 *   length    [n_nodes] branch length to the parent (>= 0, finite; the root's is ignored)
 *   tau0      root variance factor > 0
 * Every internal node must have exactly two children and no two sibling
 * subtrees may both have zero variance.  HAWKES_E_INVALID otherwise. */
hawkes_status hawkes_plan_set_tree(hawkes_plan p, int64_t n_nodes, const int64_t *parent, const double *length,
                                   double tau0);

/* log p(z) of Eq. 2 for the plan's tree, with its gradient:
 *   d_z [M] (slot order), sigma > 0;
 *   d_logp [1] = -(M log(2 pi sigma^2) + log|V| + z^T V^{-1} z / sigma^2) / 2   (may be NULL)
 *   d_grad [M] = -V^{-1} z / sigma^2                                           (may be NULL)
 *   d_quad [1] = z^T V^{-1} z                                                   (required)
 * HAWKES_E_UNSUPPORTED if no tree is set. */
hawkes_status hawkes_tree_prior(hawkes_plan p, const double *d_z, double sigma, double *d_logp, double *d_grad,
                                double *d_quad, hipStream_t stream);

/* ---- Learned preconditioner (a small network predicting the diagonal mass) ----
 *
 * Network 12 -> 64 -> 64 -> 1, tanh hidden layers, FP32.  Parameter vector
 * (hawkes_mlp_num_params() = 5057 floats, device): W1 [64][12], b1 [64],
 * W2 [64][64], b2 [64], w3 [64], b3 [1]; y = w3 . tanh(W2 tanh(W1 x + b1) + b2) + b3.
 * Inputs X are [rows][12] FP32, row-major. */
int64_t hawkes_mlp_num_params(void);
/* Floats of device workspace that hawkes_mlp_grad / hawkes_mlp_train_step need for batch B. */
int64_t hawkes_mlp_workspace_floats(int64_t B);
/* y[s] = network(X[s]) for s < B. */
hawkes_status hawkes_mlp_forward(const float *d_params, const float *d_x, int64_t B, float *d_y, hipStream_t stream);
/* Loss L = mean_s (network(X[rows[s]]) - target[rows[s]])^2 over a batch of B rows
 * of the n_rows-row arrays d_x [n_rows][12] and d_target [n_rows] (d_rows: device
 * int [B], or NULL for rows 0..B-1, which needs B <= n_rows) and its gradient by
 * back-propagation, summed over the batch in fixed order in FP64:
 * d_grad [5057] FP64, d_loss [1] FP64 (may be NULL).  A row index outside
 * [0, n_rows) is never read: that sample is dropped and *d_err |= 1 (d_err: device
 * int, may be NULL). */
hawkes_status hawkes_mlp_grad(const float *d_params, const float *d_x, int64_t n_rows, const int *d_rows,
                              const float *d_target, int64_t B, float *d_work, double *d_grad, double *d_loss,
                              int *d_err, hipStream_t stream);
/* hawkes_mlp_grad followed by one Adam update (Kingma & Ba 2015; beta1 0.9,
 * beta2 0.999, epsilon 1e-8, bias-corrected, step >= 1) of d_params in place;
 * d_adam_m, d_adam_v [5057] FP32 moment buffers (zero before step 1). */
hawkes_status hawkes_mlp_train_step(float *d_params, float *d_adam_m, float *d_adam_v, int step, float lr,
                                    const float *d_x, int64_t n_rows, const int *d_rows, const float *d_target,
                                    int64_t B, float *d_work, double *d_grad, double *d_loss, int *d_err,
                                    hipStream_t stream);

/* Allocation-free variant of hawkes_mlp_train_step, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving or
 * training loops, harnesses that forbid allocation).  Same arguments and
 * results except that the workspace and the FP64 gradient are not passed: they
 * live in a fixed device array of the library, about 4.3 MB per GPU, taken once
 * per device on the first call there and held until the process ends.  The
 * call allocates nothing and calls no allocating routine.
 *   B  at most hawkes_mlp_noalloc_max_batch() (4096); a larger batch returns
 *      HAWKES_E_CAPACITY with nothing enqueued.
 * Every call on one GPU shares that GPU's array: calls that overlap in time on
 * one GPU (different streams or host threads without ordering) race and give
 * undefined results; calls ordered on one stream are safe.  No part of the
 * array needs clearing between calls (each kernel writes what it reads). */
int64_t hawkes_mlp_noalloc_max_batch(void);
hawkes_status hawkes_mlp_train_step_noalloc(float *d_params, float *d_adam_m, float *d_adam_v, int step, float lr,
                                            const float *d_x, int64_t n_rows, const int *d_rows,
                                            const float *d_target, int64_t B, double *d_loss, int *d_err,
                                            hipStream_t stream);
/* Per-event network inputs for the subset (slot order), d_feat [m][12] FP32.
 * For free event m, with r2_e = (x_e - x_m)^2 + (y_e - y_m)^2 and dt_e = t_e - t_m:
 *   0, 1  log1p(#{e != m : r2_e < r^2}) for r = h, 3h (events in a disc)
 *   2     log1p(#{e : r2_e < (3h)^2, 0 < dt_e <= 6/omega}) (later neighbours)
 *   3..5  r = h: log1p of the events in the disc with -1/omega <= dt_e < 0,
 *         with 0 < dt_e <= 1/omega, and with 0 < dt_e <= 3/omega
 *   6, 7  the first two for r = 3h
 *   8     max(log2 S_m, -32) / 8, S_m = sum over r2_e < (3h)^2,
 *         0 < dt_e <= 6/omega of exp(-2 omega dt_e - r2_e / h^2): Eq. 5's
 *         H_m without the weights c_e / lambda_e
 *   9     z_k;  10  #{e : t_e < t_k} / N;  11  (T1 - t_k) / (T1 - T0)
 * Counts are exact: a grid of cells of size 3h (origin (gx0, gy0) <= the
 * minimum coordinates) only enumerates the candidates, each tested by its
 * FP64 distance.  S_m is summed in 64-bit fixed point relative to its largest
 * term, so it does not depend on the candidates' order.  d_t, d_xy are the arrays the plan was built from.
 * HAWKES_E_UNSUPPORTED if the grid would exceed 2^26 cells.  Uses a workspace
 * of the plan's subset (grown on demand; a growth synchronises `stream`). */
hawkes_status hawkes_features(hawkes_plan p, const hawkes_hyper *hyper, const double *d_t, const double *d_xy,
                              const double *d_z, double gx0, double gy0, float *d_feat, hipStream_t stream);

/* The log posterior's curvature in the subset's log-rates (Sec. 2.3.2: the
 * diagonal of Eq. 5 used as the HMC mass, carried to z by the chain rule; with
 * theta_k = exp(z_k + beta t_k), d theta_k / d z_k = theta_k whatever beta):
 *   c_k = -d2 log pi / dz_k^2 = theta_k^2 H_k - theta_k g_k + P_kk,
 * g, H = Eq. 4, Eq. 5 on the subset at the rates d_theta [n] (caller order,
 * read only; the subset path), P_kk the prior's precision diagonal:
 * 1/sigma_z^2 for prior = 0 (z ~ N(0, sigma_z^2 I)), (V^{-1})_kk / sigma_z^2 for
 * prior = 1 (Eq. 2 on the tree of hawkes_plan_set_tree).
 *   d_curv  [m] FP64, slot order: c_k                              -- may be NULL
 *   d_log_h [m] FP32, slot order: log max(H_k, 1e-6), the learned
 *           preconditioner's training target (Eq. 5 is 0 for an event
 *           with no later event)                                   -- may be NULL
 * HAWKES_E_UNSUPPORTED without a subset, or with prior = 1 and no tree of m tips. */
hawkes_status hawkes_subset_curvature(hawkes_plan p, const hawkes_hyper *hyper, const double *d_theta,
                                      double sigma_z, int prior, double *d_curv, float *d_log_h,
                                      hipStream_t stream);

/* Running average of the diagonal mass: d_mass[k] <- (count d_mass[k] + e_k)/(count + 1)
 * with e_k an estimate of c_k above at the rates d_theta:
 *   d_pred == NULL: exact, max(theta_k^2 H_k - theta_k g_k, 0) + P_kk (Eq. 4, Eq. 5 by
 *                   the subset path; floored at the prior's precision);
 *   d_pred != NULL: learned, theta_k^2 exp(d_pred[k]) + P_kk (d_pred [m] FP32, slot order:
 *                   the network's prediction of log H_k).
 * prior and P_kk as in hawkes_subset_curvature.  The mass stays positive, so
 * HMC remains exact whatever the estimate. */
hawkes_status hawkes_mass_update(hawkes_plan p, const hawkes_hyper *hyper, const double *d_theta,
                                 const float *d_pred, double sigma_z, int prior, int64_t count, double *d_mass,
                                 hipStream_t stream);

/* Timing of the pair passes with HIP events recorded on the launch stream.
 * hawkes_profile_enable(p, k) with k >= 1 starts recording around the row
 * pass, the column pass and the whole evaluation of every k-th evaluation of
 * plan p (the first, the (k+1)-th, ...); 0 stops and discards.  An event
 * between two dependent kernels delays the second by several microseconds,
 * so a k above 1 keeps the timing from slowing most evaluations.
 * hawkes_profile_read synchronises and fills host out[6] with
 * (total ms, count) for the row pass, the column pass and the whole evaluation
 * since the last read, then resets the totals. */
hawkes_status hawkes_profile_enable(hawkes_plan p, int on);
hawkes_status hawkes_profile_read(hawkes_plan p, double *out);

/* Calibration of the FP32 exponential.  Mean signed (d_out[0]) and mean absolute
 * (d_out[1]) relative error of the hardware exp2 over `nsamples` arguments spread
 * evenly over [lo, hi) (-126 <= lo < hi <= 0), against FP64 exp2; d_out[2] = nsamples.
 * d_out is a device FP64 [3].  The pair sums are unbiased only if this mean matches
 * hawkes_exp2_bias_constant(), the value the library corrects for. */
hawkes_status hawkes_exp2_bias(int64_t nsamples, double lo, double hi, double *d_out, hipStream_t stream);
double hawkes_exp2_bias_constant(void);

/* Issue throughput of the hardware exp2: `blocks` blocks of 256 threads, each
 * thread running 8 independent chains of `iters` exp2 steps and nothing else.
 * One untimed launch, then one launch timed by HIP events on `stream`;
 * synchronises.  h_out (host) [3]: exp2 evaluations, seconds, evaluations per
 * second.  d_sink: device FP32 [blocks], never written in practice. */
hawkes_status hawkes_exp2_rate(int64_t blocks, int iters, float *d_sink, double *h_out, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* HAWKES_H_ */
