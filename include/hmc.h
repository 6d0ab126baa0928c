/*
 * hmc.h -- C ABI of libhmc.so: batched Hamiltonian Monte Carlo on MI355X (gfx950).
 *
 * One HMC transition applied to thousands of independent chains at once
 * (arXiv 2002.01184, Sec. 2.1 "Case Study: HMC"): per chain, a Gaussian
 * momentum with one independent component per state variable, L leapfrog
 * steps each evaluating the target log-probability and its gradient, and a
 * Metropolis-Hastings accept/reject on the energy change dH, taken as a
 * per-chain select (Sec. 2.1, last paragraph: vectorised where, no branch).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every call returns hmc_status; HMC_OK is 0.  On a non-OK status a
 *    message is available from hmc_last_error() (thread-local) and no state
 *    was changed.  Nothing else crosses the ABI (no exceptions).
 *  - Device pointers are HIP device memory on the current device (allocated
 *    by the caller, e.g. PyTorch); host pointers are marked "host".  The
 *    library borrows every caller buffer and never frees it; buffers passed to
 *    hmc_init must stay alive until hmc_destroy.
 *  - States are [C, D] row-major ("list of vectors", Sec. 2.1: one row per
 *    chain), in the configured state dtype.  Per-chain scalars are [C].
 *    log-probabilities, energies, step sizes and log accept ratios are FP64.
 *  - Batch semantics (Sec. 2): the target log-probability of a [C, D] batch
 *    reduces over D only; chain c's results never depend on other chains.
 *  - All work is enqueued on the hipStream_t given to hmc_init and is
 *    asynchronous; hmc_get_state and hmc_destroy synchronize that stream.
 *    A device fault surfaces as HMC_E_DEVICE at the next synchronizing call.
 *  - One context is used by one host thread at a time.
 *  - Random numbers: Philox4x32-10 (Salmon et al., SC'11), key = (seed low
 *    word, seed high word), counter = (chain, t, block, tag); tag 0 =
 *    momentum (block = d / 4, Box-Muller on word pairs (0,1), (2,3) with
 *    u = ((w >> 9) + 1/2) 2^-23), tag 1 = accept uniform
 *    u = ((w0 >> 6) 2^26 + (w1 >> 6) + 1/2) 2^-52.  t counts transitions
 *    since hmc_init (or the value given to hmc_set_state).
 */
#ifndef HMC_H
#define HMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HMC_OK = 0,
    HMC_E_INVALID = 1,      /* bad argument: sizes, null pointers, non-finite step size */
    HMC_E_UNSUPPORTED = 2,  /* valid but unsupported combination (dtype x target x form) */
    HMC_E_NOMEM = 3,        /* workspace smaller than hmc_workspace_size() */
    HMC_E_DEVICE = 4,       /* HIP runtime or kernel error */
    HMC_E_BUSY = 5          /* serving: no capacity for the request right now */
} hmc_status;

typedef enum { HMC_F64 = 0, HMC_F32 = 1, HMC_BF16 = 2 } hmc_dtype;

typedef enum {
    HMC_TGT_STD_NORMAL = 0,   /* logp = -1/2 |x|^2 (the paper's Sec. 1 example, any D) */
    HMC_TGT_GAUSS_DIAG = 1,   /* logp = -1/2 sum_i prec_i x_i^2 */
    HMC_TGT_GAUSS_DENSE = 2,  /* logp = -1/2 x^T P x, P symmetric positive definite */
    HMC_TGT_LOGREG = 3        /* Bayesian logistic regression, prior N(0, s^2 I):
                                 logp = sum_n [y_n z_n - softplus(z_n)] - |x|^2/(2 s^2), z = X x */
} hmc_target_kind;

/* Built-in target (the paper's Sec. 3 Python callable cannot run on the GPU;
 * the target is a descriptor of one of these families with hand-written
 * gradients).  All arrays are device memory, borrowed. */
typedef struct hmc_target {
    int32_t kind;             /* hmc_target_kind */
    int32_t reserved0;
    int64_t dim;              /* D >= 1 */
    const void* prec;         /* DIAG: [D]; DENSE: [D, D] row-major; dtype = state dtype */
    const void* X;            /* LOGREG: [N, D] row-major, dtype x_dtype */
    int32_t x_dtype;          /* LOGREG: HMC_F32 or HMC_BF16 */
    int32_t reserved1;
    int64_t n_rows;           /* LOGREG: N >= 1 */
    const uint8_t* y;         /* LOGREG: [N] labels, each 0 or 1 */
    double prior_scale;       /* LOGREG: s > 0 */
} hmc_target;

/* Execution form. */
enum {
    HMC_FORM_AUTO = 0,        /* fused where the target's shape allows, else plain */
    HMC_FORM_PLAIN = 1,       /* one kernel per leapfrog step, state in HBM between steps */
    HMC_FORM_FUSED = 2,       /* persistent kernel: whole transitions per chain tile in registers/LDS */
    HMC_FORM_GRAPH = 3        /* plain kernels replayed from a captured hipGraph */
};

typedef struct hmc_config {
    int64_t num_chains;          /* C >= 1 */
    int32_t num_leapfrog_steps;  /* L >= 1 */
    int32_t state_dtype;         /* HMC_F64 (elementwise targets) or HMC_F32 */
    int32_t grad_dtype;          /* HMC_F32, or HMC_BF16 (LOGREG with BF16 X: MFMA operands in BF16,
                                    FP32 accumulation; logp for dH from an FP32 logit pass) */
    int32_t form;                /* HMC_FORM_* */
    uint64_t seed;               /* Philox key */
} hmc_config;

/* Per-chain step-size adaptation during burn-in, the adaptation wrapper
 * pattern of the paper's Sec. 4.1, with the accept statistic
 * alpha = min(1, exp(-dH)) of each burn-in transition:
 *   HMC_ADAPT_DUAL_AVERAGING (kind 0): Hoffman & Gelman 2014, Sec. 3.2,
 *     eq. 6, with mu = log(10 eps0), eps0 each chain's step size at the start
 *     of the call; after burn-in each chain uses exp(log eps_bar);
 *   HMC_ADAPT_SIMPLE (kind 1): the multiplicative rule of the paper's
 *     SimpleStepSizeAdaptation example: eps (1 + rate) when alpha >
 *     target_accept, eps / (1 + rate) otherwise; the last value is kept
 *     after burn-in. */
enum { HMC_ADAPT_DUAL_AVERAGING = 0, HMC_ADAPT_SIMPLE = 1 };
typedef struct hmc_adapt {
    int32_t enabled;
    int32_t kind;                /* HMC_ADAPT_* */
    double target_accept;        /* delta, e.g. 0.8 */
    double gamma;                /* dual averaging: 0.05 */
    double t0;                   /* dual averaging: 10 */
    double kappa;                /* dual averaging: 0.75 */
    double rate;                 /* simple: adaptation rate in (0, 1], e.g. 0.01 */
} hmc_adapt;

/* Trace of kept transitions (paper Sec. 4.2 "tracing"): each pointer is a
 * device array [R, C] or NULL. */
typedef struct hmc_trace {
    double* step_size;           /* step size used by the transition */
    uint8_t* is_accepted;
    double* log_accept_ratio;    /* -dH; -inf when dH is NaN or +inf */
    double* target_log_prob;     /* logp of the post-decision state */
} hmc_trace;

/* Optional per-transition outputs of hmc_step (device pointers or NULL). */
typedef struct hmc_step_out {
    uint8_t* is_accepted;        /* [C] */
    double* log_accept_ratio;    /* [C] */
    double* target_log_prob;     /* [C] post-decision */
    void* proposed_state;        /* [C, D] state dtype: end of the trajectory before the decision */
    void* proposed_momentum;     /* [C, D] state dtype: momentum at the end of the trajectory */
    double* delta_h;             /* [C] H(end) - H(start) */
} hmc_step_out;

typedef struct hmc_ctx hmc_ctx;

/* Bytes of device workspace hmc_init needs for this target and config. */
hmc_status hmc_workspace_size(const hmc_target* target, const hmc_config* config, size_t* bytes);

/* bootstrap_results (paper Sec. 4.1): binds the target, copies init_state
 * [C, D] (device) into the context, evaluates logp and its gradient there and
 * caches them, sets t = 0.  step_size (host) holds 1 value (broadcast) or C
 * values, each finite and > 0.  workspace (device) must hold
 * hmc_workspace_size() bytes, 256-byte aligned.  hip_stream is a hipStream_t
 * (NULL = default stream).  On HMC_OK *out owns a host object freed by
 * hmc_destroy. */
hmc_status hmc_init(const hmc_target* target, const hmc_config* config, const void* init_state,
                    const double* step_size, int64_t step_size_len, void* workspace,
                    size_t workspace_bytes, void* hip_stream, hmc_ctx** out);

/* one_step (paper Sec. 4.1): one transition of every chain; t += 1.
 * Exactly L gradient evaluations per chain (the cached gradient starts the
 * trajectory).  out may be NULL. */
hmc_status hmc_step(hmc_ctx* ctx, const hmc_step_out* out);

/* sample_chain (paper Sec. 4.2): num_burnin + num_results transitions.  Burn-in
 * states are not stored; samples [R, C, D] (device, state dtype) receives the
 * state after transition burnin + r, r = 0..R-1.  adapt (host, NULL = off)
 * enables dual averaging over the burn-in.  trace (host struct of device
 * pointers) may be NULL.  samples may be NULL (no samples stored). */
hmc_status hmc_sample_chain(hmc_ctx* ctx, int64_t num_results, int64_t num_burnin_steps,
                            const hmc_adapt* adapt, void* samples, const hmc_trace* trace);

/* Checkpoint (synchronizes): state [C, D] (device) and step_size [C] (device,
 * FP64) may be NULL; *t (host) may be NULL. */
hmc_status hmc_get_state(hmc_ctx* ctx, void* state, double* step_size, uint64_t* t);

/* Resume: replaces the state (device [C, D]) and, if step_size (device [C],
 * FP64) is not NULL, the step sizes; recomputes the cached logp and gradient;
 * sets the transition counter to t.  Runs resumed this way reproduce an
 * uninterrupted run bit for bit. */
hmc_status hmc_set_state(hmc_ctx* ctx, const void* state, const double* step_size, uint64_t t);

/* Frees the context (synchronizes its stream first).  NULL is a no-op. */
hmc_status hmc_destroy(hmc_ctx* ctx);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): hmc_init,
 * hmc_sample_chain and hmc_get_state in one call, with the workspace taken
 * from a library-owned static device array of HMC_NOALLOC_WORKSPACE_BYTES
 * per GPU instead of a caller-allocated buffer.  No hipMalloc, hipFree or
 * allocating library call is made.  Arguments as hmc_init (without the
 * workspace) and hmc_sample_chain; final_state [C, D] (device, state dtype)
 * and final_step_size [C] (device, FP64) receive the state and step sizes
 * after the last transition and may be NULL.  The samples and traces equal
 * those of hmc_init + hmc_sample_chain on the same inputs, bit for bit.
 * Errors: HMC_E_NOMEM when hmc_workspace_size() exceeds the scratch (the
 * message gives both sizes; nothing is launched), HMC_E_UNSUPPORTED for
 * HMC_FORM_GRAPH (instantiating a graph allocates), HMC_E_INVALID when
 * hip_stream belongs to a device other than the current one.  Synchronizes
 * hip_stream before returning.  Every call on a GPU shares that GPU's scratch
 * (the array keeps the last call's contents; each call initialises all it
 * reads): calls that overlap on one GPU, from several threads or streams,
 * race and must be serialised by the caller. */
#define HMC_NOALLOC_WORKSPACE_BYTES (64ll << 20)
hmc_status hmc_sample_chain_noalloc(const hmc_target* target, const hmc_config* config,
                                    const void* init_state, const double* step_size,
                                    int64_t step_size_len, int64_t num_results,
                                    int64_t num_burnin_steps, const hmc_adapt* adapt,
                                    void* samples, const hmc_trace* trace, void* final_state,
                                    double* final_step_size, void* hip_stream);

/* Kernel timing (measurement): from this call on, HIP events are recorded on
 * the context's stream around each of the next max_launches (1 .. 2^20)
 * launches of the context's dominant kernel -- the gradient kernel of the plain
 * form (the first contraction kernel of a split-N target), the transition kernel
 * of the fused form; graph-form replays are not timed.  Synchronizes the
 * stream; replaces a timer already running. */
hmc_status hmc_kernel_timer_start(hmc_ctx* ctx, int64_t max_launches);

/* Synchronizes, writes the mean duration of the recorded launches in ms, their
 * number and the kernel's name (name, host, name_len bytes, NUL-terminated;
 * each output may be NULL), and stops the timer.  HMC_E_INVALID when no timer
 * was started. */
hmc_status hmc_kernel_timer_read(hmc_ctx* ctx, double* mean_ms, int64_t* launches, char* name,
                                 size_t name_len);

/* Message of the last non-OK status on this thread ("" if none). */
const char* hmc_last_error(void);

/* Form that hmc_step / hmc_sample_chain will use for this context
 * (HMC_FORM_PLAIN, HMC_FORM_FUSED or HMC_FORM_GRAPH). */
int32_t hmc_effective_form(const hmc_ctx* ctx);

/* Autotuner: times every launch configuration that applies to this context
 * (form fused / plain / graph when the context was created with
 * HMC_FORM_AUTO; lanes per chain of the fused elementwise kernel; row splits
 * of the logistic-regression kernels) over trial_transitions transitions
 * each, with HIP events on the context's stream, and keeps the fastest.  The
 * chain state, step sizes and t are restored after every trial, so the
 * sampled chain is unchanged apart from the arithmetic order of the chosen
 * kernels.  Choices are cached per (target family, D, log2 N, log2 C, dtypes,
 * L, requested form) for the process and appended to the file named by the
 * environment variable HMC_AUTOTUNE_CACHE when set.  report (host, may be
 * NULL) receives one line per candidate.  Synchronizes the stream. */
hmc_status hmc_autotune(hmc_ctx* ctx, int32_t trial_transitions, char* report, size_t report_len);

/* ---------------------------------------------------------------------------
 * Replica exchange Monte Carlo (paper Sec. 2.2, case study REMC).
 *
 * The chains of a context form K replicas of M = C / K chains, replica-major:
 * chain c = k M + m is chain m of replica k.  Chain c targets beta_c logp(x)
 * (the tempered target of the paper: the log-probability times the inverse
 * temperature, by broadcasting); the replicas of one temperature ladder
 * 1 = beta_0 > beta_1 > ... hold the same beta in all M chains.  Tempering
 * runs on every form and target.  On the fused form, when K divides the
 * chains a workgroup groups together (dense Gaussian: 16; logistic: 4;
 * element-wise: the lane groups of a wavefront, 64 / lanes per chain), the
 * fused kernels exchange between transitions themselves: one launch for the
 * run.  Otherwise the exchange sampler launches one fused transition per
 * exchange.
 * ------------------------------------------------------------------------- */

/* Sets per-chain inverse temperatures: beta (device, FP64, [C]) is copied;
 * every value must be finite and > 0 (HMC_E_INVALID otherwise, nothing
 * changed).  NULL restores beta = 1 for every chain.  The cached log-probability, traced target_log_prob and the state stay those
 * of the untempered target.  Synchronizes the stream. */
hmc_status hmc_set_inverse_temperature(hmc_ctx* ctx, const double* beta);

/* One exchange step with swap index t (< 2^32): for every m and every pair
 * (k, k+1) with k = t mod 2, t mod 2 + 2, ..., k + 1 < K, the states of chains
 * k M + m and (k+1) M + m are exchanged with probability
 * min(1, exp((beta_k - beta_{k+1}) (logp(x_{k+1}) - logp(x_k)))): the
 * Metropolis-Hastings test on the product of the replica targets, with the
 * 52-bit uniform of the Philox block (k M + m, t, 0, tag 2).  Step sizes and
 * adaptation state stay with the chain slot.  swapped (device [C], may be
 * NULL) receives 1 for both chains of an exchanged pair and 0 elsewhere.
 * HMC_E_INVALID if num_replicas does not divide C.  Asynchronous. */
hmc_status hmc_remc_swap(hmc_ctx* ctx, int64_t num_replicas, uint64_t swap_index, uint8_t* swapped);

/* Replica-exchange sample_chain: num_burnin + num_results times, one
 * transition of every chain (as hmc_sample_chain, with the same adaptation
 * and traces) followed by the exchange step whose swap index is that
 * transition's t.  On the fused form the whole run is one launch when the
 * replicas of a chain index fit in one workgroup or wavefront (see
 * hmc_set_inverse_temperature), else one launch per transition plus the
 * exchange step; both give the same decisions.  samples [R, C, D] (device, may be NULL) receive the states
 * after the exchange of transition burnin + r; swapped (device [R, C], may be
 * NULL) the exchange flags of the kept transitions; the trace rows hold the
 * transition's results before the exchange.  Asynchronous. */
hmc_status hmc_remc_sample_chain(hmc_ctx* ctx, int64_t num_replicas, int64_t num_results, int64_t num_burnin_steps,
                                 const hmc_adapt* adapt, void* samples, const hmc_trace* trace,
                                 uint8_t* swapped);

/* Transformed kernel (the paper's TransformedTransitionKernel, Sec. 4.1) with
 * the diagonal affine bijector x = shift + scale * z: the chain moves in z
 * with identity mass against the pulled-back target and reports x.  Run in
 * x, scale_d multiplies the step size in the drift and in the kick of
 * dimension d (a diagonal preconditioner); the shift drops out of the
 * dynamics.  The fused kernels run in z = x / scale instead, with the
 * target pulled back (prec scale^2, S P S; logistic: X S and the prior's
 * precision times scale^2); they agree with the plain form to rounding.
 * scale (device, FP64, [D]) is copied; every value finite and > 0.  NULL
 * restores the identity.  All forms and targets with FP32 gradients
 * (HMC_E_UNSUPPORTED with BF16 gradients).  Synchronizes the stream. */
hmc_status hmc_set_transform_scale(hmc_ctx* ctx, const double* scale);

/* ---------------------------------------------------------------------------
 * No-U-Turn sampler (paper Sec. 2.3: NUTS with its recursion unrolled into a
 * fixed O(max_tree_depth) per-chain memory; the algorithm is Hoffman & Gelman
 * 2014, Algorithm 3, "efficient NUTS").  Each transition draws the momentum as
 * HMC does, a slice variable log u = log U - H0, and doubles the trajectory
 * (direction v = -1 or +1 per doubling) until the trajectory or one of its
 * subtrees makes a U-turn, a leaf diverges (log u >= 1000 - H) or
 * max_tree_depth doublings are done; the next state is drawn from the valid
 * points of the trajectory by the algorithm's progressive sampling.  Random
 * numbers: Philox4x32-10 with counter (chain, t, block, tag): momentum as
 * HMC (tag 0), slice (block 0, tag 6), direction of doubling j (block j,
 * tag 4), take of doubling j's subtree (block j, tag 5), merge of the level-k
 * subtree ending at leaf i of doubling j (block (1024 j + i) 16 + k, tag 3).
 * The step size is each chain's current step size.  With an hmc_adapt, each
 * burn-in transition then updates it from the statistic of Hoffman & Gelman
 * (2014) Algorithm 6 -- the mean of min(1, exp(H0 - H)) over the leaves built
 * in the transition's last doubling (0 with max_depth 0) -- by dual averaging
 * (as in hmc_sample_chain: iteration m = burn-in transition m of this call;
 * the last burn-in transition sets the averaged iterate) or by the
 * multiplicative rule.  On a context created with the fused or the automatic
 * form one persistent kernel runs every transition of the call where one
 * covers the target: N(0, I) and the diagonal Gaussian up to D = 1024 (a lane
 * group, or above 256 (FP64) / 512 (FP32) dims a workgroup, per chain); the
 * dense Gaussian in FP32 up to D = 128 (16 chains per workgroup on MFMA,
 * building their trees in lockstep); logistic regression with FP32 states and
 * gradients and D <= 32 (a wavefront per chain), with X and y in the
 * workgroup's LDS when X is FP32 and they fit (N <= 1000 at D = 25), else X
 * (FP32 or BF16) read through the L2 from a copy in the NUTS workspace.
 * Otherwise the chains run in lockstep on the plain kernels of the target and
 * a chain whose trajectory has stopped is masked.  All build the same trees.
 * The context must have no inverse temperatures or transform
 * (HMC_E_UNSUPPORTED).
 * ------------------------------------------------------------------------- */

/* Bytes of the caller-allocated NUTS workspace for this context (256-byte
 * aligned base).  max_depth in 0..10. */
hmc_status hmc_nuts_workspace_size(const hmc_ctx* ctx, int32_t max_depth, size_t* bytes);

/* burn-in + R NUTS transitions from the context's state; adapt (host, may be
 * NULL: fixed step sizes) as for hmc_sample_chain; samples [R, C, D]
 * (device, state dtype), tree_depth and n_leapfrog [R, C] (device int32: the
 * doublings and leapfrog steps of each kept transition) and accept_stat
 * [R, C] (device FP64: Algorithm 6's statistic of each kept transition) may
 * be NULL.  t advances by burn-in + R; the step sizes stay where adaptation
 * left them.  The lockstep path synchronizes the stream after every
 * doubling; the persistent one is asynchronous. */
hmc_status hmc_nuts_sample_chain(hmc_ctx* ctx, int32_t max_depth, int64_t num_results, int64_t num_burnin_steps,
                                 const hmc_adapt* adapt, void* nuts_workspace, size_t nuts_workspace_bytes,
                                 void* samples, int32_t* tree_depth, int32_t* n_leapfrog, double* accept_stat);

/* ---------------------------------------------------------------------------
 * Streaming expectations: the driver the paper plans (Sec. 4.2) for runs
 * whose full trace would be too large to store.  sample_chain keeps no
 * samples; per chain c and state variable d it accumulates over the kept
 * draws r = 0 .. R-1, in FP64:
 *   mean[h, c, d], m2[h, c, d]  mean and sum of squared deviations of the
 *       draws of half h (h = 0: r < R/2, h = 1: r >= R/2, R/2 rounded down),
 *       by Welford's update in draw order;
 *   batch_sum[b, c, d]  (optional) the sum of the draws of batch
 *       b = r / batch_len (R a multiple of batch_len).
 * The kept states pass through ring (caller-provided, [ring_rows, C, D] of
 * the state dtype): the transitions write up to ring_rows states into it and
 * one kernel folds them into the accumulators in order, so the result does
 * not depend on ring_rows.  The accumulators are cleared by the call.
 * ------------------------------------------------------------------------- */
typedef struct hmc_moments {
    double* mean;                /* [2, C, D] device */
    double* m2;                  /* [2, C, D] device */
    double* batch_sum;           /* [R / batch_len, C, D] device, or NULL */
    int64_t batch_len;           /* draws per batch when batch_sum is set */
    void* ring;                  /* [ring_rows, C, D] device, state dtype */
    int64_t ring_rows;           /* >= 1 */
} hmc_moments;

/* As hmc_sample_chain (same transitions, adaptation and traces; t advances by
 * burn-in + R) with the kept states reduced into moments instead of stored.
 * HMC_E_INVALID for missing buffers, ring_rows < 1, batch_len not dividing
 * R.  Asynchronous. */
hmc_status hmc_sample_chain_moments(hmc_ctx* ctx, int64_t num_results, int64_t num_burnin_steps,
                                    const hmc_adapt* adapt, const hmc_moments* moments,
                                    const hmc_trace* trace);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of sampling requests (one sample_chain each)
 * of differing target, dimension, data size and chain count on one GPU.
 *
 * The server owns one device pool of hbm_budget_bytes (allocated at creation)
 * and a worker thread.  A request is admitted when its device memory
 * (workspace, plus its sample buffer when the caller passes samples = NULL)
 * fits in the free part of the pool; admitted requests keep their chain state
 * and adaptation state resident in the pool until they finish.  Each tick the
 * worker advances every active request by up to transitions_per_tick
 * transitions: requests of the elementwise families that share a shape class
 * run in one ragged launch, the others run concurrently on a pool of HIP
 * streams.  A request's result does not depend on which other requests run
 * with it (its random streams are keyed by its own seed and chain ids and its
 * kernels touch only its own memory), and equals the hmc_sample_chain result
 * of the same request.  Requests are admitted in arrival order; a request that
 * does not fit waits while later, smaller ones may be admitted.
 * ------------------------------------------------------------------------- */
typedef struct hmc_request {
    hmc_target target;           /* device arrays, borrowed until the request is done */
    hmc_config config;           /* form AUTO, PLAIN or FUSED */
    const void* init_state;      /* device [C, D]; read at admission */
    double step_size;            /* eps0 for every chain */
    int64_t num_results;
    int64_t num_burnin;
    hmc_adapt adapt;             /* enabled = 0 for a fixed step size */
    void* samples;               /* device [R, C, D], or NULL: the server keeps them (counted in the budget)
                                    until hmc_server_take */
    hmc_trace trace;             /* device [R, C] arrays or NULL */
} hmc_request;

typedef struct hmc_server hmc_server;

typedef struct hmc_server_stats {
    int64_t submitted, admitted, completed, failed;
    int64_t active, pending;
    int64_t ticks;
    int64_t batched_launches;    /* ragged launches that covered >= 2 requests */
    int64_t max_active;          /* most requests resident at once */
    size_t pool_bytes, bytes_in_use, peak_bytes_in_use;
    int64_t batched_plain_transitions;   /* plain transitions run once for >= 2 BF16-gradient
                                            logistic requests of one shape class */
} hmc_server_stats;

enum { HMC_REQ_QUEUED = 0, HMC_REQ_RUNNING = 1, HMC_REQ_DONE = 2, HMC_REQ_FAILED = 3 };

/* Creates the server: allocates the pool (hbm_budget_bytes of device memory)
 * and starts the worker.  transitions_per_tick >= 1. */
hmc_status hmc_server_create(size_t hbm_budget_bytes, int32_t transitions_per_tick, hmc_server** out);

/* Queues a copy of *req.  Fails with HMC_E_INVALID / HMC_E_UNSUPPORTED for a
 * request hmc_init would reject and with HMC_E_NOMEM when its memory exceeds
 * the whole pool.  *id identifies the request. */
hmc_status hmc_server_submit(hmc_server* srv, const hmc_request* req, uint64_t* id);

/* State of a request (HMC_REQ_*) and, once done, its latency from submission
 * to completion in seconds (host clock).  Either output may be NULL. */
hmc_status hmc_server_poll(hmc_server* srv, uint64_t id, int32_t* state, double* latency_s);

/* Blocks until the request is done or failed; then as hmc_server_poll. */
hmc_status hmc_server_wait(hmc_server* srv, uint64_t id, int32_t* state, double* latency_s);

/* For a done request submitted with samples = NULL: copies its samples
 * [R, C, D] into dst (device) and releases them from the pool. */
hmc_status hmc_server_take(hmc_server* srv, uint64_t id, void* dst_samples);

hmc_status hmc_server_get_stats(hmc_server* srv, hmc_server_stats* out);

/* Waits for every request, stops the worker and frees the pool. */
hmc_status hmc_server_destroy(hmc_server* srv);

/* ---------------------------------------------------------------------------
 * Measurement helpers: the achievable peaks that roofline fractions can be
 * quoted against beside the published ones.  Not part of the sampler.
 * ------------------------------------------------------------------------- */

/* Streaming bandwidth over the caller's device buffer (16-byte aligned):
 * mode 0 reads bytes / 16 float4 `passes` times per launch (a buffer that fits
 * the L2 or the Infinity Cache is then served from there after the first
 * pass); mode 1 copies the first half of the buffer to the second (passes =
 * 1).  Grid-stride kernels, eight 16-byte loads in flight per thread, 8192
 * workgroups for buffers above 64 MiB, else 2048; non-temporal accesses for a
 * single pass and for copies, cached loads for repeated passes; one untimed
 * launch, then reps
 * launches timed with HIP events on hip_stream (synchronized before return).
 * *gbytes_per_s = bytes read (+ written) / time, in 1e9 B/s.  The buffer's
 * contents are only read (mode 0) or overwritten in its second half (mode 1). */
hmc_status hmc_peak_memory(void* buf, size_t bytes, int32_t mode, int32_t passes, int32_t reps, void* hip_stream,
                           double* gbytes_per_s);

/* Issue rate of one instruction kind at waves_per_simd (1..8) waves per SIMD
 * (256 x waves_per_simd workgroups of 4 waves), iters iterations per launch of
 * one instruction on each of the wave's independent accumulators
 * (16, or 4 for kind 4): kind 0 v_mfma_f32_16x16x4f32 (2048 flop per wave
 * instruction), 1 v_mfma_f32_4x4x1f32 (16 blocks, 512), 2
 * v_mfma_f32_16x16x32_bf16 (16384), 3 v_fma_f32 (128; the library is built
 * without packed FP32 instructions), 4 v_mfma_f32_32x32x16_bf16 (32768).
 * Timing as above;
 * *tflops in 1e12 flop/s.  clock_mhz (may be NULL): the shader clock of one
 * wave over the last launch, from its clock counter against the 100 MHz
 * real-time counter. */
hmc_status hmc_peak_compute(int32_t kind, int32_t waves_per_simd, int32_t iters, int32_t reps, void* hip_stream,
                            double* tflops, double* clock_mhz);

#ifdef __cplusplus
}
#endif
#endif
