// hmc_internal.hpp -- host-side context and launcher declarations shared by
// the translation units of libhmc.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/hmc.h"
#include "hmc_device.hpp"

namespace hmc {

// Target as the kernels see it (passed by value).
struct TargetDev {
    int32_t kind;
    int32_t x_bf16;        // LOGREG: X holds BF16 bit patterns
    int64_t D;
    const void* prec;      // state dtype
    const void* X;         // float or uint16 (bf16)
    int64_t N;
    const uint8_t* y;
    double inv_var;        // LOGREG: 1 / prior_scale^2
};

// Device workspace carve-up (all offsets 256-byte aligned).
struct Workspace {
    void* x;       // [C, D] current state
    void* g;       // [C, D] gradient at x
    double* logp;  // [C]
    double* eps;   // [C]
    DualAvg* da;   // [C]
    void* xq;      // [C, D] trajectory position (plain path)
    void* pq;      // [C, D] trajectory momentum
    void* gq;      // [C, D] trajectory gradient
    double* lpq;   // [C] data part of logp at the trajectory end (LOGREG)
    double* h0;    // [C] initial energy
    float* part_g;     // [nsplit, C, D] split-N gradient partials (LOGREG plain)
    double* part_lp;   // [nsplit, C]
    int32_t* lr_cnt;   // [ceil(C / 64)] finished splits per chain tile of the FP32 logistic step (0 between launches)
    void* xt;          // [DP, NP] BF16 zero-padded transposed copy of X (BF16 gradients only)
    void* xp;          // [NP, DP] BF16 zero-padded copy of X
    void* yp;          // [NP] labels, zeros past N
    void* bk_x;        // autotuner backup of the chain state: [C, D] x and g, [C] logp and eps, [C] da
    void* bk_g;
    double* bk_logp;
    double* bk_eps;
    DualAvg* bk_da;
    Ctrl* ctrl;
    double* beta_buf;  // [C] inverse temperatures (replica exchange)
    double* beta;      // beta_buf once temperatures are set, else NULL (every chain at beta = 1)
    double* scale_buf; // [D] diagonal scale of the transformed kernel
    double* scale;     // scale_buf once a transform is set, else NULL (identity)
    size_t bytes;
};

hmc_status fail(hmc_status st, const std::string& msg);
hmc_status validate_args(const hmc_target* tg, const hmc_config* cfg, TargetDev* out);
int64_t logreg_nsplit(int64_t N, int64_t C);
int64_t logreg_nsplit_cap(int64_t N, int64_t C);
int lb_grad_nsplit(int64_t N, int64_t C, int64_t D);
int lb_logp_nsplit(int64_t N, int64_t C, int64_t D);
bool bf16_grad_supported(const TargetDev& tg);
// bytes of the padded copy of X for the BF16 form ([NP, DP] BF16), with NP and DP
size_t lb_pad_bytes(int64_t N, int64_t D, int64_t* np, int64_t* dp);
Workspace carve_workspace(void* base, const TargetDev& tg, const hmc_config& cfg, size_t* total);
size_t elem_size(int32_t dtype);

// Launch-shape choices (0 = built-in heuristic), set by the autotuner.
struct Tune {
    int32_t lr_nsplit;     // row splits of the FP32 logistic plain kernel
    int32_t lr16_nsplit;   // row splits of the BF16 logistic kernel (1, 2, 4, 8)
    int32_t elem_gmult;    // lanes per chain multiplier of the fused elementwise kernel (1 or 2)
};

// Events recorded on the launching stream around the launches of a context's
// dominant kernel (the gradient kernel of the plain form, the transition kernel
// of the fused form), for at most cap launches once armed (host-side only).
struct KernelTimer {
    hipEvent_t* ev;        // [2 cap]: start and end of launch i at 2 i, 2 i + 1
    int64_t cap;
    int64_t n;             // launches recorded
    bool open;             // a start is recorded and its end is not
    const char* name;      // kernel of the recorded launches
};

// ---- plain path launchers (k_plain.hip) -----------------------------------
struct PlainArgs {
    TargetDev tg;
    Tune tune;
    int64_t C;
    int32_t L;
    bool f64;          // state dtype
    bool bf16_grad;    // LOGREG MFMA operands in BF16
    Key key;
    Workspace ws;
    KernelTimer* timer;   // host object or NULL (never read by a kernel)
};

inline void timer_begin(const PlainArgs& a, hipStream_t s) {
    KernelTimer* t = a.timer;
    if (!t || t->n >= t->cap) return;
    t->open = hipEventRecord(t->ev[2 * t->n], s) == hipSuccess;
}
inline void timer_end(const PlainArgs& a, hipStream_t s, const char* name) {
    KernelTimer* t = a.timer;
    if (!t || !t->open) return;
    t->open = false;
    if (hipEventRecord(t->ev[2 * t->n + 1], s) == hipSuccess) {
        t->name = name;
        ++t->n;
    }
}
int64_t logreg_nsplit_t(const PlainArgs& a);
int lb_grad_nsplit_t(const PlainArgs& a);
hipError_t launch_set_ctrl(const Ctrl& c, Ctrl* dst, hipStream_t s);
hipError_t launch_bootstrap(const PlainArgs& a, const void* x_src, hipStream_t s);
hipError_t launch_plain_transition(const PlainArgs& a, bool copy_proposal, hipStream_t s);
hipError_t launch_da_init(const PlainArgs& a, hipStream_t s);
hipError_t launch_leapfrog_step(const PlainArgs& a, double ks, hipStream_t s);

// ---- No-U-Turn sampler (k_nuts.hip) ----------------------------------------
// Per-chain buffers of the unrolled tree (state dtype T for vectors).
struct NutsWs {
    void *mx, *mr, *mg;        // [C, D] backward end of the trajectory: x, r, g
    void *px, *pr, *pg;        // [C, D] forward end
    void *lf_x, *lf_r;         // [MD, C, D] first leaf of the pending left subtree of level k
    void *lc_x, *lc_g;         // [MD, C, D] candidate of that subtree
    void *rc_x, *rc_g;         // [C, D] candidate of the finished doubling
    double *mlogp, *plogp, *wlogp, *lc_logp, *rc_logp;   // [C], [C], [C], [MD, C], [C]
    double *log_u, *seps, *ntot;                         // [C] slice, signed step, points in the tree
    double *h0, *alpha;        // [C] starting energy; sum of min(1, e^(H0 - H)) over the doubling's leaves
    int32_t *n_alpha;          // [C] and their number
    int32_t *lc_n;             // [MD, C]
    int32_t *active, *alive, *rc_n, *depth, *nleap, *moved, *dir;   // [C]
    int32_t *n_active;         // [1]
    float *xt4, *yf;           // logistic X beyond the LDS, 4-dim chunk major, and y (null when unused)
    size_t bytes;
};
// l2_rows: rows of the logistic X copy the persistent kernel reads through the L2 (nuts_l2_rows), else 0
NutsWs carve_nuts(void* base, int64_t C, int64_t D, int32_t max_depth, size_t es, int64_t l2_rows, size_t* total);
int64_t nuts_l2_rows(const PlainArgs& a);
// Step-size adaptation of a NUTS run (the fields set_adapt fills), during the
// first n_burnin transitions.
struct NutsAdapt {
    int32_t adapt;
    int32_t adapt_kind;
    double target_accept, gamma, t0, kappa, rate;
    int64_t n_burnin;
};
hipError_t launch_nuts_begin(const PlainArgs& a, const NutsWs& n, uint32_t t, hipStream_t s);
hipError_t launch_nuts_dir(const PlainArgs& a, const NutsWs& n, uint32_t t, int32_t j, hipStream_t s);
hipError_t launch_nuts_halfkick(const PlainArgs& a, const NutsWs& n, hipStream_t s);
hipError_t launch_nuts_leaf(const PlainArgs& a, const NutsWs& n, uint32_t t, int32_t j, int32_t i, hipStream_t s);
hipError_t launch_nuts_doubling_end(const PlainArgs& a, const NutsWs& n, uint32_t t, int32_t j, hipStream_t s);
bool nuts_fused_supported(const PlainArgs& a);
hipError_t launch_nuts_fused(const PlainArgs& a, const NutsWs& n, const NutsAdapt& ad, uint32_t t_begin,
                             int64_t n_trans, int32_t max_depth, void* samples, int32_t* tr_depth, int32_t* tr_nleap,
                             double* tr_stat, hipStream_t s);
// end of transition it: adaptation from the statistic, then (kept draw r, or
// r < 0) the sample and trace rows
hipError_t launch_nuts_end(const PlainArgs& a, const NutsWs& n, const NutsAdapt& ad, int64_t it, void* samples,
                           int64_t r, int32_t* tr_depth, int32_t* tr_nleap, double* tr_stat, hipStream_t s);
// Streaming moments: fold q kept states (ring rows 0..q-1 = draws r0..r0+q-1
// of R) into the per-half Welford accumulators and the batch sums.
hipError_t launch_moments(const PlainArgs& a, const void* ring, int64_t q, int64_t r0, int64_t R,
                          const hmc_moments& m, hipStream_t s);
hipError_t launch_fill_f64(double* p, int64_t n, hipStream_t s);
// Replica exchange step (K replicas of M chains, replica-major) with swap index
// t: every chain's flag into swapped and, when sample_row is not NULL, every
// chain's post-exchange state into sample_row [C, D] (both may be NULL).
hipError_t launch_remc_swap(const PlainArgs& a, int64_t K, int64_t M, uint32_t t, uint8_t* swapped,
                            void* sample_row, hipStream_t s);

// ---- BF16 gradients (k_logreg_bf16.hip) -------------------------------------
// zero-padded copies of X (row-major and transposed) and y into the workspace
hipError_t launch_pad_bf16(const PlainArgs& a, hipStream_t s);
hipError_t launch_lr16_grad(const PlainArgs& a, const float* x, const float* p, int drift, hipStream_t s);
hipError_t launch_lr16_logp(const PlainArgs& a, const float* x, hipStream_t s);

// Several BF16-gradient logistic requests of one shape class (padded width,
// lanes per chain, leapfrog count) advanced together, one launch per kernel
// of the transition: job j owns blocks begin[k] .. begin[k] + nblk[k] - 1 of
// kernel kind k (gradient and logit grids start at multiples of 8, so that a
// job's blocks keep their XCD).
enum { LR16_KIND_GROUP = 0, LR16_KIND_GRAD = 1, LR16_KIND_FINISH = 2, LR16_KIND_LOGP = 3, LR16_KIND_LPSUM = 4,
       LR16_KINDS = 5 };
struct Lr16Job {
    PlainArgs a;
    int64_t rows_g, rows_lp;        // rows per split of the gradient and logit kernels
    int32_t nsplit_g, nsplit_lp;
    int64_t begin[LR16_KINDS];
    int64_t nblk[LR16_KINDS];
};
// The job owning block b of the grid of kernel kind k and the block's index within the job (-1: a
// padding block between jobs).
__device__ __forceinline__ int lr16_job_of(const Lr16Job* __restrict__ jobs, int njobs, int kind, int64_t b,
                                           int64_t* lb) {
    for (int j = 0; j < njobs; ++j) {
        const int64_t b0 = jobs[j].begin[kind];
        if (b >= b0 && b < b0 + jobs[j].nblk[kind]) {
            *lb = b - b0;
            return j;
        }
    }
    return -1;
}
// Shape class of a request for batching (-1: not a BF16-gradient logistic plain request).
int lr16_batch_class(const PlainArgs& a);
int plain_chain_group(int64_t D);   // lanes per chain of the plain form's begin/end kernels
// Fills a job's split counts and block counts (begin is left to the caller).
void lr16_job_shape(const PlainArgs& a, Lr16Job* j);
// One launch of kernel kind k (GRAD, LOGP or LPSUM) over all jobs.
hipError_t launch_lr16_kind_multi(int kind, int64_t D, const Lr16Job* jobs_dev, int njobs, int64_t blocks,
                                  hipStream_t s);
// Block ranges of every job (fills the shapes); false if a grid would exceed 2^31 blocks.
bool lr16_layout(Lr16Job* jobs, int njobs);
// One transition of every job (host copy of the table for the grid sizes, device copy for the kernels).
hipError_t launch_lr16_transition_multi(const Lr16Job* jobs_host, const Lr16Job* jobs_dev, int njobs,
                                        hipStream_t s);

// ---- fused path (k_fused.hip) -----------------------------------------------
struct FusedRun {
    uint64_t t_begin;
    int64_t n_transitions;   // total transitions in this launch
    int64_t n_burnin;        // of which the first n_burnin are burn-in (not stored)
    int64_t m_offset;        // dual-averaging iterations done before this launch
    int64_t adapt_total;     // burn-in length of the whole run: at iteration m == adapt_total switch to eps_bar
    int32_t adapt;
    int32_t adapt_kind;      // HMC_ADAPT_DUAL_AVERAGING or HMC_ADAPT_SIMPLE
    double target_accept, gamma, t0, kappa, rate;
    void* samples;
    hmc_trace trace;
    hmc_step_out out;        // only for single-transition launches
    // replica exchange inside the launch (dense kernel; 0: none): remc_K
    // replicas of remc_M chains (chain k M + m), all replicas of one m in one
    // workgroup; after each transition the pairs of its parity exchange, and
    // the kept transitions' flags go to swapped [R, C]
    int32_t remc_K;
    int64_t remc_M;
    uint8_t* swapped;
};
// Adaptation parameters of an hmc_adapt (NULL or disabled: none) into a
// plain-path control block or a fused run.
template <typename R>
inline void set_adapt(R& r, const hmc_adapt* ad) {
    r.adapt = (ad && ad->enabled) ? 1 : 0;
    if (!r.adapt) return;
    r.adapt_kind = ad->kind;
    r.target_accept = ad->target_accept;
    r.gamma = ad->gamma;
    r.t0 = ad->t0;
    r.kappa = ad->kappa;
    r.rate = ad->rate;
}
// HMC_E_INVALID with a message when enabled parameters are out of range.
hmc_status check_adapt(const hmc_adapt* ad);

// Returns hipErrorNotSupported when no fused kernel covers this target/shape.
bool fused_supported(const PlainArgs& a);
// The fused kernel of this target can run K replicas with the exchange inside
// the launch (dense: K divides 16; element-wise: K divides the lane groups of
// a wavefront).
bool fused_remc_inline(const PlainArgs& a, int64_t K);
hipError_t launch_fused(const PlainArgs& a, const FusedRun& r, hipStream_t s);

// Ragged multi-request launch of the fused elementwise kernel: jobs of one
// shape class (state dtype, lanes per chain, blocks per lane) in one grid.
struct ElemJob {
    PlainArgs a;
    FusedRun r;
    int64_t block_begin;     // first block of this job in the grid
};
int elem_class(const PlainArgs& a);                 // -1 if the elementwise kernel does not apply
int64_t elem_blocks(const PlainArgs& a);
hipError_t launch_fused_elem_multi(int cls, const ElemJob* jobs_dev, int njobs, int64_t total_blocks,
                                   hipStream_t s);

}  // namespace hmc
