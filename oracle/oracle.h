/*
 * oracle.h -- FP64 CPU oracle of the batched HMC transition.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, obviously
 * correct reference that the GPU path is checked against.  Only tests/,
 * __graft_entry__.smoke() and the cpu_baseline leg of bench.py may load it.
 * It shares no source with the HIP library (paper_2002_01184_amd/csrc) and
 * includes nothing from it.
 *
 * What it computes (paper: "tfp.mcmc: Modern Markov Chain Monte Carlo Tools
 * Built for Modern Hardware", arXiv 2002.01184):
 *   - Sec. 2.1 (Case Study: HMC): draw one independent Gaussian momentum per
 *     state variable per chain, run a symplectic integrator for a fixed
 *     number of steps, accept or reject the proposal with a
 *     Metropolis-Hastings test; every chain is independent.
 *   - Sec. 2 (batch semantics): the target log-probability of a [C, D]
 *     batch reduces over the event axis D only, giving one value per chain.
 *   - Sec. 4.1 (TransitionKernel): bootstrap computes the target
 *     log-probability and its gradient at the initial state; one_step
 *     carries them so they are not recomputed.
 *   - Sec. 4.2 (Driver): sample_chain = burn-in (not stored), sampling
 *     (stored), tracing of kernel results.
 *   - Leapfrog integrator: Neal (2011), "MCMC using Hamiltonian dynamics",
 *     Sec. 5.2.3.3 (cited by the paper for HMC).
 *   - Step-size adaptation by dual averaging: Hoffman & Gelman (2014),
 *     Sec. 3.2, eq. (6) (cited by the paper for NUTS; the adaptation-wrapper
 *     pattern is the paper's Sec. 4.1).
 *   - Random numbers: Philox4x32-10 from Salmon, Moraes, Dror & Shaw,
 *     "Parallel Random Numbers: As Easy as 1, 2, 3" (SC'11); normals by the
 *     Box-Muller transform (Box & Muller 1958).
 *
 * All arithmetic is double precision.  Callers upcast FP32/BF16 device
 * arrays to double exactly before passing them here.
 */
#ifndef HMC_ORACLE_H
#define HMC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_STD_NORMAL = 0, ORC_GAUSS_DIAG = 1, ORC_GAUSS_DENSE = 2, ORC_LOGREG = 3 };
enum { ORC_TAG_MOMENTUM = 0, ORC_TAG_ACCEPT = 1, ORC_TAG_SWAP = 2 };

typedef struct {
    int32_t kind;          /* ORC_* target family */
    int32_t reserved;
    int64_t dim;           /* D */
    const double *prec;    /* GAUSS_DIAG: [D]; GAUSS_DENSE: [D*D] row-major precision */
    const double *X;       /* LOGREG: [N*D] row-major design matrix */
    const double *y;       /* LOGREG: [N] labels in {0, 1} */
    int64_t n_rows;        /* LOGREG: N */
    double prior_scale;    /* LOGREG: prior N(0, prior_scale^2 I) */
    double beta;           /* inverse temperature: the log-probability and its
                              gradient are multiplied by beta (1 = untempered;
                              replica exchange, paper Sec. 2.2) */
    const double *scale;   /* transformed kernel (paper Sec. 4.1): when not NULL the
                              chain moves in z with x = shift + scale * z (diagonal
                              affine bijector); logp is evaluated at x(z) and the
                              gradient is scale * grad_x.  The log-det term is
                              constant and dropped. */
    const double *shift;   /* [D] or NULL (zero) */
} orc_target;

/* Philox4x32-10 block function (SC'11, Sec. 3.2): 10 rounds, key bumped
 * by the Weyl constants between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Four standard normals from one Philox block keyed by seed with counter
 * (c0, c1, c2, tag): Box-Muller on word pairs (w0,w1) and (w2,w3). */
void orc_normal4(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t tag, double z[4]);

/* Momentum of one chain at transition t: p[i] = normal (i mod 4) of block
 * floor(i/4) with counter (chain, t, block, MOMENTUM). */
void orc_momentum(uint64_t seed, uint32_t chain, uint32_t t, int64_t D, double *p);

/* Accept uniform of one chain at transition t, in (0, 1), from the block
 * with counter (chain, t, 0, ACCEPT). */
double orc_accept_uniform(uint64_t seed, uint32_t chain, uint32_t t);

/* Batched helpers for tests: n Philox blocks (ctr [n*4] -> out [n*4]) under one
 * key; momenta of chains 0..C-1 at transition t ([C*D]); accept uniforms [C]. */
void orc_philox_many(int64_t n, const uint32_t *ctr, const uint32_t key[2], uint32_t *out);
void orc_momentum_many(uint64_t seed, int64_t C, uint32_t t, int64_t D, double *p);
void orc_accept_uniform_many(uint64_t seed, int64_t C, uint32_t t, double *u);

/* Target log-probability (up to an additive constant) and its gradient. */
double orc_logp_grad(const orc_target *tg, const double *x, double *g);

/* L leapfrog steps from (x, p) with gradient g at x.  On return x, p hold the
 * end of the trajectory, g and *logp the gradient and log-probability there. */
void orc_leapfrog(const orc_target *tg, double eps, int32_t L,
                  double *x, double *p, double *g, double *logp);

/* One HMC transition of one chain.  (x, *logp, g) is the current state with
 * its cached log-probability and gradient; it is replaced by the proposal on
 * acceptance and left unchanged otherwise.  Optional outputs (NULL allowed):
 * x_prop/p_prop [D] the end of the trajectory, logp_prop, delta_h.
 * Returns 1 if accepted.  *log_accept_ratio = -dH (-inf when dH is NaN/+inf). */
int orc_transition(const orc_target *tg, uint64_t seed, uint32_t chain, uint32_t t,
                   int32_t L, double eps, double *x, double *logp, double *g,
                   double *x_prop, double *p_prop, double *logp_prop,
                   double *delta_h, double *log_accept_ratio);

/* Dual-averaging step-size state of one chain (Hoffman & Gelman 2014, eq. 6). */
typedef struct {
    double log_eps;      /* log step size used by the next transition */
    double hbar;         /* running average of (target_accept - alpha) */
    double log_eps_bar;  /* averaged log step size */
    double mu;           /* shrinkage point log(10 * eps0) */
} orc_dual_avg;

/* Multiplicative step-size adaptation (the paper's SimpleStepSizeAdaptation
 * example of the wrapper pattern, Sec. 4.1), one chain, one burn-in
 * transition: eps (1 + rate) when the accept statistic alpha exceeds
 * target_accept, eps / (1 + rate) otherwise. */
double orc_simple_adapt(double eps, double alpha, double target_accept, double rate);

void orc_dual_avg_init(orc_dual_avg *s, double eps0);
/* Iteration m >= 1 with acceptance statistic alpha in [0, 1]. */
void orc_dual_avg_update(orc_dual_avg *s, int64_t m, double alpha, double target_accept,
                         double gamma, double t0, double kappa);

/* Batched entry points over C chains ([C, D] row-major states), OpenMP over
 * chains.  nthreads <= 0 uses the OpenMP default. */
void orc_bootstrap(const orc_target *tg, int64_t C, const double *x, double *logp, double *g,
                   int32_t nthreads);

void orc_step(const orc_target *tg, int64_t C, int32_t L, uint64_t seed, uint32_t t,
              const double *eps, double *x, double *logp, double *g,
              double *x_prop, double *p_prop, double *logp_prop, double *delta_h,
              double *log_accept_ratio, uint8_t *accepted, int32_t nthreads);

/* sample_chain: transitions t_begin .. t_begin + burnin + results - 1.
 * x [C*D] and eps [C] are read as the start and hold the final state / step
 * size on return.  adapt: 0 fixed step size; ORC_ADAPT_DUAL_AVERAGING: each
 * chain runs dual averaging during the burn-in (iteration m = 1..burnin) and
 * then uses exp(log_eps_bar); ORC_ADAPT_SIMPLE: orc_simple_adapt after every
 * burn-in transition (rate), the last value kept afterwards.
 * samples [R*C*D] and traces [R*C] may be NULL.  Returns 0. */
enum { ORC_ADAPT_DUAL_AVERAGING = 1, ORC_ADAPT_SIMPLE = 2 };
int orc_sample_chain(const orc_target *tg, int64_t C, int32_t L, uint64_t seed,
                     uint32_t t_begin, double *x, double *eps,
                     int64_t num_burnin, int64_t num_results,
                     int32_t adapt, double target_accept, double gamma, double t0, double kappa,
                     double rate, double *samples, double *tr_step, uint8_t *tr_acc, double *tr_lar,
                     double *tr_logp, int32_t nthreads);

/* ---- Replica exchange Monte Carlo (paper Sec. 2.2, case study REMC) ----
 * K replicas of M chains each, replica-major: chain c = k*M + m is chain m of
 * replica k, whose target is tgs[k] (the same target with inverse temperature
 * beta_k; replica k's log-probability is beta_k times the target's).
 *
 * orc_remc_swap: the exchange step with swap index t.  The pairs (k, k+1)
 * with k = (t mod 2), (t mod 2) + 2, ... (k + 1 < K) exchange the states of
 * their chain m with probability min(1, exp((beta_k - beta_{k+1}) (l(x_{k+1,m})
 * - l(x_{k,m})))), l the untempered log-probability: accept iff
 * log u < that exponent, u the 52-bit uniform of block (k*M + m, t, 0, SWAP).
 * x [K*M*D], logp [K*M] and g [K*M*D] are each chain's state with the
 * log-probability and gradient of its own replica's target; after an
 * exchange both are recomputed for the chain's replica.  swapped [K*M]
 * (may be NULL) gets 1 for both chains of an exchanged pair, 0 elsewhere. */
void orc_remc_swap(const orc_target *tgs, int64_t K, int64_t M, uint64_t seed, uint32_t t,
                   double *x, double *logp, double *g, uint8_t *swapped);

/* REMC driver: transitions t_begin .. t_begin + burnin + results - 1; each is
 * one HMC transition of every chain on its replica's target (chain c uses
 * tgs[c / M], step eps[c], the counters of chain c) followed by the exchange
 * step with swap index t.  Step-size adaptation (adapt as in
 * orc_sample_chain) works per chain on the burn-in; step sizes stay with the
 * chain slot.
 * samples [R*C*D] hold the states after the exchange of transition
 * burnin + r; tr_acc [R*C] the HMC accept flags, tr_swap [R*C] the exchange
 * flags (each may be NULL).  x and eps hold the final state / step sizes. */
int orc_remc_sample_chain(const orc_target *tgs, int64_t K, int64_t M, int32_t L, uint64_t seed,
                          uint32_t t_begin, double *x, double *eps, int64_t num_burnin,
                          int64_t num_results, int32_t adapt, double target_accept, double gamma,
                          double t0, double kappa, double rate, double *samples, uint8_t *tr_acc,
                          uint8_t *tr_swap, int32_t nthreads);

/* ---- No-U-Turn sampler (paper Sec. 2.3; Hoffman & Gelman 2014, Algorithm 3,
 * "efficient NUTS") ----
 * One transition of one chain from (x, *logp, g): momentum r0 as HMC's;
 * slice log u = log U - H0 with U the uniform of block (chain, t, 0, tag 6);
 * doubling j = 0, 1, ... picks direction v = -1 when the uniform of block
 * (chain, t, j, tag 4) is below 1/2, else +1, and builds a subtree of 2^j
 * leapfrog steps of size v eps from the trajectory's end in that direction by
 * the recursive BuildTree; a leaf counts (n' = 1) when log u <= -H and
 * continues (s' = 1) when log u < 1000 - H; merging two halves of a subtree
 * takes the second half's candidate with probability n''/(n' + n'') (uniform
 * of block (chain, t, (j * 1024 + i) * 16 + k, tag 3), i the index of the
 * subtree's last leaf within doubling j, k the merged subtree's depth) and
 * ends the subtree when (x+ - x-).r- < 0 or (x+ - x-).r+ < 0; the transition
 * takes the subtree's candidate with probability min(1, n'/n) (uniform of block
 * (chain, t, j, tag 5)) when s' = 1, then stops when s' = 0, the whole
 * trajectory makes a U-turn, or j reaches max_depth.  (x, logp, g) become the
 * chosen state's; *depth receives the number of doublings, *n_leapfrog the
 * leapfrog steps taken, *accept_stat the step-size adaptation statistic of
 * Hoffman & Gelman's Algorithm 6: the mean of min(1, exp(H0 - H)) over the
 * leaves built in the last doubling (0 when none was built).  leaf_x
 * [(2^max_depth - 1) * D] and leaf_j [2^max_depth - 1], when not NULL,
 * receive every leaf's position and doubling in build order (a check of the
 * statistic against closed forms).  Returns 1 if the state moved. */
enum { ORC_TAG_NUTS_MERGE = 3, ORC_TAG_NUTS_DIR = 4, ORC_TAG_NUTS_TOP = 5, ORC_TAG_NUTS_SLICE = 6 };
int orc_nuts_transition(const orc_target *tg, uint64_t seed, uint32_t chain, uint32_t t, double eps,
                        int32_t max_depth, double *x, double *logp, double *g, int32_t *depth,
                        int32_t *n_leapfrog, double *accept_stat, double *leaf_x, int32_t *leaf_j);

/* NUTS sample_chain (eps [C] in: initial step sizes; out: final ones):
 * transitions t_begin .. t_begin + burnin + results - 1; samples [R*C*D],
 * depth, n_leapfrog and accept-statistic traces [R*C] (each may be NULL).
 * adapt (0 none, ORC_ADAPT_DUAL_AVERAGING, ORC_ADAPT_SIMPLE): during burn-in
 * each transition's statistic updates the chain's step size as in
 * orc_sample_chain (Hoffman & Gelman Algorithm 6 for dual averaging).
 * x holds the final state. */
int orc_nuts_sample_chain(const orc_target *tg, int64_t C, uint64_t seed, uint32_t t_begin, double *x,
                          double *eps, int32_t max_depth, int64_t num_burnin, int64_t num_results,
                          int32_t adapt, double target_accept, double gamma, double t0, double kappa,
                          double rate, double *samples, int32_t *tr_depth, int32_t *tr_nleap, double *tr_stat,
                          int32_t nthreads);

#ifdef __cplusplus
}
#endif
#endif
