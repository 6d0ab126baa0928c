/*
 * oracle.c -- FP64 CPU oracle of the batched HMC transition.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h): tests/, __graft_entry__.smoke()
 * and bench.py's cpu_baseline leg are its only users.  Nothing here is
 * blocked, fused or reordered beyond the definitions it follows, so each
 * function can be checked against the cited passage by eye.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------
 * Philox4x32-10 (Salmon et al., SC'11, Sec. 3.2 and Table 2).
 * One round: two 32x32->64 products of the even counter words with the
 * round multipliers; the odd words and the key are xor-ed into the high
 * halves and the words are permuted.  The key is bumped by the Weyl
 * constants (golden ratio, sqrt(3)-1) between rounds.
 * ---------------------------------------------------------------------- */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t prod0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void philox_block(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                         uint32_t w[4])
{
    const uint32_t ctr[4] = {c0, c1, c2, c3};
    const uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, w);
}

/* Uniform in (0,1) from the top 23 bits of a word: (k + 1/2) / 2^23.  The
 * value is exactly representable in binary32 as well as binary64. */
static double uniform23(uint32_t w)
{
    return ((double)(w >> 9) + 0.5) * (1.0 / 8388608.0);
}

/* Box & Muller (1958): (u1, u2) uniform -> two independent N(0,1). */
void orc_normal4(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t tag, double z[4])
{
    uint32_t w[4];
    philox_block(seed, c0, c1, c2, tag, w);
    for (int pair = 0; pair < 2; ++pair) {
        double u1 = uniform23(w[2 * pair]);
        double u2 = uniform23(w[2 * pair + 1]);
        double radius = sqrt(-2.0 * log(u1));
        double angle = 2.0 * M_PI * u2;
        z[2 * pair] = radius * cos(angle);
        z[2 * pair + 1] = radius * sin(angle);
    }
}

/* Paper Sec. 2.1: one independent momentum per state variable per chain. */
void orc_momentum(uint64_t seed, uint32_t chain, uint32_t t, int64_t D, double *p)
{
    for (int64_t i = 0; i < D; ++i) {
        double z[4];
        orc_normal4(seed, chain, t, (uint32_t)(i / 4), ORC_TAG_MOMENTUM, z);
        p[i] = z[i % 4];
    }
}

/* Uniform in (0,1) with 52 random bits: (k + 1/2) / 2^52, k from the top
 * 26 bits of the first two words of the block (chain, t, 0, tag). */
static double uniform52(uint64_t seed, uint32_t chain, uint32_t t, uint32_t tag)
{
    uint32_t w[4];
    philox_block(seed, chain, t, 0, tag, w);
    double k = (double)(w[0] >> 6) * 67108864.0 + (double)(w[1] >> 6);
    return (k + 0.5) * (1.0 / 4503599627370496.0);
}

double orc_accept_uniform(uint64_t seed, uint32_t chain, uint32_t t)
{
    return uniform52(seed, chain, t, ORC_TAG_ACCEPT);
}

void orc_philox_many(int64_t n, const uint32_t *ctr, const uint32_t key[2], uint32_t *out)
{
    for (int64_t i = 0; i < n; ++i)
        orc_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

void orc_momentum_many(uint64_t seed, int64_t C, uint32_t t, int64_t D, double *p)
{
    for (int64_t c = 0; c < C; ++c)
        orc_momentum(seed, (uint32_t)c, t, D, p + c * D);
}

void orc_accept_uniform_many(uint64_t seed, int64_t C, uint32_t t, double *u)
{
    for (int64_t c = 0; c < C; ++c)
        u[c] = orc_accept_uniform(seed, (uint32_t)c, t);
}

/* ------------------------------------------------------------------------
 * Targets: log-probability up to a constant and its gradient.  Batch
 * semantics (paper Sec. 2): each chain's value reduces over its own event
 * axis only.
 * ---------------------------------------------------------------------- */
static double softplus(double s)
{
    /* log(1 + e^s) without overflow */
    return (s > 0.0 ? s : 0.0) + log1p(exp(-fabs(s)));
}

static double sigmoid(double s)
{
    if (s >= 0.0)
        return 1.0 / (1.0 + exp(-s));
    double e = exp(s);
    return e / (1.0 + e);
}

static double logp_grad_x(const orc_target *tg, const double *x, double *g);

/* TransformedTransitionKernel (paper Sec. 4.1) with the diagonal affine
 * bijector x = shift + scale z: the inner kernel sees the pulled-back target
 * l(x(z)) (+ the constant log-det), whose gradient is scale * grad_x l. */
double orc_logp_grad(const orc_target *tg, const double *z, double *g)
{
    if (!tg->scale)
        return logp_grad_x(tg, z, g);
    const int64_t D = tg->dim;
    double *x = (double *)calloc((size_t)(D > 0 ? D : 1), sizeof(double));
    for (int64_t i = 0; i < D; ++i)
        x[i] = (tg->shift ? tg->shift[i] : 0.0) + tg->scale[i] * z[i];
    double lp = logp_grad_x(tg, x, g);
    for (int64_t i = 0; i < D; ++i)
        g[i] *= tg->scale[i];
    free(x);
    return lp;
}

static double logp_grad_x(const orc_target *tg, const double *x, double *g)
{
    const int64_t D = tg->dim;
    double logp = 0.0;
    switch (tg->kind) {
    case ORC_STD_NORMAL:
        /* log N(x; 0, I) = -1/2 x.x */
        for (int64_t i = 0; i < D; ++i) {
            g[i] = -x[i];
            logp += -0.5 * x[i] * x[i];
        }
        break;
    case ORC_GAUSS_DIAG:
        /* precision diag(prec): -1/2 sum prec_i x_i^2 */
        for (int64_t i = 0; i < D; ++i) {
            g[i] = -tg->prec[i] * x[i];
            logp += -0.5 * tg->prec[i] * x[i] * x[i];
        }
        break;
    case ORC_GAUSS_DENSE:
        /* precision P: logp = -1/2 x^T P x, grad = -P x */
        for (int64_t i = 0; i < D; ++i) {
            double row = 0.0;
            for (int64_t j = 0; j < D; ++j)
                row += tg->prec[i * D + j] * x[j];
            g[i] = -row;
            logp += -0.5 * x[i] * row;
        }
        break;
    case ORC_LOGREG: {
        /* Bayesian logistic regression, prior N(0, s^2 I):
         *   logp = sum_n [y_n z_n - softplus(z_n)] - |theta|^2 / (2 s^2),  z = X theta
         *   grad = X^T (y - sigmoid(z)) - theta / s^2 */
        const double inv_var = 1.0 / (tg->prior_scale * tg->prior_scale);
        for (int64_t i = 0; i < D; ++i) {
            g[i] = -x[i] * inv_var;
            logp += -0.5 * x[i] * x[i] * inv_var;
        }
        for (int64_t n = 0; n < tg->n_rows; ++n) {
            const double *row = tg->X + n * D;
            double z = 0.0;
            for (int64_t i = 0; i < D; ++i)
                z += row[i] * x[i];
            logp += tg->y[n] * z - softplus(z);
            double r = tg->y[n] - sigmoid(z);
            for (int64_t i = 0; i < D; ++i)
                g[i] += row[i] * r;
        }
        break;
    }
    default:
        logp = NAN;
    }
    /* tempered target (replica exchange, paper Sec. 2.2): beta * logp */
    if (tg->beta != 1.0) {
        logp *= tg->beta;
        for (int64_t i = 0; i < D; ++i)
            g[i] *= tg->beta;
    }
    return logp;
}

/* ------------------------------------------------------------------------
 * Leapfrog (Neal 2011, Sec. 5.2.3.3): half step in momentum, full step in
 * position, half step in momentum; potential U = -logp, so -dU/dx = grad.
 * Written as L complete steps (the half kicks are not merged).
 * ---------------------------------------------------------------------- */
void orc_leapfrog(const orc_target *tg, double eps, int32_t L,
                  double *x, double *p, double *g, double *logp)
{
    const int64_t D = tg->dim;
    for (int32_t l = 0; l < L; ++l) {
        for (int64_t i = 0; i < D; ++i)
            p[i] += 0.5 * eps * g[i];
        for (int64_t i = 0; i < D; ++i)
            x[i] += eps * p[i];
        *logp = orc_logp_grad(tg, x, g);
        for (int64_t i = 0; i < D; ++i)
            p[i] += 0.5 * eps * g[i];
    }
}

static double kinetic(const double *p, int64_t D)
{
    /* identity mass matrix: K(p) = 1/2 p.p */
    double k = 0.0;
    for (int64_t i = 0; i < D; ++i)
        k += 0.5 * p[i] * p[i];
    return k;
}

/* Paper Sec. 2.1 (HMC case study) with the Metropolis-Hastings correction
 * of Sec. 4.1; H(x, p) = -logp(x) + K(p). */
int orc_transition(const orc_target *tg, uint64_t seed, uint32_t chain, uint32_t t,
                   int32_t L, double eps, double *x, double *logp, double *g,
                   double *x_prop, double *p_prop, double *logp_prop,
                   double *delta_h, double *log_accept_ratio)
{
    const int64_t D = tg->dim;
    double *buf = (double *)malloc(sizeof(double) * 3 * (size_t)D);
    double *xn = buf, *pn = buf + D, *gn = buf + 2 * D;

    /* 1. momentum draw */
    orc_momentum(seed, chain, t, D, pn);
    double h0 = -(*logp) + kinetic(pn, D);

    /* 2. trajectory from the current state with its cached gradient */
    memcpy(xn, x, sizeof(double) * (size_t)D);
    memcpy(gn, g, sizeof(double) * (size_t)D);
    double lp = *logp;
    orc_leapfrog(tg, eps, L, xn, pn, gn, &lp);
    double h1 = -lp + kinetic(pn, D);
    double dh = h1 - h0;

    /* 3. Metropolis-Hastings: accept iff log u < -dH; NaN/+inf dH rejects */
    double lar = -dh;
    if (isnan(dh) || (isinf(dh) && dh > 0))
        lar = -INFINITY;
    double u = orc_accept_uniform(seed, chain, t);
    int accepted = log(u) < lar;

    if (x_prop) memcpy(x_prop, xn, sizeof(double) * (size_t)D);
    if (p_prop) memcpy(p_prop, pn, sizeof(double) * (size_t)D);
    if (logp_prop) *logp_prop = lp;
    if (delta_h) *delta_h = dh;
    if (log_accept_ratio) *log_accept_ratio = lar;

    /* 4. select (the paper's vectorised where: rejected chains keep state) */
    if (accepted) {
        memcpy(x, xn, sizeof(double) * (size_t)D);
        memcpy(g, gn, sizeof(double) * (size_t)D);
        *logp = lp;
    }
    free(buf);
    return accepted;
}

/* ------------------------------------------------------------------------
 * Dual averaging (Hoffman & Gelman 2014, Sec. 3.2, eq. 6):
 *   Hbar_m     = (1 - 1/(m + t0)) Hbar_{m-1} + (delta - alpha_m) / (m + t0)
 *   log eps_m  = mu - sqrt(m) / gamma * Hbar_m
 *   log ebar_m = m^-kappa log eps_m + (1 - m^-kappa) log ebar_{m-1}
 * with mu = log(10 eps0), Hbar_0 = 0, ebar_0 = 1.
 * ---------------------------------------------------------------------- */
/* Paper Sec. 4.1 names SimpleStepSizeAdaptation as a wrapper that tunes the
 * inner kernel's step size during burn-in: grow it after a transition whose
 * accept statistic is above the target, shrink it otherwise. */
double orc_simple_adapt(double eps, double alpha, double target_accept, double rate)
{
    return alpha > target_accept ? eps * (1.0 + rate) : eps / (1.0 + rate);
}

void orc_dual_avg_init(orc_dual_avg *s, double eps0)
{
    s->log_eps = log(eps0);
    s->hbar = 0.0;
    s->log_eps_bar = 0.0;
    s->mu = log(10.0 * eps0);
}

void orc_dual_avg_update(orc_dual_avg *s, int64_t m, double alpha, double target_accept,
                         double gamma, double t0, double kappa)
{
    double md = (double)m;
    double w = 1.0 / (md + t0);
    s->hbar = (1.0 - w) * s->hbar + w * (target_accept - alpha);
    s->log_eps = s->mu - sqrt(md) / gamma * s->hbar;
    double eta = pow(md, -kappa);
    s->log_eps_bar = eta * s->log_eps + (1.0 - eta) * s->log_eps_bar;
}

/* ------------------------------------------------------------------------
 * Batched entry points.  Chains are independent (paper Sec. 2), so the
 * OpenMP loop runs each chain on its own; results do not depend on the
 * thread count.
 * ---------------------------------------------------------------------- */
static void set_threads(int32_t nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

void orc_bootstrap(const orc_target *tg, int64_t C, const double *x, double *logp, double *g,
                   int32_t nthreads)
{
    const int64_t D = tg->dim;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < C; ++c)
        logp[c] = orc_logp_grad(tg, x + c * D, g + c * D);
}

void orc_step(const orc_target *tg, int64_t C, int32_t L, uint64_t seed, uint32_t t,
              const double *eps, double *x, double *logp, double *g,
              double *x_prop, double *p_prop, double *logp_prop, double *delta_h,
              double *log_accept_ratio, uint8_t *accepted, int32_t nthreads)
{
    const int64_t D = tg->dim;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < C; ++c) {
        int a = orc_transition(tg, seed, (uint32_t)c, t, L, eps[c], x + c * D, logp + c, g + c * D,
                               x_prop ? x_prop + c * D : NULL, p_prop ? p_prop + c * D : NULL,
                               logp_prop ? logp_prop + c : NULL, delta_h ? delta_h + c : NULL,
                               log_accept_ratio ? log_accept_ratio + c : NULL);
        if (accepted)
            accepted[c] = (uint8_t)a;
    }
}

/* Paper Sec. 4.2 (sample_chain): burn-in transitions are not stored; the
 * state after transition burnin + r is kept sample r; tracing records the
 * kernel results of each kept transition. */
int orc_sample_chain(const orc_target *tg, int64_t C, int32_t L, uint64_t seed,
                     uint32_t t_begin, double *x, double *eps,
                     int64_t num_burnin, int64_t num_results,
                     int32_t adapt, double target_accept, double gamma, double t0, double kappa,
                     double rate, double *samples, double *tr_step, uint8_t *tr_acc, double *tr_lar,
                     double *tr_logp, int32_t nthreads)
{
    const int64_t D = tg->dim;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < C; ++c) {
        double *xc = x + c * D;
        double *gc = (double *)malloc(sizeof(double) * (size_t)D);
        double lp = orc_logp_grad(tg, xc, gc);   /* bootstrap */
        orc_dual_avg da;
        orc_dual_avg_init(&da, eps[c]);
        double step = eps[c];
        for (int64_t i = 0; i < num_burnin + num_results; ++i) {
            uint32_t t = t_begin + (uint32_t)i;
            double lar;
            int a = orc_transition(tg, seed, (uint32_t)c, t, L, step, xc, &lp, gc,
                                   NULL, NULL, NULL, NULL, &lar);
            double used = step;
            if (adapt && i < num_burnin) {
                double alpha = lar < 0.0 ? exp(lar) : 1.0;   /* min(1, e^-dH); 0 for NaN */
                if (adapt == ORC_ADAPT_SIMPLE) {
                    step = orc_simple_adapt(step, alpha, target_accept, rate);
                } else {
                    orc_dual_avg_update(&da, i + 1, alpha, target_accept, gamma, t0, kappa);
                    step = (i + 1 < num_burnin) ? exp(da.log_eps) : exp(da.log_eps_bar);
                }
            }
            if (i >= num_burnin) {
                int64_t r = i - num_burnin;
                if (samples)
                    memcpy(samples + (r * C + c) * D, xc, sizeof(double) * (size_t)D);
                if (tr_step) tr_step[r * C + c] = used;
                if (tr_acc) tr_acc[r * C + c] = (uint8_t)a;
                if (tr_lar) tr_lar[r * C + c] = lar;
                if (tr_logp) tr_logp[r * C + c] = lp;
            }
        }
        eps[c] = step;
        free(gc);
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Replica exchange (paper Sec. 2.2): replica k targets p(x)^beta_k; the
 * exchange of the states x_a (replica a) and x_b (replica b) is a
 * Metropolis-Hastings move on the product of the replica targets, with ratio
 *   p(x_b)^beta_a p(x_a)^beta_b / (p(x_a)^beta_a p(x_b)^beta_b)
 *   = exp((beta_a - beta_b) (l(x_b) - l(x_a))).
 * ---------------------------------------------------------------------- */
void orc_remc_swap(const orc_target *tgs, int64_t K, int64_t M, uint64_t seed, uint32_t t,
                   double *x, double *logp, double *g, uint8_t *swapped)
{
    const int64_t D = tgs[0].dim;
    orc_target base = tgs[0];
    base.beta = 1.0;
    double *tmp = (double *)malloc(sizeof(double) * (size_t)D);
    if (swapped)
        memset(swapped, 0, (size_t)(K * M));
    for (int64_t k = (int64_t)(t % 2); k + 1 < K; k += 2) {
        for (int64_t m = 0; m < M; ++m) {
            const int64_t a = k * M + m, b = (k + 1) * M + m;
            double la = orc_logp_grad(&base, x + a * D, tmp);   /* untempered l(x_a) */
            double lb = orc_logp_grad(&base, x + b * D, tmp);
            double log_ratio = (tgs[k].beta - tgs[k + 1].beta) * (lb - la);
            double u = uniform52(seed, (uint32_t)a, t, ORC_TAG_SWAP);
            if (!(log(u) < log_ratio))
                continue;   /* rejected (also when the ratio is NaN) */
            for (int64_t i = 0; i < D; ++i) {
                double v = x[a * D + i];
                x[a * D + i] = x[b * D + i];
                x[b * D + i] = v;
            }
            /* each chain's cached values belong to its own replica's target */
            logp[a] = orc_logp_grad(&tgs[k], x + a * D, g + a * D);
            logp[b] = orc_logp_grad(&tgs[k + 1], x + b * D, g + b * D);
            if (swapped)
                swapped[a] = swapped[b] = 1;
        }
    }
    free(tmp);
}

int orc_remc_sample_chain(const orc_target *tgs, int64_t K, int64_t M, int32_t L, uint64_t seed,
                          uint32_t t_begin, double *x, double *eps, int64_t num_burnin,
                          int64_t num_results, int32_t adapt, double target_accept, double gamma,
                          double t0, double kappa, double rate, double *samples, uint8_t *tr_acc,
                          uint8_t *tr_swap, int32_t nthreads)
{
    const int64_t D = tgs[0].dim, C = K * M;
    double *logp = (double *)malloc(sizeof(double) * (size_t)C);
    double *g = (double *)malloc(sizeof(double) * (size_t)(C * D));
    orc_dual_avg *da = (orc_dual_avg *)malloc(sizeof(orc_dual_avg) * (size_t)C);
    uint8_t *acc = (uint8_t *)malloc((size_t)C);
    uint8_t *swp = (uint8_t *)malloc((size_t)C);
    set_threads(nthreads);
    for (int64_t c = 0; c < C; ++c) {   /* bootstrap on each chain's own replica */
        logp[c] = orc_logp_grad(&tgs[c / M], x + c * D, g + c * D);
        orc_dual_avg_init(&da[c], eps[c]);
    }
    for (int64_t i = 0; i < num_burnin + num_results; ++i) {
        const uint32_t t = t_begin + (uint32_t)i;
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t c = 0; c < C; ++c) {
            double lar;
            acc[c] = (uint8_t)orc_transition(&tgs[c / M], seed, (uint32_t)c, t, L, eps[c], x + c * D,
                                             &logp[c], g + c * D, NULL, NULL, NULL, NULL, &lar);
            if (adapt && i < num_burnin) {
                double alpha = lar < 0.0 ? exp(lar) : 1.0;
                if (adapt == ORC_ADAPT_SIMPLE) {
                    eps[c] = orc_simple_adapt(eps[c], alpha, target_accept, rate);
                } else {
                    orc_dual_avg_update(&da[c], i + 1, alpha, target_accept, gamma, t0, kappa);
                    eps[c] = (i + 1 < num_burnin) ? exp(da[c].log_eps) : exp(da[c].log_eps_bar);
                }
            }
        }
        orc_remc_swap(tgs, K, M, seed, t, x, logp, g, swp);
        if (i >= num_burnin) {
            const int64_t r = i - num_burnin;
            if (samples)
                memcpy(samples + r * C * D, x, sizeof(double) * (size_t)(C * D));
            if (tr_acc)
                memcpy(tr_acc + r * C, acc, (size_t)C);
            if (tr_swap)
                memcpy(tr_swap + r * C, swp, (size_t)C);
        }
    }
    free(logp);
    free(g);
    free(da);
    free(acc);
    free(swp);
    return 0;
}

/* ------------------------------------------------------------------------
 * No-U-Turn sampler, Hoffman & Gelman (2014), Algorithm 3 (the paper's
 * Sec. 2.3 case study vectorises this recursion).  A state carries its
 * position, momentum, gradient and log-probability so that each leapfrog
 * step starts from the cached gradient.
 * ---------------------------------------------------------------------- */
typedef struct {
    double *x, *r, *g;
    double logp;
} nuts_pt;

typedef struct {
    const orc_target *tg;
    uint64_t seed;
    uint32_t chain, t;
    int32_t doubling;      /* j of the top-level loop */
    int32_t leaves;        /* leaves built so far in this doubling */
    int32_t n_leapfrog;
    double eps, log_u;
    int64_t D;
    double H0;             /* energy of the starting point */
    double alpha;          /* sum of min(1, exp(H0 - H)) over this doubling's leaves */
    int32_t n_alpha;       /* and their number */
    double *leaf_x;        /* optional record of every leaf's position, in build order */
    int32_t *leaf_j;       /* and the doubling it belongs to */
} nuts_ctx;

static nuts_pt pt_new(int64_t D)
{
    nuts_pt p;
    p.x = (double *)malloc(sizeof(double) * (size_t)D);
    p.r = (double *)malloc(sizeof(double) * (size_t)D);
    p.g = (double *)malloc(sizeof(double) * (size_t)D);
    p.logp = 0.0;
    return p;
}

static void pt_free(nuts_pt *p)
{
    free(p->x);
    free(p->r);
    free(p->g);
}

static void pt_copy(nuts_pt *dst, const nuts_pt *src, int64_t D)
{
    memcpy(dst->x, src->x, sizeof(double) * (size_t)D);
    memcpy(dst->r, src->r, sizeof(double) * (size_t)D);
    memcpy(dst->g, src->g, sizeof(double) * (size_t)D);
    dst->logp = src->logp;
}

/* 52-bit uniform of block (chain, t, block, tag), as the accept uniform */
static double uniform52_block(uint64_t seed, uint32_t chain, uint32_t t, uint32_t block, uint32_t tag)
{
    uint32_t w[4];
    philox_block(seed, chain, t, block, tag, w);
    double k = (double)(w[0] >> 6) * 67108864.0 + (double)(w[1] >> 6);
    return (k + 0.5) * (1.0 / 4503599627370496.0);
}

/* no-U-turn indicator of a span from its backward end m to its forward end p */
static int no_uturn(const nuts_pt *m, const nuts_pt *p, int64_t D)
{
    double dm = 0.0, dp = 0.0;
    for (int64_t i = 0; i < D; ++i) {
        double dx = p->x[i] - m->x[i];
        dm += dx * m->r[i];
        dp += dx * p->r[i];
    }
    return dm >= 0.0 && dp >= 0.0;
}

/* BuildTree(state, v, depth): extends from `edge` (updated in place to the
 * subtree's far end in direction v); `cand` receives the subtree's candidate;
 * the subtree's near end (first leaf) is written to `first` when not NULL. */
static void nuts_build(nuts_ctx *c, nuts_pt *edge, int v, int depth, nuts_pt *cand, nuts_pt *first,
                       int32_t *n_out, int32_t *s_out)
{
    const int64_t D = c->D;
    if (depth == 0) {
        orc_leapfrog(c->tg, v * c->eps, 1, edge->x, edge->r, edge->g, &edge->logp);
        c->n_leapfrog += 1;
        c->leaves += 1;
        double H = -edge->logp + kinetic(edge->r, D);
        *n_out = (c->log_u <= -H) ? 1 : 0;
        *s_out = (c->log_u < 1000.0 - H) ? 1 : 0;     /* NaN H fails both */
        /* Algorithm 6's per-leaf acceptance probability (NaN H counts 0) */
        double dh0 = c->H0 - H;
        c->alpha += isnan(dh0) ? 0.0 : (dh0 >= 0.0 ? 1.0 : exp(dh0));
        c->n_alpha += 1;
        if (c->leaf_x) {
            memcpy(c->leaf_x + (int64_t)(c->n_leapfrog - 1) * D, edge->x, sizeof(double) * (size_t)D);
            c->leaf_j[c->n_leapfrog - 1] = c->doubling;
        }
        pt_copy(cand, edge, D);
        if (first)
            pt_copy(first, edge, D);
        return;
    }
    nuts_pt first_half_start = pt_new(D);
    int32_t n1, s1;
    nuts_build(c, edge, v, depth - 1, cand, &first_half_start, &n1, &s1);
    if (first)
        pt_copy(first, &first_half_start, D);
    if (s1) {
        nuts_pt cand2 = pt_new(D);
        int32_t n2, s2;
        nuts_build(c, edge, v, depth - 1, &cand2, NULL, &n2, &s2);
        /* merged at the last leaf of the second half */
        const uint32_t i = (uint32_t)(c->leaves - 1);
        const uint32_t block = ((uint32_t)c->doubling * 1024u + i) * 16u + (uint32_t)depth;
        const double u = uniform52_block(c->seed, c->chain, c->t, block, ORC_TAG_NUTS_MERGE);
        if (n1 + n2 > 0 && u < (double)n2 / (double)(n1 + n2))
            pt_copy(cand, &cand2, D);
        /* span of the merged subtree: from its first leaf to its last (= edge) */
        const nuts_pt *m = (v > 0) ? &first_half_start : edge;
        const nuts_pt *p = (v > 0) ? edge : &first_half_start;
        s1 = s2 && no_uturn(m, p, D);
        n1 += n2;
        pt_free(&cand2);
    }
    pt_free(&first_half_start);
    *n_out = n1;
    *s_out = s1;
}

int orc_nuts_transition(const orc_target *tg, uint64_t seed, uint32_t chain, uint32_t t, double eps,
                        int32_t max_depth, double *x, double *logp, double *g, int32_t *depth,
                        int32_t *n_leapfrog, double *accept_stat, double *leaf_x, int32_t *leaf_j)
{
    const int64_t D = tg->dim;
    nuts_ctx c = {tg, seed, chain, t, 0, 0, 0, eps, 0.0, D, 0.0, 0.0, 0, leaf_x, leaf_j};
    nuts_pt minus = pt_new(D), plus = pt_new(D), cand = pt_new(D), chosen = pt_new(D);
    memcpy(minus.x, x, sizeof(double) * (size_t)D);
    memcpy(minus.g, g, sizeof(double) * (size_t)D);
    minus.logp = *logp;
    orc_momentum(seed, chain, t, D, minus.r);
    pt_copy(&plus, &minus, D);
    pt_copy(&chosen, &minus, D);
    const double H0 = -(*logp) + kinetic(minus.r, D);
    c.H0 = H0;
    c.log_u = log(uniform52_block(seed, chain, t, 0, ORC_TAG_NUTS_SLICE)) - H0;
    int32_t n = 1, s = 1, j = 0, moved = 0;
    while (s && j < max_depth) {
        const int v = uniform52_block(seed, chain, t, (uint32_t)j, ORC_TAG_NUTS_DIR) < 0.5 ? -1 : 1;
        c.doubling = j;
        c.leaves = 0;
        c.alpha = 0.0;             /* the statistic is the last doubling's */
        c.n_alpha = 0;
        int32_t n1, s1;
        nuts_build(&c, v > 0 ? &plus : &minus, v, j, &cand, NULL, &n1, &s1);
        if (s1 && uniform52_block(seed, chain, t, (uint32_t)j, ORC_TAG_NUTS_TOP) < (double)n1 / (double)n) {
            pt_copy(&chosen, &cand, D);
            moved = 1;
        }
        n += n1;
        s = s1 && no_uturn(&minus, &plus, D);
        j += 1;
    }
    memcpy(x, chosen.x, sizeof(double) * (size_t)D);
    memcpy(g, chosen.g, sizeof(double) * (size_t)D);
    *logp = chosen.logp;
    if (depth) *depth = j;
    if (n_leapfrog) *n_leapfrog = c.n_leapfrog;
    if (accept_stat) *accept_stat = c.n_alpha > 0 ? c.alpha / (double)c.n_alpha : 0.0;
    pt_free(&minus);
    pt_free(&plus);
    pt_free(&cand);
    pt_free(&chosen);
    return moved;
}

int orc_nuts_sample_chain(const orc_target *tg, int64_t C, uint64_t seed, uint32_t t_begin, double *x,
                          double *eps, int32_t max_depth, int64_t num_burnin, int64_t num_results,
                          int32_t adapt, double target_accept, double gamma, double t0, double kappa,
                          double rate, double *samples, int32_t *tr_depth, int32_t *tr_nleap, double *tr_stat,
                          int32_t nthreads)
{
    const int64_t D = tg->dim;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < C; ++c) {
        double *xc = x + c * D;
        double *gc = (double *)malloc(sizeof(double) * (size_t)D);
        double lp = orc_logp_grad(tg, xc, gc);
        orc_dual_avg da;
        orc_dual_avg_init(&da, eps[c]);
        for (int64_t i = 0; i < num_burnin + num_results; ++i) {
            int32_t dep, nl;
            double stat;
            orc_nuts_transition(tg, seed, (uint32_t)c, t_begin + (uint32_t)i, eps[c], max_depth, xc, &lp, gc,
                                &dep, &nl, &stat, NULL, NULL);
            /* Algorithm 6: the step size of the next transition from the
             * statistic of this one, during burn-in only */
            if (adapt && i < num_burnin) {
                if (adapt == ORC_ADAPT_SIMPLE) {
                    eps[c] = orc_simple_adapt(eps[c], stat, target_accept, rate);
                } else {
                    orc_dual_avg_update(&da, i + 1, stat, target_accept, gamma, t0, kappa);
                    eps[c] = (i + 1 < num_burnin) ? exp(da.log_eps) : exp(da.log_eps_bar);
                }
            }
            if (i >= num_burnin) {
                int64_t r = i - num_burnin;
                if (samples)
                    memcpy(samples + (r * C + c) * D, xc, sizeof(double) * (size_t)D);
                if (tr_depth) tr_depth[r * C + c] = dep;
                if (tr_nleap) tr_nleap[r * C + c] = nl;
                if (tr_stat) tr_stat[r * C + c] = stat;
            }
        }
        free(gc);
    }
    return 0;
}
