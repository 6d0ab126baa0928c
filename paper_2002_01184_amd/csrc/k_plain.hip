// k_plain.hip -- the plain form of the HMC transition: one kernel per phase,
// the trajectory state in HBM between leapfrog steps ([C, D] row-major).
//
//   k_begin       momentum draw, initial energy H0, first half kick      (Sec. 2.1)
//   leapfrog x L  drift x += eps p, target gradient, kick p += eps g
//   k_end         energy at the trajectory end, dH, Metropolis test,
//                 per-chain select, dual averaging, sample/trace writes  (Sec. 2.1, 4.2)
//   k_tick        t += 1 (device-resident, so a captured graph replays unchanged)
//   k_remc_exchange  replica exchange between neighbouring temperatures (Sec. 2.2)
//
// Inverse temperatures (replica exchange): chain c targets beta_c logp.  The
// cached logp and gradient stay those of the untempered target; beta_c
// multiplies the gradient in every kick and logp in both energies, so the
// exchange step moves states without recomputing anything.  With no
// temperatures set (ws.beta == NULL) every factor is exactly 1.
//
// Transformed kernel (diagonal affine bijector x = shift + scale z, Sec. 4.1):
// the momentum is that of z, so scale_d multiplies eps in the drift and the
// kick of dimension d; with no transform (ws.scale == NULL) nothing changes.
//
// Gradient kernels:
//   elementwise   N(0, I) and diagonal Gaussians: one thread per (chain, dim)
//   dense         g = -P x on MFMA (v_mfma_f32_16x16x4f32), 16 chains per workgroup
//   logreg        s = X theta, r = y - sigmoid(s), g = X^T r - theta/s^2 on MFMA,
//                 rows split across workgroups with partials reduced in a fixed order
#include "hmc_internal.hpp"

namespace hmc {

typedef float floatx4 __attribute__((ext_vector_type(4)));

__global__ void k_set_ctrl(Ctrl* dst, Ctrl v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = v;
}

__global__ void k_tick(Ctrl* c) {
    if (threadIdx.x == 0 && blockIdx.x == 0) c->t += 1;
}

// ---------------------------------------------------------------------------
// Chain-group kernels: G lanes of a wavefront share one chain; each lane owns
// the 4-dim Philox blocks b = lane, lane + G, ...
// ---------------------------------------------------------------------------
template <typename T, int G>
__device__ __forceinline__ void begin_body(const PlainArgs& a, int64_t blk) {
    const int64_t gid = blk * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x % G;
    const int64_t c = gid / G;
    const bool active = c < a.C;
    const int64_t D = a.tg.D;
    const uint32_t t = (uint32_t)a.ws.ctrl->t;
    const T* x = (const T*)a.ws.x;
    const T* g = (const T*)a.ws.g;
    T* xq = (T*)a.ws.xq;
    T* pq = (T*)a.ws.pq;
    const double bt = (active && a.ws.beta) ? a.ws.beta[c] : 1.0;
    const T half_eps = active ? (T)(0.5 * a.ws.eps[c] * bt) : (T)0;
    double k0 = 0.0;
    const int64_t nblk = (D + 3) / 4;
    if (active) {
        for (int64_t b = lane; b < nblk; b += G) {
            T z[4];
            momentum4<T>(a.key, (uint32_t)c, t, (uint32_t)b, z, 4 * b + 2 < D);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t d = 4 * b + j;
                if (d < D) {
                    const int64_t i = c * D + d;
                    xq[i] = x[i];
                    k0 += 0.5 * (double)z[j] * (double)z[j];
                    const T hk = a.ws.scale ? (T)(0.5 * a.ws.eps[c] * bt * a.ws.scale[d]) : half_eps;
                    pq[i] = z[j] + hk * g[i];
                }
            }
        }
    }
    k0 = group_sum<G>(k0);
    if (active && lane == 0) a.ws.h0[c] = -(bt * a.ws.logp[c]) + k0;
}

template <typename T, int G>
__global__ __launch_bounds__(256) void k_begin(PlainArgs a) { begin_body<T, G>(a, blockIdx.x); }

// logp at (x, g) from the closed form that remains after the gradient kernel:
// Gaussians 1/2 x.g; logistic regression -|x|^2/(2 s^2) + the data part in lpq.
template <typename T, int G>
__device__ __forceinline__ double chain_logp(const PlainArgs& a, int64_t c, bool active, const T* x, const T* g,
                                             int lane) {
    const int64_t D = a.tg.D;
    double s = 0.0;
    if (active) {
        if (a.tg.kind == HMC_TGT_LOGREG) {
            for (int64_t d = lane; d < D; d += G) {
                const double v = (double)x[c * D + d];
                s += -0.5 * v * v * a.tg.inv_var;
            }
        } else {
            for (int64_t d = lane; d < D; d += G)
                s += 0.5 * (double)x[c * D + d] * (double)g[c * D + d];
        }
    }
    s = group_sum<G>(s);
    if (active && a.tg.kind == HMC_TGT_LOGREG) s += a.ws.lpq[c];
    return s;
}

template <typename T, int G>
__global__ __launch_bounds__(256) void k_logp_finish(PlainArgs a) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x % G;
    const int64_t c = gid / G;
    const bool active = c < a.C;
    const double lp = chain_logp<T, G>(a, c, active, (const T*)a.ws.x, (const T*)a.ws.g, lane);
    if (active && lane == 0) a.ws.logp[c] = lp;
}

__device__ __forceinline__ void end_scalars(const PlainArgs& a, const Ctrl& ct, int64_t c, int64_t i, bool acc,
                                            double lar, double dh, double lp_new, double eps_used);

template <typename T, int G>
__device__ __forceinline__ void end_body(const PlainArgs& a, int64_t blk) {
    const int64_t gid = blk * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x % G;
    const int64_t c = gid / G;
    const bool active = c < a.C;
    const int64_t D = a.tg.D;
    const Ctrl& ct = *a.ws.ctrl;
    const uint64_t t = ct.t;
    T* x = (T*)a.ws.x;
    T* g = (T*)a.ws.g;
    const T* xq = (const T*)a.ws.xq;
    const T* pq = (const T*)a.ws.pq;
    const T* gq = (const T*)a.ws.gq;

    double k1 = 0.0;
    if (active)
        for (int64_t d = lane; d < D; d += G) {
            const double p = (double)pq[c * D + d];
            k1 += 0.5 * p * p;
        }
    k1 = group_sum<G>(k1);
    const double lp1 = chain_logp<T, G>(a, c, active, xq, gq, lane);
    if (!active) return;

    const double bt = a.ws.beta ? a.ws.beta[c] : 1.0;
    const double dh = (-(bt * lp1) + k1) - a.ws.h0[c];
    const double lar = log_accept_ratio_of(dh);
    const bool acc = log_accept_uniform(a.key, (uint32_t)c, (uint32_t)t) < lar;

    // per-chain select (vectorised where of the paper, Sec. 2.1)
    if (acc)
        for (int64_t d = lane; d < D; d += G) {
            x[c * D + d] = xq[c * D + d];
            g[c * D + d] = gq[c * D + d];
        }
    const double lp_new = acc ? lp1 : a.ws.logp[c];
    const double eps_used = a.ws.eps[c];
    const int64_t i = (int64_t)(t - ct.t_begin);

    if (ct.samples && i >= ct.n_burnin && i < ct.n_burnin + ct.n_results) {
        const int64_t r = i - ct.n_burnin;
        T* smp = (T*)ct.samples + (r * a.C + c) * D;
        for (int64_t d = lane; d < D; d += G) smp[d] = x[c * D + d];
    }
    if (lane != 0) return;
    a.ws.logp[c] = lp_new;
    end_scalars(a, ct, c, i, acc, lar, dh, lp_new, eps_used);
}

template <typename T, int G>
__global__ __launch_bounds__(256) void k_end(PlainArgs a) { end_body<T, G>(a, blockIdx.x); }

// The per-chain scalars at the end of transition i of the call (one lane per
// chain): step-size adaptation during the burn-in, the trace row of a kept
// transition, and the hmc_step outputs.
__device__ __forceinline__ void end_scalars(const PlainArgs& a, const Ctrl& ct, int64_t c, int64_t i, bool acc,
                                            double lar, double dh, double lp_new, double eps_used) {
    if (ct.adapt && i < ct.n_burnin) {
        const double alpha = lar < 0.0 ? exp(lar) : 1.0;
        if (ct.adapt_kind == HMC_ADAPT_SIMPLE) {
            a.ws.eps[c] = simple_adapt(eps_used, alpha, ct.target_accept, ct.rate);
        } else {
            DualAvg s = a.ws.da[c];
            const double log_eps = dual_avg_update(s, (double)(i + 1), alpha, ct.target_accept, ct.gamma, ct.t0,
                                                   ct.kappa);
            a.ws.da[c] = s;
            a.ws.eps[c] = (i + 1 < ct.n_burnin) ? exp(log_eps) : exp(s.log_eps_bar);
        }
    }
    if (i >= ct.n_burnin && i < ct.n_burnin + ct.n_results) {
        const int64_t r = i - ct.n_burnin;
        if (ct.tr_step) ct.tr_step[r * a.C + c] = eps_used;
        if (ct.tr_acc) ct.tr_acc[r * a.C + c] = acc ? 1 : 0;
        if (ct.tr_lar) ct.tr_lar[r * a.C + c] = lar;
        if (ct.tr_logp) ct.tr_logp[r * a.C + c] = lp_new;
    }
    if (ct.out_acc) ct.out_acc[c] = acc ? 1 : 0;
    if (ct.out_lar) ct.out_lar[c] = lar;
    if (ct.out_logp) ct.out_logp[c] = lp_new;
    if (ct.out_dh) ct.out_dh[c] = dh;
}

// proposal copies for hmc_step outputs (kept out of k_end's hot loop)
template <typename T>
__global__ __launch_bounds__(256) void k_copy_proposal(PlainArgs a) {
    const Ctrl& ct = *a.ws.ctrl;
    const int64_t n = a.C * a.tg.D;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (ct.out_xprop) ((T*)ct.out_xprop)[i] = ((const T*)a.ws.xq)[i];
        if (ct.out_pprop) ((T*)ct.out_pprop)[i] = ((const T*)a.ws.pq)[i];
    }
}

// Replica exchange (Sec. 2.2): chain c = k M + m is chain m of replica k.  The
// pairs (k, k+1) of the parity class of t exchange the states (x, g, logp) of
// chains k M + m and (k+1) M + m with probability
// min(1, exp((beta_k - beta_{k+1}) (logp_{k+1} - logp_k))) (untempered logp),
// testing log u < that exponent with the 52-bit uniform of block
// (k M + m, t, 0, SWAP).  Step sizes and adaptation state stay with the slot.
// One wavefront per pair, then one per chain of the unpaired replicas (0 when
// the parity is odd, the last ones when too few remain): every chain gets its
// flag (0 outside the pairs) and, when sample_row is given, its post-exchange
// state written there, so the step needs no fill or copy besides.
template <typename T>
__global__ __launch_bounds__(256) void k_remc_exchange(PlainArgs a, int64_t K, int64_t M, int32_t parity, uint32_t t,
                                                       uint8_t* swapped, T* sample_row) {
    const int64_t item = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t npairs = (K - parity) / 2;      // k = parity, parity + 2, ... with k + 1 < K
    const int64_t D = a.tg.D;
    T* x = (T*)a.ws.x;
    T* g = (T*)a.ws.g;
    if (item < npairs * M) {
        const int64_t k = parity + 2 * (item / M), m = item % M;
        const int64_t ca = k * M + m, cb = (k + 1) * M + m;
        const double ba = a.ws.beta ? a.ws.beta[ca] : 1.0, bb = a.ws.beta ? a.ws.beta[cb] : 1.0;
        const double la = a.ws.logp[ca], lb = a.ws.logp[cb];
        const bool acc = log_uniform52(a.key, (uint32_t)ca, t, TAG_SWAP) < (ba - bb) * (lb - la);
        if (swapped && lane == 0) {
            swapped[ca] = acc ? 1 : 0;
            swapped[cb] = acc ? 1 : 0;
        }
        for (int64_t d = lane; d < D; d += 64) {
            const T xa = x[ca * D + d], xb = x[cb * D + d];
            if (acc) {
                x[ca * D + d] = xb;
                x[cb * D + d] = xa;
                const T ga = g[ca * D + d], gb = g[cb * D + d];
                g[ca * D + d] = gb;
                g[cb * D + d] = ga;
            }
            if (sample_row) {
                sample_row[ca * D + d] = acc ? xb : xa;
                sample_row[cb * D + d] = acc ? xa : xb;
            }
        }
        if (acc && lane == 0) {
            a.ws.logp[ca] = lb;
            a.ws.logp[cb] = la;
        }
        return;
    }
    // unpaired replicas: 0 if the parity is odd, then parity + 2 npairs .. K - 1
    const int64_t u = item - npairs * M, kr = u / M, m = u % M;
    if (kr >= K - 2 * npairs) return;
    const int64_t k = parity ? (kr == 0 ? 0 : 1 + 2 * npairs + (kr - 1)) : 2 * npairs + kr;
    const int64_t c = k * M + m;
    if (swapped && lane == 0) swapped[c] = 0;
    if (sample_row)
        for (int64_t d = lane; d < D; d += 64) sample_row[c * D + d] = x[c * D + d];
}

template <typename T>
__global__ __launch_bounds__(256) void k_da_init(PlainArgs a) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.C) return;
    DualAvg s;
    s.hbar = 0.0;
    s.log_eps_bar = 0.0;
    s.mu = log(10.0 * a.ws.eps[c]);
    a.ws.da[c] = s;
}

// ---------------------------------------------------------------------------
// Elementwise targets: one thread per (chain, dim).  mode bits: 1 = drift
// before the gradient, 2 = kick after it; kick_scale is 1 or 1/2 (last step).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_elem_leapfrog(PlainArgs a, const T* __restrict__ xs, T* __restrict__ xd,
                                                       T* __restrict__ pd, T* __restrict__ gd, int mode,
                                                       double kick_scale) {
    const int64_t D = a.tg.D;
    const int64_t n = a.C * D;
    const T* prec = (const T*)a.tg.prec;
    const bool diag = a.tg.kind == HMC_TGT_GAUSS_DIAG;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = i / D;
        const double sd = a.ws.scale ? a.ws.scale[i - c * D] : 1.0;
        const T eps = a.ws.scale ? (T)(a.ws.eps[c] * sd) : (T)a.ws.eps[c];
        T x = xs[i];
        T p = (mode & 3) ? pd[i] : (T)0;
        if (mode & 1) x = fma(eps, p, x);
        const T gv = diag ? -prec[i - c * D] * x : -x;
        if (mode & 2) p = fma((T)(kick_scale * a.ws.eps[c] * (a.ws.beta ? a.ws.beta[c] : 1.0) * sd), gv, p);
        if (mode & 1) xd[i] = x;
        if (mode & 2) pd[i] = p;
        if (gd) gd[i] = gv;
    }
}

// ---------------------------------------------------------------------------
// Element-wise targets, merged transition: L launches per transition, each
// one leapfrog step that reads and writes the trajectory once.
//   k_elem_first  momentum draw, H0, first half kick, then leapfrog step 1
//   k_elem_mid    leapfrog steps 2 .. L-1 on (xq, pq)
//   k_elem_last   leapfrog step L, energy at the end, Metropolis test; an
//                 accepted chain writes its new x, g and logp from registers,
//                 a rejected one leaves them as they are (no select copy)
// G lanes per chain (as chain_group); the arithmetic and the order of every
// FP64 sum are those of k_begin / k_elem_leapfrog / k_end, so both sequences
// give bitwise the same chains.  Needs L >= 2.
// ---------------------------------------------------------------------------

// n (1..4) consecutive elements at p; vector loads when vec (p 16-byte aligned)
__device__ __forceinline__ void load4(const float* p, int n, bool vec, float v[4]) {
    if (vec && n == 4) {
        const float4 q = *(const float4*)p;
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = j < n ? p[j] : 0.f;
    }
}
__device__ __forceinline__ void load4(const double* p, int n, bool vec, double v[4]) {
    if (vec && n == 4) {
        const double2 q0 = *(const double2*)p, q1 = *(const double2*)(p + 2);
        v[0] = q0.x; v[1] = q0.y; v[2] = q1.x; v[3] = q1.y;
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = j < n ? p[j] : 0.0;
    }
}
__device__ __forceinline__ void store4(float* p, int n, bool vec, const float v[4]) {
    if (vec && n == 4) {
        *(float4*)p = make_float4(v[0], v[1], v[2], v[3]);
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (j < n) p[j] = v[j];
    }
}
__device__ __forceinline__ void store4(double* p, int n, bool vec, const double v[4]) {
    if (vec && n == 4) {
        *(double2*)p = make_double2(v[0], v[1]);
        *(double2*)(p + 2) = make_double2(v[2], v[3]);
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (j < n) p[j] = v[j];
    }
}

// vec: every row of [C, D] starts 16-byte aligned (D % 4 == 0 in FP32, D even in FP64)
template <typename T, int G>
__global__ __launch_bounds__(256) void k_elem_first(PlainArgs a, int vec) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x % G;
    const int64_t c = gid / G;
    const bool active = c < a.C;
    const int64_t D = a.tg.D;
    const uint32_t t = (uint32_t)a.ws.ctrl->t;
    const T* x = (const T*)a.ws.x;
    const T* g = (const T*)a.ws.g;
    T* xq = (T*)a.ws.xq;
    T* pq = (T*)a.ws.pq;
    const T* prec = (const T*)a.tg.prec;
    const bool diag = a.tg.kind == HMC_TGT_GAUSS_DIAG;
    const double eps = active ? a.ws.eps[c] : 0.0;
    const double bt = (active && a.ws.beta) ? a.ws.beta[c] : 1.0;
    const T half_eps = (T)(0.5 * eps * bt);
    double k0 = 0.0;
    const int64_t nblk = (D + 3) / 4;
    if (active) {
        for (int64_t b = lane; b < nblk; b += G) {
            T z[4], xv[4], gv[4], xo[4], po[4];
            // the state's loads first: the draw below runs while they are in flight
            const int n = D - 4 * b < 4 ? (int)(D - 4 * b) : 4;
            load4(x + c * D + 4 * b, n, vec != 0, xv);
            load4(g + c * D + 4 * b, n, vec != 0, gv);
            momentum4<T>(a.key, (uint32_t)c, t, (uint32_t)b, z, 4 * b + 2 < D);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                xo[j] = (T)0;
                po[j] = (T)0;
                if (j < n) {
                    const int64_t d = 4 * b + j;
                    k0 += 0.5 * (double)z[j] * (double)z[j];
                    const double sd = a.ws.scale ? a.ws.scale[d] : 1.0;
                    const T hk = a.ws.scale ? (T)(0.5 * eps * bt * sd) : half_eps;
                    T p = z[j] + hk * gv[j];
                    const T e = a.ws.scale ? (T)(eps * sd) : (T)eps;
                    const T xx = fma(e, p, xv[j]);
                    const T gg = diag ? -prec[d] * xx : -xx;
                    p = fma((T)(1.0 * eps * bt * sd), gg, p);
                    xo[j] = xx;
                    po[j] = p;
                }
            }
            store4(xq + c * D + 4 * b, n, vec != 0, xo);
            store4(pq + c * D + 4 * b, n, vec != 0, po);
        }
    }
    k0 = group_sum<G>(k0);
    if (active && lane == 0) a.ws.h0[c] = -(bt * a.ws.logp[c]) + k0;
}

template <typename T, int G>
__global__ __launch_bounds__(256) void k_elem_mid(PlainArgs a) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x % G;
    const int64_t c = gid / G;
    if (c >= a.C) return;
    const int64_t D = a.tg.D;
    T* xq = (T*)a.ws.xq;
    T* pq = (T*)a.ws.pq;
    const T* prec = (const T*)a.tg.prec;
    const bool diag = a.tg.kind == HMC_TGT_GAUSS_DIAG;
    const double eps = a.ws.eps[c];
    const double bt = a.ws.beta ? a.ws.beta[c] : 1.0;
    for (int64_t d = lane; d < D; d += G) {
        const int64_t i = c * D + d;
        const double sd = a.ws.scale ? a.ws.scale[d] : 1.0;
        const T e = a.ws.scale ? (T)(eps * sd) : (T)eps;
        const T xx = fma(e, pq[i], xq[i]);
        const T gg = diag ? -prec[d] * xx : -xx;
        const T p = fma((T)(1.0 * eps * bt * sd), gg, pq[i]);
        xq[i] = xx;
        pq[i] = p;
    }
}

// NE >= ceil(D / G): dimension lane + G k of the chain is held in slot k
template <typename T, int G, int NE>
__global__ __launch_bounds__(256) void k_elem_last(PlainArgs a) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x % G;
    const int64_t c = gid / G;
    const bool active = c < a.C;
    const int64_t D = a.tg.D;
    const Ctrl& ct = *a.ws.ctrl;
    const uint64_t t = ct.t;
    T* x = (T*)a.ws.x;
    T* g = (T*)a.ws.g;
    const T* xq = (const T*)a.ws.xq;
    const T* pq = (const T*)a.ws.pq;
    const T* prec = (const T*)a.tg.prec;
    const bool diag = a.tg.kind == HMC_TGT_GAUSS_DIAG;
    const double eps = active ? a.ws.eps[c] : 0.0;
    const double bt = (active && a.ws.beta) ? a.ws.beta[c] : 1.0;
    T xl[NE], gl[NE], pl[NE], pr[NE];
    double k1 = 0.0, lp1 = 0.0;
    // every slot's loads first (addresses clamped into the chain's row), then the arithmetic
    const int64_t cr = (active ? c : 0) * D;
#pragma unroll
    for (int k = 0; k < NE; ++k) {
        const int64_t d = lane + (int64_t)G * k;
        const int64_t dd = d < D ? d : 0;
        xl[k] = xq[cr + dd];
        pl[k] = pq[cr + dd];
        pr[k] = diag ? prec[dd] : (T)0;
    }
#pragma unroll
    for (int k = 0; k < NE; ++k) {
        const int64_t d = lane + (int64_t)G * k;
        const T xq0 = xl[k];
        xl[k] = (T)0;
        gl[k] = (T)0;
        if (active && d < D) {
            const int64_t i = c * D + d;
            const double sd = a.ws.scale ? a.ws.scale[d] : 1.0;
            const T e = a.ws.scale ? (T)(eps * sd) : (T)eps;
            const T pv0 = pl[k];
            const T xx = fma(e, pv0, xq0);
            const T gg = diag ? -pr[k] * xx : -xx;
            const T p = fma((T)(0.5 * eps * bt * sd), gg, pv0);
            k1 += 0.5 * (double)p * (double)p;
            lp1 += 0.5 * (double)xx * (double)gg;
            xl[k] = xx;
            gl[k] = gg;
            if (ct.out_xprop) ((T*)ct.out_xprop)[i] = xx;
            if (ct.out_pprop) ((T*)ct.out_pprop)[i] = p;
        }
    }
    k1 = group_sum<G>(k1);
    lp1 = group_sum<G>(lp1);
    if (!active) return;

    const double dh = (-(bt * lp1) + k1) - a.ws.h0[c];
    const double lar = log_accept_ratio_of(dh);
    const bool acc = log_accept_uniform(a.key, (uint32_t)c, (uint32_t)t) < lar;
    const int64_t i = (int64_t)(t - ct.t_begin);
    const bool keep = ct.samples && i >= ct.n_burnin && i < ct.n_burnin + ct.n_results;
    T* smp = keep ? (T*)ct.samples + ((i - ct.n_burnin) * a.C + c) * D : nullptr;
    if (acc) {
#pragma unroll
        for (int k = 0; k < NE; ++k) {
            const int64_t d = lane + (int64_t)G * k;
            if (d < D) {
                x[c * D + d] = xl[k];
                g[c * D + d] = gl[k];
                if (keep) smp[d] = xl[k];
            }
        }
    } else if (keep) {
        for (int64_t d = lane; d < D; d += G) smp[d] = x[c * D + d];
    }
    if (lane != 0) return;
    double lp_new = lp1;
    if (acc) a.ws.logp[c] = lp1;
    else lp_new = a.ws.logp[c];
    end_scalars(a, ct, c, i, acc, lar, dh, lp_new, eps);
}

// ---------------------------------------------------------------------------
// Dense Gaussian: g = -P x with v_mfma_f32_16x16x4f32.
// Operand layouts (16x16x4, wave64): A[i][k] at lane i + 16 k; B[k][j] at
// lane j + 16 k; D[i][j] in VGPR v of lane j + 16 (i / 4) with v = i % 4.
// Chains are the N dimension (16 per workgroup), rows of P the M dimension;
// wave w owns M-tiles w, w + 4, ...  x^T is staged in LDS as xs[d][chain].
// ---------------------------------------------------------------------------
template <int MT>
__global__ __launch_bounds__(256) void k_dense_leapfrog(PlainArgs a, const float* __restrict__ xsrc,
                                                        float* __restrict__ xdst, float* __restrict__ pd,
                                                        float* __restrict__ gd, int mode, double kick_scale) {
    extern __shared__ float lds[];
    const int64_t D = a.tg.D;
    const int ntiles = (int)((D + 15) / 16);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i16 = lane & 15, g4 = lane >> 4;
    const int64_t c = (int64_t)blockIdx.x * 16 + i16;
    const bool cvalid = c < a.C;
    const float* P = (const float*)a.tg.prec;
    const float eps = cvalid ? (float)a.ws.eps[c] : 0.f;
    const float keps = cvalid ? (float)(kick_scale * a.ws.eps[c] * (a.ws.beta ? a.ws.beta[c] : 1.0)) : 0.f;
    float* xs = lds;   // [16 * ntiles][17]

    float xr[MT][4], pr[MT][4];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        const int mt = w + 4 * m;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t d = 16 * mt + 4 * g4 + v;
            const bool ok = mt < ntiles && d < D && cvalid;
            float xv = ok ? xsrc[c * D + d] : 0.f;
            float pv = (ok && (mode & 3)) ? pd[c * D + d] : 0.f;
            const float ed = (ok && a.ws.scale) ? (float)(a.ws.eps[c] * a.ws.scale[d]) : eps;
            if (mode & 1) xv = fmaf(ed, pv, xv);
            xr[m][v] = xv;
            pr[m][v] = pv;
            if (mt < ntiles) xs[(16 * mt + 4 * g4 + v) * 17 + i16] = xv;
        }
    }
    __syncthreads();
    const int KM = 4 * ntiles;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        const int mt = w + 4 * m;
        if (mt >= ntiles) break;
        // k-step ks, lane group g4 takes dim g4 KM + ks, with KM = 4 ntiles; even
        // and odd k-steps in two accumulators: the same MFMA sequence as the
        // fused kernel, so both forms give bitwise the same gradient
        floatx4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
        const int64_t row = 16 * mt + i16;
        for (int ks = 0; ks < KM; ks += 2) {
            const int64_t col = (int64_t)g4 * KM + ks;
            const float av0 = (row < D && col < D) ? P[row * D + col] : 0.f;
            const float av1 = (row < D && col + 1 < D) ? P[row * D + col + 1] : 0.f;
            acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av0, xs[col * 17 + i16], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av1, xs[(col + 1) * 17 + i16], acc1, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t d = 16 * mt + 4 * g4 + v;
            if (!(d < D && cvalid)) continue;
            const float gv = -(acc0[v] + acc1[v]);
            const float kd = a.ws.scale ? (float)(kick_scale * a.ws.eps[c] * (a.ws.beta ? a.ws.beta[c] : 1.0) *
                                                  a.ws.scale[d])
                                        : keps;
            if (mode & 1) xdst[c * D + d] = xr[m][v];
            if (mode & 2) pd[c * D + d] = fmaf(kd, gv, pr[m][v]);
            if (gd) gd[c * D + d] = gv;
        }
    }
}

// ---------------------------------------------------------------------------
// Dense Gaussian, merged transition (D <= 128): one launch per leapfrog step,
// 16 chains per workgroup of 8 waves, wave w owning M-tile w of g = -P x.
// P is loaded once per launch into VGPRs as the A operands of
// v_mfma_f32_16x16x4f32 (zero-padded, so the 4 NT k-steps run unrolled), and
// x is staged chain-major in LDS for the B operands: the operand layout and
// MFMA sequence of the fused dense kernel (k = g4 KM + ks, even and odd
// k-steps in two accumulators), so the gradient is bitwise the one of
// k_dense_leapfrog and of the fused form.  Lane (i16, g4) of wave w holds
// dims 16 w + 4 g4 + v of chain i16.  FIRST also draws the momentum (Philox
// block 4 w + g4), forms H0 and makes the first half kick; LAST forms H at the
// trajectory's end, takes the Metropolis decision and writes the accepted
// chain's x, g and logp (a rejected chain's are left as they are).
// ---------------------------------------------------------------------------
constexpr int DS_NW = 8;

template <int NT, bool FIRST, bool LAST>
__global__ __launch_bounds__(64 * DS_NW) void k_dense_step(PlainArgs a) {
    constexpr int KM = 4 * NT;
    constexpr int XS = 16 * NT + 4;        // floats per chain row of the staged x, and per row of the staged P
    extern __shared__ float plds[];        // P [16 NT][XS], zero-padded
    __shared__ __attribute__((aligned(16))) float xs[16 * XS];
    __shared__ double red[3 * DS_NW * 16];
    const int64_t D = a.tg.D;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i16 = lane & 15, g4 = lane >> 4;
    const int64_t c = (int64_t)blockIdx.x * 16 + i16;
    const bool cvalid = c < a.C;
    const int64_t cc = cvalid ? c : 0;
    const bool tile_ok = w < NT;
    const float* P = (const float*)a.tg.prec;
    const Ctrl& ct = *a.ws.ctrl;
    const uint64_t t = ct.t;
    const double eps = a.ws.eps[cc];
    const double bt = a.ws.beta ? a.ws.beta[cc] : 1.0;
    const double* sc = a.ws.scale;
    float* xq = (float*)a.ws.xq;
    float* pq = (float*)a.ws.pq;
    float* X = (float*)a.ws.x;
    float* Gs = (float*)a.ws.g;

    // this chain's state first (its loads are in flight while P is staged)
    float xv[4], pv[4], gv[4];
    bool ok[4];
    double k0 = 0.0;
    const int64_t d0 = 16 * w + 4 * g4;
    if (FIRST) {
        float z[4] = {0.f, 0.f, 0.f, 0.f};
        if (tile_ok && d0 < D) momentum4<float>(a.key, (uint32_t)cc, (uint32_t)t, (uint32_t)(4 * w + g4), z, d0 + 2 < D);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t d = d0 + v;
            ok[v] = tile_ok && cvalid && d < D;
            const float x0 = ok[v] ? X[c * D + d] : 0.f;
            const float g0 = ok[v] ? Gs[c * D + d] : 0.f;
            const float p0 = ok[v] ? z[v] : 0.f;
            if (ok[v]) k0 += 0.5 * (double)p0 * (double)p0;
            const float hk = (sc && ok[v]) ? (float)(0.5 * eps * bt * sc[d]) : (float)(0.5 * eps * bt);
            pv[v] = p0 + hk * g0;
            xv[v] = x0;
        }
    } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t d = d0 + v;
            ok[v] = tile_ok && cvalid && d < D;
            xv[v] = ok[v] ? xq[c * D + d] : 0.f;
            pv[v] = ok[v] ? pq[c * D + d] : 0.f;
        }
    }
    // P into LDS with contiguous loads (16 bytes at a time when rows are 16-byte
    // aligned), the padding rows and columns zero; then each lane's A operands
    // pa[ks] = P[16 w + i16][g4 KM + ks] with 16-byte LDS reads
    {
        // every load of a thread is issued before the first LDS store (D <= 16 NT:
        // at most 16 NT x 16 NT / (4 x 512) 16-byte loads per thread)
        const int Di = (int)D;
        constexpr int PV = (16 * NT * 16 * NT + 4 * 64 * DS_NW - 1) / (4 * 64 * DS_NW);
        if ((Di & 3) == 0 && ((uintptr_t)P & 15) == 0) {
            floatx4 pv4[PV];
#pragma unroll
            for (int k = 0; k < PV; ++k) {
                const int e = 4 * ((int)threadIdx.x + k * 64 * DS_NW);
                if (e < Di * Di) pv4[k] = *(const floatx4*)(P + e);
            }
#pragma unroll
            for (int k = 0; k < PV; ++k) {
                const int e = 4 * ((int)threadIdx.x + k * 64 * DS_NW);
                if (e < Di * Di) {
                    const int row = e / Di, col = e - row * Di;
                    *(floatx4*)(plds + row * XS + col) = pv4[k];
                }
            }
        } else {
            for (int e0 = 0; e0 < Di * Di; e0 += 8 * 64 * DS_NW) {
                float pv1[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int e = e0 + (int)threadIdx.x + k * 64 * DS_NW;
                    if (e < Di * Di) pv1[k] = P[e];
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int e = e0 + (int)threadIdx.x + k * 64 * DS_NW;
                    if (e < Di * Di) {
                        const int row = e / Di, col = e - row * Di;
                        plds[row * XS + col] = pv1[k];
                    }
                }
            }
        }
        const int pad = 16 * NT - Di;
        for (int e = threadIdx.x; e < pad * 16 * NT; e += 64 * DS_NW) {
            const int r = e / (16 * NT), k = e - r * 16 * NT;
            plds[(Di + r) * XS + k] = 0.f;          // rows D .. 16 NT
            plds[k * XS + Di + r] = 0.f;            // columns D .. 16 NT
        }
    }
    __syncthreads();
    float pa[KM];
    if (tile_ok) {
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const floatx4 v4 = *(const floatx4*)(plds + (16 * w + i16) * XS + g4 * KM + 4 * j);
            pa[4 * j] = v4[0];
            pa[4 * j + 1] = v4[1];
            pa[4 * j + 2] = v4[2];
            pa[4 * j + 3] = v4[3];
        }
    } else {
#pragma unroll
        for (int ks = 0; ks < KM; ++ks) pa[ks] = 0.f;
    }

    // drift, then x of the tile into LDS
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const float e = (sc && ok[v]) ? (float)(eps * sc[d0 + v]) : (float)eps;
        xv[v] = fmaf(e, pv[v], xv[v]);
    }
    if (tile_ok) *(floatx4*)(xs + i16 * XS + 16 * w + 4 * g4) = floatx4{xv[0], xv[1], xv[2], xv[3]};
    __syncthreads();
    if (tile_ok) {
        floatx4 bq[NT];
#pragma unroll
        for (int q = 0; q < NT; ++q) bq[q] = *(const floatx4*)(xs + i16 * XS + g4 * KM + 4 * q);
        floatx4 acc[2] = {floatx4{0.f, 0.f, 0.f, 0.f}, floatx4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
        for (int ks = 0; ks < KM; ++ks)
            acc[ks & 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(pa[ks], bq[ks >> 2][ks & 3], acc[ks & 1], 0, 0, 0);
        // all operand reads first (one LDS latency), then the MFMAs
        __builtin_amdgcn_sched_group_barrier(0x100, NT, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, KM, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) gv[v] = -(acc[0][v] + acc[1][v]);
    } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) gv[v] = 0.f;
    }
    const double ksc = LAST ? 0.5 : 1.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const float kd = (sc && ok[v]) ? (float)(ksc * eps * bt * sc[d0 + v]) : (float)(ksc * eps * bt);
        pv[v] = fmaf(kd, gv[v], pv[v]);
    }

    if (!LAST) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
            if (ok[v]) {
                xq[c * D + d0 + v] = xv[v];
                pq[c * D + d0 + v] = pv[v];
            }
        if (FIRST) {
            k0 += __shfl_xor(k0, 16, 64);
            k0 += __shfl_xor(k0, 32, 64);
            if (g4 == 0) red[w * 16 + i16] = k0;
            __syncthreads();
            if (threadIdx.x < 16 && cvalid) {
                double s0 = 0.0;
                for (int ww = 0; ww < DS_NW; ++ww) s0 += red[ww * 16 + i16];
                a.ws.h0[c] = -(bt * a.ws.logp[c]) + s0;
            }
        }
        return;
    }

    // end of the trajectory: kinetic energy and logp = 1/2 x.g, summed over the
    // lane groups, then over the waves in wave order
    double k1 = 0.0, lp1 = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v)
        if (ok[v]) {
            k1 += 0.5 * (double)pv[v] * (double)pv[v];
            lp1 += 0.5 * (double)xv[v] * (double)gv[v];
            if (ct.out_xprop) ((float*)ct.out_xprop)[c * D + d0 + v] = xv[v];
            if (ct.out_pprop) ((float*)ct.out_pprop)[c * D + d0 + v] = pv[v];
        }
    k0 += __shfl_xor(k0, 16, 64);
    k0 += __shfl_xor(k0, 32, 64);
    k1 += __shfl_xor(k1, 16, 64);
    k1 += __shfl_xor(k1, 32, 64);
    lp1 += __shfl_xor(lp1, 16, 64);
    lp1 += __shfl_xor(lp1, 32, 64);
    if (g4 == 0) {
        red[w * 16 + i16] = k0;
        red[(DS_NW + w) * 16 + i16] = k1;
        red[(2 * DS_NW + w) * 16 + i16] = lp1;
    }
    __syncthreads();
    if (!cvalid) return;
    double s0 = 0.0, s1 = 0.0, sl = 0.0;
    for (int ww = 0; ww < DS_NW; ++ww) {
        s0 += red[ww * 16 + i16];
        s1 += red[(DS_NW + ww) * 16 + i16];
        sl += red[(2 * DS_NW + ww) * 16 + i16];
    }
    const double lp_old = a.ws.logp[c];
    const double h0 = FIRST ? -(bt * lp_old) + s0 : a.ws.h0[c];
    const double dh = (-(bt * sl) + s1) - h0;
    const double lar = log_accept_ratio_of(dh);
    const bool acc = log_accept_uniform(a.key, (uint32_t)c, (uint32_t)t) < lar;
    const int64_t i = (int64_t)(t - ct.t_begin);
    const bool keep = ct.samples && i >= ct.n_burnin && i < ct.n_burnin + ct.n_results;
    float* smp = keep ? (float*)ct.samples + ((i - ct.n_burnin) * a.C + c) * D : nullptr;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        if (!ok[v]) continue;
        const int64_t d = d0 + v;
        if (acc) {
            X[c * D + d] = xv[v];
            Gs[c * D + d] = gv[v];
            if (keep) smp[d] = xv[v];
        } else if (keep) {
            smp[d] = X[c * D + d];
        }
    }
    if (threadIdx.x >= 16) return;
    if (acc) a.ws.logp[c] = sl;
    end_scalars(a, ct, c, i, acc, lar, dh, acc ? sl : lp_old, eps);
}

// ---------------------------------------------------------------------------
// Logistic regression, split over rows.  Workgroup (chain tile of 16, split s)
// handles rows [s*rows, (s+1)*rows).  Per 16-row tile:
//   S = X_tile theta^T   (M = rows, N = chains, K = dims)      16x16x4 MFMA
//   R = y - sigmoid(S)   (rows beyond N give 0)
//   G += X_tile^T R      (M = dims, N = chains, K = 4 rows)    K-step v takes the
//       rows {4k + v}, so the B operand is the S accumulator's own VGPR v.
// Wave partials are summed in LDS in wave order, then written to part_g[s].
// ---------------------------------------------------------------------------
template <typename XT>
__device__ __forceinline__ float ld_x(const XT* X, int64_t i);
template <>
__device__ __forceinline__ float ld_x<float>(const float* X, int64_t i) { return X[i]; }
template <>
__device__ __forceinline__ float ld_x<uint16_t>(const uint16_t* X, int64_t i) { return bf16_to_f32(X[i]); }

__device__ __forceinline__ float sigmoidf_(float s) {
    // 1 / (1 + e^-s) evaluated without overflow on either side
    const float e = expf(-fabsf(s));
    const float r = 1.0f / (1.0f + e);
    return s >= 0.f ? r : e * r;
}

__device__ __forceinline__ float softplusf_(float s) {
    return fmaxf(s, 0.f) + log1pf(expf(-fabsf(s)));
}

// ---------------------------------------------------------------------------
// Logistic regression, FP32 operands: one launch per leapfrog step.
// A workgroup (4 waves) owns 64 chains and one split of the rows; wave w runs
// both contractions for chains c0 + 16 w + i16 over the split's rows on
// v_mfma_f32_16x16x4f32, 16 rows at a time:
//   S = X_sub theta^T  (M = 16 rows, N = 16 chains, K = 4 dims): k-step (b, v)
//                      takes dims 16 b + 4 q + v at lane group q, so one
//                      16-byte LDS read gives the A operands of 4 k-steps and
//                      lane (i16, q) holds theta of dims 16 b + 4 q .. + 3 as B
//   R = y - sigmoid(S) (0 for rows outside the split)
//   G += X_sub^T R     (M = 16 dims, N = 16 chains, K = 4 rows): k-step v takes
//                      rows 4 q + v, the S accumulator's own VGPR v
// theta (drifted) stays in VGPRs, G in KT accumulators; 16-row stages of X
// (FP32, upcast when stored BF16) are double-buffered in LDS through
// registers and shared by the 4 waves (row stride 16 KT + 4 floats: both
// operand reads hit distinct banks).  Each workgroup writes its partial G and
// logp to part_g / part_lp; the last one of a chain tile to finish (an atomic
// count per tile, reset by that workgroup) sums the partials in split order,
// adds the prior gradient, kicks and writes x, p, g and the data part of logp
// -- the partial-sum and finish passes in one launch, in a fixed order.
// ---------------------------------------------------------------------------
constexpr int LR32_CT = 64;      // chains per workgroup
constexpr int LR32_RS = 16;      // rows per sub-tile (one M tile of S)

// rows per LDS stage: 16 for 128 dims and more, else 128 / KT (8 stage elements
// per thread in every case below 256 dims), so that narrow problems do not wait
// on one global load latency per 16 rows
template <int KT>
constexpr int lr32_rs() { return KT >= 8 ? 16 : 128 / KT; }

template <typename XT>
struct Lr32Stage;
// FP32 X: 16-byte loads when rows are 16-byte aligned (D % 4 == 0)
template <>
struct Lr32Stage<float> {
    static constexpr int V = 4;
    typedef float4 raw;
    __device__ static raw load(const float* X, int64_t e) { return *(const float4*)(X + e); }
    __device__ static void to_f32(raw r, float f[4]) { f[0] = r.x; f[1] = r.y; f[2] = r.z; f[3] = r.w; }
    __device__ static float one(const float* X, int64_t e) { return X[e]; }
};
// BF16 X: 8 values (16 bytes) per load when D % 8 == 0
template <>
struct Lr32Stage<uint16_t> {
    static constexpr int V = 8;
    typedef uint4 raw;
    __device__ static raw load(const uint16_t* X, int64_t e) { return *(const uint4*)(X + e); }
    __device__ static void to_f32(raw r, float f[8]) {
        const uint32_t u[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            f[2 * k] = __uint_as_float(u[k] << 16);
            f[2 * k + 1] = __uint_as_float(u[k] & 0xffff0000u);
        }
    }
    __device__ static float one(const uint16_t* X, int64_t e) { return bf16_to_f32(X[e]); }
};

// Registers of the next stage: thread t holds elements (k 256 + t) V .. + V - 1
// (VEC: one 16-byte load each; rows 16-byte aligned) or k 256 + t of the
// stage's RS x D block of X, which is contiguous in the row-major array.
template <typename XT, int KT, bool VEC>
struct Lr32Pre {
    typedef Lr32Stage<XT> SL;
    static constexpr int XS = 16 * KT + 4;
    static constexpr int RS = lr32_rs<KT>();
    static constexpr int NV = (RS * 16 * KT) / (SL::V * 256) > 0 ? (RS * 16 * KT) / (SL::V * 256) : 1;
    static constexpr int NS = VEC ? 1 : NV * SL::V;
    typename SL::raw r[VEC ? NV : 1];
    float f[NS];

    __device__ __forceinline__ void fetch(const XT* X, int64_t D, int64_t r_begin, int64_t r_end, int st) {
        const int64_t r0 = r_begin + (int64_t)st * RS;
        const int64_t lim = ((r_end - r0) < RS ? (r_end - r0) : RS) * D;   // valid elements
        if (VEC) {
            // an element past the valid rows loads the last valid vector (zeroed at the store)
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                const int64_t e = ((int64_t)k * 256 + threadIdx.x) * SL::V;
                r[k] = SL::load(X, r0 * D + (e < lim ? e : lim - SL::V));
            }
        } else {
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                const int64_t e = (int64_t)k * 256 + threadIdx.x;
                f[k] = e < lim ? SL::one(X, r0 * D + e) : 0.f;
            }
        }
    }
    __device__ __forceinline__ void store(float* lds, int64_t D, int64_t r_begin, int64_t r_end, int st, int buf) const {
        const int64_t r0 = r_begin + (int64_t)st * RS;
        const int lim = (int)(((r_end - r0) < RS ? (r_end - r0) : RS) * D);
        const int nel = RS * (int)D;
        float* xb = lds + buf * RS * XS;
        if (VEC) {
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                const int e = (k * 256 + (int)threadIdx.x) * SL::V;
                if (e >= nel) continue;
                float v[SL::V];
                SL::to_f32(r[k], v);
                const bool ok = e < lim;
                const int row = e / (int)D, col = e - row * (int)D;
#pragma unroll
                for (int j = 0; j < SL::V; j += 4)
                    *(floatx4*)(xb + row * XS + col + j) = ok ? floatx4{v[j], v[j + 1], v[j + 2], v[j + 3]}
                                                              : floatx4{0.f, 0.f, 0.f, 0.f};
            }
        } else {
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                const int e = k * 256 + (int)threadIdx.x;
                if (e >= nel) continue;
                const int row = e / (int)D, col = e - row * (int)D;
                xb[row * XS + col] = f[k];
            }
        }
    }
};

// The label of row threadIdx.x of a stage as its raw byte (0 past the split):
// converted only at the LDS store, so that its load is not waited for (with
// the stage's X loads ahead of it) before the current stage is computed.
template <int RS>
__device__ __forceinline__ uint32_t lr32_label(const uint8_t* y, int64_t r_begin, int64_t r_end, int st) {
    const int64_t r = r_begin + (int64_t)st * RS + threadIdx.x;
    return (threadIdx.x < RS && r < r_end) ? (uint32_t)y[r] : 0u;
}

template <typename XT, int KT, bool VEC>
__global__ __launch_bounds__(256) void k_lr32_step(PlainArgs a, float* __restrict__ xio, float* __restrict__ pio,
                                                   float* __restrict__ gout, int drift, int kick, double kick_scale,
                                                   int want_logp, int nsplit, int64_t rows_per_split) {
    constexpr int XS = 16 * KT + 4;                       // LDS row stride (floats)
    constexpr int RS = lr32_rs<KT>();                    // rows per stage
    constexpr int STAGE = RS * XS;
    extern __shared__ float lds[];                        // [2][RS][XS] X stages, then [2][RS] labels
    float* ys = lds + 2 * STAGE;
    __shared__ int s_last;
    const int64_t D = a.tg.D, N = a.tg.N, C = a.C;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i16 = lane & 15, q = lane >> 4;
    const int tile = blockIdx.x, split = blockIdx.y;
    const int64_t c = (int64_t)tile * LR32_CT + 16 * w + i16;
    const bool cv = c < C;
    const XT* X = (const XT*)a.tg.X;
    const uint8_t* y = a.tg.y;
    const double* sc = a.ws.scale;
    const double eps = cv ? a.ws.eps[c] : 0.0;

    // theta (drifted) as B operands: th[b][v] = theta[c][16 b + 4 q + v], loaded
    // four 16-dim blocks at a time with every load of a group issued before its
    // arithmetic (the drift is the same fmaf as the finish below, which stores
    // the drifted x)
    float th[KT][4];
    const int64_t cr = (cv ? c : 0) * D;
    constexpr int PB = KT < 4 ? KT : 4;
#pragma unroll
    for (int b0 = 0; b0 < KT; b0 += PB) {
        float pm[PB][4];
#pragma unroll
        for (int bb = 0; bb < PB; ++bb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t d = 16 * (b0 + bb) + 4 * q + v;
                const int64_t dd = d < D ? d : 0;
                th[b0 + bb][v] = xio[cr + dd];
                pm[bb][v] = drift ? pio[cr + dd] : 0.f;
            }
#pragma unroll
        for (int bb = 0; bb < PB; ++bb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t d = 16 * (b0 + bb) + 4 * q + v;
                const bool ok = cv && d < D;
                float t = th[b0 + bb][v];
                if (drift) t = fmaf(sc ? (float)(eps * sc[ok ? d : 0]) : (float)eps, pm[bb][v], t);
                th[b0 + bb][v] = ok ? t : 0.f;
            }
    }

    const int64_t r_begin = (int64_t)split * rows_per_split;
    const int64_t r_end = r_begin + rows_per_split < N ? r_begin + rows_per_split : N;
    const int nst = (int)((r_end - r_begin + RS - 1) / RS);

    // columns D .. 16 KT of both stage buffers stay zero
    for (int idx = threadIdx.x; idx < 2 * RS * (16 * KT - (int)D); idx += 256) {
        const int pad = 16 * KT - (int)D;
        const int row = idx / pad, col = (int)D + idx % pad;
        lds[row * XS + col] = 0.f;
    }
    // stage loads: element e of the stage's RS x D block of X (contiguous rows)
    Lr32Pre<XT, KT, VEC> pre;
    uint32_t pre_y = 0u;
    floatx4 gacc[KT];
#pragma unroll
    for (int b = 0; b < KT; ++b) gacc[b] = floatx4{0.f, 0.f, 0.f, 0.f};
    double lp = 0.0;
    if (nst > 0) {
        pre.fetch(X, D, r_begin, r_end, 0);
        pre_y = lr32_label<RS>(y, r_begin, r_end, 0);
        pre.store(lds, D, r_begin, r_end, 0, 0);
        if (threadIdx.x < RS) ys[threadIdx.x] = (float)pre_y;
    }
    __syncthreads();
    for (int st = 0; st < nst; ++st) {
        const int buf = st & 1;
        if (st + 1 < nst) {
            pre.fetch(X, D, r_begin, r_end, st + 1);
            pre_y = lr32_label<RS>(y, r_begin, r_end, st + 1);
        }
        const float* xst = lds + buf * STAGE;
#pragma unroll
        for (int h = 0; h < RS / LR32_RS; ++h) {
            const int64_t r0 = r_begin + (int64_t)st * RS + LR32_RS * h;
            if (RS > LR32_RS && r0 >= r_end) continue;     // sub-tiles past the split's end (uniform)
            const float* xb = xst + LR32_RS * h * XS;
            // S = X_sub theta^T
            floatx4 s0 = {0.f, 0.f, 0.f, 0.f}, s1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int b = 0; b < KT; ++b) {
                const floatx4 a4 = *(const floatx4*)(xb + i16 * XS + 16 * b + 4 * q);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    if (b & 1) s1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[v], th[b][v], s1, 0, 0, 0);
                    else s0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[v], th[b][v], s0, 0, 0, 0);
                }
            }
            float rr[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float sv = s0[v] + s1[v];
                const bool ok = r0 + 4 * q + v < r_end;
                const float yv = ys[buf * RS + LR32_RS * h + 4 * q + v];
                rr[v] = ok ? yv - sigmoidf_(sv) : 0.f;
                if (want_logp && ok) lp -= (double)softplusf_(yv > 0.5f ? -sv : sv);
            }
            // G += X_sub^T R
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int b = 0; b < KT; ++b)
                    gacc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(xb[(4 * q + v) * XS + 16 * b + i16], rr[v],
                                                                   gacc[b], 0, 0, 0);
        }
        if (st + 1 < nst) {
            pre.store(lds, D, r_begin, r_end, st + 1, buf ^ 1);
            if (threadIdx.x < RS) ys[(buf ^ 1) * RS + threadIdx.x] = (float)pre_y;
        }
        __syncthreads();
    }

    // this workgroup's partials: lane (i16, q) holds G[c][16 b + 4 q + v]
    const int64_t CD = C * D;
    if (cv) {
        float* pg = a.ws.part_g + (int64_t)split * CD + c * D;
#pragma unroll
        for (int b = 0; b < KT; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t d = 16 * b + 4 * q + v;
                if (d < D) pg[d] = gacc[b][v];
            }
    }
    lp += __shfl_xor(lp, 16, 64);
    lp += __shfl_xor(lp, 32, 64);
    if (want_logp && cv && q == 0) a.ws.part_lp[(int64_t)split * C + c] = lp;
    // release this workgroup's partials (agent scope: the other splits may run on other XCDs),
    // then count it; the last one to count acquires them all
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) s_last = atomicAdd(&a.ws.lr_cnt[tile], 1) == nsplit - 1;
    __syncthreads();
    if (!s_last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");

    // last workgroup of the tile: drift (the same fmaf), split sum in split order,
    // prior gradient, kick -- four elements per thread at a time, every load of
    // the four (state, step size, split partials) issued before the arithmetic
    const int64_t c0 = (int64_t)tile * LR32_CT;
    const int64_t nc = C - c0 < LR32_CT ? C - c0 : LR32_CT;
    const int64_t ne = nc * D;
    constexpr int U = 4;
    for (int64_t base = threadIdx.x; base < ne; base += 256 * U) {
        float xv[U], pv[U], gs[U];
        double ec[U], sd[U], bt[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t idx = base + 256 * u < ne ? base + 256 * u : ne - 1;    // clamped: loads stay in range
            const int64_t i = c0 * D + idx;
            const int64_t cc = i / D, d = i - cc * D;
            ec[u] = a.ws.eps[cc];
            sd[u] = sc ? sc[d] : 1.0;
            bt[u] = a.ws.beta ? a.ws.beta[cc] : 1.0;
            xv[u] = xio[i];
            pv[u] = (drift || kick) ? pio[i] : 0.f;
            gs[u] = 0.f;
        }
        for (int s0 = 0; s0 < nsplit; s0 += 8) {
            float v[U][8];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t idx = base + 256 * u < ne ? base + 256 * u : ne - 1;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int sk = s0 + k < nsplit ? s0 + k : nsplit - 1;
                    v[u][k] = a.ws.part_g[(int64_t)sk * CD + c0 * D + idx];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (s0 + k < nsplit) gs[u] += v[u][k];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (base + 256 * u >= ne) continue;
            const int64_t i = c0 * D + base + 256 * u;
            float x = xv[u];
            if (drift) {
                x = fmaf(sc ? (float)(ec[u] * sd[u]) : (float)ec[u], pv[u], x);
                xio[i] = x;
            }
            const float gv = gs[u] - x * (float)a.tg.inv_var;
            if (kick) pio[i] = fmaf((float)(kick_scale * ec[u] * bt[u] * sd[u]), gv, pv[u]);
            if (gout) gout[i] = gv;
        }
    }
    if (want_logp && threadIdx.x < nc) {
        const int64_t cc = c0 + threadIdx.x;
        // eight loads in flight, then the sums in split order
        double l = 0.0;
        for (int s0 = 0; s0 < nsplit; s0 += 8) {
            double v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = a.ws.part_lp[(int64_t)(s0 + k < nsplit ? s0 + k : nsplit - 1) * C + cc];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (s0 + k < nsplit) l += v[k];
        }
        a.ws.lpq[cc] = l;
    }
    if (threadIdx.x == 0) a.ws.lr_cnt[tile] = 0;
}

// drift (same fmaf as the partial kernel), sum the split partials in split
// order, add the prior gradient, kick.
__device__ __forceinline__ void finish_body(const PlainArgs& a, float* __restrict__ xd, float* __restrict__ pd,
                                            float* __restrict__ gd, int nsplit, int drift, int kick,
                                            double kick_scale, int want_logp, int64_t blk, int64_t nblk) {
    const int64_t D = a.tg.D, C = a.C;
    const int64_t n = C * D;
    for (int64_t i = blk * blockDim.x + threadIdx.x; i < n; i += nblk * blockDim.x) {
        const int64_t c = i / D;
        const double sd = a.ws.scale ? a.ws.scale[i - c * D] : 1.0;
        float x = xd[i];
        const float p = (drift || kick) ? pd[i] : 0.f;
        if (drift) {
            x = fmaf(a.ws.scale ? (float)(a.ws.eps[c] * sd) : (float)a.ws.eps[c], p, x);
            xd[i] = x;
        }
        float gsum = 0.f;
        for (int s = 0; s < nsplit; ++s) gsum += a.ws.part_g[(int64_t)s * n + i];
        const float gv = gsum - x * (float)a.tg.inv_var;
        if (kick) pd[i] = fmaf((float)(kick_scale * a.ws.eps[c] * (a.ws.beta ? a.ws.beta[c] : 1.0) * sd), gv, p);
        if (gd) gd[i] = gv;
        if (want_logp && i - c * D == 0) {
            double l = 0.0;
            for (int s = 0; s < nsplit; ++s) l += a.ws.part_lp[(int64_t)s * C + c];
            a.ws.lpq[c] = l;
        }
    }
}

__global__ __launch_bounds__(256) void k_logreg_finish(PlainArgs a, float* __restrict__ xd, float* __restrict__ pd,
                                                       float* __restrict__ gd, int nsplit, int drift, int kick,
                                                       double kick_scale, int want_logp) {
    finish_body(a, xd, pd, gd, nsplit, drift, kick, kick_scale, want_logp, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// Several BF16-gradient logistic requests in one launch per kernel (serving):
// the one-request bodies with job-local block indices (see Lr16Job).
// ---------------------------------------------------------------------------
template <int G>
__global__ __launch_bounds__(256) void k_begin_multi(const Lr16Job* __restrict__ jobs, int njobs) {
    int64_t lb;
    const int j = lr16_job_of(jobs, njobs, LR16_KIND_GROUP, blockIdx.x, &lb);
    if (j < 0) return;
    const PlainArgs a = jobs[j].a;
    begin_body<float, G>(a, lb);
}

template <int G>
__global__ __launch_bounds__(256) void k_end_multi(const Lr16Job* __restrict__ jobs, int njobs) {
    int64_t lb;
    const int j = lr16_job_of(jobs, njobs, LR16_KIND_GROUP, blockIdx.x, &lb);
    if (j < 0) return;
    const PlainArgs a = jobs[j].a;
    end_body<float, G>(a, lb);
}

// leapfrog step of the transition: drift, split sums, kick (ks), the gradient kept on the last step
__global__ __launch_bounds__(256) void k_finish_multi(const Lr16Job* __restrict__ jobs, int njobs, int last) {
    int64_t lb;
    const int j = lr16_job_of(jobs, njobs, LR16_KIND_FINISH, blockIdx.x, &lb);
    if (j < 0) return;
    const PlainArgs a = jobs[j].a;
    finish_body(a, (float*)a.ws.xq, (float*)a.ws.pq, last ? (float*)a.ws.gq : nullptr, jobs[j].nsplit_g, 1, 1,
                last ? 0.5 : 1.0, 0, lb, jobs[j].nblk[LR16_KIND_FINISH]);
}

__global__ void k_tick_multi(const Lr16Job* __restrict__ jobs, int njobs) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < njobs) jobs[j].a.ws.ctrl->t += 1;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static int chain_group(int64_t D) {
    if (D <= 4) return 1;
    if (D <= 16) return 4;
    if (D <= 64) return 16;
    return 64;
}

int plain_chain_group(int64_t D) { return chain_group(D); }

#define HMC_GROUP_DISPATCH(KERNEL, T, a, s)                                                       \
    do {                                                                                          \
        const int G = chain_group((a).tg.D);                                                      \
        const int64_t threads = (a).C * G;                                                        \
        const dim3 grid((unsigned)((threads + 255) / 256));                                       \
        if (G == 1) hipLaunchKernelGGL((KERNEL<T, 1>), grid, dim3(256), 0, s, a);                 \
        else if (G == 4) hipLaunchKernelGGL((KERNEL<T, 4>), grid, dim3(256), 0, s, a);            \
        else if (G == 16) hipLaunchKernelGGL((KERNEL<T, 16>), grid, dim3(256), 0, s, a);          \
        else hipLaunchKernelGGL((KERNEL<T, 64>), grid, dim3(256), 0, s, a);                       \
    } while (0)

static dim3 elem_grid(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

int64_t logreg_nsplit(int64_t N, int64_t C) {
    // about two workgroups per CU (64 chains each), splits of >= 8 stages of rows
    // (the last workgroup of a tile sums one partial per split)
    const int64_t tiles = (C + 63) / 64;
    int64_t want = (512 + tiles - 1) / tiles;
    const int64_t maxs = (N + 127) / 128;
    if (want > maxs) want = maxs;
    if (want < 1) want = 1;
    if (want > 32) want = 32;
    return want;
}

static size_t dense_lds(int64_t D) { return (size_t)16 * ((D + 15) / 16) * 17 * sizeof(float); }

template <typename K>
static void allow_lds(K kernel, size_t lds) {
    if (lds > 65536) (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

static hipError_t launch_dense(const PlainArgs& a, const float* xs, float* xd, float* pd, float* gd, int mode,
                               double ks, hipStream_t s) {
    const int ntiles = (int)((a.tg.D + 15) / 16);
    const dim3 grid((unsigned)((a.C + 15) / 16));
    const size_t lds = dense_lds(a.tg.D);
    allow_lds(k_dense_leapfrog<16>, lds);
    if (ntiles <= 4) hipLaunchKernelGGL(k_dense_leapfrog<1>, grid, dim3(256), lds, s, a, xs, xd, pd, gd, mode, ks);
    else if (ntiles <= 8) hipLaunchKernelGGL(k_dense_leapfrog<2>, grid, dim3(256), lds, s, a, xs, xd, pd, gd, mode, ks);
    else if (ntiles <= 16) hipLaunchKernelGGL(k_dense_leapfrog<4>, grid, dim3(256), lds, s, a, xs, xd, pd, gd, mode, ks);
    else hipLaunchKernelGGL(k_dense_leapfrog<16>, grid, dim3(256), lds, s, a, xs, xd, pd, gd, mode, ks);
    return hipGetLastError();
}

// largest split count the workspace is sized for (the autotuner tries up to 2x the default)
int64_t logreg_nsplit_cap(int64_t N, int64_t C) {
    int64_t cap = 2 * logreg_nsplit(N, C);
    const int64_t maxs = (N + 4 * LR32_RS - 1) / (4 * LR32_RS);
    if (cap > maxs) cap = maxs;
    if (cap > 64) cap = 64;
    return cap < 1 ? 1 : cap;
}

int64_t logreg_nsplit_t(const PlainArgs& a) {
    if (a.tune.lr_nsplit > 0) {
        const int64_t cap = logreg_nsplit_cap(a.tg.N, a.C);
        return a.tune.lr_nsplit < cap ? a.tune.lr_nsplit : cap;
    }
    return logreg_nsplit(a.tg.N, a.C);
}

template <int KT>
static size_t lr32_lds() {
    constexpr int RS = lr32_rs<KT>();
    return (size_t)(2 * RS * (16 * KT + 4) + 2 * RS) * sizeof(float);
}

template <typename XT, int KT>
static void launch_lr32_kt(const PlainArgs& a, dim3 grid, hipStream_t s, float* x, float* p, float* gd, int drift,
                           int kick, double ks, int want_logp, int nsplit, int64_t rows, int vec) {
    const size_t lds = lr32_lds<KT>();
    if (vec) {
        allow_lds(k_lr32_step<XT, KT, true>, lds);
        hipLaunchKernelGGL((k_lr32_step<XT, KT, true>), grid, dim3(256), lds, s, a, x, p, gd, drift, kick, ks,
                           want_logp, nsplit, rows);
    } else {
        allow_lds(k_lr32_step<XT, KT, false>, lds);
        hipLaunchKernelGGL((k_lr32_step<XT, KT, false>), grid, dim3(256), lds, s, a, x, p, gd, drift, kick, ks,
                           want_logp, nsplit, rows);
    }
}

template <typename XT>
static void launch_lr32(const PlainArgs& a, dim3 grid, hipStream_t s, float* x, float* p, float* gd, int drift,
                        int kick, double ks, int want_logp, int nsplit, int64_t rows, int vec) {
    const int kt = (int)((a.tg.D + 15) / 16);
    if (kt <= 1) launch_lr32_kt<XT, 1>(a, grid, s, x, p, gd, drift, kick, ks, want_logp, nsplit, rows, vec);
    else if (kt <= 2) launch_lr32_kt<XT, 2>(a, grid, s, x, p, gd, drift, kick, ks, want_logp, nsplit, rows, vec);
    else if (kt <= 4) launch_lr32_kt<XT, 4>(a, grid, s, x, p, gd, drift, kick, ks, want_logp, nsplit, rows, vec);
    else if (kt <= 8) launch_lr32_kt<XT, 8>(a, grid, s, x, p, gd, drift, kick, ks, want_logp, nsplit, rows, vec);
    else if (kt <= 16) launch_lr32_kt<XT, 16>(a, grid, s, x, p, gd, drift, kick, ks, want_logp, nsplit, rows, vec);
    else launch_lr32_kt<XT, 32>(a, grid, s, x, p, gd, drift, kick, ks, want_logp, nsplit, rows, vec);
}

// One FP32 gradient evaluation of logistic regression at x (drifted in place
// first when drift), kicking p when kick, the gradient into gd if not null and
// the data part of logp into lpq when want_logp.
static hipError_t launch_logreg(const PlainArgs& a, float* x, float* p, float* gd, int drift, int kick, double ks,
                                int want_logp, hipStream_t s) {
    int64_t nsplit = logreg_nsplit_t(a);
    int64_t rows = (a.tg.N + nsplit - 1) / nsplit;
    rows = (rows + LR32_RS - 1) / LR32_RS * LR32_RS;
    nsplit = (a.tg.N + rows - 1) / rows;
    const dim3 grid((unsigned)((a.C + LR32_CT - 1) / LR32_CT), (unsigned)nsplit);
    const bool x_aligned = ((uintptr_t)a.tg.X & 15) == 0;
    timer_begin(a, s);
    if (a.tg.x_bf16)
        launch_lr32<uint16_t>(a, grid, s, x, p, gd, drift, kick, ks, want_logp, (int)nsplit, rows,
                              a.tg.D % 8 == 0 && x_aligned);
    else
        launch_lr32<float>(a, grid, s, x, p, gd, drift, kick, ks, want_logp, (int)nsplit, rows,
                           a.tg.D % 4 == 0 && x_aligned);
    timer_end(a, s, "k_lr32_step");
    return hipGetLastError();
}

hipError_t launch_set_ctrl(const Ctrl& c, Ctrl* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_set_ctrl, dim3(1), dim3(64), 0, s, dst, c);
    return hipGetLastError();
}

hipError_t launch_da_init(const PlainArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_da_init<float>, dim3((unsigned)((a.C + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

// Streaming expectations: element e = (c, d) of q kept states in draw order.
// Welford (1962): n-th draw of a half, delta = x - mean, mean += delta / n,
// m2 += delta (x - mean); batch sums accumulate in a register and are added
// to memory when the batch changes (a batch may span chunks).
template <typename T>
__global__ __launch_bounds__(256) void k_moments(const T* __restrict__ ring, int64_t n_el, int64_t q, int64_t r0,
                                                 int64_t R, double* __restrict__ mean, double* __restrict__ m2,
                                                 double* __restrict__ bsum, int64_t blen) {
    const int64_t half = R / 2;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_el; e += (int64_t)gridDim.x * blockDim.x) {
        double mu[2] = {mean[e], mean[n_el + e]};
        double ss[2] = {m2[e], m2[n_el + e]};
        int64_t cur_b = -1;
        double bacc = 0.0;
        for (int64_t j = 0; j < q; ++j) {
            const int64_t r = r0 + j;
            const double x = (double)ring[j * n_el + e];
            const int h = r < half ? 0 : 1;
            const double n = (double)(h ? r - half + 1 : r + 1);
            const double delta = x - mu[h];
            mu[h] += delta / n;
            ss[h] += delta * (x - mu[h]);
            if (bsum) {
                const int64_t b = r / blen;
                if (b != cur_b) {
                    if (cur_b >= 0) bsum[cur_b * n_el + e] += bacc;
                    cur_b = b;
                    bacc = 0.0;
                }
                bacc += x;
            }
        }
        if (bsum && cur_b >= 0) bsum[cur_b * n_el + e] += bacc;
        mean[e] = mu[0];
        mean[n_el + e] = mu[1];
        m2[e] = ss[0];
        m2[n_el + e] = ss[1];
    }
}

__global__ void k_zero_i32(int32_t* p, int64_t n) {
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

__global__ void k_fill_f64(double* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

hipError_t launch_fill_f64(double* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_moments(const PlainArgs& a, const void* ring, int64_t q, int64_t r0, int64_t R,
                          const hmc_moments& m, hipStream_t s) {
    const int64_t n_el = a.C * a.tg.D;
    const int64_t blocks = (n_el + 255) / 256 < 8192 ? (n_el + 255) / 256 : 8192;
    if (a.f64)
        hipLaunchKernelGGL(k_moments<double>, dim3((unsigned)blocks), dim3(256), 0, s, (const double*)ring, n_el, q, r0,
                           R, m.mean, m.m2, m.batch_sum, m.batch_len);
    else
        hipLaunchKernelGGL(k_moments<float>, dim3((unsigned)blocks), dim3(256), 0, s, (const float*)ring, n_el, q, r0,
                           R, m.mean, m.m2, m.batch_sum, m.batch_len);
    return hipGetLastError();
}

hipError_t launch_remc_swap(const PlainArgs& a, int64_t K, int64_t M, uint32_t t, uint8_t* swapped,
                            void* sample_row, hipStream_t s) {
    if (K <= 0 || M <= 0) return hipSuccess;
    const int32_t parity = (int32_t)(t & 1u);
    const int64_t npairs = (K - parity) / 2;
    const int64_t waves = (K - npairs) * M;       // one per pair, one per unpaired chain
    const dim3 grid((unsigned)((waves + 3) / 4));
    if (a.f64)
        hipLaunchKernelGGL(k_remc_exchange<double>, grid, dim3(256), 0, s, a, K, M, parity, t, swapped,
                           (double*)sample_row);
    else
        hipLaunchKernelGGL(k_remc_exchange<float>, grid, dim3(256), 0, s, a, K, M, parity, t, swapped,
                           (float*)sample_row);
    return hipGetLastError();
}

static bool launch_dense_logp(const PlainArgs& a, hipStream_t s);

// gradient (and logp) at ws.x into ws.g / ws.logp
hipError_t launch_bootstrap(const PlainArgs& a_in, const void* x_src, hipStream_t s) {
    PlainArgs a = a_in;
    a.timer = nullptr;       // the kernel timer covers transitions only
    const size_t es = a.f64 ? 8 : 4;
    if (x_src && x_src != a.ws.x) {
        hipError_t e = hipMemcpyAsync(a.ws.x, x_src, (size_t)a.C * a.tg.D * es, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    switch (a.tg.kind) {
    case HMC_TGT_STD_NORMAL:
    case HMC_TGT_GAUSS_DIAG:
        if (a.f64)
            hipLaunchKernelGGL(k_elem_leapfrog<double>, elem_grid(a.C * a.tg.D), dim3(256), 0, s, a,
                               (const double*)a.ws.x, (double*)nullptr, (double*)nullptr, (double*)a.ws.g, 0, 0.0);
        else
            hipLaunchKernelGGL(k_elem_leapfrog<float>, elem_grid(a.C * a.tg.D), dim3(256), 0, s, a,
                               (const float*)a.ws.x, (float*)nullptr, (float*)nullptr, (float*)a.ws.g, 0, 0.0);
        break;
    case HMC_TGT_GAUSS_DENSE:
        (void)launch_dense(a, (const float*)a.ws.x, nullptr, nullptr, (float*)a.ws.g, 0, 0.0, s);
        break;
    case HMC_TGT_LOGREG:
        if (a.bf16_grad) {
            (void)launch_lr16_grad(a, (const float*)a.ws.x, nullptr, 0, s);
            hipLaunchKernelGGL(k_logreg_finish, elem_grid(a.C * a.tg.D), dim3(256), 0, s, a, (float*)a.ws.x,
                               (float*)nullptr, (float*)a.ws.g, lb_grad_nsplit_t(a), 0, 0, 0.0, 0);
            (void)launch_lr16_logp(a, (const float*)a.ws.x, s);
        } else {
            hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(256), 0, s, a.ws.lr_cnt, (a.C + LR32_CT - 1) / LR32_CT);
            (void)launch_logreg(a, (float*)a.ws.x, nullptr, (float*)a.ws.g, 0, 0, 0.0, 1, s);
        }
        break;
    }
    if (a.tg.kind == HMC_TGT_GAUSS_DENSE && launch_dense_logp(a, s)) return hipGetLastError();
    if (a.f64) HMC_GROUP_DISPATCH(k_logp_finish, double, a, s);
    else HMC_GROUP_DISPATCH(k_logp_finish, float, a, s);
    return hipGetLastError();
}

// One leapfrog drift + gradient + kick (scale ks) on the trajectory buffers
// (xq, pq, gq), the gradient always written to gq and, for logistic
// regression, the data part of logp to lpq.  Used by the NUTS leaves.
hipError_t launch_leapfrog_step(const PlainArgs& a, double ks, hipStream_t s) {
    switch (a.tg.kind) {
    case HMC_TGT_STD_NORMAL:
    case HMC_TGT_GAUSS_DIAG:
        if (a.f64)
            hipLaunchKernelGGL(k_elem_leapfrog<double>, elem_grid(a.C * a.tg.D), dim3(256), 0, s, a,
                               (const double*)a.ws.xq, (double*)a.ws.xq, (double*)a.ws.pq, (double*)a.ws.gq, 3, ks);
        else
            hipLaunchKernelGGL(k_elem_leapfrog<float>, elem_grid(a.C * a.tg.D), dim3(256), 0, s, a,
                               (const float*)a.ws.xq, (float*)a.ws.xq, (float*)a.ws.pq, (float*)a.ws.gq, 3, ks);
        break;
    case HMC_TGT_GAUSS_DENSE:
        (void)launch_dense(a, (const float*)a.ws.xq, (float*)a.ws.xq, (float*)a.ws.pq, (float*)a.ws.gq, 3, ks, s);
        break;
    case HMC_TGT_LOGREG:
        if (a.bf16_grad) {
            (void)launch_lr16_grad(a, (const float*)a.ws.xq, (const float*)a.ws.pq, 1, s);
            hipLaunchKernelGGL(k_logreg_finish, elem_grid(a.C * a.tg.D), dim3(256), 0, s, a, (float*)a.ws.xq,
                               (float*)a.ws.pq, (float*)a.ws.gq, lb_grad_nsplit_t(a), 1, 1, ks, 0);
            (void)launch_lr16_logp(a, (const float*)a.ws.xq, s);
            break;
        }
        (void)launch_logreg(a, (float*)a.ws.xq, (float*)a.ws.pq, (float*)a.ws.gq, 1, 1, ks, 1, s);
        break;
    }
    return hipGetLastError();
}

// Slots per lane of k_elem_last for G lanes per chain (0: D beyond the merged kernels).
static int elem_last_slots(int64_t D, int G) {
    const int64_t need = (D + G - 1) / G;
    const int cap = G == 64 ? 32 : 4;
    for (int ne = 1; ne <= cap; ne *= 2)
        if (need <= ne) return ne;
    return 0;
}

template <typename T>
static void launch_elem_last(const PlainArgs& a, int G, int NE, dim3 grid, hipStream_t s) {
#define HMC_ELEM_LAST(GG, NN)                                                              \
    if (G == GG && NE == NN) {                                                             \
        hipLaunchKernelGGL((k_elem_last<T, GG, NN>), grid, dim3(256), 0, s, a);            \
        return;                                                                            \
    }
    HMC_ELEM_LAST(1, 1) HMC_ELEM_LAST(1, 2) HMC_ELEM_LAST(1, 4)
    HMC_ELEM_LAST(4, 1) HMC_ELEM_LAST(4, 2) HMC_ELEM_LAST(4, 4)
    HMC_ELEM_LAST(16, 1) HMC_ELEM_LAST(16, 2) HMC_ELEM_LAST(16, 4)
    HMC_ELEM_LAST(64, 1) HMC_ELEM_LAST(64, 2) HMC_ELEM_LAST(64, 4) HMC_ELEM_LAST(64, 8)
    HMC_ELEM_LAST(64, 16) HMC_ELEM_LAST(64, 32)
#undef HMC_ELEM_LAST
}

template <typename T>
static void launch_elem_group(int which, const PlainArgs& a, int G, dim3 grid, int vec, hipStream_t s) {
    // which: 0 = first step, 1 = middle step
    if (which == 0) {
        if (G == 1) hipLaunchKernelGGL((k_elem_first<T, 1>), grid, dim3(256), 0, s, a, vec);
        else if (G == 4) hipLaunchKernelGGL((k_elem_first<T, 4>), grid, dim3(256), 0, s, a, vec);
        else if (G == 16) hipLaunchKernelGGL((k_elem_first<T, 16>), grid, dim3(256), 0, s, a, vec);
        else hipLaunchKernelGGL((k_elem_first<T, 64>), grid, dim3(256), 0, s, a, vec);
    } else {
        if (G == 1) hipLaunchKernelGGL((k_elem_mid<T, 1>), grid, dim3(256), 0, s, a);
        else if (G == 4) hipLaunchKernelGGL((k_elem_mid<T, 4>), grid, dim3(256), 0, s, a);
        else if (G == 16) hipLaunchKernelGGL((k_elem_mid<T, 16>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_elem_mid<T, 64>), grid, dim3(256), 0, s, a);
    }
}

// Merged element-wise transition (k_elem_first, k_elem_mid x (L-2), k_elem_last);
// false when the shape is not covered (L < 2 or D > 2048).
static bool launch_elem_transition(const PlainArgs& a, hipStream_t s) {
    const int G = chain_group(a.tg.D);
    const int NE = elem_last_slots(a.tg.D, G);
    if (a.L < 2 || NE == 0) return false;
    const dim3 grid((unsigned)((a.C * G + 255) / 256));
    const int vec = a.f64 ? (a.tg.D % 2 == 0) : (a.tg.D % 4 == 0);
    for (int l = 0; l < a.L; ++l) {
        timer_begin(a, s);
        if (l == a.L - 1) {
            if (a.f64) launch_elem_last<double>(a, G, NE, grid, s);
            else launch_elem_last<float>(a, G, NE, grid, s);
        } else if (a.f64) {
            launch_elem_group<double>(l == 0 ? 0 : 1, a, G, grid, vec, s);
        } else {
            launch_elem_group<float>(l == 0 ? 0 : 1, a, G, grid, vec, s);
        }
        timer_end(a, s, "k_elem_first/mid/last");
    }
    hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, s, a.ws.ctrl);
    return true;
}

// logp = 1/2 x.g of the state (after the bootstrap gradient), summed in the
// order of k_dense_step's end-of-trajectory sum, so that a chain's cached logp
// is bitwise the same whether it was reset or reached in a transition.
template <int NT>
__global__ __launch_bounds__(64 * DS_NW) void k_dense_logp(PlainArgs a) {
    __shared__ double red[DS_NW * 16];
    const int64_t D = a.tg.D;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i16 = lane & 15, g4 = lane >> 4;
    const int64_t c = (int64_t)blockIdx.x * 16 + i16;
    const bool cvalid = c < a.C;
    const int64_t d0 = 16 * w + 4 * g4;
    const float* X = (const float*)a.ws.x;
    const float* Gs = (const float*)a.ws.g;
    double lp = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t d = d0 + v;
        if (w < NT && cvalid && d < D) lp += 0.5 * (double)X[c * D + d] * (double)Gs[c * D + d];
    }
    lp += __shfl_xor(lp, 16, 64);
    lp += __shfl_xor(lp, 32, 64);
    if (g4 == 0) red[w * 16 + i16] = lp;
    __syncthreads();
    if (threadIdx.x < 16 && cvalid) {
        double sl = 0.0;
        for (int ww = 0; ww < DS_NW; ++ww) sl += red[ww * 16 + i16];
        a.ws.logp[c] = sl;
    }
}

static bool launch_dense_logp(const PlainArgs& a, hipStream_t s) {
    const int nt = (int)((a.tg.D + 15) / 16);
    if (nt > DS_NW) return false;
    const dim3 grid((unsigned)((a.C + 15) / 16)), blk(64 * DS_NW);
    switch (nt) {
    case 1: hipLaunchKernelGGL(k_dense_logp<1>, grid, blk, 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_dense_logp<2>, grid, blk, 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_dense_logp<3>, grid, blk, 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_dense_logp<4>, grid, blk, 0, s, a); break;
    case 5: hipLaunchKernelGGL(k_dense_logp<5>, grid, blk, 0, s, a); break;
    case 6: hipLaunchKernelGGL(k_dense_logp<6>, grid, blk, 0, s, a); break;
    case 7: hipLaunchKernelGGL(k_dense_logp<7>, grid, blk, 0, s, a); break;
    default: hipLaunchKernelGGL(k_dense_logp<8>, grid, blk, 0, s, a); break;
    }
    return true;
}

template <int NT>
static void launch_dense_step_nt(const PlainArgs& a, int first, int last, hipStream_t s) {
    const dim3 grid((unsigned)((a.C + 15) / 16));
    const size_t lds = (size_t)16 * NT * (16 * NT + 4) * sizeof(float);
    if (first && last) {
        allow_lds(k_dense_step<NT, true, true>, lds);
        hipLaunchKernelGGL((k_dense_step<NT, true, true>), grid, dim3(64 * DS_NW), lds, s, a);
    } else if (first) {
        allow_lds(k_dense_step<NT, true, false>, lds);
        hipLaunchKernelGGL((k_dense_step<NT, true, false>), grid, dim3(64 * DS_NW), lds, s, a);
    } else if (last) {
        allow_lds(k_dense_step<NT, false, true>, lds);
        hipLaunchKernelGGL((k_dense_step<NT, false, true>), grid, dim3(64 * DS_NW), lds, s, a);
    } else {
        allow_lds(k_dense_step<NT, false, false>, lds);
        hipLaunchKernelGGL((k_dense_step<NT, false, false>), grid, dim3(64 * DS_NW), lds, s, a);
    }
}

// Merged dense transition (k_dense_step x L); false when D > 128.
static bool launch_dense_transition(const PlainArgs& a, hipStream_t s) {
    const int nt = (int)((a.tg.D + 15) / 16);
    if (nt > DS_NW) return false;
    for (int l = 0; l < a.L; ++l) {
        const int first = l == 0, last = l == a.L - 1;
        timer_begin(a, s);
        switch (nt) {
        case 1: launch_dense_step_nt<1>(a, first, last, s); break;
        case 2: launch_dense_step_nt<2>(a, first, last, s); break;
        case 3: launch_dense_step_nt<3>(a, first, last, s); break;
        case 4: launch_dense_step_nt<4>(a, first, last, s); break;
        case 5: launch_dense_step_nt<5>(a, first, last, s); break;
        case 6: launch_dense_step_nt<6>(a, first, last, s); break;
        case 7: launch_dense_step_nt<7>(a, first, last, s); break;
        default: launch_dense_step_nt<8>(a, first, last, s); break;
        }
        timer_end(a, s, "k_dense_step");
    }
    hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, s, a.ws.ctrl);
    return true;
}

hipError_t launch_plain_transition(const PlainArgs& a, bool copy_proposal, hipStream_t s) {
    if ((a.tg.kind == HMC_TGT_STD_NORMAL || a.tg.kind == HMC_TGT_GAUSS_DIAG) && launch_elem_transition(a, s))
        return hipGetLastError();
    if (a.tg.kind == HMC_TGT_GAUSS_DENSE && launch_dense_transition(a, s)) return hipGetLastError();
    if (a.f64) HMC_GROUP_DISPATCH(k_begin, double, a, s);
    else HMC_GROUP_DISPATCH(k_begin, float, a, s);
    for (int l = 0; l < a.L; ++l) {
        const bool last = l == a.L - 1;
        const double ks = last ? 0.5 : 1.0;
        switch (a.tg.kind) {
        case HMC_TGT_STD_NORMAL:
        case HMC_TGT_GAUSS_DIAG:
            timer_begin(a, s);
            if (a.f64)
                hipLaunchKernelGGL(k_elem_leapfrog<double>, elem_grid(a.C * a.tg.D), dim3(256), 0, s, a,
                                   (const double*)a.ws.xq, (double*)a.ws.xq, (double*)a.ws.pq,
                                   last ? (double*)a.ws.gq : (double*)nullptr, 3, ks);
            else
                hipLaunchKernelGGL(k_elem_leapfrog<float>, elem_grid(a.C * a.tg.D), dim3(256), 0, s, a,
                                   (const float*)a.ws.xq, (float*)a.ws.xq, (float*)a.ws.pq,
                                   last ? (float*)a.ws.gq : (float*)nullptr, 3, ks);
            timer_end(a, s, "k_elem_leapfrog");
            break;
        case HMC_TGT_GAUSS_DENSE:
            timer_begin(a, s);
            (void)launch_dense(a, (const float*)a.ws.xq, (float*)a.ws.xq, (float*)a.ws.pq,
                         last ? (float*)a.ws.gq : nullptr, 3, ks, s);
            timer_end(a, s, "k_dense_leapfrog");
            break;
        case HMC_TGT_LOGREG:
            if (a.bf16_grad) {
                timer_begin(a, s);
                (void)launch_lr16_grad(a, (const float*)a.ws.xq, (const float*)a.ws.pq, 1, s);
                timer_end(a, s, "k_lr16_grad");
                hipLaunchKernelGGL(k_logreg_finish, elem_grid(a.C * a.tg.D), dim3(256), 0, s, a, (float*)a.ws.xq,
                                   (float*)a.ws.pq, last ? (float*)a.ws.gq : (float*)nullptr,
                                   lb_grad_nsplit_t(a), 1, 1, ks, 0);
                if (last) (void)launch_lr16_logp(a, (const float*)a.ws.xq, s);
                break;
            }
            (void)launch_logreg(a, (float*)a.ws.xq, (float*)a.ws.pq, last ? (float*)a.ws.gq : nullptr, 1, 1, ks,
                          last ? 1 : 0, s);
            break;
        }
    }
    if (a.f64) HMC_GROUP_DISPATCH(k_end, double, a, s);
    else HMC_GROUP_DISPATCH(k_end, float, a, s);
    if (copy_proposal) {
        if (a.f64) hipLaunchKernelGGL(k_copy_proposal<double>, elem_grid(a.C * a.tg.D), dim3(256), 0, s, a);
        else hipLaunchKernelGGL(k_copy_proposal<float>, elem_grid(a.C * a.tg.D), dim3(256), 0, s, a);
    }
    hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, s, a.ws.ctrl);
    return hipGetLastError();
}

// One transition of every job, in the order of launch_plain_transition for a
// BF16-gradient logistic request: begin, L x (gradient, finish), logit pass and
// its split sum after the last gradient, end, tick.  Every job has the same
// lanes per chain G, padded width and L (the batch class).
hipError_t launch_lr16_transition_multi(const Lr16Job* jobs_host, const Lr16Job* jobs_dev, int njobs,
                                        hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    const PlainArgs& a0 = jobs_host[0].a;
    const int G = chain_group(a0.tg.D);
    int64_t tot[LR16_KINDS];
    for (int k = 0; k < LR16_KINDS; ++k)
        tot[k] = jobs_host[njobs - 1].begin[k] + jobs_host[njobs - 1].nblk[k];
    const dim3 gg((unsigned)tot[LR16_KIND_GROUP]);
    if (G == 1) hipLaunchKernelGGL(k_begin_multi<1>, gg, dim3(256), 0, s, jobs_dev, njobs);
    else if (G == 4) hipLaunchKernelGGL(k_begin_multi<4>, gg, dim3(256), 0, s, jobs_dev, njobs);
    else if (G == 16) hipLaunchKernelGGL(k_begin_multi<16>, gg, dim3(256), 0, s, jobs_dev, njobs);
    else hipLaunchKernelGGL(k_begin_multi<64>, gg, dim3(256), 0, s, jobs_dev, njobs);
    for (int l = 0; l < a0.L; ++l) {
        const int last = l == a0.L - 1;
        hipError_t e = launch_lr16_kind_multi(LR16_KIND_GRAD, a0.tg.D, jobs_dev, njobs, tot[LR16_KIND_GRAD], s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_finish_multi, dim3((unsigned)tot[LR16_KIND_FINISH]), dim3(256), 0, s, jobs_dev, njobs,
                           last);
        if (last) {
            e = launch_lr16_kind_multi(LR16_KIND_LOGP, a0.tg.D, jobs_dev, njobs, tot[LR16_KIND_LOGP], s);
            if (e != hipSuccess) return e;
            e = launch_lr16_kind_multi(LR16_KIND_LPSUM, a0.tg.D, jobs_dev, njobs, tot[LR16_KIND_LPSUM], s);
            if (e != hipSuccess) return e;
        }
    }
    if (G == 1) hipLaunchKernelGGL(k_end_multi<1>, gg, dim3(256), 0, s, jobs_dev, njobs);
    else if (G == 4) hipLaunchKernelGGL(k_end_multi<4>, gg, dim3(256), 0, s, jobs_dev, njobs);
    else if (G == 16) hipLaunchKernelGGL(k_end_multi<16>, gg, dim3(256), 0, s, jobs_dev, njobs);
    else hipLaunchKernelGGL(k_end_multi<64>, gg, dim3(256), 0, s, jobs_dev, njobs);
    hipLaunchKernelGGL(k_tick_multi, dim3((unsigned)((njobs + 63) / 64)), dim3(64), 0, s, jobs_dev, njobs);
    return hipGetLastError();
}

// Grid layout of a batch: block ranges of every job for every kernel kind
// (gradient and logit ranges start at multiples of 8); false if a grid would
// exceed 2^31 blocks.
bool lr16_layout(Lr16Job* jobs, int njobs) {
    int64_t next[LR16_KINDS] = {0, 0, 0, 0, 0};
    for (int j = 0; j < njobs; ++j) {
        Lr16Job& jb = jobs[j];
        lr16_job_shape(jb.a, &jb);
        const int G = chain_group(jb.a.tg.D);
        jb.nblk[LR16_KIND_GROUP] = (jb.a.C * G + 255) / 256;
        jb.nblk[LR16_KIND_FINISH] = elem_grid(jb.a.C * jb.a.tg.D).x;
        for (int k = 0; k < LR16_KINDS; ++k) {
            if (k == LR16_KIND_GRAD || k == LR16_KIND_LOGP) next[k] = (next[k] + 7) / 8 * 8;
            jb.begin[k] = next[k];
            next[k] += jb.nblk[k];
            if (next[k] > 0x7fffffffLL) return false;
        }
    }
    return true;
}

}  // namespace hmc
