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
__global__ __launch_bounds__(256) void k_begin(PlainArgs a) {
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

template <typename T, int G>
__global__ __launch_bounds__(256) void k_end(PlainArgs a) {
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

template <typename XT, int GT>
__global__ __launch_bounds__(256) void k_logreg_partial(PlainArgs a, const float* __restrict__ xsrc,
                                                        const float* __restrict__ psrc, int drift, int want_logp,
                                                        int64_t rows_per_split) {
    extern __shared__ float lds[];
    const int64_t D = a.tg.D, N = a.tg.N, C = a.C;
    const int K4 = (int)((D + 3) / 4);
    const int ntiles = (int)((D + 15) / 16);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i16 = lane & 15, g4 = lane >> 4;
    const int64_t c0 = (int64_t)blockIdx.x * 16;
    const int s = blockIdx.y;
    const XT* X = (const XT*)a.tg.X;
    const uint8_t* y = a.tg.y;
    float* th = lds;                         // [4*K4][17] theta^T (after drift)
    float* red = lds + 4 * K4 * 17;          // [16*ntiles][17] gradient reduction
    double* redlp = (double*)(lds + ((4 * K4 * 17 + 16 * ntiles * 17 + 1) & ~1));   // [16]

    // theta tile (with drift): thread loops over (d, chain)
    for (int idx = threadIdx.x; idx < 4 * K4 * 16; idx += blockDim.x) {
        const int d = idx / 16, j = idx % 16;
        const int64_t c = c0 + j;
        float v = 0.f;
        if (d < D && c < C) {
            v = xsrc[c * D + d];
            // the drift is recomputed (same fmaf) and stored by k_logreg_finish
            if (drift)
                v = fmaf(a.ws.scale ? (float)(a.ws.eps[c] * a.ws.scale[d]) : (float)a.ws.eps[c], psrc[c * D + d], v);
        }
        th[d * 17 + j] = v;
    }
    __syncthreads();

    const int64_t r_begin = (int64_t)s * rows_per_split;
    const int64_t r_end = r_begin + rows_per_split < N ? r_begin + rows_per_split : N;
    floatx4 gacc[GT];
#pragma unroll
    for (int m = 0; m < GT; ++m) gacc[m] = floatx4{0.f, 0.f, 0.f, 0.f};
    double lp = 0.0;

    for (int64_t n0 = r_begin + 16 * w; n0 < r_end; n0 += 64) {
        floatx4 sacc = {0.f, 0.f, 0.f, 0.f};
        const int64_t arow = n0 + i16;
        const bool arow_ok = arow < r_end;
        for (int ks = 0; ks < K4; ++ks) {
            const int64_t col = 4 * ks + g4;
            const float av = (arow_ok && col < D) ? ld_x<XT>(X, arow * D + col) : 0.f;
            const float bv = th[(4 * ks + g4) * 17 + i16];
            sacc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, sacc, 0, 0, 0);
        }
        float r[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t row = n0 + 4 * g4 + v;
            const bool ok = row < r_end;
            const float yv = ok ? (float)y[row] : 0.f;
            r[v] = ok ? yv - sigmoidf_(sacc[v]) : 0.f;
            if (want_logp && ok) lp -= (double)softplusf_(yv > 0.5f ? -sacc[v] : sacc[v]);
        }
#pragma unroll
        for (int m = 0; m < GT; ++m) {
            if (m >= ntiles) break;
            const int64_t dcol = 16 * m + i16;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = n0 + 4 * g4 + v;
                const float av = (row < r_end && dcol < D) ? ld_x<XT>(X, row * D + dcol) : 0.f;
                gacc[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, r[v], gacc[m], 0, 0, 0);
            }
        }
    }
    // log-prob partial: lanes of the same chain are i16, i16+16, +32, +48
    lp += __shfl_xor(lp, 16, 64);
    lp += __shfl_xor(lp, 32, 64);

    // wave partials summed in wave order (deterministic)
    for (int ww = 0; ww < 4; ++ww) {
        if (w == ww) {
#pragma unroll
            for (int m = 0; m < GT; ++m) {
                if (m >= ntiles) break;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int d = 16 * m + 4 * g4 + v;
                    float* dst = &red[d * 17 + i16];
                    *dst = (ww == 0) ? gacc[m][v] : *dst + gacc[m][v];
                }
            }
            if (lane < 16) redlp[lane] = (ww == 0) ? lp : redlp[lane] + lp;
        }
        __syncthreads();
    }
    for (int idx = threadIdx.x; idx < 16 * D; idx += blockDim.x) {
        const int j = idx / (int)D;
        const int d = idx % (int)D;
        const int64_t c = c0 + j;
        if (c < C) a.ws.part_g[((int64_t)s * C + c) * D + d] = red[d * 17 + j];
    }
    if (want_logp && threadIdx.x < 16 && c0 + threadIdx.x < C)
        a.ws.part_lp[(int64_t)s * C + c0 + threadIdx.x] = redlp[threadIdx.x];
}

// drift (same fmaf as the partial kernel), sum the split partials in split
// order, add the prior gradient, kick.
__global__ __launch_bounds__(256) void k_logreg_finish(PlainArgs a, float* __restrict__ xd, float* __restrict__ pd,
                                                       float* __restrict__ gd, int nsplit, int drift, int kick,
                                                       double kick_scale, int want_logp) {
    const int64_t D = a.tg.D, C = a.C;
    const int64_t n = C * D;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
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

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static int chain_group(int64_t D) {
    if (D <= 4) return 1;
    if (D <= 16) return 4;
    if (D <= 64) return 16;
    return 64;
}

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
    // enough workgroups to fill 256 CUs several times, splits of >= 64 rows
    const int64_t tiles = (C + 15) / 16;
    int64_t want = (1024 + tiles - 1) / tiles;
    int64_t maxs = (N + 63) / 64;
    if (want > maxs) want = maxs;
    if (want < 1) want = 1;
    if (want > 64) want = 64;
    return want;
}

static size_t logreg_lds(int64_t D) {
    const int K4 = (int)((D + 3) / 4);
    const int ntiles = (int)((D + 15) / 16);
    return (size_t)((4 * K4 * 17 + 16 * ntiles * 17 + 1) & ~1) * sizeof(float) + 16 * sizeof(double);
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

template <typename XT>
static void launch_logreg_partial_t(const PlainArgs& a, dim3 grid, size_t lds, hipStream_t s, const float* xs,
                                    const float* ps, int drift, int want_logp, int64_t rows) {
    const int ntiles = (int)((a.tg.D + 15) / 16);
    if (ntiles <= 2) hipLaunchKernelGGL((k_logreg_partial<XT, 2>), grid, dim3(256), lds, s, a, xs, ps, drift, want_logp, rows);
    else if (ntiles <= 4) hipLaunchKernelGGL((k_logreg_partial<XT, 4>), grid, dim3(256), lds, s, a, xs, ps, drift, want_logp, rows);
    else if (ntiles <= 8) hipLaunchKernelGGL((k_logreg_partial<XT, 8>), grid, dim3(256), lds, s, a, xs, ps, drift, want_logp, rows);
    else if (ntiles <= 16) hipLaunchKernelGGL((k_logreg_partial<XT, 16>), grid, dim3(256), lds, s, a, xs, ps, drift, want_logp, rows);
    else {
        allow_lds(k_logreg_partial<XT, 32>, lds);
        hipLaunchKernelGGL((k_logreg_partial<XT, 32>), grid, dim3(256), lds, s, a, xs, ps, drift, want_logp, rows);
    }
}

// x (in place, drifted when drift), p (kicked when kick), g into gd if not null
// largest split count the workspace is sized for (the autotuner tries up to 2x the default)
int64_t logreg_nsplit_cap(int64_t N, int64_t C) {
    int64_t cap = 2 * logreg_nsplit(N, C);
    const int64_t maxs = (N + 63) / 64;
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

static hipError_t launch_logreg(const PlainArgs& a, float* x, float* p, float* gd, int drift, int kick, double ks,
                                int want_logp, hipStream_t s) {
    const int64_t nsplit = logreg_nsplit_t(a);
    const int64_t rows = (a.tg.N + nsplit - 1) / nsplit;
    const size_t lds = logreg_lds(a.tg.D);
    const dim3 grid((unsigned)((a.C + 15) / 16), (unsigned)nsplit);
    timer_begin(a, s);
    if (a.tg.x_bf16)
        launch_logreg_partial_t<uint16_t>(a, grid, lds, s, x, p, drift, want_logp, rows);
    else
        launch_logreg_partial_t<float>(a, grid, lds, s, x, p, drift, want_logp, rows);
    timer_end(a, s, "k_logreg_partial");
    hipLaunchKernelGGL(k_logreg_finish, elem_grid(a.C * a.tg.D), dim3(256), 0, s, a, x, p, gd, (int)nsplit, drift,
                       kick, ks, want_logp);
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
            (void)launch_logreg(a, (float*)a.ws.x, nullptr, (float*)a.ws.g, 0, 0, 0.0, 1, s);
        }
        break;
    }
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

hipError_t launch_plain_transition(const PlainArgs& a, bool copy_proposal, hipStream_t s) {
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

}  // namespace hmc
