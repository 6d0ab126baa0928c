// k_fused.hip -- fused persistent form: each workgroup owns a tile of chains
// and runs whole transitions (momentum, L leapfrog steps, energy, accept,
// select, dual averaging, sample and trace writes) with the chain state in
// registers and LDS.  HBM traffic per transition is the kept sample and
// trace rows; target data stays in registers/LDS/L2.
//
//   elementwise  N(0, I), diagonal Gaussian: G lanes per chain, 4-dim Philox
//                blocks per lane, reductions across the lane group
//   dense        g = -P x on v_mfma_f32_16x16x4f32; 16 chains per workgroup,
//                P held in VGPRs as A operands, x^T staged in LDS (double
//                buffered, one barrier per leapfrog step)
//   logreg       see k_fused_logreg.hip
#include "hmc_internal.hpp"

namespace hmc {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Per-chain bookkeeping at the end of a transition, executed identically by
// every lane that holds a part of the chain.
struct ChainCtl {
    double logp, eps;
    DualAvg da;
};

__device__ __forceinline__ void after_decision(const FusedRun& r, int64_t C, int64_t c, int64_t i, bool acc,
                                               double lar, double dh, double lp_new, ChainCtl& s, bool writer) {
    const double eps_used = s.eps;
    if (r.adapt && i < r.n_burnin) {
        const double alpha = lar < 0.0 ? exp(lar) : 1.0;
        if (r.adapt_kind == HMC_ADAPT_SIMPLE) {
            s.eps = simple_adapt(s.eps, alpha, r.target_accept, r.rate);
        } else {
            const int64_t m = r.m_offset + i + 1;
            const double log_eps = dual_avg_update(s.da, (double)m, alpha, r.target_accept, r.gamma, r.t0, r.kappa);
            s.eps = (m < r.adapt_total) ? exp(log_eps) : exp(s.da.log_eps_bar);
        }
    }
    if (!writer) return;
    if (i >= r.n_burnin) {
        const int64_t k = (i - r.n_burnin) * C + c;
        if (r.trace.step_size) r.trace.step_size[k] = eps_used;
        if (r.trace.is_accepted) r.trace.is_accepted[k] = acc ? 1 : 0;
        if (r.trace.log_accept_ratio) r.trace.log_accept_ratio[k] = lar;
        if (r.trace.target_log_prob) r.trace.target_log_prob[k] = lp_new;
    }
    if (r.out.is_accepted) r.out.is_accepted[c] = acc ? 1 : 0;
    if (r.out.log_accept_ratio) r.out.log_accept_ratio[c] = lar;
    if (r.out.target_log_prob) r.out.target_log_prob[c] = lp_new;
    if (r.out.delta_h) r.out.delta_h[c] = dh;
}

// ---------------------------------------------------------------------------
// Elementwise targets.  NB blocks of 4 dims per lane; lane j of a group owns
// blocks j, j + G, ...
// ---------------------------------------------------------------------------
// EX: a transform and / or the replica exchange inside the launch (a template
// parameter, so that plain runs carry neither).  With the exchange, lane group
// (slot) s holds replica s % K of chain index s / K; K divides the 64 / G slots
// of a wavefront, so the two chains of every pair exchange by shuffles G lanes
// apart.
template <typename T, int G, int NB, bool EX>
__device__ __forceinline__ void fused_elem_body(const PlainArgs& a, const FusedRun& r, int64_t lblock) {
    const int64_t gid = lblock * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x % G;
    const int nrep = EX ? r.remc_K : 0;
    const int64_t slot = gid / G;
    const int krep = nrep > 1 ? (int)(slot % nrep) : 0;
    const int64_t c = nrep > 1 ? krep * r.remc_M + slot / nrep : slot;
    const bool active = slot < a.C;                  // with the exchange: chain index slot / K < M
    const int64_t cc = active ? c : 0;
    const int64_t D = a.tg.D;
    const bool diag = a.tg.kind == HMC_TGT_GAUSS_DIAG;
    T* X = (T*)a.ws.x;
    T* Gr = (T*)a.ws.g;
    const T* prec = (const T*)a.tg.prec;

    // Transformed kernel (x = shift + scale z): the chain runs in z = x / scale,
    // whose precision is prec scale^2; states are converted at load and store.
    const double* sc = EX ? a.ws.scale : nullptr;
    const bool trs = sc != nullptr;
    // the scale in the state's precision, staged once in LDS for the stores
    // of x (a lane group covers 4 G NB >= D dims)
    __shared__ T sc_lds[EX ? 4 * G * NB : 1];
    if (EX) {
        if (trs)
            for (int64_t d = threadIdx.x; d < D; d += blockDim.x) sc_lds[d] = (T)sc[d];
        __syncthreads();
    }
    T x[NB][4], g[NB][4], pr[NB][4];
    bool ok[NB][4];
#pragma unroll
    for (int k = 0; k < NB; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t d = 4 * (lane + (int64_t)G * k) + j;
            ok[k][j] = active && d < D;
            x[k][j] = ok[k][j] ? X[cc * D + d] : (T)0;
            g[k][j] = ok[k][j] ? Gr[cc * D + d] : (T)0;
            pr[k][j] = ok[k][j] ? (diag ? prec[d] : (T)1) : (T)0;
            if (sc && ok[k][j]) {
                const double sd = sc[d];
                pr[k][j] = (T)((double)pr[k][j] * sd * sd);
                x[k][j] = (T)((double)x[k][j] / sd);
                g[k][j] = (T)((double)g[k][j] * sd);
            }
        }
    ChainCtl s;
    s.logp = a.ws.logp[cc];
    s.eps = a.ws.eps[cc];
    s.da = a.ws.da[cc];
    const double bt = a.ws.beta ? a.ws.beta[cc] : 1.0;   // inverse temperature of the chain

    for (int64_t i = 0; i < r.n_transitions; ++i) {
        const uint32_t t = (uint32_t)(r.t_begin + i);
        const T eps = (T)s.eps;                   // drift
        const T half = (T)(0.5 * s.eps * bt);     // kicks: beta eps (replica exchange; beta = 1 otherwise)
        const T keps = (T)(s.eps * bt);
        T xn[NB][4], pn[NB][4], gn[NB][4];
        double dk = 0.0;
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            T z[4];
            momentum4<T>(a.key, (uint32_t)cc, t, (uint32_t)(lane + G * k), z,
                         4 * (lane + (int64_t)G * k) + 2 < D);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const T p0 = ok[k][j] ? z[j] : (T)0;
                dk -= 0.5 * (double)p0 * (double)p0;
                xn[k][j] = x[k][j];
                pn[k][j] = fma(half, g[k][j], p0);
            }
        }
        for (int l = 0; l < a.L; ++l) {
            const T ke = (l == a.L - 1) ? half : keps;
#pragma unroll
            for (int k = 0; k < NB; ++k)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    xn[k][j] = fma(eps, pn[k][j], xn[k][j]);
                    gn[k][j] = -pr[k][j] * xn[k][j];
                    pn[k][j] = fma(ke, gn[k][j], pn[k][j]);
                }
        }
        double lp = 0.0;
#pragma unroll
        for (int k = 0; k < NB; ++k)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                dk += 0.5 * (double)pn[k][j] * (double)pn[k][j];
                lp += 0.5 * (double)xn[k][j] * (double)gn[k][j];
            }
        dk = group_sum<G>(dk);
        lp = group_sum<G>(lp);
        const double dh = -(bt * lp) + bt * s.logp + dk;
        const double lar = log_accept_ratio_of(dh);
        const bool acc = log_accept_uniform(a.key, (uint32_t)cc, t) < lar;
        if (acc) {
#pragma unroll
            for (int k = 0; k < NB; ++k)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    x[k][j] = xn[k][j];
                    g[k][j] = gn[k][j];
                }
            s.logp = lp;
        }
        // kept sample and proposal outputs of this transition
        auto store_outputs = [&]() {
            if (r.samples && i >= r.n_burnin) {
                T* smp = (T*)r.samples + ((i - r.n_burnin) * a.C + c) * D;
                if (EX && trs) {
                    // an index the compiler cannot see through keeps the LDS
                    // reads here: hoisted out of the transition loop they
                    // would hold NB 4 registers for the whole run
                    int l4 = 4 * lane;
                    asm volatile("" : "+v"(l4));
#pragma unroll
                    for (int k = 0; k < NB; ++k)
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            if (ok[k][j]) smp[4 * (lane + (int64_t)G * k) + j] = x[k][j] * sc_lds[l4 + 4 * G * k + j];
                } else {
#pragma unroll
                    for (int k = 0; k < NB; ++k)
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            if (ok[k][j]) smp[4 * (lane + (int64_t)G * k) + j] = x[k][j];
                }
            }
            if (r.out.proposed_state || r.out.proposed_momentum) {
                int l4 = 4 * lane;
                if (EX) asm volatile("" : "+v"(l4));
#pragma unroll
                for (int k = 0; k < NB; ++k)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (ok[k][j]) {
                            const int64_t d = 4 * (lane + (int64_t)G * k) + j;
                            if (r.out.proposed_state)
                                ((T*)r.out.proposed_state)[c * D + d] = (EX && trs) ? xn[k][j] * sc_lds[l4 + 4 * G * k + j] : xn[k][j];
                            if (r.out.proposed_momentum) ((T*)r.out.proposed_momentum)[c * D + d] = pn[k][j];
                        }
            }
        };
        if (EX) {
            // traces and adaptation record the transition; the exchange follows
            // it, and the kept sample is the state after the exchange
            if (active) after_decision(r, a.C, c, i, acc, lar, dh, s.logp, s, lane == 0);
            if (nrep > 1) {
                const int par = (int)(t & 1u);
                const bool a_side = krep >= par && ((krep - par) & 1) == 0 && krep + 1 < nrep;
                const bool b_side = krep >= par + 1 && ((krep - 1 - par) & 1) == 0;
                const int wl = threadIdx.x & 63;
                const int src = a_side ? wl + G : (b_side ? wl - G : wl);
                const double lp_o = __shfl(s.logp, src, 64);
                const double bt_o = __shfl(bt, src, 64);
                bool swp = false;
                if (active && (a_side || b_side)) {
                    const int64_t ca = a_side ? c : c - r.remc_M;
                    const double la = a_side ? s.logp : lp_o, lb = a_side ? lp_o : s.logp;
                    const double ba = a_side ? bt : bt_o, bb = a_side ? bt_o : bt;
                    swp = log_uniform52(a.key, (uint32_t)ca, t, TAG_SWAP) < (ba - bb) * (lb - la);
                }
#pragma unroll
                for (int k = 0; k < NB; ++k)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const T xo = __shfl(x[k][j], src, 64), go = __shfl(g[k][j], src, 64);
                        if (swp) {
                            x[k][j] = xo;
                            g[k][j] = go;
                        }
                    }
                if (swp) s.logp = lp_o;
                if (active && r.swapped && i >= r.n_burnin && lane == 0)
                    r.swapped[(i - r.n_burnin) * a.C + c] = swp ? 1 : 0;
            }
            if (active) store_outputs();
        } else if (active) {
            store_outputs();
            after_decision(r, a.C, c, i, acc, lar, dh, s.logp, s, lane == 0);
        }
    }
    if (!active) return;
    // a fresh read of the scale: reusing the values loaded before the loop
    // would hold them in registers for the whole run
    if (EX) asm volatile("" ::: "memory");
#pragma unroll
    for (int k = 0; k < NB; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (ok[k][j]) {
                const int64_t d = 4 * (lane + (int64_t)G * k) + j;
                X[c * D + d] = (EX && trs) ? (T)((double)x[k][j] * sc[d]) : x[k][j];
                Gr[c * D + d] = (EX && trs) ? (T)((double)g[k][j] / sc[d]) : g[k][j];
            }
    if (lane == 0) {
        a.ws.logp[c] = s.logp;
        a.ws.eps[c] = s.eps;
        a.ws.da[c] = s.da;
    }
}

template <typename T, int G, int NB, bool EX>
__global__ __launch_bounds__(256) void k_fused_elem(PlainArgs a, FusedRun r) {
    fused_elem_body<T, G, NB, EX>(a, r, blockIdx.x);
}

// Several requests of one shape class in one grid: block b runs job j with
// jobs[j].block_begin <= b < jobs[j + 1].block_begin.
template <typename T, int G, int NB>
__global__ __launch_bounds__(256) void k_fused_elem_multi(const ElemJob* __restrict__ jobs, int njobs) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].block_begin <= (int64_t)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const PlainArgs a = jobs[lo].a;
    const FusedRun r = jobs[lo].r;
    fused_elem_body<T, G, NB, false>(a, r, (int64_t)blockIdx.x - jobs[lo].block_begin);
}

// ---------------------------------------------------------------------------
// Dense Gaussian on MFMA.  16 chains per workgroup (the N dimension), 8 waves
// (two per SIMD, so that one wave's MFMAs cover the other's LDS and barrier
// waits), wave w owns M-tiles w, w + NW, ...; lane (g4 = lane/16, i16 = lane%16) holds rows
// 16 mt + 4 g4 + v (v = 0..3) of chain i16 -- exactly the 4 dims of Philox
// block 4 mt + g4, so each lane draws its own momenta.
//
// NT = ceil(D / 16) tiles is a template parameter, so the contraction over
// the 4 NT k-steps is fully unrolled with no guards: P is zero-padded in the
// A operands and rows D .. 16 NT of x stay exactly zero, so the padding adds
// zeros.  Every wave runs MT tiles (a wave's tiles past NT multiply zeros on
// its own SIMD while the other SIMDs finish theirs), and each tile keeps two
// accumulators (even / odd k-steps) so that consecutive MFMAs are independent.
//
// The contraction index is assigned as k = g4 KM + ks (lane group g4 supplies
// dims g4 KM .. g4 KM + KM - 1 over the k-steps ks), so with x staged chain-
// major in LDS ([16 chains][16 NT + 4], the pad making the 16 chains of a
// lane group hit distinct bank quads) each lane fetches the B operands of 4
// consecutive k-steps with one ds_read_b128 and writes its own 4 dims of a
// tile with one ds_write_b128.
// ---------------------------------------------------------------------------
constexpr int DENSE_NW = 8;                 // waves per workgroup (2 per SIMD)

// EX: a transform and / or the replica exchange inside the launch (a template
// parameter, so that plain runs carry neither).  With the exchange, slot i16
// of the workgroup holds replica i16 % K of chain m = 16 / K * block + i16 / K,
// so the two chains of every pair sit in neighbouring lanes of one wavefront
// and exchange by shuffles.
template <int NT, bool EX>
__global__ __launch_bounds__(64 * DENSE_NW) void k_fused_dense(PlainArgs a, FusedRun r) {
    constexpr int MT = (NT + DENSE_NW - 1) / DENSE_NW;
    constexpr int KM = 4 * NT;
    extern __shared__ float lds[];
    const int64_t D = a.tg.D;
    const int ntiles = NT;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i16 = lane & 15, g4 = lane >> 4;
    const int nrep = EX ? r.remc_K : 0;
    const int krep = nrep > 1 ? i16 % nrep : 0;
    const int64_t mrep = nrep > 1 ? (int64_t)blockIdx.x * (16 / nrep) + i16 / nrep : 0;
    const int64_t c = nrep > 1 ? krep * r.remc_M + mrep : (int64_t)blockIdx.x * 16 + i16;
    const bool cvalid = nrep > 1 ? mrep < r.remc_M : c < a.C;
    const int64_t cc = cvalid ? c : 0;
    constexpr int XS = 16 * NT + 4;                 // floats per chain row in LDS
    float* xs0 = lds;                               // [16][XS] x 2 buffers
    float* xs1 = lds + 16 * XS;
    double* red = (double*)(lds + 2 * 16 * XS);     // [2][NW][16] (dk, lp)
    const float* P = (const float*)a.tg.prec;
    float* X = (float*)a.ws.x;
    float* Gr = (float*)a.ws.g;

    // Transformed kernel (x = shift + scale z, EX): the chain runs in
    // z = x / scale, whose precision matrix is S P S (S = diag(scale)); states
    // are converted at load and store.
    const double* sc = EX ? a.ws.scale : nullptr;
    const bool trs = sc != nullptr;
    __shared__ float sc_lds[EX ? 16 * NT : 1];     // the scale, for the stores of x
    if (EX) {
        if (trs)
            for (int d = threadIdx.x; d < D; d += blockDim.x) sc_lds[d] = (float)sc[d];
        __syncthreads();
    }
    // P as A operands: pa[m][ks] = P[16 mt + i16][g4 KM + ks]
    float pa[MT][KM];
    bool tile_ok[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        const int mt = w + DENSE_NW * m;
        tile_ok[m] = mt < ntiles;
        const int64_t row = 16 * mt + i16;
#pragma unroll
        for (int ks = 0; ks < KM; ++ks) {
            const int64_t col = (int64_t)g4 * KM + ks;
            const bool in = tile_ok[m] && row < D && col < D;
            pa[m][ks] = in ? P[row * D + col] : 0.f;
            if (sc && in) pa[m][ks] = (float)((double)pa[m][ks] * sc[row] * sc[col]);
        }
    }
    float x[MT][4], g[MT][4];
    bool ok[MT][4];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t d = 16 * (w + DENSE_NW * m) + 4 * g4 + v;
            ok[m][v] = tile_ok[m] && cvalid && d < D;
            x[m][v] = ok[m][v] ? X[cc * D + d] : 0.f;
            g[m][v] = ok[m][v] ? Gr[cc * D + d] : 0.f;
            if (sc && ok[m][v]) {
                x[m][v] = (float)((double)x[m][v] / sc[d]);
                g[m][v] = (float)((double)g[m][v] * sc[d]);
            }
        }
    ChainCtl s;
    s.logp = a.ws.logp[cc];
    s.eps = a.ws.eps[cc];
    s.da = a.ws.da[cc];
    const double bt = a.ws.beta ? a.ws.beta[cc] : 1.0;   // inverse temperature of the chain
    int buf = 0;

    for (int64_t i = 0; i < r.n_transitions; ++i) {
        const uint32_t t = (uint32_t)(r.t_begin + i);
        const float eps = (float)s.eps, half = (float)(0.5 * s.eps * bt), keps = (float)(s.eps * bt);
        float xn[MT][4], pn[MT][4], gn[MT][4];
        double dk = 0.0;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            float z[4];
            momentum4<float>(a.key, (uint32_t)cc, t, (uint32_t)(4 * (w + DENSE_NW * m) + g4), z);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float p0 = ok[m][v] ? z[v] : 0.f;
                dk -= 0.5 * (double)p0 * (double)p0;
                xn[m][v] = x[m][v];
                pn[m][v] = fmaf(half, g[m][v], p0);
                gn[m][v] = 0.f;
            }
        }
        for (int l = 0; l < a.L; ++l) {
            const float ke = (l == a.L - 1) ? half : keps;
            float* xs = buf ? xs1 : xs0;
#pragma unroll
            for (int m = 0; m < MT; ++m) {
#pragma unroll
                for (int v = 0; v < 4; ++v) xn[m][v] = fmaf(eps, pn[m][v], xn[m][v]);
                if (tile_ok[m])
                    *(floatx4*)(xs + i16 * XS + 16 * (w + DENSE_NW * m) + 4 * g4) =
                        floatx4{xn[m][0], xn[m][1], xn[m][2], xn[m][3]};
            }
            __syncthreads();
            floatx4 bq[NT];
#pragma unroll
            for (int q = 0; q < NT; ++q) bq[q] = *(const floatx4*)(xs + i16 * XS + g4 * KM + 4 * q);
            floatx4 acc[MT][2];
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                acc[m][0] = floatx4{0.f, 0.f, 0.f, 0.f};
                acc[m][1] = floatx4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int ks = 0; ks < KM; ++ks) {
                const float bv = bq[ks >> 2][ks & 3];
#pragma unroll
                for (int m = 0; m < MT; ++m)
                    acc[m][ks & 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(pa[m][ks], bv, acc[m][ks & 1], 0, 0, 0);
            }
            // all operand reads first (one LDS latency per step), then the MFMAs
            __builtin_amdgcn_sched_group_barrier(0x100, NT, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, KM * MT, 0);
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    gn[m][v] = -(acc[m][0][v] + acc[m][1][v]);
                    pn[m][v] = fmaf(ke, gn[m][v], pn[m][v]);
                }
            buf ^= 1;
        }
        double lp = 0.0;
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                if (ok[m][v]) {
                    dk += 0.5 * (double)pn[m][v] * (double)pn[m][v];
                    lp += 0.5 * (double)xn[m][v] * (double)gn[m][v];
                }
        dk += __shfl_xor(dk, 16, 64);
        dk += __shfl_xor(dk, 32, 64);
        lp += __shfl_xor(lp, 16, 64);
        lp += __shfl_xor(lp, 32, 64);
        double* rb = red + (i & 1) * (2 * DENSE_NW * 16);
        if (g4 == 0) {
            rb[(2 * w) * 16 + i16] = dk;
            rb[(2 * w + 1) * 16 + i16] = lp;
        }
        __syncthreads();
        dk = 0.0;
        lp = 0.0;
#pragma unroll
        for (int ww = 0; ww < DENSE_NW; ++ww) {
            dk += rb[(2 * ww) * 16 + i16];
            lp += rb[(2 * ww + 1) * 16 + i16];
        }
        const double dh = -(bt * lp) + bt * s.logp + dk;
        const double lar = log_accept_ratio_of(dh);
        const bool acc = log_accept_uniform(a.key, (uint32_t)cc, t) < lar;
        if (acc) {
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    x[m][v] = xn[m][v];
                    g[m][v] = gn[m][v];
                }
            s.logp = lp;
        }
        // traces and adaptation record the transition; the exchange follows it,
        // and the kept sample is the state after the exchange
        if (cvalid) after_decision(r, a.C, c, i, acc, lar, dh, s.logp, s, w == 0 && g4 == 0);
        if (EX && nrep > 1) {
            const int par = (int)(t & 1u);
            const bool a_side = krep >= par && ((krep - par) & 1) == 0 && krep + 1 < nrep;
            const bool b_side = krep >= par + 1 && ((krep - 1 - par) & 1) == 0;
            const int src = a_side ? lane + 1 : (b_side ? lane - 1 : lane);
            const double lp_o = __shfl(s.logp, src, 64);
            const double bt_o = __shfl(bt, src, 64);
            bool swp = false;
            if (cvalid && (a_side || b_side)) {
                const int64_t ca = a_side ? c : c - r.remc_M;
                const double la = a_side ? s.logp : lp_o, lb = a_side ? lp_o : s.logp;
                const double ba = a_side ? bt : bt_o, bb = a_side ? bt_o : bt;
                swp = log_uniform52(a.key, (uint32_t)ca, t, TAG_SWAP) < (ba - bb) * (lb - la);
            }
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float xo = __shfl(x[m][v], src, 64), go = __shfl(g[m][v], src, 64);
                    if (swp) {
                        x[m][v] = xo;
                        g[m][v] = go;
                    }
                }
            if (swp) s.logp = lp_o;
            if (cvalid && r.swapped && i >= r.n_burnin && w == 0 && g4 == 0)
                r.swapped[(i - r.n_burnin) * a.C + c] = swp ? 1 : 0;
        }
        if (cvalid) {
            const bool want_smp = r.samples && i >= r.n_burnin;
            int q = 16 * w + 4 * g4;                 // opaque: keeps the LDS reads of the scale here
            if (EX) asm volatile("" : "+v"(q));
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (ok[m][v]) {
                        const int64_t d = 16 * (w + DENSE_NW * m) + 4 * g4 + v;
                        const float sd = (EX && trs) ? sc_lds[q + 16 * DENSE_NW * m + v] : 1.f;
                        if (want_smp)
                            ((float*)r.samples)[((i - r.n_burnin) * a.C + c) * D + d] =
                                (EX && trs) ? x[m][v] * sd : x[m][v];
                        if (r.out.proposed_state)
                            ((float*)r.out.proposed_state)[c * D + d] = (EX && trs) ? xn[m][v] * sd : xn[m][v];
                        if (r.out.proposed_momentum) ((float*)r.out.proposed_momentum)[c * D + d] = pn[m][v];
                    }
        }
    }
    if (!cvalid) return;
    if (EX) asm volatile("" ::: "memory");   // a fresh read of the scale (see the element-wise kernel)
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            if (ok[m][v]) {
                const int64_t d = 16 * (w + DENSE_NW * m) + 4 * g4 + v;
                X[c * D + d] = sc ? (float)((double)x[m][v] * sc[d]) : x[m][v];
                Gr[c * D + d] = sc ? (float)((double)g[m][v] / sc[d]) : g[m][v];
            }
    if (w == 0 && g4 == 0) {
        a.ws.logp[c] = s.logp;
        a.ws.eps[c] = s.eps;
        a.ws.da[c] = s.da;
    }
}

// ---------------------------------------------------------------------------
// Launch selection
// ---------------------------------------------------------------------------
bool fused_logreg_supported(const PlainArgs& a);
hipError_t launch_fused_logreg(const PlainArgs& a, const FusedRun& r, hipStream_t s);

static int elem_nb(int64_t D, int* G) {
    // lanes per chain and 4-blocks per lane
    const int64_t nblk = (D + 3) / 4;
    if (nblk <= 1) { *G = 1; return 1; }
    if (nblk <= 4) { *G = 4; return 1; }
    if (nblk <= 16) { *G = 16; return 1; }
    if (nblk <= 64) { *G = 64; return 1; }
    if (nblk <= 128) { *G = 64; return 2; }
    if (nblk <= 256) { *G = 64; return 4; }
    if (nblk <= 512) { *G = 64; return 8; }
    *G = 0;
    return 0;
}

bool fused_supported(const PlainArgs& a) {
    switch (a.tg.kind) {
    case HMC_TGT_STD_NORMAL:
    case HMC_TGT_GAUSS_DIAG: {
        int G;
        return elem_nb(a.tg.D, &G) > 0;
    }
    case HMC_TGT_GAUSS_DENSE:
        return !a.f64 && a.tg.D <= 128;
    case HMC_TGT_LOGREG:
        return fused_logreg_supported(a);
    }
    return false;
}

static int elem_class_of(int G, int NB) {
    if (G == 1) return 0;
    if (G == 4) return 1;
    if (G == 16) return 2;
    return NB == 1 ? 3 : (NB == 2 ? 4 : (NB == 4 ? 5 : 6));
}

// lanes per chain G and 4-blocks per lane NB, after the tuned multiplier
// (doubling G halves NB when the blocks still cover D)
static int elem_shape(const PlainArgs& a, int* G) {
    int NB = elem_nb(a.tg.D, G);
    if (NB == 0) return 0;
    if (a.tune.elem_gmult == 2 && *G < 64) *G = *G == 1 ? 4 : 4 * *G;   // next wider lane group
    return NB;
}

int elem_class(const PlainArgs& a) {
    if (a.tg.kind != HMC_TGT_STD_NORMAL && a.tg.kind != HMC_TGT_GAUSS_DIAG) return -1;
    int G;
    const int NB = elem_shape(a, &G);
    if (NB == 0) return -1;
    return (a.f64 ? 8 : 0) + elem_class_of(G, NB);
}

int64_t elem_blocks(const PlainArgs& a) {
    int G;
    elem_shape(a, &G);
    return (a.C * G + 255) / 256;
}

bool fused_remc_inline(const PlainArgs& a, int64_t K) {
    if (K < 2 || a.C % K != 0 || !fused_supported(a)) return false;
    if (a.tg.kind == HMC_TGT_GAUSS_DENSE) return 16 % K == 0;
    if (a.tg.kind == HMC_TGT_STD_NORMAL || a.tg.kind == HMC_TGT_GAUSS_DIAG) {
        int G;
        elem_shape(a, &G);
        return G <= 64 && (64 / G) % K == 0;       // a pair's two lane groups in one wavefront
    }
    if (a.tg.kind == HMC_TGT_LOGREG) return 4 % K == 0;   // 4 chains per workgroup
    return false;
}

#define HMC_ELEM_DISPATCH(CLS, MACRO)                  \
    switch ((CLS) & 7) {                               \
    case 0: MACRO(1, 1); break;                        \
    case 1: MACRO(4, 1); break;                        \
    case 2: MACRO(16, 1); break;                       \
    case 3: MACRO(64, 1); break;                       \
    case 4: MACRO(64, 2); break;                       \
    case 5: MACRO(64, 4); break;                       \
    default: MACRO(64, 8); break;                      \
    }

template <typename T>
static hipError_t launch_elem(const PlainArgs& a, const FusedRun& r, hipStream_t s) {
    const int cls = elem_class(a);
    const dim3 grid((unsigned)elem_blocks(a));
    if (r.remc_K > 1 && !fused_remc_inline(a, r.remc_K)) return hipErrorInvalidValue;
    if (a.ws.scale || r.remc_K > 1) {
#define HMC_ELEM(GG, NN) hipLaunchKernelGGL((k_fused_elem<T, GG, NN, true>), grid, dim3(256), 0, s, a, r)
        HMC_ELEM_DISPATCH(cls, HMC_ELEM)
#undef HMC_ELEM
    } else {
#define HMC_ELEM(GG, NN) hipLaunchKernelGGL((k_fused_elem<T, GG, NN, false>), grid, dim3(256), 0, s, a, r)
        HMC_ELEM_DISPATCH(cls, HMC_ELEM)
#undef HMC_ELEM
    }
    return hipGetLastError();
}

hipError_t launch_fused_elem_multi(int cls, const ElemJob* jobs_dev, int njobs, int64_t total_blocks,
                                   hipStream_t s) {
    const dim3 grid((unsigned)total_blocks);
    if (cls & 8) {
#define HMC_ELEM_M(GG, NN) hipLaunchKernelGGL((k_fused_elem_multi<double, GG, NN>), grid, dim3(256), 0, s, jobs_dev, njobs)
        HMC_ELEM_DISPATCH(cls, HMC_ELEM_M)
#undef HMC_ELEM_M
    } else {
#define HMC_ELEM_M(GG, NN) hipLaunchKernelGGL((k_fused_elem_multi<float, GG, NN>), grid, dim3(256), 0, s, jobs_dev, njobs)
        HMC_ELEM_DISPATCH(cls, HMC_ELEM_M)
#undef HMC_ELEM_M
    }
    return hipGetLastError();
}

static hipError_t launch_dense_fused(const PlainArgs& a, const FusedRun& r, hipStream_t s) {
    const int ntiles = (int)((a.tg.D + 15) / 16);
    const size_t lds = (size_t)2 * 16 * (16 * ntiles + 4) * sizeof(float) + 2 * 2 * DENSE_NW * 16 * sizeof(double);
    if (r.remc_K > 1 && (!fused_remc_inline(a, r.remc_K) || r.remc_K * r.remc_M != a.C)) return hipErrorInvalidValue;
    const int64_t per = r.remc_K > 1 ? 16 / r.remc_K : 16;      // values of m (or chains) per workgroup
    const int64_t units = r.remc_K > 1 ? r.remc_M : a.C;
    const dim3 grid((unsigned)((units + per - 1) / per));
    const bool ex = a.ws.scale || r.remc_K > 1;
    switch (ntiles) {
#define HMC_DENSE_NT(N)                                                                   \
    case N:                                                                               \
        if (ex) hipLaunchKernelGGL((k_fused_dense<N, true>), grid, dim3(64 * DENSE_NW), lds, s, a, r); \
        else hipLaunchKernelGGL((k_fused_dense<N, false>), grid, dim3(64 * DENSE_NW), lds, s, a, r);            \
        break;
        HMC_DENSE_NT(1) HMC_DENSE_NT(2) HMC_DENSE_NT(3) HMC_DENSE_NT(4)
        HMC_DENSE_NT(5) HMC_DENSE_NT(6) HMC_DENSE_NT(7) HMC_DENSE_NT(8)
#undef HMC_DENSE_NT
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fused(const PlainArgs& a, const FusedRun& r, hipStream_t s) {
    switch (a.tg.kind) {
    case HMC_TGT_STD_NORMAL:
    case HMC_TGT_GAUSS_DIAG:
        return a.f64 ? launch_elem<double>(a, r, s) : launch_elem<float>(a, r, s);
    case HMC_TGT_GAUSS_DENSE:
        return launch_dense_fused(a, r, s);
    case HMC_TGT_LOGREG:
        return launch_fused_logreg(a, r, s);
    }
    return hipErrorNotSupported;
}

}  // namespace hmc
