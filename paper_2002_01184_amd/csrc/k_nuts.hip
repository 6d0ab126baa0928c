// k_nuts.hip -- the No-U-Turn sampler with its recursion unrolled (paper
// Sec. 2.3; Hoffman & Gelman 2014, Algorithm 3, "efficient NUTS").
//
// All chains advance in lockstep through the same schedule: doubling j builds
// a subtree of 2^j leaves; leaf i is one leapfrog step (a half kick here, then
// the plain drift + gradient + half kick kernels of the target) from the end of
// the trajectory in the chain's direction.  The recursion's stack is replaced
// by one record per tree level k (the paper's O(max_tree_depth) memory): the
// first leaf and the candidate of the pending left subtree of level k.  After
// leaf i the subtrees that end at i are merged bottom-up -- the levels k with
// bit k-1 of i set -- exactly where the recursive BuildTree merges them, with
// the same counter-keyed uniforms, and the first unset bit parks the finished
// subtree as the pending left of its level.  A chain whose leaf diverges or
// whose merged subtree makes a U-turn stops for the rest of the transition
// (masked), as the recursion would.
//
// Step-size adaptation (Hoffman & Gelman 2014, Algorithm 6): each leaf adds
// min(1, exp(H0 - H)) to its chain's sum for the current doubling; at the end
// of the transition the mean over the last doubling's leaves is the statistic
// of dual averaging or of the multiplicative rule, during burn-in only.
//
// Random numbers (Philox4x32-10, counter (chain, t, block, tag)): momentum as
// HMC (tag 0), slice u (block 0, tag 6), direction of doubling j (block j,
// tag 4), take of doubling j's subtree (block j, tag 5), merge of level k at
// leaf i of doubling j (block (1024 j + i) 16 + k, tag 3).
#include "hmc_internal.hpp"

namespace hmc {

typedef float floatx4 __attribute__((ext_vector_type(4)));

enum : uint32_t { TAG_NUTS_MERGE = 3, TAG_NUTS_DIR = 4, TAG_NUTS_TOP = 5, TAG_NUTS_SLICE = 6 };

// (k + 1/2) 2^-52 uniform of block (chain, t, block, tag), as the accept uniform
__device__ __forceinline__ double nuts_u52(Key key, uint32_t chain, uint32_t t, uint32_t block, uint32_t tag) {
    const uint4 w = philox(chain, t, block, tag, key);
    const double k = (double)(w.x >> 6) * 67108864.0 + (double)(w.y >> 6);
    return (k + 0.5) * 0x1p-52;
}

// a leaf's min(1, exp(H0 - H)), 0 for NaN
__device__ __forceinline__ double leaf_accept_prob(double dh0) {
    return isnan(dh0) ? 0.0 : (dh0 >= 0.0 ? 1.0 : exp(dh0));
}

// Adaptation after transition it from its statistic; returns the new step
// size (eps unchanged outside burn-in or without adaptation).  Out of line:
// inlined, its FP64 pow / exp / sqrt raised the persistent kernel's register
// pressure in the tree loop into spills.
__device__ __attribute__((noinline)) double nuts_adapt(const NutsAdapt& ad, int64_t it, double stat, double eps,
                                                       DualAvg& da) {
    if (!ad.adapt || it >= ad.n_burnin) return eps;
    if (ad.adapt_kind == HMC_ADAPT_SIMPLE) return simple_adapt(eps, stat, ad.target_accept, ad.rate);
    const double log_eps = dual_avg_update(da, (double)(it + 1), stat, ad.target_accept, ad.gamma, ad.t0, ad.kappa);
    return (it + 1 < ad.n_burnin) ? exp(log_eps) : exp(da.log_eps_bar);
}

static size_t al256(size_t n) { return (n + 255) & ~(size_t)255; }

NutsWs carve_nuts(void* base, int64_t C, int64_t D, int32_t max_depth, size_t es, int64_t l2_rows, size_t* total) {
    char* p = (char*)base;
    size_t off = 0;
    auto take = [&](size_t n) {
        void* r = p ? (void*)(p + off) : nullptr;
        off += al256(n);
        return r;
    };
    const size_t vec = (size_t)C * D * es, lev = (size_t)(max_depth > 0 ? max_depth : 1) * C * D * es;
    const size_t md = (size_t)(max_depth > 0 ? max_depth : 1);
    NutsWs n;
    n.mx = take(vec); n.mr = take(vec); n.mg = take(vec);
    n.px = take(vec); n.pr = take(vec); n.pg = take(vec);
    n.lf_x = take(lev); n.lf_r = take(lev); n.lc_x = take(lev); n.lc_g = take(lev);
    n.rc_x = take(vec); n.rc_g = take(vec);
    n.mlogp = (double*)take((size_t)C * 8); n.plogp = (double*)take((size_t)C * 8);
    n.wlogp = (double*)take((size_t)C * 8); n.lc_logp = (double*)take(md * C * 8);
    n.rc_logp = (double*)take((size_t)C * 8);
    n.log_u = (double*)take((size_t)C * 8); n.seps = (double*)take((size_t)C * 8);
    n.ntot = (double*)take((size_t)C * 8);
    n.h0 = (double*)take((size_t)C * 8); n.alpha = (double*)take((size_t)C * 8);
    n.n_alpha = (int32_t*)take((size_t)C * 4);
    n.lc_n = (int32_t*)take(md * C * 4);
    n.active = (int32_t*)take((size_t)C * 4); n.alive = (int32_t*)take((size_t)C * 4);
    n.rc_n = (int32_t*)take((size_t)C * 4); n.depth = (int32_t*)take((size_t)C * 4);
    n.nleap = (int32_t*)take((size_t)C * 4); n.moved = (int32_t*)take((size_t)C * 4);
    n.dir = (int32_t*)take((size_t)C * 4);
    n.n_active = (int32_t*)take(4);
    n.xt4 = (float*)take((size_t)((D + 3) / 4) * 16 * l2_rows);
    n.yf = (float*)take((size_t)l2_rows * 4);
    if (l2_rows == 0) n.xt4 = n.yf = nullptr;
    n.bytes = off;
    if (total) *total = off;
    return n;
}

// One wavefront per chain, four chains per 256-thread block.
#define NUTS_CHAIN                                                   \
    const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); \
    const int lane = threadIdx.x & 63;                               \
    if (c >= a.C) return;                                            \
    const int64_t D = a.tg.D;

template <typename T>
__global__ __launch_bounds__(256) void k_nuts_begin(PlainArgs a, NutsWs n, uint32_t t) {
    NUTS_CHAIN
    const T* x = (const T*)a.ws.x;
    const T* g = (const T*)a.ws.g;
    T *mx = (T*)n.mx, *mr = (T*)n.mr, *mg = (T*)n.mg, *px = (T*)n.px, *pr = (T*)n.pr, *pg = (T*)n.pg;
    double k0 = 0.0;
    const int64_t nblk = (D + 3) / 4;
    for (int64_t b = lane; b < nblk; b += 64) {
        T z[4];
        momentum4<T>(a.key, (uint32_t)c, t, (uint32_t)b, z, 4 * b + 2 < D);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t d = 4 * b + j;
            if (d < D) {
                const int64_t i = c * D + d;
                mx[i] = px[i] = x[i];
                mg[i] = pg[i] = g[i];
                mr[i] = pr[i] = z[j];
                k0 += 0.5 * (double)z[j] * (double)z[j];
            }
        }
    }
    k0 = group_sum<64>(k0);
    if (lane == 0) {
        const double lp = a.ws.logp[c];
        n.mlogp[c] = n.plogp[c] = lp;
        n.h0[c] = -lp + k0;
        n.log_u[c] = log(nuts_u52(a.key, (uint32_t)c, t, 0u, TAG_NUTS_SLICE)) - (-lp + k0);
        n.ntot[c] = 1.0;
        n.alpha[c] = 0.0;
        n.n_alpha[c] = 0;
        n.active[c] = 1;
        n.depth[c] = 0;
        n.nleap[c] = 0;
        n.moved[c] = 0;
    }
}

// direction of doubling j; the trajectory end in that direction becomes the
// working leaf state (xq, pq, gq)
template <typename T>
__global__ __launch_bounds__(256) void k_nuts_dir(PlainArgs a, NutsWs n, uint32_t t, int32_t j) {
    NUTS_CHAIN
    const bool act = n.active[c] != 0;
    const int v = (act && nuts_u52(a.key, (uint32_t)c, t, (uint32_t)j, TAG_NUTS_DIR) < 0.5) ? -1 : 1;
    const T* sx = (const T*)(v > 0 ? n.px : n.mx);
    const T* sr = (const T*)(v > 0 ? n.pr : n.mr);
    const T* sg = (const T*)(v > 0 ? n.pg : n.mg);
    T *xq = (T*)a.ws.xq, *pq = (T*)a.ws.pq, *gq = (T*)a.ws.gq;
    for (int64_t d = lane; d < D; d += 64) {
        const int64_t i = c * D + d;
        xq[i] = sx[i];
        pq[i] = sr[i];
        gq[i] = sg[i];
    }
    if (lane == 0) {
        if (act) {                              // the statistic is the last doubling's
            n.alpha[c] = 0.0;
            n.n_alpha[c] = 0;
        }
        n.dir[c] = v;
        n.seps[c] = act ? (double)v * a.ws.eps[c] : 0.0;
        n.alive[c] = act ? 1 : 0;
        n.wlogp[c] = v > 0 ? n.plogp[c] : n.mlogp[c];
    }
}

// first half kick of a leaf's leapfrog step: p += (v eps / 2) g
template <typename T>
__global__ __launch_bounds__(256) void k_nuts_halfkick(PlainArgs a, NutsWs n) {
    const int64_t D = a.tg.D, tot = a.C * D;
    T* pq = (T*)a.ws.pq;
    const T* gq = (const T*)a.ws.gq;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x)
        pq[i] = pq[i] + (T)(0.5 * n.seps[i / D]) * gq[i];
}

// leaf i of doubling j: its energy, then the merges of the subtrees that end here
template <typename T>
__global__ __launch_bounds__(256) void k_nuts_leaf(PlainArgs a, NutsWs n, uint32_t t, int32_t j, int32_t i) {
    NUTS_CHAIN
    if (!n.alive[c]) return;
    const T *xq = (const T*)a.ws.xq, *pq = (const T*)a.ws.pq, *gq = (const T*)a.ws.gq;
    const bool logreg = a.tg.kind == HMC_TGT_LOGREG;
    // summed in the order k_nuts_begin sums the starting kinetic energy (lane
    // by lane over 4-dim blocks), so that H - H0 is exactly 0 where the energy
    // is exactly conserved
    double lp = 0.0, kin = 0.0;
    for (int64_t b = lane; b < (D + 3) / 4; b += 64)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t d = 4 * b + q;
            if (d >= D) break;
            const int64_t e = c * D + d;
            const double xv = (double)xq[e], pv = (double)pq[e];
            kin += 0.5 * pv * pv;
            lp += logreg ? -0.5 * xv * xv * a.tg.inv_var : 0.5 * xv * (double)gq[e];
        }
    lp = group_sum<64>(lp);
    kin = group_sum<64>(kin);
    if (logreg) lp += a.ws.lpq[c];
    const double H = -lp + kin, lu = n.log_u[c];
    int32_t n_node = (lu <= -H) ? 1 : 0;
    const bool s_leaf = lu < 1000.0 - H;        // NaN H fails
    if (lane == 0) {
        n.nleap[c] += 1;
        n.wlogp[c] = lp;
        n.alpha[c] += leaf_accept_prob(n.h0[c] - H);
        n.n_alpha[c] += 1;
    }
    if (!s_leaf) {
        if (lane == 0) n.alive[c] = 0;
        return;
    }
    const int64_t C = a.C;
    const int v = n.dir[c];
    T *lfx = (T*)n.lf_x, *lfr = (T*)n.lf_r, *lcx = (T*)n.lc_x, *lcg = (T*)n.lc_g;
    int cand = -1, first = -1;                  // -1: the leaf itself, k: the record of level k
    double cand_lp = lp;
    for (int k = 1; k <= j; ++k) {
        const int64_t rk = ((int64_t)k * C + c) * D;
        if (((i >> (k - 1)) & 1) == 0) {
            // the finished subtree is the left child at level k: park it
            const int64_t rf = first < 0 ? 0 : ((int64_t)first * C + c) * D;
            const int64_t rc = cand < 0 ? 0 : ((int64_t)cand * C + c) * D;
            for (int64_t d = lane; d < D; d += 64) {
                lfx[rk + d] = first < 0 ? xq[c * D + d] : lfx[rf + d];
                lfr[rk + d] = first < 0 ? pq[c * D + d] : lfr[rf + d];
                lcx[rk + d] = cand < 0 ? xq[c * D + d] : lcx[rc + d];
                lcg[rk + d] = cand < 0 ? gq[c * D + d] : lcg[rc + d];
            }
            if (lane == 0) {
                n.lc_n[k * C + c] = n_node;
                n.lc_logp[k * C + c] = cand_lp;
            }
            return;
        }
        // the finished subtree is the right child at level k: merge with the parked left
        const int32_t nl = n.lc_n[k * C + c];
        const uint32_t block = ((uint32_t)j * 1024u + (uint32_t)i) * 16u + (uint32_t)k;
        const double u = nuts_u52(a.key, (uint32_t)c, t, block, TAG_NUTS_MERGE);
        const bool keep_right = (nl + n_node > 0) && u < (double)n_node / (double)(nl + n_node);
        if (!keep_right) {
            cand = k;
            cand_lp = n.lc_logp[k * C + c];
        }
        n_node += nl;
        // U-turn over the merged span: from its first leaf (level k's record) to this leaf
        double dm = 0.0, dp = 0.0;
        for (int64_t d = lane; d < D; d += 64) {
            const double fx = (double)lfx[rk + d], fr = (double)lfr[rk + d];
            const double lx = (double)xq[c * D + d], lr = (double)pq[c * D + d];
            const double dx = v > 0 ? lx - fx : fx - lx;     // forward end minus backward end
            dm += dx * (v > 0 ? fr : lr);
            dp += dx * (v > 0 ? lr : fr);
        }
        dm = group_sum<64>(dm);
        dp = group_sum<64>(dp);
        first = k;
        if (!(dm >= 0.0 && dp >= 0.0)) {
            if (lane == 0) n.alive[c] = 0;
            return;
        }
    }
    // every subtree of doubling j ends at this leaf: the doubling's tree is complete
    T *rcx = (T*)n.rc_x, *rcg = (T*)n.rc_g;
    const int64_t rc = cand < 0 ? 0 : ((int64_t)cand * C + c) * D;
    for (int64_t d = lane; d < D; d += 64) {
        rcx[c * D + d] = cand < 0 ? xq[c * D + d] : lcx[rc + d];
        rcg[c * D + d] = cand < 0 ? gq[c * D + d] : lcg[rc + d];
    }
    if (lane == 0) {
        n.rc_n[c] = n_node;
        n.rc_logp[c] = cand_lp;
    }
}

// end of doubling j: the working state becomes the trajectory end, the
// subtree's candidate is taken with probability min(1, n'/n), and the whole
// trajectory's U-turn decides whether the chain continues
template <typename T>
__global__ __launch_bounds__(256) void k_nuts_doubling_end(PlainArgs a, NutsWs n, uint32_t t, int32_t j) {
    NUTS_CHAIN
    if (!n.active[c]) return;
    const int v = n.dir[c];
    T* ex = (T*)(v > 0 ? n.px : n.mx);
    T* er = (T*)(v > 0 ? n.pr : n.mr);
    T* eg = (T*)(v > 0 ? n.pg : n.mg);
    const T *xq = (const T*)a.ws.xq, *pq = (const T*)a.ws.pq, *gq = (const T*)a.ws.gq;
    for (int64_t d = lane; d < D; d += 64) {
        const int64_t e = c * D + d;
        ex[e] = xq[e];
        er[e] = pq[e];
        eg[e] = gq[e];
    }
    if (lane == 0) (v > 0 ? n.plogp : n.mlogp)[c] = n.wlogp[c];
    bool s = false;
    if (n.alive[c]) {
        const double ntot = n.ntot[c];
        const int32_t nsub = n.rc_n[c];
        if (nuts_u52(a.key, (uint32_t)c, t, (uint32_t)j, TAG_NUTS_TOP) < (double)nsub / ntot) {
            T* x = (T*)a.ws.x;
            T* g = (T*)a.ws.g;
            const T *rcx = (const T*)n.rc_x, *rcg = (const T*)n.rc_g;
            for (int64_t d = lane; d < D; d += 64) {
                x[c * D + d] = rcx[c * D + d];
                g[c * D + d] = rcg[c * D + d];
            }
            if (lane == 0) {
                a.ws.logp[c] = n.rc_logp[c];
                n.moved[c] = 1;
            }
        }
        if (lane == 0) n.ntot[c] = ntot + (double)nsub;
        // U-turn of the whole trajectory (each lane reads the elements it wrote)
        const T *mx = (const T*)n.mx, *mr = (const T*)n.mr, *px = (const T*)n.px, *pr = (const T*)n.pr;
        double dm = 0.0, dp = 0.0;
        for (int64_t d = lane; d < D; d += 64) {
            const int64_t e = c * D + d;
            const double dx = (double)px[e] - (double)mx[e];
            dm += dx * (double)mr[e];
            dp += dx * (double)pr[e];
        }
        dm = group_sum<64>(dm);
        dp = group_sum<64>(dp);
        s = dm >= 0.0 && dp >= 0.0;
    }
    if (lane == 0) {
        n.depth[c] = j + 1;
        if (s) atomicAdd(n.n_active, 1);
        else n.active[c] = 0;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_nuts_end(PlainArgs a, NutsWs n, NutsAdapt ad, int64_t it, T* samples,
                                                  int64_t r, int32_t* tr_depth, int32_t* tr_nleap, double* tr_stat) {
    NUTS_CHAIN
    if (r >= 0 && samples) {
        const T* x = (const T*)a.ws.x;
        for (int64_t d = lane; d < D; d += 64) samples[(r * a.C + c) * D + d] = x[c * D + d];
    }
    if (lane == 0) {
        const int32_t na = n.n_alpha[c];
        const double stat = na > 0 ? n.alpha[c] / (double)na : 0.0;
        if (ad.adapt && it < ad.n_burnin) {
            DualAvg da = a.ws.da[c];
            a.ws.eps[c] = nuts_adapt(ad, it, stat, a.ws.eps[c], da);
            a.ws.da[c] = da;
        }
        if (r >= 0) {
            if (tr_depth) tr_depth[r * a.C + c] = n.depth[c];
            if (tr_nleap) tr_nleap[r * a.C + c] = n.nleap[c];
            if (tr_stat) tr_stat[r * a.C + c] = stat;
        }
    }
}

// ---------------------------------------------------------------------------
// Persistent NUTS for the element-wise targets (N(0, I), diagonal Gaussian):
// a group of G lanes owns one chain (NB blocks of 4 dims per lane) and runs
// whole transitions -- every doubling and leaf -- in registers, so a chain
// waits only for the chains of its own wavefront, not for the whole batch.
// The levels' parked first leaves and candidates live in the NutsWs buffers
// (each lane touches only its own dims); their counts and log-probabilities
// in registers (levels unrolled).  With a workgroup per chain (G = 256) a
// leaf's sums (energies, the U-turn products of every subtree ending at it)
// share one LDS exchange and barrier, the per-level counts sit in LDS and the
// records move between levels by slot index, a park writing only the records
// it creates.  Same tree, same uniforms, same arithmetic order per leaf as the
// lockstep kernels.
// ---------------------------------------------------------------------------
constexpr int NUTS_MAXD = 10;

// Sums over a chain's lanes for the persistent element-wise kernel.  G <= 64:
// shuffles inside the wavefront.  G = 256 (one chain per workgroup): the four
// waves' shuffle sums through LDS (gsr [2 parity][2 values][4 waves]), one
// barrier per call; every call is made by the whole workgroup, whose control
// flow is the chain's.
template <int G>
__device__ __forceinline__ void nuts_gsum2(double& a0, double& a1, double* gsr, int& gk) {
    if constexpr (G <= 64) {
        a0 = group_sum<G>(a0);
        a1 = group_sum<G>(a1);
    } else {
        constexpr int NWG = G / 64;
        a0 = group_sum<64>(a0);
        a1 = group_sum<64>(a1);
        double* slot = gsr + (gk & 1) * 2 * NWG;
        if ((threadIdx.x & 63) == 0) {
            slot[threadIdx.x >> 6] = a0;
            slot[NWG + (threadIdx.x >> 6)] = a1;
        }
        __syncthreads();
        a0 = 0.0;
        a1 = 0.0;
#pragma unroll
        for (int q = 0; q < NWG; ++q) {
            a0 += slot[q];
            a1 += slot[NWG + q];
        }
        ++gk;
    }
}

// Logistic regression on the persistent path (GK = 1): one wavefront per
// chain (G = 64, NB = 1: lane l holds dims 4 l .. 4 l + 3, D <= 4 LR_DQ), X
// (FP32, rows padded to 4 DQ floats) and y staged once per workgroup in LDS
// and shared by its 4 chains.  A leaf's gradient reads each row of X once:
// s = x . theta with theta broadcast from LDS, r = y - sigmoid(s), the row's
// term of the log-likelihood, then r x_row into per-lane partials, which the
// wave sums column by column through LDS in a fixed order.
constexpr int LR_DQ = 8;                    // 4-dim chunks of theta (D <= 32)
constexpr int LR_SCR = 4 * LR_DQ + 1;       // row stride of the transposition scratch

// One row's residual y - sigmoid(s) and log-likelihood term
// -softplus(y ? -s : s), from a single e = exp(-|s|) on the hardware exp2,
// reciprocal and log2 (a few ulp; softplus(z) = max(z, 0) + ln(1 + e), where
// ln(1 + e) loses e below 2^-24 relative to 1, an absolute error < 6e-8).
__device__ __forceinline__ float nuts_lr_row(float s, float yv, double& lpd) {
    const float e = __builtin_amdgcn_exp2f(-fabsf(s) * 1.44269504f);
    const float inv = __builtin_amdgcn_rcpf(1.f + e);
    const float sig = s >= 0.f ? inv : e * inv;
    const float z = yv > 0.5f ? -s : s;
    lpd -= (double)(fmaxf(z, 0.f) + __builtin_amdgcn_logf(1.f + e) * 0.693147181f);
    return yv - sig;
}

// LDS floats of the logistic persistent kernel: X [N][4 DQ], y [N rounded up
// to 4, keeping what follows 16-byte aligned], per wave theta [4 DQ], the
// gradient [4 DQ] and the scratch [64][LR_SCR]; then, per wave, the parked
// records (4 arrays of 4 DQ floats) of as many shallow tree levels as the
// rest of the 160 KB holds (at most 9).
__host__ __device__ inline int64_t nuts_lr_lds_fixed(int64_t N, int64_t D) {
    const int64_t dp = 4 * ((D + 3) / 4);
    return N * dp + ((N + 3) & ~(int64_t)3) + 4 * (2 * dp + 64 * LR_SCR);
}
__host__ __device__ inline int nuts_lr_lds_levels(int64_t N, int64_t D) {
    const int64_t dp = 4 * ((D + 3) / 4);
    const int64_t room = 163840 / 4 - 16 - nuts_lr_lds_fixed(N, D);   // 64 bytes kept for static LDS
    const int64_t lv = room > 0 ? room / (4 * 4 * dp) : 0;
    return (int)(lv > 9 ? 9 : lv);
}
inline size_t nuts_lr_lds_bytes(int64_t N, int64_t D) {
    const int64_t dp = 4 * ((D + 3) / 4);
    return (size_t)(nuts_lr_lds_fixed(N, D) + (int64_t)nuts_lr_lds_levels(N, D) * 4 * 4 * dp) * sizeof(float);
}

// The L2 variant (GK = 2, X beyond the LDS): X and y stay in global memory, so
// a workgroup holds only the per-wave buffers and as many parked levels as fit
// in a third of the LDS, and three workgroups (12 waves) share a CU.
constexpr int NUTS_L2_LDS = 53248;
__host__ __device__ inline int nuts_l2_lds_levels(int64_t D) {
    const int64_t dp = 4 * ((D + 3) / 4);
    const int64_t room = NUTS_L2_LDS / 4 - 16 - nuts_lr_lds_fixed(0, D);
    const int64_t lv = room > 0 ? room / (4 * 4 * dp) : 0;
    return (int)(lv > 9 ? 9 : lv);
}
inline size_t nuts_l2_lds_bytes(int64_t D) {
    const int64_t dp = 4 * ((D + 3) / 4);
    return (size_t)(nuts_lr_lds_fixed(0, D) + (int64_t)nuts_l2_lds_levels(D) * 4 * 4 * dp) * sizeof(float);
}

// Copy of X for the L2 variant, 4-dim chunk major: xt4[q][r] holds dims
// 4q .. 4q + 3 of row r (zeros past D), so that the 64 lanes of a wave, on 64
// consecutive rows, read 1 KB of consecutive bytes per chunk; y as floats.
__global__ __launch_bounds__(256) void k_nuts_pad_x(const void* __restrict__ X, int x_bf16,
                                                    const uint8_t* __restrict__ y, float* __restrict__ xt4,
                                                    float* __restrict__ yf, int64_t N, int64_t D) {
    const int64_t dq = (D + 3) / 4;
    const int64_t n = dq * N;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = i / N, r = i - q * N;
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t d = 4 * q + e;
            v[e] = 0.f;
            if (d < D)
                v[e] = x_bf16 ? bf16_to_f32(((const uint16_t*)X)[r * D + d]) : ((const float*)X)[r * D + d];
        }
        *(float4*)(xt4 + 4 * i) = make_float4(v[0], v[1], v[2], v[3]);
        if (q == 0) yf[r] = y[r] ? 1.f : 0.f;
    }
}

// ST: the run adapts the step size or traces the statistic (a template
// parameter, so that plain runs carry none of it).  GK: 0 element-wise
// Gaussian gradient, 1 logistic regression with X in LDS, 2 logistic
// regression with X read from global memory (the L2 holds it).
template <typename T, int G, int NB, bool ST, int GK>
__global__ __launch_bounds__(256) void k_nuts_fused_elem(PlainArgs a, NutsWs n, NutsAdapt ad, uint32_t t_begin,
                                                         int64_t n_trans, int32_t max_depth, T* samples,
                                                         int32_t* tr_depth, int32_t* tr_nleap, double* tr_stat) {
    const int64_t n_burnin = ad.n_burnin;
    extern __shared__ float lr_lds[];
    __shared__ double gsr[G > 64 ? 2 * 2 * (G / 64) : 1];
    __shared__ double gsb[G > 64 ? 2 * 2 * NUTS_MAXD * (G / 64) : 1];   // [2 parity][values][waves]
    // a workgroup per chain: per pending level its slice leaf count and candidate logp
    // (written by thread 0 at the park, read at a merge one barrier or more later) and the
    // slots of its first-leaf and candidate records (read before the next barrier, so each
    // wave keeps its own copy, written by its lane 0: a wave's LDS accesses run in order)
    __shared__ int32_t wg_cn[G > 64 ? NUTS_MAXD : 1];
    __shared__ double wg_lp[G > 64 ? NUTS_MAXD : 1];
    __shared__ int32_t wg_fsa[G > 64 ? (G / 64) * NUTS_MAXD : 1], wg_csa[G > 64 ? (G / 64) * NUTS_MAXD : 1];
    int32_t* const wg_fs = wg_fsa + (G > 64 ? (threadIdx.x >> 6) * NUTS_MAXD : 0);
    int32_t* const wg_cs = wg_csa + (G > 64 ? (threadIdx.x >> 6) * NUTS_MAXD : 0);
    int gk = 0;
    const int64_t NR = GK >= 1 ? a.tg.N : 0;
    const int64_t NL = GK == 1 ? NR : 0;                 // rows of X held in LDS
    const int dq = GK >= 1 ? (int)((a.tg.D + 3) / 4) : 0;
    const int dp = 4 * dq;
    float* xl = lr_lds;                                  // [N][dp] (GK = 1)
    float* yl = xl + NL * dp;                            // [N] (GK = 1)
    const floatx4* xg4 = (const floatx4*)n.xt4;          // [dq][N] (GK = 2)
    const float* yg = n.yf;                              // [N] (GK = 2)
    float* thl = yl + ((NL + 3) & ~(int64_t)3) + (threadIdx.x >> 6) * (2 * dp + 64 * LR_SCR);   // wave's theta [dp]
    float* gsl = thl + dp;                               // gradient sums [dp]
    float* scr = gsl + dp;                               // [64][LR_SCR]
    const int nlv = GK == 1 ? nuts_lr_lds_levels(NR, a.tg.D) : GK == 2 ? nuts_l2_lds_levels(a.tg.D) : 0;
    float* lvl = lr_lds + (GK >= 1 ? nuts_lr_lds_fixed(NL, a.tg.D) : 0) +
                 (int64_t)(threadIdx.x >> 6) * nlv * 4 * dp;  // this wave's level records [nlv][4][dp]
    if (GK == 1) {
        const float* Xg = (const float*)a.tg.X;
        const int64_t D0 = a.tg.D;
        for (int64_t e = threadIdx.x; e < NR * dp; e += blockDim.x) {
            const int64_t r = e / dp, d = e - r * dp;
            xl[e] = d < D0 ? Xg[r * D0 + d] : 0.f;
        }
        for (int64_t r = threadIdx.x; r < NR; r += blockDim.x) yl[r] = a.tg.y[r] ? 1.f : 0.f;
        __syncthreads();                                 // the only barrier: the chains are independent after it
    }
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x % G;
    const int64_t c = gid / G;
    const bool active = c < a.C;
    const int64_t cc = active ? c : 0;
    const int64_t C = a.C, D = a.tg.D;
    const bool diag = a.tg.kind == HMC_TGT_GAUSS_DIAG;
    const T* X = (const T*)a.ws.x;
    const T* Gr = (const T*)a.ws.g;
    const T* prec = (const T*)a.tg.prec;
    T *lfx = (T*)n.lf_x, *lfr = (T*)n.lf_r, *lcx = (T*)n.lc_x, *lcg = (T*)n.lc_g;

    T pc[NB][4], x[NB][4], g[NB][4];
    bool ok[NB][4];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t d = 4 * (lane + (int64_t)G * b) + e;
            ok[b][e] = active && d < D;
            x[b][e] = ok[b][e] ? X[cc * D + d] : (T)0;
            g[b][e] = ok[b][e] ? Gr[cc * D + d] : (T)0;
            pc[b][e] = ok[b][e] ? (diag ? prec[d] : (T)1) : (T)0;
        }
    auto dim_of = [&](int b, int e) -> int64_t { return 4 * (lane + (int64_t)G * b) + e; };
    // level k's record q (0 first x, 1 first r, 2 candidate x, 3 candidate g),
    // indexed by dim: the shallow levels of the logistic path in LDS (a flat
    // pointer), the rest in the NutsWs buffers
    T* const grec[4] = {lfx, lfr, lcx, lcg};
    auto recp = [&](int k, int q) -> T* {
        if (GK >= 1 && k <= nlv) return (T*)(lvl + ((k - 1) * 4 + q) * dp);
        // formed where it is used: the empty asm keeps the compiler from hoisting
        // one 64-bit address per level and record out of the leaf loop
        int64_t off = ((int64_t)k * C + cc) * D;
        asm volatile("" : "+v"(off));
        return grec[q] + off;
    };
    // logistic data gradient X^T (y - sigmoid(X theta)) at theta = wxa into
    // wga (the lane's dims), and the data log-likelihood (wave-uniform).  The
    // LDS traffic between lanes stays inside the wave, whose LDS operations
    // run in order; the empty asm statements keep the compiler from moving
    // them across each other.
    auto logreg_grad_lds = [&](T (&wxa)[NB][4], T (&wga)[NB][4]) -> double {
        if (lane < dq) *(floatx4*)(thl + 4 * lane) = floatx4{(float)wxa[0][0], (float)wxa[0][1], (float)wxa[0][2],
                                                            (float)wxa[0][3]};
        asm volatile("" ::: "memory");
        floatx4 th[LR_DQ];
#pragma unroll
        for (int q = 0; q < LR_DQ; ++q) th[q] = q < dq ? *(const floatx4*)(thl + 4 * q) : floatx4{0.f, 0.f, 0.f, 0.f};
        floatx4 gacc[LR_DQ];
#pragma unroll
        for (int q = 0; q < LR_DQ; ++q) gacc[q] = floatx4{0.f, 0.f, 0.f, 0.f};
        double lpd = 0.0;
        const int nr = (int)NR;
#pragma unroll 2
        for (int r = lane; r < nr; r += 64) {
            const float* xr = xl + r * dp;
            floatx4 xq[LR_DQ];
            float sv = 0.f;
#pragma unroll
            for (int q = 0; q < LR_DQ; ++q) {
                if constexpr (GK == 2) xq[q] = q < dq ? xg4[(int64_t)q * nr + r] : floatx4{0.f, 0.f, 0.f, 0.f};
                else xq[q] = q < dq ? *(const floatx4*)(xr + 4 * q) : floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int e = 0; e < 4; ++e) sv = fmaf(xq[q][e], th[q][e], sv);
            }
            const float res = nuts_lr_row(sv, GK == 2 ? yg[r] : yl[r], lpd);
#pragma unroll
            for (int q = 0; q < LR_DQ; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) gacc[q][e] = fmaf(xq[q][e], res, gacc[q][e]);
        }
        asm volatile("" ::: "memory");
#pragma unroll
        for (int q = 0; q < LR_DQ; ++q)
            if (q < dq)
#pragma unroll
                for (int e = 0; e < 4; ++e) scr[lane * LR_SCR + 4 * q + e] = gacc[q][e];
        asm volatile("" ::: "memory");
        if (lane < dp) {
            float col = 0.f;
            for (int rr = 0; rr < 64; ++rr) col += scr[rr * LR_SCR + lane];
            gsl[lane] = col;
        }
        asm volatile("" ::: "memory");
        const floatx4 gq = lane < dq ? *(const floatx4*)(gsl + 4 * lane) : floatx4{0.f, 0.f, 0.f, 0.f};
        asm volatile("" ::: "memory");
#pragma unroll
        for (int e = 0; e < 4; ++e) wga[0][e] = (T)gq[e];
        return group_sum<64>(lpd);
    };
    double logp = a.ws.logp[cc];
    double eps = a.ws.eps[cc];
    DualAvg da{};
    if (ST) da = a.ws.da[cc];

    for (int64_t it = 0; it < n_trans; ++it) {
        const uint32_t t = t_begin + (uint32_t)it;
        T mx[NB][4], mr[NB][4], mg[NB][4], px[NB][4], pr[NB][4], pg[NB][4];
        double k0 = 0.0;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            T z[4];
            momentum4<T>(a.key, (uint32_t)cc, t, (uint32_t)(lane + G * b), z, 4 * (lane + (int64_t)G * b) + 2 < D);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const T r0 = ok[b][e] ? z[e] : (T)0;
                k0 += 0.5 * (double)r0 * (double)r0;
                mx[b][e] = px[b][e] = x[b][e];
                mg[b][e] = pg[b][e] = g[b][e];
                mr[b][e] = pr[b][e] = r0;
            }
        }
        double k0_unused = 0.0;
        nuts_gsum2<G>(k0, k0_unused, gsr, gk);
        const double h0 = -logp + k0;
        const double log_u = log(nuts_u52(a.key, (uint32_t)cc, t, 0u, TAG_NUTS_SLICE)) - (-logp + k0);
        double mlogp = logp, plogp = logp, ntot = 1.0;
        double alpha = 0.0;                     // the last doubling's acceptance-probability sum
        int32_t n_alpha = 0;
        int32_t depth = 0, nleap = 0;
        bool s = active;                        // lanes past the last chain build no tree
        for (int j = 0; j < max_depth && s; ++j) {
            const int v = nuts_u52(a.key, (uint32_t)cc, t, (uint32_t)j, TAG_NUTS_DIR) < 0.5 ? -1 : 1;
            const T se = (T)((double)v * eps), hse = (T)(0.5 * ((double)v * eps));
            T wx[NB][4], wr[NB][4], wg[NB][4];
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    wx[b][e] = v > 0 ? px[b][e] : mx[b][e];
                    wr[b][e] = v > 0 ? pr[b][e] : mr[b][e];
                    wg[b][e] = v > 0 ? pg[b][e] : mg[b][e];
                }
            double wlogp = v > 0 ? plogp : mlogp;
            bool alive = true, complete = false;
            alpha = 0.0;
            n_alpha = 0;
            int32_t lcn[NUTS_MAXD];
            double lclp[NUTS_MAXD];
            T rcx[NB][4], rcg[NB][4];
            // a workgroup per chain: each pending level's first-leaf and candidate records
            // live in slots of the level buffers, handed from level to level by index, so a
            // park writes only the records it creates (bit s of ffree / cfree: slot s free)
            uint32_t ffree = ~0u, cfree = ~0u;
            double rclp = 0.0;
            int32_t rcn = 0;
            const int nleaves = 1 << j;
            for (int i = 0; i < nleaves; ++i) {
                double lp = 0.0, kin = 0.0;
#pragma unroll
                for (int b = 0; b < NB; ++b)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        wr[b][e] = wr[b][e] + hse * wg[b][e];
                        wx[b][e] = fma(se, wr[b][e], wx[b][e]);
                        if (GK == 0) {
                            wg[b][e] = -pc[b][e] * wx[b][e];
                            wr[b][e] = fma(hse, wg[b][e], wr[b][e]);
                            lp += 0.5 * (double)wx[b][e] * (double)wg[b][e];
                            kin += 0.5 * (double)wr[b][e] * (double)wr[b][e];
                        }
                    }
                if constexpr (G > 64) {
                    // a workgroup per chain: one reduction (one barrier) carries the leaf's
                    // energies and the U-turn products of every subtree that ends at the
                    // leaf (levels 1 .. nm: bit k-1 of i set, k <= j); each value's wave
                    // sums go to gsb as they are formed and are read where they are used
                    static_assert(GK == 0, "a workgroup per chain runs element-wise targets only");
                    constexpr int NWG = G / 64;
                    const int nm = min(__builtin_ctz(~(unsigned)i), j);
                    double* gb = gsb + (gk & 1) * (2 * NUTS_MAXD * NWG);
                    auto put = [&](int q, double val) {
                        val = group_sum<64>(val);
                        if ((threadIdx.x & 63) == 0) gb[q * NWG + (threadIdx.x >> 6)] = val;
                    };
                    auto get = [&](int q) -> double {
                        double acc = 0.0;
#pragma unroll
                        for (int q2 = 0; q2 < NWG; ++q2) acc += gb[q * NWG + q2];
                        return acc;
                    };
                    put(0, lp);
                    put(1, kin);
                    for (int k = 1; k <= nm; ++k) {
                        const T *kfx = recp(wg_fs[k - 1], 0), *kfr = recp(wg_fs[k - 1], 1);
                        double dm = 0.0, dp = 0.0;
#pragma unroll
                        for (int b = 0; b < NB; ++b)
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                if (ok[b][e]) {
                                    const int64_t d = dim_of(b, e);
                                    const double fx = (double)kfx[d], fr = (double)kfr[d];
                                    const double lx = (double)wx[b][e], lr = (double)wr[b][e];
                                    const double dx = v > 0 ? lx - fx : fx - lx;
                                    dm += dx * (v > 0 ? fr : lr);
                                    dp += dx * (v > 0 ? lr : fr);
                                }
                        put(2 * k, dm);
                        put(2 * k + 1, dp);
                    }
                    __syncthreads();
                    ++gk;
                    lp = get(0);
                    kin = get(1);
                    wlogp = lp;
                    nleap += 1;
                    const double H = -lp + kin;
                    if (ST) {
                        alpha += leaf_accept_prob(h0 - H);
                        n_alpha += 1;
                    }
                    int32_t n_node = (log_u <= -H) ? 1 : 0;
                    if (!(log_u < 1000.0 - H)) {
                        alive = false;
                        break;
                    }
                    int cand = -1;
                    double cand_lp = lp;
                    for (int k = 1; k <= nm; ++k) {
                        const int32_t nl = wg_cn[k - 1];
                        const uint32_t block = ((uint32_t)j * 1024u + (uint32_t)i) * 16u + (uint32_t)k;
                        const double u = nuts_u52(a.key, (uint32_t)cc, t, block, TAG_NUTS_MERGE);
                        if (!((nl + n_node > 0) && u < (double)n_node / (double)(nl + n_node))) {
                            cand = k;
                            cand_lp = wg_lp[k - 1];
                        }
                        n_node += nl;
                        if (!(get(2 * k) >= 0.0 && get(2 * k + 1) >= 0.0)) {
                            alive = false;
                            break;
                        }
                    }
                    if (!alive) break;
                    if (nm < j) {           // park the merged tree at level nm + 1
                        const int kp = nm + 1;
                        // its first leaf: this leaf's (x, r) in a free slot, or level nm's slot;
                        // the slots of levels 1 .. nm - 1 are released
                        if (nm == 0) {
                            const int sf = __builtin_ctz(ffree);
                            ffree &= ~(1u << sf);
                            if ((threadIdx.x & 63) == 0) wg_fs[kp - 1] = sf;
                            T *kfx = recp(sf, 0), *kfr = recp(sf, 1);
#pragma unroll
                            for (int b = 0; b < NB; ++b)
#pragma unroll
                                for (int e = 0; e < 4; ++e)
                                    if (ok[b][e]) {
                                        kfx[dim_of(b, e)] = wx[b][e];
                                        kfr[dim_of(b, e)] = wr[b][e];
                                    }
                        } else {
                            const int32_t sfn = wg_fs[nm - 1];
                            if ((threadIdx.x & 63) == 0) wg_fs[kp - 1] = sfn;
                            for (int k = 1; k < nm; ++k) ffree |= 1u << wg_fs[k - 1];
                        }
                        // its candidate: level cand's slot, or this leaf's (x, g) in a slot freed
                        // from the merged levels first
                        for (int k = 1; k <= nm; ++k)
                            if (k != cand) cfree |= 1u << wg_cs[k - 1];
                        if (cand < 0) {
                            const int sc = __builtin_ctz(cfree);
                            cfree &= ~(1u << sc);
                            if ((threadIdx.x & 63) == 0) wg_cs[kp - 1] = sc;
                            T *kcx = recp(sc, 2), *kcg = recp(sc, 3);
#pragma unroll
                            for (int b = 0; b < NB; ++b)
#pragma unroll
                                for (int e = 0; e < 4; ++e)
                                    if (ok[b][e]) {
                                        kcx[dim_of(b, e)] = wx[b][e];
                                        kcg[dim_of(b, e)] = wg[b][e];
                                    }
                        } else {
                            const int32_t scn = wg_cs[cand - 1];
                            if ((threadIdx.x & 63) == 0) wg_cs[kp - 1] = scn;
                        }
                        if (threadIdx.x == 0) {
                            wg_cn[kp - 1] = n_node;
                            wg_lp[kp - 1] = cand_lp;
                        }
                    } else {                // the last leaf: every subtree of doubling j ends here
                        const T* ccx = recp(cand < 0 ? 0 : wg_cs[cand - 1], 2);
                        const T* ccg = recp(cand < 0 ? 0 : wg_cs[cand - 1], 3);
#pragma unroll
                        for (int b = 0; b < NB; ++b)
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const int64_t d = dim_of(b, e);
                                rcx[b][e] = cand < 0 ? wx[b][e] : (ok[b][e] ? ccx[d] : (T)0);
                                rcg[b][e] = cand < 0 ? wg[b][e] : (ok[b][e] ? ccg[d] : (T)0);
                            }
                        rclp = cand_lp;
                        rcn = n_node;
                        complete = true;
                    }
                    continue;
                }
                if (GK >= 1) {
                    const double lpd = logreg_grad_lds(wx, wg);
#pragma unroll
                    for (int b = 0; b < NB; ++b)
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            wg[b][e] = ok[b][e] ? wg[b][e] - (float)wx[b][e] * (float)a.tg.inv_var : (T)0;
                            wr[b][e] = fma(hse, wg[b][e], wr[b][e]);
                            if (ok[b][e]) lp += -0.5 * (double)wx[b][e] * (double)wx[b][e] * a.tg.inv_var;
                            kin += 0.5 * (double)wr[b][e] * (double)wr[b][e];
                        }
                    nuts_gsum2<G>(lp, kin, gsr, gk);
                    lp += lpd;
                } else {
                    nuts_gsum2<G>(lp, kin, gsr, gk);
                }
                wlogp = lp;
                nleap += 1;
                const double H = -lp + kin;
                if (ST) {
                    alpha += leaf_accept_prob(h0 - H);
                    n_alpha += 1;
                }
                int32_t n_node = (log_u <= -H) ? 1 : 0;
                if (!(log_u < 1000.0 - H)) {
                    alive = false;
                    break;
                }
                int cand = -1, first = -1;
                double cand_lp = lp;
                bool parked = false;
#pragma unroll
                for (int k = 1; k <= NUTS_MAXD; ++k) {
                    if (k > j) break;
                    T *kfx = recp(k, 0), *kfr = recp(k, 1), *kcx = recp(k, 2), *kcg = recp(k, 3);
                    if (((i >> (k - 1)) & 1) == 0) {
                        const T* ffx = recp(first < 0 ? 1 : first, 0);
                        const T* ffr = recp(first < 0 ? 1 : first, 1);
                        const T* ccx = recp(cand < 0 ? 1 : cand, 2);
                        const T* ccg = recp(cand < 0 ? 1 : cand, 3);
#pragma unroll
                        for (int b = 0; b < NB; ++b)
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                if (ok[b][e]) {
                                    const int64_t d = dim_of(b, e);
                                    kfx[d] = first < 0 ? wx[b][e] : ffx[d];
                                    kfr[d] = first < 0 ? wr[b][e] : ffr[d];
                                    kcx[d] = cand < 0 ? wx[b][e] : ccx[d];
                                    kcg[d] = cand < 0 ? wg[b][e] : ccg[d];
                                }
                        lcn[k - 1] = n_node;
                        lclp[k - 1] = cand_lp;
                        parked = true;
                        break;
                    }
                    const int32_t nl = lcn[k - 1];
                    const uint32_t block = ((uint32_t)j * 1024u + (uint32_t)i) * 16u + (uint32_t)k;
                    const double u = nuts_u52(a.key, (uint32_t)cc, t, block, TAG_NUTS_MERGE);
                    if (!((nl + n_node > 0) && u < (double)n_node / (double)(nl + n_node))) {
                        cand = k;
                        cand_lp = lclp[k - 1];
                    }
                    n_node += nl;
                    double dm = 0.0, dp = 0.0;
#pragma unroll
                    for (int b = 0; b < NB; ++b)
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (ok[b][e]) {
                                const int64_t d = dim_of(b, e);
                                const double fx = (double)kfx[d], fr = (double)kfr[d];
                                const double lx = (double)wx[b][e], lr = (double)wr[b][e];
                                const double dx = v > 0 ? lx - fx : fx - lx;
                                dm += dx * (v > 0 ? fr : lr);
                                dp += dx * (v > 0 ? lr : fr);
                            }
                    nuts_gsum2<G>(dm, dp, gsr, gk);
                    first = k;
                    if (!(dm >= 0.0 && dp >= 0.0)) {
                        alive = false;
                        break;
                    }
                }
                if (!alive) break;
                if (!parked) {          // the last leaf: every subtree of doubling j ends here
                    const T* ccx = recp(cand < 0 ? 1 : cand, 2);
                    const T* ccg = recp(cand < 0 ? 1 : cand, 3);
#pragma unroll
                    for (int b = 0; b < NB; ++b)
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int64_t d = dim_of(b, e);
                            rcx[b][e] = cand < 0 ? wx[b][e] : (ok[b][e] ? ccx[d] : (T)0);
                            rcg[b][e] = cand < 0 ? wg[b][e] : (ok[b][e] ? ccg[d] : (T)0);
                        }
                    rclp = cand_lp;
                    rcn = n_node;
                    complete = true;
                }
            }
            // the working state becomes the trajectory end in direction v
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (v > 0) {
                        px[b][e] = wx[b][e];
                        pr[b][e] = wr[b][e];
                        pg[b][e] = wg[b][e];
                    } else {
                        mx[b][e] = wx[b][e];
                        mr[b][e] = wr[b][e];
                        mg[b][e] = wg[b][e];
                    }
                }
            if (v > 0) plogp = wlogp;
            else mlogp = wlogp;
            depth = j + 1;
            s = false;
            if (alive && complete) {
                if (nuts_u52(a.key, (uint32_t)cc, t, (uint32_t)j, TAG_NUTS_TOP) < (double)rcn / ntot) {
#pragma unroll
                    for (int b = 0; b < NB; ++b)
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            x[b][e] = rcx[b][e];
                            g[b][e] = rcg[b][e];
                        }
                    logp = rclp;
                }
                ntot += (double)rcn;
                double dm = 0.0, dp = 0.0;
#pragma unroll
                for (int b = 0; b < NB; ++b)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const double dx = (double)px[b][e] - (double)mx[b][e];
                        dm += dx * (double)mr[b][e];
                        dp += dx * (double)pr[b][e];
                    }
                nuts_gsum2<G>(dm, dp, gsr, gk);
                s = dm >= 0.0 && dp >= 0.0;
            }
        }
        const double stat = n_alpha > 0 ? alpha / (double)n_alpha : 0.0;
        if (ST && ad.adapt && it < n_burnin) eps = nuts_adapt(ad, it, stat, eps, da);
        if (active && it >= n_burnin) {
            const int64_t r = it - n_burnin;
            if (samples)
#pragma unroll
                for (int b = 0; b < NB; ++b)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (ok[b][e]) samples[(r * C + c) * D + dim_of(b, e)] = x[b][e];
            if (lane == 0) {
                if (tr_depth) tr_depth[r * C + c] = depth;
                if (tr_nleap) tr_nleap[r * C + c] = nleap;
                if (ST && tr_stat) tr_stat[r * C + c] = stat;
            }
        }
    }
    if (!active) return;
    T* Xw = (T*)a.ws.x;
    T* Gw = (T*)a.ws.g;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (ok[b][e]) {
                Xw[c * D + dim_of(b, e)] = x[b][e];
                Gw[c * D + dim_of(b, e)] = g[b][e];
            }
    if (lane == 0) {
        a.ws.logp[c] = logp;
        if (ST) {
            a.ws.eps[c] = eps;
            a.ws.da[c] = da;
        }
    }
}

// ---------------------------------------------------------------------------
// Persistent NUTS for the dense Gaussian on MFMA (FP32, D <= 128).  A
// workgroup of 8 waves (two per SIMD) owns 16 chains in the layout of the
// fused dense HMC kernel: P as the A operands of v_mfma_f32_16x16x4f32 in
// VGPRs, x staged chain-major in LDS as the B operands, lane (g4, i16) of wave
// w holding dims 16 (w + 8 m) + 4 g4 + v of chain i16.  The 16 chains build
// their trees in lockstep -- the same doubling and leaf at a time, a chain
// that has stopped masked -- and the tile moves on as soon as none of them is
// running, so a chain waits for the 15 others of its tile only, and there is
// one launch for the whole run.  A chain's sums over its dims (energies,
// U-turn products) are summed over its 4 lane rows with register-only lane
// swaps and over the 8 waves through one LDS exchange; every reduction sits
// where the control flow is uniform across the workgroup (their count depends
// on the leaf index only).  The trajectory ends, the levels' parked first
// leaves and candidates and the doubling's candidate live in the NutsWs
// buffers, each lane touching only its own dims, except the parked records of
// the shallow levels (the merges of all but a few of the leaves) and every
// level's parked leaf count and candidate logp, which sit in LDS: a global
// read there is latency that nothing hides.  Every wave holds all 16 chains,
// so whether any chain of the tile is still running is a wave-local ballot
// (every wave computes the same flags from the same sums and random numbers);
// a leaf costs two barriers, the drifted x and one reduction that carries the
// leaf's energies and every U-turn check ending at it.
// Same tree, uniforms and arithmetic order per lane as the lockstep kernels
// up to the order of the FP64 sums.
// ---------------------------------------------------------------------------
constexpr int ND_NW = 8;                    // waves per workgroup (2 per SIMD)
constexpr int ND_LDS_MAX = 163840;          // LDS bytes of a gfx950 workgroup
constexpr int ND_RV = 2;                    // values per chain in a per-transition / per-doubling reduction
constexpr int ND_LV = 2 * NUTS_MAXD;        // values per chain in a leaf's reduction: the two energies and
                                            // the two U-turn products of each subtree that ends at the leaf
constexpr int ND_LRS = 10;                  // doubles per (value, chain) row of the leaf reduction: the 8
                                            // waves' partials, padded so 16 chains' rows hit distinct banks

template <int NT>
constexpr int nd_xs() { return 16 * NT + 4; }
// LDS bytes before the level records: x staging, the leaf reduction, the
// other reductions, each level's parked leaf count and candidate logp
template <int NT>
constexpr int nd_fixed_bytes() {
    return 16 * nd_xs<NT>() * 4 + ND_LV * 16 * ND_LRS * 8 + 2 * ND_RV * ND_NW * 16 * 8 + NUTS_MAXD * 16 * (8 + 4);
}
// levels whose records (first leaf x, r; candidate x, g of 16 chains) fit in LDS
template <int NT>
constexpr int nd_lds_levels() {
    constexpr int lv = (ND_LDS_MAX - nd_fixed_bytes<NT>()) / (4 * 16 * nd_xs<NT>() * 4);
    return lv > NUTS_MAXD - 1 ? NUTS_MAXD - 1 : lv;
}
template <int NT>
constexpr int nd_lds_bytes() { return nd_fixed_bytes<NT>() + nd_lds_levels<NT>() * 4 * 16 * nd_xs<NT>() * 4; }

// Sums over each chain's dims of the first nv (<= NV, the same for the whole
// workgroup) of sv's values, returned to every lane of the chain: two
// shuffles over the chain's 4 lane rows, then the waves' partials through the
// LDS buffer rb (one barrier; the caller makes sure no wave still reads rb
// from the previous use).
template <int NV>
__device__ __forceinline__ void nd_chain_sum(double* sv, int nv, double* rb, int w, int g4, int i16) {
#pragma unroll
    for (int q = 0; q < NV; ++q)
        if (q < nv) {
            sv[q] += __shfl_xor(sv[q], 16, 64);
            sv[q] += __shfl_xor(sv[q], 32, 64);
        }
    if (g4 == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q)
            if (q < nv) rb[(q * ND_NW + w) * 16 + i16] = sv[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q)
        if (q < nv) {
            double acc = 0.0;
#pragma unroll
            for (int ww = 0; ww < ND_NW; ++ww) acc += rb[(q * ND_NW + ww) * 16 + i16];
            sv[q] = acc;
        }
}

// Sum of v over lanes l, l ^ 16, l ^ 32, l ^ 48 (a chain's 4 lane rows),
// exact in rows 0 (the lanes that store it): register-only lane swaps of
// gfx950 instead of LDS permutes.  v_permlane32_swap trades the upper 32 lanes
// of its first operand for the lower 32 of its second, so the second result
// holds x[l + 32] in rows 0, 1; v_permlane16_swap trades the odd rows of its
// first operand for the even rows of its second, so the second result holds
// x[l + 16] in rows 0, 2.
__device__ __forceinline__ double nd_rows_sum(double v) {
    uint32_t lo = (uint32_t)__double_as_longlong(v), hi = (uint32_t)((uint64_t)__double_as_longlong(v) >> 32);
    const auto l32 = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto h32 = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    const double s = v + __longlong_as_double((long long)(((uint64_t)h32[1] << 32) | l32[1]));
    lo = (uint32_t)__double_as_longlong(s);
    hi = (uint32_t)((uint64_t)__double_as_longlong(s) >> 32);
    const auto l16 = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h16 = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    return s + __longlong_as_double((long long)(((uint64_t)h16[1] << 32) | l16[1]));
}

template <int NT, bool ST>
__global__ __launch_bounds__(64 * ND_NW) void k_nuts_fused_dense(PlainArgs a, NutsWs n, NutsAdapt ad, uint32_t t_begin,
                                                          int64_t n_trans, int32_t max_depth, float* samples,
                                                          int32_t* tr_depth, int32_t* tr_nleap, double* tr_stat) {
    constexpr int MT = (NT + ND_NW - 1) / ND_NW;
    constexpr int KM = 4 * NT;
    constexpr int XS = nd_xs<NT>();
    constexpr int LV = nd_lds_levels<NT>();
    static_assert(LV >= 1, "the level records need at least one LDS level");
    extern __shared__ float lds[];
    const int64_t C = a.C, D = a.tg.D;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i16 = lane & 15, g4 = lane >> 4;
    const int64_t c = (int64_t)blockIdx.x * 16 + i16;
    const bool cvalid = c < C;
    const int64_t cc = cvalid ? c : 0;
    float* xs = lds;                                     // [16 chains][XS]
    double* lred = (double*)(lds + 16 * XS);             // [ND_LV values][16 chains][ND_LRS]
    double* red = lred + ND_LV * 16 * ND_LRS;            // [2 parity][ND_RV values][NW][16]
    double* lclp = red + 2 * ND_RV * ND_NW * 16;         // [NUTS_MAXD levels][16]: candidate logp
    int32_t* lcn = (int32_t*)(lclp + NUTS_MAXD * 16);    // [NUTS_MAXD levels][16]: slice leaf count
    float* lvl = (float*)(lcn + NUTS_MAXD * 16);         // [LV][4 records][16 chains][XS]
    const float* P = (const float*)a.tg.prec;
    float *mx = (float*)n.mx, *mr = (float*)n.mr, *mg = (float*)n.mg;
    float *px = (float*)n.px, *pr = (float*)n.pr, *pg = (float*)n.pg;
    float *lfx = (float*)n.lf_x, *lfr = (float*)n.lf_r, *lcx = (float*)n.lc_x, *lcg = (float*)n.lc_g;
    float *rcx = (float*)n.rc_x, *rcg = (float*)n.rc_g;

    float pa[MT][KM];
    bool tile_ok[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        const int mt = w + ND_NW * m;
        tile_ok[m] = mt < NT;
        const int64_t row = 16 * mt + i16;
#pragma unroll
        for (int ks = 0; ks < KM; ++ks) {
            const int64_t col = (int64_t)g4 * KM + ks;
            pa[m][ks] = (tile_ok[m] && row < D && col < D) ? P[row * D + col] : 0.f;
        }
    }
    auto dim_of = [&](int m, int v) -> int64_t { return 16 * (w + ND_NW * m) + 4 * g4 + v; };
    float x[MT][4], g[MT][4];
    bool ok[MT][4];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            ok[m][v] = tile_ok[m] && cvalid && dim_of(m, v) < D;
            x[m][v] = ok[m][v] ? ((const float*)a.ws.x)[cc * D + dim_of(m, v)] : 0.f;
            g[m][v] = ok[m][v] ? ((const float*)a.ws.g)[cc * D + dim_of(m, v)] : 0.f;
        }
    // parked records of level k (1 ..): 0 first leaf x, 1 first leaf r, 2
    // candidate x, 3 candidate g; the lane's 4 dims of tile m
    float* const grec[4] = {lfx, lfr, lcx, lcg};
    // element offset of level k's record of this lane's chain; formed where it
    // is used (the empty asm keeps the compiler from hoisting one 64-bit
    // address per level and record out of the leaf loop into registers)
    auto rec_off = [&](int k) -> int64_t {
        int64_t off = ((int64_t)k * C + cc) * D;
        asm volatile("" : "+v"(off));
        return off;
    };
    auto rec_load = [&](int k, int q, int m, float out[4]) {
        if (k <= LV) {
            const floatx4 v4 = *(const floatx4*)(lvl + (((k - 1) * 4 + q) * 16 + i16) * XS + 16 * (w + ND_NW * m) +
                                                  4 * g4);
#pragma unroll
            for (int v = 0; v < 4; ++v) out[v] = v4[v];
        } else {
            const float* gp = grec[q] + rec_off(k);
#pragma unroll
            for (int v = 0; v < 4; ++v) out[v] = ok[m][v] ? gp[dim_of(m, v)] : 0.f;
        }
    };
    auto rec_store = [&](int k, int q, int m, const float in[4]) {
        if (k <= LV) {
            *(floatx4*)(lvl + (((k - 1) * 4 + q) * 16 + i16) * XS + 16 * (w + ND_NW * m) + 4 * g4) =
                floatx4{in[0], in[1], in[2], in[3]};
        } else {
            float* gp = grec[q] + rec_off(k);
#pragma unroll
            for (int v = 0; v < 4; ++v)
                if (ok[m][v]) gp[dim_of(m, v)] = in[v];
        }
    };
    // the two halves of rec_load for a level known to sit in LDS (1 .. LV; any
    // lane may pass its own) or in global memory (lanes of dims beyond D read 0)
    auto rec_lds = [&](int k, int q, int m) -> floatx4 {
        return *(const floatx4*)(lvl + (((k - 1) * 4 + q) * 16 + i16) * XS + 16 * (w + ND_NW * m) + 4 * g4);
    };
    auto rec_glb = [&](int k, int q, int m, float out[4]) {
        const float* gp = grec[q] + rec_off(k);
#pragma unroll
        for (int v = 0; v < 4; ++v) out[v] = ok[m][v] ? gp[dim_of(m, v)] : 0.f;
    };
    double logp = a.ws.logp[cc];
    double eps = a.ws.eps[cc];
    DualAvg da{};
    if (ST) da = a.ws.da[cc];
    int rk = 0;

    // the per-transition and per-doubling reductions alternate two buffers,
    // so one barrier each suffices
    auto chain_sum2 = [&](double& s0, double& s1) {
        double sv[2] = {s0, s1};
        nd_chain_sum<2>(sv, 2, red + (rk & 1) * (ND_RV * ND_NW * 16), w, g4, i16);
        ++rk;
        s0 = sv[0];
        s1 = sv[1];
    };
    // does any chain of the tile satisfy pred (one value per chain, the same
    // in every wave)
    auto tile_any = [&](bool pred) -> bool { return __ballot(pred ? 1 : 0) != 0ull; };

    for (int64_t it = 0; it < n_trans; ++it) {
        const uint32_t t = t_begin + (uint32_t)it;
        double k0 = 0.0, unused = 0.0;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            float z[4];
            momentum4<float>(a.key, (uint32_t)cc, t, (uint32_t)(4 * (w + ND_NW * m) + g4), z);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float r0 = ok[m][v] ? z[v] : 0.f;
                k0 += 0.5 * (double)r0 * (double)r0;
                if (ok[m][v]) {
                    const int64_t e = c * D + dim_of(m, v);
                    mx[e] = px[e] = x[m][v];
                    mr[e] = pr[e] = r0;
                    mg[e] = pg[e] = g[m][v];
                }
            }
        }
        chain_sum2(k0, unused);
        const double h0 = -logp + k0;
        const double log_u = log(nuts_u52(a.key, (uint32_t)cc, t, 0u, TAG_NUTS_SLICE)) - h0;
        double mlogp = logp, plogp = logp, ntot = 1.0;
        bool active = cvalid;
        int32_t depth = 0, nleap = 0;
        double alpha = 0.0;
        int32_t n_alpha = 0;
        for (int j = 0; j < max_depth; ++j) {
            if (!tile_any(active)) break;
            const int dir = (active && nuts_u52(a.key, (uint32_t)cc, t, (uint32_t)j, TAG_NUTS_DIR) < 0.5) ? -1 : 1;
            const float se = (float)((double)dir * eps), hse = (float)(0.5 * ((double)dir * eps));
            float wx[MT][4], wr[MT][4], wg[MT][4];
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t e = cc * D + dim_of(m, v);
                    wx[m][v] = ok[m][v] ? (dir > 0 ? px[e] : mx[e]) : 0.f;
                    wr[m][v] = ok[m][v] ? (dir > 0 ? pr[e] : mr[e]) : 0.f;
                    wg[m][v] = ok[m][v] ? (dir > 0 ? pg[e] : mg[e]) : 0.f;
                }
            double wlogp = dir > 0 ? plogp : mlogp;
            bool alive = active, complete = false;
            if (ST && active) {
                alpha = 0.0;
                n_alpha = 0;
            }
            double rclp = 0.0;
            int32_t rcn = 0;
            const int nleaves = 1 << j;
            for (int i = 0; i < nleaves; ++i) {
                if (!tile_any(alive)) break;
                // one leapfrog step of size dir eps for every chain of the tile
#pragma unroll
                for (int m = 0; m < MT; ++m) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        wr[m][v] = wr[m][v] + hse * wg[m][v];
                        wx[m][v] = fmaf(se, wr[m][v], wx[m][v]);
                    }
                    if (tile_ok[m])
                        *(floatx4*)(xs + i16 * XS + 16 * (w + ND_NW * m) + 4 * g4) =
                            floatx4{wx[m][0], wx[m][1], wx[m][2], wx[m][3]};
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
                __builtin_amdgcn_sched_group_barrier(0x100, NT, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, KM * MT, 0);
                // the leaf's energies, then for each subtree that ends at this leaf
                // (levels k = 1 .. nm: bit k-1 of i set, k <= j) the U-turn products of
                // its first leaf (parked at level k) and this leaf: each value's lane
                // partials go to the leaf reduction buffer as they are formed, and one
                // barrier later the chain's sums are read where they are used
                const int nm = min(__builtin_ctz(~(unsigned)i), j);
                // two values' lane partials summed over the chain's 4 lane rows and
                // stored (from row 0) as this wave's partials of values q, q + 1
                auto lred_put2 = [&](int q, double v0, double v1) {
                    v0 = nd_rows_sum(v0);
                    v1 = nd_rows_sum(v1);
                    if (g4 == 0) {
                        lred[(q * 16 + i16) * ND_LRS + w] = v0;
                        lred[((q + 1) * 16 + i16) * ND_LRS + w] = v1;
                    }
                };
                auto lred_get = [&](int q) -> double {
                    const double2* r2 = (const double2*)(lred + (q * 16 + i16) * ND_LRS);
                    double2 pv[ND_NW / 2];
#pragma unroll
                    for (int h = 0; h < ND_NW / 2; ++h) pv[h] = r2[h];
                    double acc = pv[0].x;
#pragma unroll
                    for (int h = 0; h < ND_NW / 2; ++h) {
                        if (h > 0) acc += pv[h].x;
                        acc += pv[h].y;
                    }
                    return acc;
                };
                {
                    double lp = 0.0, kin = 0.0;
#pragma unroll
                    for (int m = 0; m < MT; ++m)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            // dims beyond D (and chains beyond C) hold zeros
                            wg[m][v] = -(acc[m][0][v] + acc[m][1][v]);
                            wr[m][v] = fmaf(hse, wg[m][v], wr[m][v]);
                            kin += 0.5 * (double)wr[m][v] * (double)wr[m][v];
                            lp += 0.5 * (double)wx[m][v] * (double)wg[m][v];
                        }
                    lred_put2(0, lp, kin);
                }
                // (the levels in LDS first, as straight-line reads; the deep ones, at few
                // leaves, from global memory)
                auto uturn_part = [&](int k, const float (&f0)[4], const float (&f1)[4], int m, double& dm,
                                      double& dp) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const double fx = (double)f0[v], fr = (double)f1[v];
                        const double lx = (double)wx[m][v], lr = (double)wr[m][v];
                        const double dx = dir > 0 ? lx - fx : fx - lx;
                        dm += dx * (dir > 0 ? fr : lr);
                        dp += dx * (dir > 0 ? lr : fr);
                    }
                };
                const int nm_l = min(nm, LV);
                for (int k = 1; k <= nm_l; ++k) {
                    double dm = 0.0, dp = 0.0;
#pragma unroll
                    for (int m = 0; m < MT; ++m) {
                        if (!tile_ok[m]) continue;
                        const floatx4 a0 = rec_lds(k, 0, m), a1 = rec_lds(k, 1, m);
                        const float f0[4] = {a0[0], a0[1], a0[2], a0[3]}, f1[4] = {a1[0], a1[1], a1[2], a1[3]};
                        uturn_part(k, f0, f1, m, dm, dp);
                    }
                    lred_put2(2 * k, dm, dp);
                }
                for (int k = LV + 1; k <= nm; ++k) {
                    double dm = 0.0, dp = 0.0;
#pragma unroll
                    for (int m = 0; m < MT; ++m) {
                        if (!tile_ok[m]) continue;
                        float f0[4], f1[4];
                        rec_glb(k, 0, m, f0);
                        rec_glb(k, 1, m, f1);
                        uturn_part(k, f0, f1, m, dm, dp);
                    }
                    lred_put2(2 * k, dm, dp);
                }
                __syncthreads();
                const double lp = lred_get(0), kin = lred_get(1);
                int32_t n_node = 0;
                if (alive) {
                    wlogp = lp;
                    nleap += 1;
                    const double H = -lp + kin;
                    if (ST) {
                        alpha += leaf_accept_prob(h0 - H);
                        n_alpha += 1;
                    }
                    n_node = (log_u <= -H) ? 1 : 0;
                    if (!(log_u < 1000.0 - H)) alive = false;
                }
                // merge the subtrees that end here (levels 1 .. nm), then park the
                // merged tree at level nm + 1, or, at the doubling's last leaf
                // (nm == j), keep its candidate
                int cand = -1;
                double cand_lp = lp;
                for (int k = 1; k <= nm; ++k) {
                    if (alive) {
                        const int32_t nl = lcn[(k - 1) * 16 + i16];
                        const uint32_t block = ((uint32_t)j * 1024u + (uint32_t)i) * 16u + (uint32_t)k;
                        const double u = nuts_u52(a.key, (uint32_t)cc, t, block, TAG_NUTS_MERGE);
                        if (!((nl + n_node > 0) && u < (double)n_node / (double)(nl + n_node))) {
                            cand = k;
                            cand_lp = lclp[(k - 1) * 16 + i16];
                        }
                        n_node += nl;
                    }
                    if (alive && !(lred_get(2 * k) >= 0.0 && lred_get(2 * k + 1) >= 0.0)) alive = false;
                }
                if (nm < j) {
                    // park at level nm + 1 (the same for the whole tile): its first leaf is
                    // that of level nm's subtree (this leaf when nm = 0).  Stopped chains
                    // park too (their records are never merged again), so the stores are
                    // not divergent; the candidate's level is per chain: its LDS record
                    // is read from a clamped level by every lane, the global one only when
                    // some chain's candidate sits there.  The count and the candidate's
                    // logp go to LDS, read back by every lane of the chain at the merge
                    // (one barrier or more later).
                    const int kp = nm + 1;
                    const int cl = min(max(cand, 1), LV);
                    const bool cand_glb = __ballot(cand > LV ? 1 : 0) != 0ull;
#pragma unroll
                    for (int m = 0; m < MT; ++m) {
                        if (!tile_ok[m]) continue;
                        float f0[4], f1[4], c0[4], c1[4];
                        if (nm == 0) {
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                f0[v] = wx[m][v];
                                f1[v] = wr[m][v];
                            }
                        } else if (nm <= LV) {
                            const floatx4 a0 = rec_lds(nm, 0, m), a1 = rec_lds(nm, 1, m);
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                f0[v] = a0[v];
                                f1[v] = a1[v];
                            }
                        } else {
                            rec_glb(nm, 0, m, f0);
                            rec_glb(nm, 1, m, f1);
                        }
                        const floatx4 l0 = rec_lds(cl, 2, m), l1 = rec_lds(cl, 3, m);
                        float g0[4] = {0.f, 0.f, 0.f, 0.f}, g1[4] = {0.f, 0.f, 0.f, 0.f};
                        if (cand_glb) {
                            rec_glb(max(cand, LV + 1), 2, m, g0);
                            rec_glb(max(cand, LV + 1), 3, m, g1);
                        }
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            c0[v] = cand < 0 ? wx[m][v] : (cand <= LV ? l0[v] : g0[v]);
                            c1[v] = cand < 0 ? wg[m][v] : (cand <= LV ? l1[v] : g1[v]);
                        }
                        if (kp <= LV) {
                            float* base = lvl + (((kp - 1) * 4) * 16 + i16) * XS + 16 * (w + ND_NW * m) + 4 * g4;
                            *(floatx4*)(base) = floatx4{f0[0], f0[1], f0[2], f0[3]};
                            *(floatx4*)(base + 16 * XS) = floatx4{f1[0], f1[1], f1[2], f1[3]};
                            *(floatx4*)(base + 2 * 16 * XS) = floatx4{c0[0], c0[1], c0[2], c0[3]};
                            *(floatx4*)(base + 3 * 16 * XS) = floatx4{c1[0], c1[1], c1[2], c1[3]};
                        } else {
                            rec_store(kp, 0, m, f0);
                            rec_store(kp, 1, m, f1);
                            rec_store(kp, 2, m, c0);
                            rec_store(kp, 3, m, c1);
                        }
                    }
                    if (w == 0 && g4 == 0) {
                        lcn[(kp - 1) * 16 + i16] = n_node;
                        lclp[(kp - 1) * 16 + i16] = cand_lp;
                    }
                } else if (alive) {         // the last leaf: every subtree of doubling j ends here
#pragma unroll
                    for (int m = 0; m < MT; ++m) {
                        if (!tile_ok[m]) continue;
                        float c0[4], c1[4];
                        if (cand < 0) {
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                c0[v] = wx[m][v];
                                c1[v] = wg[m][v];
                            }
                        } else {
                            rec_load(cand, 2, m, c0);
                            rec_load(cand, 3, m, c1);
                        }
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            if (ok[m][v]) {
                                rcx[cc * D + dim_of(m, v)] = c0[v];
                                rcg[cc * D + dim_of(m, v)] = c1[v];
                            }
                    }
                    rclp = cand_lp;
                    rcn = n_node;
                    complete = true;
                }
            }
            // the working state becomes the trajectory end in direction dir
            if (active) {
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (ok[m][v]) {
                            const int64_t e = cc * D + dim_of(m, v);
                            (dir > 0 ? px : mx)[e] = wx[m][v];
                            (dir > 0 ? pr : mr)[e] = wr[m][v];
                            (dir > 0 ? pg : mg)[e] = wg[m][v];
                        }
                if (dir > 0) plogp = wlogp;
                else mlogp = wlogp;
                depth = j + 1;
            }
            const bool grown = active && alive && complete;
            double dm = 0.0, dp = 0.0;
            if (grown) {
                if (nuts_u52(a.key, (uint32_t)cc, t, (uint32_t)j, TAG_NUTS_TOP) < (double)rcn / ntot) {
#pragma unroll
                    for (int m = 0; m < MT; ++m)
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            if (ok[m][v]) {
                                x[m][v] = rcx[cc * D + dim_of(m, v)];
                                g[m][v] = rcg[cc * D + dim_of(m, v)];
                            }
                    logp = rclp;
                }
                ntot += (double)rcn;
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (ok[m][v]) {
                            const int64_t e = cc * D + dim_of(m, v);
                            const double dx = (double)px[e] - (double)mx[e];
                            dm += dx * (double)mr[e];
                            dp += dx * (double)pr[e];
                        }
            }
            chain_sum2(dm, dp);
            active = grown && dm >= 0.0 && dp >= 0.0;
        }
        const double stat = n_alpha > 0 ? alpha / (double)n_alpha : 0.0;
        if (ST && ad.adapt && it < ad.n_burnin) eps = nuts_adapt(ad, it, stat, eps, da);
        if (cvalid && it >= ad.n_burnin) {
            const int64_t r = it - ad.n_burnin;
            if (samples)
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (ok[m][v]) samples[(r * C + c) * D + dim_of(m, v)] = x[m][v];
            if (w == 0 && g4 == 0) {
                if (tr_depth) tr_depth[r * C + c] = depth;
                if (tr_nleap) tr_nleap[r * C + c] = nleap;
                if (ST && tr_stat) tr_stat[r * C + c] = stat;
            }
        }
    }
    if (!cvalid) return;
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            if (ok[m][v]) {
                ((float*)a.ws.x)[c * D + dim_of(m, v)] = x[m][v];
                ((float*)a.ws.g)[c * D + dim_of(m, v)] = g[m][v];
            }
    if (w == 0 && g4 == 0) {
        a.ws.logp[c] = logp;
        if (ST) {
            a.ws.eps[c] = eps;
            a.ws.da[c] = da;
        }
    }
}

// lanes per chain and 4-dim blocks per lane of the persistent kernel, 0 if it
// does not apply (registers: FP64 keeps one block per lane, FP32 two)
// the logistic persistent kernel: FP32 states and X, D <= 4 LR_DQ, X and y in LDS
static bool nuts_lr_supported(const PlainArgs& a) {
    return a.tg.kind == HMC_TGT_LOGREG && !a.f64 && !a.tg.x_bf16 && !a.bf16_grad && a.tg.D >= 1 &&
           a.tg.D <= 4 * LR_DQ && nuts_lr_lds_bytes(a.tg.N, a.tg.D) <= (size_t)ND_LDS_MAX - 64;
}

// the L2 variant: FP32 states, X (FP32 or BF16) beyond the LDS or stored in BF16,
// D <= 4 LR_DQ
static bool nuts_l2_supported(const PlainArgs& a) {
    return a.tg.kind == HMC_TGT_LOGREG && !a.f64 && !a.bf16_grad && a.tg.D >= 1 && a.tg.D <= 4 * LR_DQ &&
           a.tg.N >= 1 && !nuts_lr_supported(a);
}

int64_t nuts_l2_rows(const PlainArgs& a) { return nuts_l2_supported(a) ? a.tg.N : 0; }

static int nuts_elem_shape(const PlainArgs& a, int* G) {
    if (nuts_lr_supported(a) || nuts_l2_supported(a)) { *G = 64; return 1; }
    if (a.tg.kind != HMC_TGT_STD_NORMAL && a.tg.kind != HMC_TGT_GAUSS_DIAG) return 0;
    const int64_t nblk = (a.tg.D + 3) / 4;
    if (nblk <= 1) { *G = 1; return 1; }
    if (nblk <= 4) { *G = 4; return 1; }
    if (nblk <= 16) { *G = 16; return 1; }
    if (nblk <= 64) { *G = 64; return 1; }
    if (nblk <= 128 && !a.f64) { *G = 64; return 2; }
    if (nblk <= 256) { *G = 256; return 1; }      // one chain per workgroup
    return 0;
}

// the persistent dense kernel: FP32 states, D <= 128 (P resident in VGPRs)
static bool nuts_dense_supported(const PlainArgs& a) {
    return a.tg.kind == HMC_TGT_GAUSS_DENSE && !a.f64 && a.tg.D >= 1 && a.tg.D <= 128;
}

bool nuts_fused_supported(const PlainArgs& a) {
    int G;
    return nuts_elem_shape(a, &G) > 0 || nuts_dense_supported(a);
}

static hipError_t launch_nuts_dense(const PlainArgs& a, const NutsWs& n, const NutsAdapt& ad, uint32_t t_begin,
                                    int64_t n_trans, int32_t max_depth, void* samples, int32_t* tr_depth,
                                    int32_t* tr_nleap, double* tr_stat, hipStream_t s) {
    const int nt = (int)((a.tg.D + 15) / 16);
    const dim3 grid((unsigned)((a.C + 15) / 16));
    const bool st = ad.adapt || tr_stat;
    switch (nt) {
#define HMC_NUTS_D(N)                                                                                               \
    case N: {                                                                                                       \
        constexpr size_t lds = nd_lds_bytes<N>();                                                                   \
        if (st) {                                                                                                   \
            if (lds > 65536)                                                                                        \
                (void)hipFuncSetAttribute((const void*)k_nuts_fused_dense<N, true>,                                 \
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                    \
            hipLaunchKernelGGL((k_nuts_fused_dense<N, true>), grid, dim3(64 * ND_NW), lds, s, a, n, ad, t_begin, n_trans,  \
                               max_depth, (float*)samples, tr_depth, tr_nleap, tr_stat);                            \
        } else {                                                                                                    \
            if (lds > 65536)                                                                                        \
                (void)hipFuncSetAttribute((const void*)k_nuts_fused_dense<N, false>,                                \
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                    \
            hipLaunchKernelGGL((k_nuts_fused_dense<N, false>), grid, dim3(64 * ND_NW), lds, s, a, n, ad, t_begin, n_trans, \
                               max_depth, (float*)samples, tr_depth, tr_nleap, tr_stat);                            \
        }                                                                                                           \
        break;                                                                                                      \
    }
        HMC_NUTS_D(1) HMC_NUTS_D(2) HMC_NUTS_D(3) HMC_NUTS_D(4)
        HMC_NUTS_D(5) HMC_NUTS_D(6) HMC_NUTS_D(7) HMC_NUTS_D(8)
#undef HMC_NUTS_D
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_nuts_fused(const PlainArgs& a, const NutsWs& n, const NutsAdapt& ad, uint32_t t_begin,
                             int64_t n_trans, int32_t max_depth, void* samples, int32_t* tr_depth, int32_t* tr_nleap,
                             double* tr_stat, hipStream_t s) {
    if (nuts_dense_supported(a))
        return launch_nuts_dense(a, n, ad, t_begin, n_trans, max_depth, samples, tr_depth, tr_nleap, tr_stat, s);
    int G = 0;
    const int NB = nuts_elem_shape(a, &G);
    if (NB == 0) return hipErrorNotSupported;
    const dim3 grid((unsigned)((a.C * G + 255) / 256));
    const bool st = ad.adapt || tr_stat;
#define HMC_NUTS_F(TT, GG, NN)                                                                                       \
    do {                                                                                                             \
        if (st)                                                                                                      \
            hipLaunchKernelGGL((k_nuts_fused_elem<TT, GG, NN, true, 0>), grid, dim3(256), 0, s, a, n, ad, t_begin,   \
                               n_trans, max_depth, (TT*)samples, tr_depth, tr_nleap, tr_stat);                       \
        else                                                                                                         \
            hipLaunchKernelGGL((k_nuts_fused_elem<TT, GG, NN, false, 0>), grid, dim3(256), 0, s, a, n, ad, t_begin,  \
                               n_trans, max_depth, (TT*)samples, tr_depth, tr_nleap, tr_stat);                       \
    } while (0)
    if (nuts_l2_supported(a)) {
        if (!n.xt4 || !n.yf) return hipErrorInvalidValue;
        const int64_t ne = (a.tg.D + 3) / 4 * a.tg.N;
        int64_t pb = (ne + 255) / 256;
        if (pb > 4096) pb = 4096;
        hipLaunchKernelGGL(k_nuts_pad_x, dim3((unsigned)pb), dim3(256), 0, s, a.tg.X, a.tg.x_bf16 ? 1 : 0, a.tg.y,
                           n.xt4, n.yf, a.tg.N, a.tg.D);
        const size_t lds = nuts_l2_lds_bytes(a.tg.D);
        if (st)
            hipLaunchKernelGGL((k_nuts_fused_elem<float, 64, 1, true, 2>), grid, dim3(256), lds, s, a, n, ad, t_begin,
                               n_trans, max_depth, (float*)samples, tr_depth, tr_nleap, tr_stat);
        else
            hipLaunchKernelGGL((k_nuts_fused_elem<float, 64, 1, false, 2>), grid, dim3(256), lds, s, a, n, ad,
                               t_begin, n_trans, max_depth, (float*)samples, tr_depth, tr_nleap, tr_stat);
    } else if (nuts_lr_supported(a)) {
        const size_t lds = nuts_lr_lds_bytes(a.tg.N, a.tg.D);
        if (st) {
            if (lds > 65536)
                (void)hipFuncSetAttribute((const void*)k_nuts_fused_elem<float, 64, 1, true, 1>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            hipLaunchKernelGGL((k_nuts_fused_elem<float, 64, 1, true, 1>), grid, dim3(256), lds, s, a, n, ad, t_begin,
                               n_trans, max_depth, (float*)samples, tr_depth, tr_nleap, tr_stat);
        } else {
            if (lds > 65536)
                (void)hipFuncSetAttribute((const void*)k_nuts_fused_elem<float, 64, 1, false, 1>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            hipLaunchKernelGGL((k_nuts_fused_elem<float, 64, 1, false, 1>), grid, dim3(256), lds, s, a, n, ad,
                               t_begin, n_trans, max_depth, (float*)samples, tr_depth, tr_nleap, tr_stat);
        }
    } else if (a.f64) {
        if (G == 1) HMC_NUTS_F(double, 1, 1);
        else if (G == 4) HMC_NUTS_F(double, 4, 1);
        else if (G == 16) HMC_NUTS_F(double, 16, 1);
        else if (G == 64) HMC_NUTS_F(double, 64, 1);
        else HMC_NUTS_F(double, 256, 1);
    } else {
        if (G == 1) HMC_NUTS_F(float, 1, 1);
        else if (G == 4) HMC_NUTS_F(float, 4, 1);
        else if (G == 16) HMC_NUTS_F(float, 16, 1);
        else if (G == 64 && NB == 1) HMC_NUTS_F(float, 64, 1);
        else if (G == 64) HMC_NUTS_F(float, 64, 2);
        else HMC_NUTS_F(float, 256, 1);
    }
#undef HMC_NUTS_F
    return hipGetLastError();
}

__global__ void k_nuts_zero(int32_t* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

static dim3 nuts_grid(int64_t C) { return dim3((unsigned)((C + 3) / 4)); }

hipError_t launch_nuts_begin(const PlainArgs& a, const NutsWs& n, uint32_t t, hipStream_t s) {
    if (a.f64) hipLaunchKernelGGL(k_nuts_begin<double>, nuts_grid(a.C), dim3(256), 0, s, a, n, t);
    else hipLaunchKernelGGL(k_nuts_begin<float>, nuts_grid(a.C), dim3(256), 0, s, a, n, t);
    return hipGetLastError();
}

hipError_t launch_nuts_dir(const PlainArgs& a, const NutsWs& n, uint32_t t, int32_t j, hipStream_t s) {
    if (a.f64) hipLaunchKernelGGL(k_nuts_dir<double>, nuts_grid(a.C), dim3(256), 0, s, a, n, t, j);
    else hipLaunchKernelGGL(k_nuts_dir<float>, nuts_grid(a.C), dim3(256), 0, s, a, n, t, j);
    return hipGetLastError();
}

hipError_t launch_nuts_halfkick(const PlainArgs& a, const NutsWs& n, hipStream_t s) {
    const int64_t tot = a.C * a.tg.D;
    const dim3 grid((unsigned)((tot + 255) / 256 < 65536 ? (tot + 255) / 256 : 65536));
    if (a.f64) hipLaunchKernelGGL(k_nuts_halfkick<double>, grid, dim3(256), 0, s, a, n);
    else hipLaunchKernelGGL(k_nuts_halfkick<float>, grid, dim3(256), 0, s, a, n);
    return hipGetLastError();
}

hipError_t launch_nuts_leaf(const PlainArgs& a, const NutsWs& n, uint32_t t, int32_t j, int32_t i, hipStream_t s) {
    if (a.f64) hipLaunchKernelGGL(k_nuts_leaf<double>, nuts_grid(a.C), dim3(256), 0, s, a, n, t, j, i);
    else hipLaunchKernelGGL(k_nuts_leaf<float>, nuts_grid(a.C), dim3(256), 0, s, a, n, t, j, i);
    return hipGetLastError();
}

hipError_t launch_nuts_doubling_end(const PlainArgs& a, const NutsWs& n, uint32_t t, int32_t j, hipStream_t s) {
    hipLaunchKernelGGL(k_nuts_zero, dim3(1), dim3(64), 0, s, n.n_active);
    if (a.f64) hipLaunchKernelGGL(k_nuts_doubling_end<double>, nuts_grid(a.C), dim3(256), 0, s, a, n, t, j);
    else hipLaunchKernelGGL(k_nuts_doubling_end<float>, nuts_grid(a.C), dim3(256), 0, s, a, n, t, j);
    return hipGetLastError();
}

hipError_t launch_nuts_end(const PlainArgs& a, const NutsWs& n, const NutsAdapt& ad, int64_t it, void* samples,
                           int64_t r, int32_t* tr_depth, int32_t* tr_nleap, double* tr_stat, hipStream_t s) {
    if (a.f64)
        hipLaunchKernelGGL(k_nuts_end<double>, nuts_grid(a.C), dim3(256), 0, s, a, n, ad, it, (double*)samples, r,
                           tr_depth, tr_nleap, tr_stat);
    else
        hipLaunchKernelGGL(k_nuts_end<float>, nuts_grid(a.C), dim3(256), 0, s, a, n, ad, it, (float*)samples, r,
                           tr_depth, tr_nleap, tr_stat);
    return hipGetLastError();
}

}  // namespace hmc
