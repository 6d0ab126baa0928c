// k_fused_logreg.hip -- fused persistent kernel for Bayesian logistic
// regression with a small event dimension (D <= 32) and a data set that fits
// on chip (N <= 512 * TPW rows).
//
// One workgroup (8 waves) owns 4 chains and runs whole transitions.  The two
// contractions of every gradient evaluation,
//     S = X theta            (rows x chains, K = dims)
//     G = X^T (y - sigmoid(S))  (chains x dims, K = rows)
// run on v_mfma_f32_4x4x1f32 (16 independent 4x4 blocks per instruction):
// with only 4 chains per workgroup the 4-wide chain dimension is fully used,
// so C = 1024 chains occupy all 256 CUs.
//
// Lane layouts (wave64, lane = 4 b + j, b = 0..15 block, j = 0..3):
//   first contraction, one instruction per dim d:
//     A[b][i] = X[row0 + 4b + i][d]   (lane l holds its own row l)
//     B[b][j] = theta[chain j][d]     (one lane group broadcast to all by BLGP)
//     D[b][i][j] -> VGPR i of lane 4b + j = S[row0 + 4b + i][chain j]
//   second contraction, one instruction per (row offset v, dim group q):
//     A[b][i] = R[row0 + 4b + v][chain i]   = VGPR v of the S result (no shuffles)
//     B[b][j] = X[row0 + 4b + v][4q + j]
//     D[b][i][j] accumulates G[chain i][4q + j] over the rows of block b
// The 16 block partials of G are summed inside the wave: a reduce-scatter over
// the four 16-lane rows (v_permlane32_swap, v_permlane16_swap) leaves chain i's
// values in row i, and two DPP rotates finish each row.  The 8 wave partials are
// summed in LDS in a fixed order, so results are bitwise reproducible.
//
// Each wave keeps the X rows of its tiles in VGPRs, in both operand layouts,
// for the whole kernel.  Threads 0..127 own (chain i = t / 32, dim d = t % 32)
// of the chain state: theta, momentum, gradient and the accepted state; they
// sum the wave partials, kick, drift and take the accept decision.  The other
// waves draw momenta for the next 32 transitions, and accept uniforms and
// dual-averaging factors for the next 128, into LDS whenever a block of them
// runs out; they would otherwise wait for the owners at the transition boundary.
#include "exp_f64.hpp"
#include "hmc_internal.hpp"

namespace hmc {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int LR_NW = 8;          // waves per workgroup
constexpr int LR_PS = 36;         // row stride (floats) of the per-wave gradient partials
constexpr int LR_ZT = 32;         // transitions of momenta drawn at a time
constexpr int LR_UT = 128;        // transitions of accept uniforms / DA factors drawn at a time

__device__ __forceinline__ float dpp_ror(float v, int n) {
    // rotate right within a row of 16 lanes
    int r;
    if (n == 4)
        r = __builtin_amdgcn_mov_dpp(__float_as_int(v), 0x124, 0xf, 0xf, true);
    else
        r = __builtin_amdgcn_mov_dpp(__float_as_int(v), 0x128, 0xf, 0xf, true);
    return __int_as_float(r);
}

// 4x4x1 MFMA whose B operand is lane group g (lanes 16g..16g+15) broadcast to
// all four groups (BLGP = 4 + g); g is a constant after unrolling.
__device__ __forceinline__ floatx4 mfma4_bgroup(int g, float a, float b, floatx4 c) {
    switch (g) {
    case 0: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 4);
    case 1: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 5);
    case 2: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 6);
    default: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 7);
    }
}

// Row k (lanes 16k..16k+15) of the result holds, per lane position, the sum
// of input k over the four rows.  permlane32_swap(x, y) gives
// ([x.lo, y.lo], [x.hi, y.hi]) and permlane16_swap(x, y) gives rows
// ([x0, y0, x2, y2], [x1, y1, x3, y3]).
__device__ __forceinline__ float rows4_scatter(float a0, float a1, float a2, float a3) {
    const auto s02 = __builtin_amdgcn_permlane32_swap(__float_as_uint(a0), __float_as_uint(a2), false, false);
    const auto s13 = __builtin_amdgcn_permlane32_swap(__float_as_uint(a1), __float_as_uint(a3), false, false);
    const float c02 = __uint_as_float(s02[0]) + __uint_as_float(s02[1]);
    const float c13 = __uint_as_float(s13[0]) + __uint_as_float(s13[1]);
    const auto t = __builtin_amdgcn_permlane16_swap(__float_as_uint(c02), __float_as_uint(c13), false, false);
    return __uint_as_float(t[0]) + __uint_as_float(t[1]);
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xf, 0xf, true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Sum of rows 2k and 2k+1 (k = 0, 1), in both rows.
__device__ __forceinline__ double rows2_sum(double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)u, (uint32_t)u, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(u >> 32), (uint32_t)(u >> 32), false, false);
    const double a = __longlong_as_double((long long)(((uint64_t)hi[0] << 32) | lo[0]));
    const double b = __longlong_as_double((long long)(((uint64_t)hi[1] << 32) | lo[1]));
    return a + b;
}

// Sum over the 32 lanes of each half wave, as a butterfly: every step adds a
// lane's value and its partner's, so all 32 lanes end with the same bits.
__device__ __forceinline__ double half_wave_sum(double v) {
    v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]: partner lane ^ 1
    v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]: partner lane ^ 2
    v += dpp_f64<0x141>(v);   // row_half_mirror: the two quads of each 8 lanes
    v += dpp_f64<0x140>(v);   // row_mirror: the two halves of each row
    return rows2_sum(v);
}

// Sum over the 16 lanes of equal lane % 4; lanes 0..3 hold the result.
__device__ __forceinline__ double same_j_sum(double v) {
    v += dpp_f64<0x124>(v);   // row_ror 4
    v += dpp_f64<0x128>(v);   // row_ror 8
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)u, (uint32_t)u, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(u >> 32), (uint32_t)(u >> 32), false, false);
    v = __longlong_as_double((long long)(((uint64_t)hi[0] << 32) | lo[0])) +
        __longlong_as_double((long long)(((uint64_t)hi[1] << 32) | lo[1]));
    return rows2_sum(v);
}

// The logistic link of one row from e = e^-|s| (hardware exp2, about 1 ulp):
// sigmoid(s) = 1 / (1 + e) for s >= 0 and e / (1 + e) below, and
// log1p(e), from which softplus(+-s) = max(+-s, 0) + log1p(e).  log1p(e) for
// e in (0, 1] is the hardware log2 of 1 + e when e >= 2^-10, else the series
// e - e^2/2 + e^3/3 (error < e^4/4).
struct Link {
    float e, rc;     // e^-|s|, 1 / (1 + e^-|s|)
};
__device__ __forceinline__ Link link_of(float s) {
    const float e = __builtin_amdgcn_exp2f(-1.4426950408889634f * fabsf(s));
    return Link{e, __builtin_amdgcn_rcpf(1.0f + e)};
}
__device__ __forceinline__ float sigmoid_of(float s, Link k) { return s >= 0.f ? k.rc : k.e * k.rc; }
__device__ __forceinline__ float log1p_of(Link k) {
    const float big = 0.69314718055994531f * __builtin_amdgcn_logf(1.0f + k.e);
    const float small = k.e * (1.0f - k.e * (0.5f - k.e * 0.33333333f));
    return k.e >= 0x1p-10f ? big : small;
}

struct ChainSt {       // per-chain scalars of the owners, kept in LDS
    double logp, eps;
    DualAvg da;
};

// Output pointers, kept in LDS: read where a transition ends instead of
// occupying registers through the leapfrog steps.  They are global-memory
// pointers, so stores through them are global stores, not flat ones.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
struct OutPtrs {
    gptr<float> samples;
    gptr<double> tr_step;
    gptr<uint8_t> tr_acc;
    gptr<double> tr_lar;
    gptr<double> tr_tlp;
    gptr<float> ps;
    gptr<float> pm;
    gptr<uint8_t> acc;
    gptr<double> lar;
    gptr<double> tlp;
    gptr<double> dh;
};

// TP: the chains carry inverse temperatures and / or the context a transform
// (a template parameter, so that plain runs compile without either).  The
// transformed kernel (x = shift + scale z) runs in z: X scaled by column
// where it is loaded into VGPRs (X S), the prior's precision inv_var scale^2
// per dim, states divided by scale at load and multiplied back where x is
// stored.
template <int TPW, int QQ, typename XT, bool TP>
__global__ __launch_bounds__(512) void k_fused_logreg4(PlainArgs a, FusedRun r) {
    extern __shared__ float lds[];
    constexpr int NW = LR_NW, PS = LR_PS, ZT = LR_ZT, UT = LR_UT;
    const int64_t D = a.tg.D, N = a.tg.N, C = a.C, T = r.n_transitions;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int q4 = lane & 3, b16 = lane >> 2;
    const int64_t c0 = (int64_t)blockIdx.x * 4;
    // chain of slot s (0..3): s itself, or with the exchange inside the launch
    // replica s % K of chain index 4 / K * block + s / K (chain k M + m), so
    // that all replicas of a chain index share the workgroup
    const int nrep = TP ? r.remc_K : 0;
    auto chain_of = [&](int sl) -> int64_t {
        return nrep > 1 ? (int64_t)(sl % nrep) * r.remc_M + (int64_t)blockIdx.x * (4 / nrep) + sl / nrep : c0 + sl;
    };
    auto slot_valid = [&](int sl) -> bool {
        return nrep > 1 ? (int64_t)blockIdx.x * (4 / nrep) + sl / nrep < r.remc_M : c0 + sl < C;
    };
    const float inv_var = (float)a.tg.inv_var;

    float* th = lds;                                    // [4][32] theta of the 4 chains (dim order)
    float* part = th + 128;                             // [NW][4][PS] wave partials of G
    float* zb = part + NW * 4 * PS;                     // [ZT][4][32] momenta
    double* lpp = (double*)(zb + ZT * 128);             // [NW][4] wave partials of the data log-likelihood
    double* lub = lpp + NW * 4;                         // [2][UT][4] log accept uniforms, two blocks
    double* dac = lub + 2 * UT * 4;                     // [2][UT][4] dual-averaging factors (w, k, eta)
    ChainSt* cst = (ChainSt*)(dac + 2 * UT * 4);        // [4]
    OutPtrs* optr = (OutPtrs*)(cst + 4);
    double* ecf = (double*)(optr + 1);                  // [EXP_NC] 1 / n!
    float* xgr = (float*)(ecf + EXP_NC);                // [4][32] gradients posted for the exchange

    // ---- X and y of this wave's tiles, in the two operand layouts, kept in VGPRs ----
    const XT* X = (const XT*)a.tg.X;
    const double* sc = TP ? a.ws.scale : nullptr;
    auto ldx = [&](int64_t row, int64_t d) -> float {
        if (row >= N || d >= D) return 0.f;
        float v;
        if constexpr (sizeof(XT) == 2) v = bf16_to_f32(((const uint16_t*)X)[row * D + d]);
        else v = ((const float*)X)[row * D + d];
        return sc ? (float)((double)v * sc[d]) : v;
    };
    float xa[TPW][4 * QQ];     // first contraction: X[row0 + lane][d]
    float xb[TPW][4][QQ];      // second contraction: X[row0 + 4 b16 + v][4 q + q4]
    uint32_t ybits = 0, rbits = 0;   // bit 4 tt + v: label of row 4 b16 + v of tile tt is 1 / row exists
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
        const int64_t row0 = (int64_t)(w + NW * tt) * 64;
#pragma unroll
        for (int d = 0; d < 4 * QQ; ++d) xa[tt][d] = ldx(row0 + lane, d);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t row = row0 + 4 * b16 + v;
            if (row < N) {
                rbits |= 1u << (4 * tt + v);
                if (a.tg.y[row]) ybits |= 1u << (4 * tt + v);
            }
#pragma unroll
            for (int q = 0; q < QQ; ++q) xb[tt][v][q] = ldx(row, 4 * q + q4);
        }
    }

    // ---- draws, by waves 2..7 ----
    auto draw_momenta = [&](int64_t i0) {               // transitions i0 .. i0 + ZT - 1
        const int nb = (int)((D + 3) / 4);
        for (int task = (int)threadIdx.x - 128; task < ZT * 32; task += 384) {
            const int k = task >> 5, ci = (task >> 3) & 3, blk = task & 7;
            float z[4] = {0.f, 0.f, 0.f, 0.f};
            if (i0 + k < T && slot_valid(ci) && blk < nb)
                momentum4<float>(a.key, (uint32_t)chain_of(ci), (uint32_t)(r.t_begin + i0 + k), (uint32_t)blk, z);
            *(float4*)&zb[(k * 4 + ci) * 32 + 4 * blk] = make_float4(z[0], z[1], z[2], z[3]);
        }
    };
    auto draw_accept = [&](int64_t i0) {                // transitions i0 .. i0 + UT - 1, block (i0 / UT) % 2
        const int hb = (int)((i0 / UT) & 1);
        for (int task = (int)threadIdx.x - 128; task < UT * 4; task += 384) {
            const int k = task >> 2, ci = task & 3;
            double lu = 0.0;
            if (i0 + k < T && slot_valid(ci))
                lu = log_accept_uniform(a.key, (uint32_t)chain_of(ci), (uint32_t)(r.t_begin + i0 + k));
            lub[(hb * UT + k) * 4 + ci] = lu;
        }
        if (r.adapt)
            for (int k = (int)threadIdx.x - 128; k < UT; k += 384)
                if (i0 + k < T) {
                    const DaConst f = dual_avg_const((double)(r.m_offset + i0 + k + 1), r.gamma, r.t0, r.kappa);
                    double* o = dac + (hb * UT + k) * 4;
                    o[0] = f.w;
                    o[1] = f.k;
                    o[2] = f.eta;
                }
    };
    if (threadIdx.x >= 128 && T > 0) {
        draw_momenta(0);
        draw_accept(0);
    }

    // ---- owners: thread t < 128 holds (chain oi, dim od) ----
    const bool owner = threadIdx.x < 128;
    const int oi = (threadIdx.x >> 5) & 3, od = threadIdx.x & 31;
    const int64_t oc = chain_of(oi);
    const bool cval = slot_valid(oi);
    const bool ovalid = owner && cval && od < D;
    const int64_t occ = (owner && cval) ? oc : 0;
    float* Xw = (float*)a.ws.x;
    float* Gw = (float*)a.ws.g;
    float th0 = ovalid ? Xw[occ * D + od] : 0.f;
    float g0 = ovalid ? Gw[occ * D + od] : 0.f;
    // transform: this owner's scale and prior precision in z
    const double sod = (sc && ovalid) ? sc[od] : 1.0;
    const float pv_z = sc ? (float)((double)inv_var * sod * sod) : inv_var;
    if (sc && ovalid) {
        th0 = (float)((double)th0 / sod);
        g0 = (float)((double)g0 * sod);
    }
    // step size of the owner's chain in FP32; half steps are eps / 2 (halving
    // commutes with rounding to float)
    float eps = owner ? (float)a.ws.eps[occ] : 0.f;
    // inverse temperature of the owner's chain (replica exchange): it scales
    // every kick (keps = beta eps) and both energies
    const double btd = (TP && owner && a.ws.beta) ? a.ws.beta[occ] : 1.0;
    float keps = TP ? (owner ? (float)(a.ws.eps[occ] * btd) : 0.f) : 0.f;
    auto kick_eps = [&]() -> float { return TP ? keps : eps; };
    if (owner && od == 0 && cval) cst[oi] = ChainSt{a.ws.logp[oc], a.ws.eps[oc], a.ws.da[oc]};
    if (threadIdx.x == 0)
        *optr = OutPtrs{(gptr<float>)r.samples,          (gptr<double>)r.trace.step_size,
                        (gptr<uint8_t>)r.trace.is_accepted, (gptr<double>)r.trace.log_accept_ratio,
                        (gptr<double>)r.trace.target_log_prob, (gptr<float>)r.out.proposed_state,
                        (gptr<float>)r.out.proposed_momentum, (gptr<uint8_t>)r.out.is_accepted,
                        (gptr<double>)r.out.log_accept_ratio, (gptr<double>)r.out.target_log_prob,
                        (gptr<double>)r.out.delta_h};
    if (threadIdx.x < EXP_NC) ecf[threadIdx.x] = exp_coef((int)threadIdx.x);
    float p = 0.f, thq = th0, gq = 0.f;
    __syncthreads();

    auto step = [&](auto last_c) {
        constexpr bool LAST = decltype(last_c)::value;
        if (owner) {
            thq = fmaf(eps, p, thq);
            th[oi * 32 + od] = ovalid ? thq : 0.f;
        }
        __syncthreads();
        // B operands of the first contraction: lane 16 g + 4 b + j of tb[k] holds
        // theta[chain j][4 k + g]; the MFMA for dim 4 k + g broadcasts lane group g
        // to all four groups (BLGP = 4 + g)
        float tb[QQ];
#pragma unroll
        for (int k = 0; k < QQ; ++k) tb[k] = th[q4 * 32 + 4 * k + (lane >> 4)];
        // S = X theta (two accumulation chains per tile); tile tt + 1's S, tile tt's
        // residuals and tile tt's G contribution form one scheduling region, so MFMA
        // and VALU work of neighbouring tiles interleave
        const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
        floatx4 sa[TPW][2];
        float sv[TPW][4], rr[TPW][4];
        floatx4 gacc[QQ];
        float ll[TPW][4];        // log-likelihood terms of the rows (last step)
#pragma unroll
        for (int d = 0; d < 4 * QQ; d += 4)
#pragma unroll
            for (int u = 0; u < 4; ++u)
                sa[0][u & 1] = mfma4_bgroup(u, xa[0][d + u], tb[d / 4], (d == 0 && u < 2) ? zero : sa[0][u & 1]);
#pragma unroll
        for (int tt = 0; tt < TPW; ++tt) {
            __builtin_amdgcn_sched_barrier(0);
            if (tt + 1 < TPW) {
#pragma unroll
                for (int d = 0; d < 4 * QQ; d += 4)
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        sa[tt + 1][u & 1] = mfma4_bgroup(u, xa[tt + 1][d + u], tb[d / 4],
                                                         (d == 0 && u < 2) ? zero : sa[tt + 1][u & 1]);
            }
            // residuals y - sigmoid(S); padded rows have X = 0 and add nothing to G
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int bit = 4 * tt + v;
                sv[tt][v] = sa[tt][0][v] + sa[tt][1][v];
                const bool yb = (ybits >> bit) & 1u;
                const Link k = link_of(sv[tt][v]);
                rr[tt][v] = (yb ? 1.f : 0.f) - sigmoid_of(sv[tt][v], k);
                if constexpr (LAST) {
                    // y log sigmoid(s) + (1 - y) log(1 - sigmoid(s)) = -softplus(y ? -s : s)
                    const float sp = fmaxf(yb ? -sv[tt][v] : sv[tt][v], 0.f) + log1p_of(k);
                    ll[tt][v] = ((rbits >> bit) & 1u) ? -sp : 0.f;
                }
            }
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int q = 0; q < QQ; ++q)
                    gacc[q] = __builtin_amdgcn_mfma_f32_4x4x1f32(rr[tt][v], xb[tt][v][q],
                                                                 (tt == 0 && v == 0) ? zero : gacc[q], 0, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
        // block sums: chain i to row i, then the 4 blocks of each row (dims 4q + lane % 4)
        float gsum[QQ];
#pragma unroll
        for (int q = 0; q < QQ; ++q) {
            float v = rows4_scatter(gacc[q][0], gacc[q][1], gacc[q][2], gacc[q][3]);
            v += dpp_ror(v, 4);
            v += dpp_ror(v, 8);
            gsum[q] = v;
        }
        if ((lane & 15) < 4) {
            float* dst = part + (w * 4 + (lane >> 4)) * PS + q4;
#pragma unroll
            for (int q = 0; q < QQ; ++q) dst[4 * q] = gsum[q];
        }
        if constexpr (LAST) {
            // FP64 pairwise sum of the lane's rows, then over the 16 lanes of each chain
            double t[TPW * 4];
#pragma unroll
            for (int k = 0; k < TPW * 4; ++k) t[k] = (double)ll[k / 4][k % 4];
#pragma unroll
            for (int hh = TPW * 2; hh >= 1; hh >>= 1)
#pragma unroll
                for (int k = 0; k < hh; ++k) t[k] = t[2 * k] + t[2 * k + 1];
            const double lp = same_j_sum(t[0]);
            if (lane < 4) lpp[w * 4 + lane] = lp;
        }
        __syncthreads();
        if (owner) {
            float gs = 0.f;
            if (od < 4 * QQ) {
                // fixed-order pairwise sum over the wave partials
                float v[NW];
#pragma unroll
                for (int ww = 0; ww < NW; ++ww) v[ww] = part[(ww * 4 + oi) * PS + od];
#pragma unroll
                for (int hh = NW / 2; hh >= 1; hh >>= 1)
#pragma unroll
                    for (int k = 0; k < hh; ++k) v[k] = v[2 * k] + v[2 * k + 1];
                gs = v[0];
            }
            gq = gs - thq * (TP ? pv_z : inv_var);
            p = fmaf(LAST ? 0.5f * kick_eps() : kick_eps(), gq, p);
        }
    };

    for (int64_t itr = 0; itr < T; ++itr) {
        double dk = 0.0;
        if (owner) {
            const float z = ovalid ? zb[((int)(itr % ZT) * 4 + oi) * 32 + od] : 0.f;
            dk = -0.5 * (double)z * (double)z;
            thq = th0;
            p = fmaf(0.5f * kick_eps(), g0, z);
        }
        for (int l = 0; l + 1 < a.L; ++l) step(std::false_type{});
        step(std::true_type{});

        const bool refill_z = itr + 1 < T && (itr + 1) % ZT == 0;
        if (owner) {
            // energy change and decision (the 32 lanes of a chain agree bitwise)
            const int hb = (int)((itr / UT) & 1), ku = (int)(itr % UT);
            ChainSt cs = cst[oi];
            double prior = ovalid ? -0.5 * (double)thq * (double)thq * a.tg.inv_var * (TP ? sod * sod : 1.0) : 0.0;
            dk += ovalid ? 0.5 * (double)p * (double)p : 0.0;
            dk = half_wave_sum(dk);
            prior = half_wave_sum(prior);
            double lpdata = 0.0;
#pragma unroll
            for (int ww = 0; ww < NW; ++ww) lpdata += lpp[ww * 4 + oi];
            const double lp1 = lpdata + prior;
            const double dh = TP ? -(btd * lp1) + btd * cs.logp + dk : -lp1 + cs.logp + dk;
            const double lar = log_accept_ratio_of(dh);
            const bool acc = lub[(hb * UT + ku) * 4 + oi] < lar;
            if (acc) {
                th0 = thq;
                g0 = gq;
                cs.logp = lp1;
            }
            if (cval) {
                const OutPtrs o = *optr;
                if (ovalid) {
                    if (o.samples && itr >= r.n_burnin && !(TP && nrep > 1))
                        o.samples[((itr - r.n_burnin) * C + oc) * D + od] = TP && sc ? (float)((double)th0 * sod) : th0;
                    if (o.ps) o.ps[oc * D + od] = TP && sc ? (float)((double)thq * sod) : thq;
                    if (o.pm) o.pm[oc * D + od] = p;
                }
                const double eps_used = cs.eps;
                if (r.adapt && itr < r.n_burnin) {
                    const double alpha = lar < 0.0 ? exp_lds(lar, ecf) : 1.0;
                    if (r.adapt_kind == HMC_ADAPT_SIMPLE) {
                        cs.eps = simple_adapt(cs.eps, alpha, r.target_accept, r.rate);
                    } else {
                        const int64_t m = r.m_offset + itr + 1;
                        const double* f = dac + (hb * UT + ku) * 4;
                        const double log_eps =
                            dual_avg_apply(cs.da, DaConst{f[0], f[1], f[2]}, alpha, r.target_accept);
                        cs.eps = exp_lds((m < r.adapt_total) ? log_eps : cs.da.log_eps_bar, ecf);
                    }
                }
                eps = (float)cs.eps;
                if (TP) keps = (float)(cs.eps * btd);
                if (od == 0) {
                    if (itr >= r.n_burnin) {
                        const int64_t k = (itr - r.n_burnin) * C + oc;
                        if (o.tr_step) o.tr_step[k] = eps_used;
                        if (o.tr_acc) o.tr_acc[k] = acc ? 1 : 0;
                        if (o.tr_lar) o.tr_lar[k] = lar;
                        if (o.tr_tlp) o.tr_tlp[k] = cs.logp;
                    }
                    if (o.acc) o.acc[oc] = acc ? 1 : 0;
                    if (o.lar) o.lar[oc] = lar;
                    if (o.tlp) o.tlp[oc] = cs.logp;
                    if (o.dh) o.dh[oc] = dh;
                    cst[oi] = cs;
                }
            }
        } else if (itr + 1 < T) {
            if (refill_z) draw_momenta(itr + 1);
            if ((itr + 1) % UT == 0) draw_accept(itr + 1);
        }
        // the owners read the next momenta before the next barrier of a step
        if (refill_z) __syncthreads();
        if (TP && nrep > 1) {
            // the exchange: the owners post their chains' states in the theta buffer
            // (no wave reads it between the last barrier of a trajectory and the
            // first drift of the next) and their gradients in a buffer of their own;
            // after a barrier every owner reads its partner's state and both
            // log-probabilities, and the swap is applied after another barrier
            float* xth = th;                    // [4][32]
            if (owner) {
                xth[oi * 32 + od] = th0;
                xgr[oi * 32 + od] = g0;
            }
            __syncthreads();
            bool swp = false;
            float th_n = th0, g_n = g0;
            double lp_n = 0.0;
            const uint32_t tt = (uint32_t)(r.t_begin + itr);
            if (owner && cval) {
                const int krep = oi % nrep, par = (int)(tt & 1u);
                const bool a_side = krep >= par && ((krep - par) & 1) == 0 && krep + 1 < nrep;
                const bool b_side = krep >= par + 1 && ((krep - 1 - par) & 1) == 0;
                if (a_side || b_side) {
                    const int po = a_side ? oi + 1 : oi - 1;        // the partner's slot (same chain index)
                    const int64_t pc = chain_of(po);
                    const double lo = cst[oi].logp, lq = cst[po].logp;
                    const double bq = a.ws.beta ? a.ws.beta[pc] : 1.0;
                    const int64_t ca = a_side ? oc : pc;
                    const double la = a_side ? lo : lq, lb = a_side ? lq : lo;
                    const double ba = a_side ? btd : bq, bb = a_side ? bq : btd;
                    swp = log_uniform52(a.key, (uint32_t)ca, tt, TAG_SWAP) < (ba - bb) * (lb - la);
                    if (swp) {
                        th_n = xth[po * 32 + od];
                        g_n = xgr[po * 32 + od];
                        lp_n = lq;
                    }
                }
            }
            __syncthreads();
            if (owner && cval) {
                if (swp) {
                    th0 = th_n;
                    g0 = g_n;
                    if (od == 0) cst[oi].logp = lp_n;
                }
                const OutPtrs o = *optr;
                if (itr >= r.n_burnin) {
                    if (od == 0 && r.swapped) r.swapped[(itr - r.n_burnin) * C + oc] = swp ? 1 : 0;
                    if (o.samples && od < D)
                        o.samples[((itr - r.n_burnin) * C + oc) * D + od] = sc ? (float)((double)th0 * sod) : th0;
                }
            }
        }
    }
    if (ovalid) {
        Xw[oc * D + od] = TP && sc ? (float)((double)th0 * sod) : th0;
        Gw[oc * D + od] = TP && sc ? (float)((double)g0 / sod) : g0;
    }
    if (owner && od == 0 && cval) {
        const ChainSt cs = cst[oi];
        a.ws.logp[oc] = cs.logp;
        a.ws.eps[oc] = cs.eps;
        a.ws.da[oc] = cs.da;
    }
}

static size_t logreg4_lds(int) {
    return (size_t)(128 + LR_NW * 4 * LR_PS + LR_ZT * 128) * sizeof(float) +
           (size_t)(LR_NW * 4 + 4 * LR_UT * 4 + EXP_NC) * sizeof(double) + 4 * sizeof(ChainSt) + sizeof(OutPtrs) +
           128 * sizeof(float);
}

bool fused_logreg_supported(const PlainArgs& a) {
    return !a.bf16_grad && a.tg.D <= 32 && a.tg.N <= (int64_t)LR_NW * 2 * 64;
}

template <int TPW, int QQ, typename XT>
static hipError_t launch_lr4(const PlainArgs& a, const FusedRun& r, hipStream_t s) {
    const size_t lds = logreg4_lds(TPW);
    if (r.remc_K > 1 && (4 % r.remc_K != 0 || r.remc_K * r.remc_M != a.C)) return hipErrorInvalidValue;
    const int64_t per = r.remc_K > 1 ? 4 / r.remc_K : 4;      // chain indices (or chains) per workgroup
    const int64_t units = r.remc_K > 1 ? r.remc_M : a.C;
    const dim3 grid((unsigned)((units + per - 1) / per));
    if (a.ws.beta || a.ws.scale || r.remc_K > 1)
        hipLaunchKernelGGL((k_fused_logreg4<TPW, QQ, XT, true>), grid, dim3(64 * LR_NW), lds, s, a, r);
    else
        hipLaunchKernelGGL((k_fused_logreg4<TPW, QQ, XT, false>), grid, dim3(64 * LR_NW), lds, s, a, r);
    return hipGetLastError();
}

template <int TPW, typename XT>
static hipError_t launch_lr4_q(const PlainArgs& a, const FusedRun& r, hipStream_t s) {
    switch ((a.tg.D + 3) / 4) {
    case 1: return launch_lr4<TPW, 1, XT>(a, r, s);
    case 2: return launch_lr4<TPW, 2, XT>(a, r, s);
    case 3: return launch_lr4<TPW, 3, XT>(a, r, s);
    case 4: return launch_lr4<TPW, 4, XT>(a, r, s);
    case 5: return launch_lr4<TPW, 5, XT>(a, r, s);
    case 6: return launch_lr4<TPW, 6, XT>(a, r, s);
    case 7: return launch_lr4<TPW, 7, XT>(a, r, s);
    default: return launch_lr4<TPW, 8, XT>(a, r, s);
    }
}

hipError_t launch_fused_logreg(const PlainArgs& a, const FusedRun& r, hipStream_t s) {
    if (!fused_logreg_supported(a)) return hipErrorNotSupported;
    const bool one = a.tg.N <= LR_NW * 64;
    if (a.tg.x_bf16) return one ? launch_lr4_q<1, uint16_t>(a, r, s) : launch_lr4_q<2, uint16_t>(a, r, s);
    return one ? launch_lr4_q<1, float>(a, r, s) : launch_lr4_q<2, float>(a, r, s);
}

}  // namespace hmc
