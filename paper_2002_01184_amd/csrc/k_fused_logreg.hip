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
//     B[b][j] = theta[chain j][d]
//     D[b][i][j] -> VGPR i of lane 4b + j = S[row0 + 4b + i][chain j]
//   second contraction, one instruction per (row offset v, dim group q):
//     A[b][i] = R[row0 + 4b + v][chain i]   = VGPR v of the S result (no shuffles)
//     B[b][j] = X[row0 + 4b + v][4q + j]
//     D[b][i][j] accumulates G[chain i][4q + j] over the rows of block b
// Block partials are summed across a 16-lane row with DPP rotates, across
// rows and waves in LDS in a fixed order (bitwise-reproducible).
//
// X lives in LDS with permuted columns (stored column (d % 4) * 8 + d / 4) so
// that the 8 dims 4q + j a lane needs for the second contraction are two
// 16-byte reads; each wave keeps the first-contraction rows of its tiles in
// VGPRs for the whole kernel.  Threads 0..127 own (chain i = t / 32,
// dim d = t % 32) of the chain state: theta, momentum, gradient, the accepted
// state, and do the momentum draw, kicks, drifts and the accept test.
#include "hmc_internal.hpp"

namespace hmc {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int LR_NW = 8;          // waves per workgroup
constexpr int LR_PART = 512;      // floats per wave in the gradient partial buffer: 4 rows x 8 q x 16

__device__ __forceinline__ float dpp_ror(float v, int n) {
    // rotate right within a row of 16 lanes
    int r;
    if (n == 4)
        r = __builtin_amdgcn_mov_dpp(__float_as_int(v), 0x124, 0xf, 0xf, true);
    else
        r = __builtin_amdgcn_mov_dpp(__float_as_int(v), 0x128, 0xf, 0xf, true);
    return __int_as_float(r);
}

// 1 / (1 + e^-s) with the hardware exp2 and reciprocal (about 1 ulp each);
// e^-s overflowing to +inf gives the correct limit 0.
__device__ __forceinline__ float sigmoid_fast(float s) {
    const float e = __builtin_amdgcn_exp2f(-1.4426950408889634f * s);
    return __builtin_amdgcn_rcpf(1.0f + e);
}

// log(1 + e^s) = max(s, 0) + log1p(e^-|s|); log1p(e) for e in (0, 1] from the
// hardware log2 when e >= 2^-10, else its series e - e^2/2 + e^3/3 (error < e^4/4).
__device__ __forceinline__ float softplus_f(float s) {
    const float e = __builtin_amdgcn_exp2f(-1.4426950408889634f * fabsf(s));
    const float l = e >= 0x1p-10f ? 0.69314718055994531f * __builtin_amdgcn_logf(1.0f + e)
                                  : e * (1.0f - e * (0.5f - e * 0.33333333f));
    return fmaxf(s, 0.f) + l;
}

// stored column of dim d and its inverse
__device__ __forceinline__ int lr_col(int d) { return (d & 3) * 8 + (d >> 2); }
__device__ __forceinline__ int lr_dim(int k) { return (k & 7) * 4 + (k >> 3); }

struct ChainCtlL {
    double logp, eps;
    DualAvg da;
};

template <int TPW, int QQ, typename XT>
__global__ __launch_bounds__(512) void k_fused_logreg4(PlainArgs a, FusedRun r) {
    extern __shared__ float lds[];
    constexpr int NW = LR_NW;
    const int64_t D = a.tg.D, N = a.tg.N, C = a.C;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int q4 = lane & 3, b16 = lane >> 2;
    const int64_t c0 = (int64_t)blockIdx.x * 4;
    const float inv_var = (float)a.tg.inv_var;

    float* th = lds;                         // [4][32] theta of the 4 chains (dim order)
    float* part = th + 128;                  // [NW][4 rows][4 j][32]: row partials, (q, i) inner
    double* lpp = (double*)(part + NW * LR_PART);   // [NW][4]

    // ---- X and y of this wave's tiles, in the two operand layouts, kept in VGPRs ----
    const XT* X = (const XT*)a.tg.X;
    auto ldx = [&](int64_t row, int64_t d) -> float {
        if (row >= N || d >= D) return 0.f;
        if constexpr (sizeof(XT) == 2) return bf16_to_f32(((const uint16_t*)X)[row * D + d]);
        else return ((const float*)X)[row * D + d];
    };
    float xa[TPW][4 * QQ];     // first contraction: X[row0 + lane][d]
    float xb[TPW][4][QQ];      // second contraction: X[row0 + 4 b16 + v][4 q + q4]
    float yv[TPW][4];
    bool rv[TPW][4];
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
        const int64_t row0 = (int64_t)(w + NW * tt) * 64;
#pragma unroll
        for (int d = 0; d < 4 * QQ; ++d) xa[tt][d] = ldx(row0 + lane, d);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t row = row0 + 4 * b16 + v;
            rv[tt][v] = row < N;
            yv[tt][v] = row < N ? (float)a.tg.y[row] : 0.f;
#pragma unroll
            for (int q = 0; q < QQ; ++q) xb[tt][v][q] = ldx(row, 4 * q + q4);
        }
    }

    // ---- owners: thread t < 128 holds (chain oi, dim od) ----
    const bool owner = threadIdx.x < 128;
    const int oi = (threadIdx.x >> 5) & 3, od = threadIdx.x & 31;
    const int64_t oc = c0 + oi;
    const bool ovalid = owner && oc < C && od < D;
    const int64_t occ = (owner && oc < C) ? oc : 0;
    float* Xw = (float*)a.ws.x;
    float* Gw = (float*)a.ws.g;
    float th0 = ovalid ? Xw[occ * D + od] : 0.f;
    float g0 = ovalid ? Gw[occ * D + od] : 0.f;
    ChainCtlL s;
    s.logp = a.ws.logp[occ];
    s.eps = a.ws.eps[occ];
    s.da = a.ws.da[occ];

    for (int64_t itr = 0; itr < r.n_transitions; ++itr) {
        const uint32_t t = (uint32_t)(r.t_begin + itr);
        const float eps = (float)s.eps, half = (float)(0.5 * s.eps);
        float p = 0.f, thq = th0, gq = 0.f;
        double dk = 0.0, lpdata = 0.0;
        if (owner) {
            float z[4];
            momentum4<float>(a.key, (uint32_t)occ, t, (uint32_t)(od >> 2), z);
            const int jj = od & 3;
            const float zj = jj == 0 ? z[0] : (jj == 1 ? z[1] : (jj == 2 ? z[2] : z[3]));
            const float p0 = ovalid ? zj : 0.f;
            dk = -0.5 * (double)p0 * (double)p0;
            p = fmaf(half, g0, p0);
        }
        for (int l = 0; l < a.L; ++l) {
            const bool last = l == a.L - 1;
            if (owner) {
                thq = fmaf(eps, p, thq);
                th[oi * 32 + od] = ovalid ? thq : 0.f;
            }
            __syncthreads();
            float tb[4 * QQ];
#pragma unroll
            for (int k = 0; k < 4 * QQ; k += 4) {
                const float4 v = *(const float4*)&th[q4 * 32 + k];
                tb[k] = v.x;
                tb[k + 1] = v.y;
                tb[k + 2] = v.z;
                tb[k + 3] = v.w;
            }
            floatx4 gacc[QQ];
#pragma unroll
            for (int q = 0; q < QQ; ++q) gacc[q] = floatx4{0.f, 0.f, 0.f, 0.f};
            double lp = 0.0;
            // S = X theta for all tiles, four independent accumulation chains per tile
            floatx4 sa[TPW][4];
#pragma unroll
            for (int tt = 0; tt < TPW; ++tt)
#pragma unroll
                for (int u = 0; u < 4; ++u) sa[tt][u] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int d = 0; d < 4 * QQ; d += 4)
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int tt = 0; tt < TPW; ++tt)
                        sa[tt][u] = __builtin_amdgcn_mfma_f32_4x4x1f32(xa[tt][d + u], tb[d + u], sa[tt][u], 0, 0, 0);
#pragma unroll
            for (int tt = 0; tt < TPW; ++tt) {
                if ((w + NW * tt) * 64 >= N) break;
                float rr[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float sv = (sa[tt][0][v] + sa[tt][1][v]) + (sa[tt][2][v] + sa[tt][3][v]);
                    rr[v] = yv[tt][v] - sigmoid_fast(sv);
                    if (last && rv[tt][v]) lp -= (double)softplus_f(yv[tt][v] > 0.5f ? -sv : sv);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v)
#pragma unroll
                    for (int q = 0; q < QQ; ++q)
                        gacc[q] = __builtin_amdgcn_mfma_f32_4x4x1f32(rr[v], xb[tt][v][q], gacc[q], 0, 0, 0);
            }
            // sum the 4 blocks of each 16-lane row (lanes of equal j), write row partials
#pragma unroll
            for (int q = 0; q < QQ; ++q)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float v = gacc[q][i];
                    v += dpp_ror(v, 4);
                    v += dpp_ror(v, 8);
                    gacc[q][i] = v;
                }
            if ((lane & 15) < 4) {
                float* dst = part + w * LR_PART + ((lane >> 4) * 4 + q4) * 32;
#pragma unroll
                for (int q = 0; q < QQ; ++q) *(floatx4*)(dst + 4 * q) = gacc[q];
            }
            if (last) {
                lp += __shfl_xor(lp, 4, 64);
                lp += __shfl_xor(lp, 8, 64);
                lp += __shfl_xor(lp, 16, 64);
                lp += __shfl_xor(lp, 32, 64);
                if (lane < 4) lpp[w * 4 + lane] = lp;
            }
            __syncthreads();
            if (owner) {
                float gs = 0.f;
                if (od < 4 * QQ) {
                    // fixed-order pairwise tree over the NW x 4 row partials
                    const int q = od >> 2, j = od & 3;
                    float v[NW * 4];
#pragma unroll
                    for (int ww = 0; ww < NW; ++ww)
#pragma unroll
                        for (int rrow = 0; rrow < 4; ++rrow)
                            v[ww * 4 + rrow] = part[ww * LR_PART + (rrow * 4 + j) * 32 + 4 * q + oi];
#pragma unroll
                    for (int h = NW * 2; h >= 1; h >>= 1)
#pragma unroll
                        for (int k = 0; k < h; ++k) v[k] = v[2 * k] + v[2 * k + 1];
                    gs = v[0];
                }
                gq = gs - thq * inv_var;
                p = fmaf(last ? half : eps, gq, p);
                if (last) {
#pragma unroll
                    for (int ww = 0; ww < NW; ++ww) lpdata += lpp[ww * 4 + oi];
                }
            }
        }
        if (!owner) continue;
        // energy change and decision (the 32 lanes of a chain agree)
        double prior = ovalid ? -0.5 * (double)thq * (double)thq * a.tg.inv_var : 0.0;
        dk += ovalid ? 0.5 * (double)p * (double)p : 0.0;
#pragma unroll
        for (int off = 1; off < 32; off <<= 1) {
            dk += __shfl_xor(dk, off, 64);
            prior += __shfl_xor(prior, off, 64);
        }
        const double lp1 = lpdata + prior;
        const double dh = -lp1 + s.logp + dk;
        const double lar = log_accept_ratio_of(dh);
        const bool acc = log_accept_uniform(a.key, (uint32_t)occ, t) < lar;
        if (acc) {
            th0 = thq;
            g0 = gq;
            s.logp = lp1;
        }
        if (oc < C) {
            if (ovalid) {
                if (r.samples && itr >= r.n_burnin) ((float*)r.samples)[((itr - r.n_burnin) * C + oc) * D + od] = th0;
                if (r.out.proposed_state) ((float*)r.out.proposed_state)[oc * D + od] = thq;
                if (r.out.proposed_momentum) ((float*)r.out.proposed_momentum)[oc * D + od] = p;
            }
            // dual averaging, traces and step outputs (lane od == 0 writes)
            const double eps_used = s.eps;
            if (r.adapt && itr < r.n_burnin) {
                const double alpha = lar < 0.0 ? exp(lar) : 1.0;
                const int64_t m = r.m_offset + itr + 1;
                const double log_eps = dual_avg_update(s.da, (double)m, alpha, r.target_accept, r.gamma, r.t0,
                                                       r.kappa);
                s.eps = (m < r.adapt_total) ? exp(log_eps) : exp(s.da.log_eps_bar);
            }
            if (od == 0) {
                if (itr >= r.n_burnin) {
                    const int64_t k = (itr - r.n_burnin) * C + oc;
                    if (r.trace.step_size) r.trace.step_size[k] = eps_used;
                    if (r.trace.is_accepted) r.trace.is_accepted[k] = acc ? 1 : 0;
                    if (r.trace.log_accept_ratio) r.trace.log_accept_ratio[k] = lar;
                    if (r.trace.target_log_prob) r.trace.target_log_prob[k] = s.logp;
                }
                if (r.out.is_accepted) r.out.is_accepted[oc] = acc ? 1 : 0;
                if (r.out.log_accept_ratio) r.out.log_accept_ratio[oc] = lar;
                if (r.out.target_log_prob) r.out.target_log_prob[oc] = s.logp;
                if (r.out.delta_h) r.out.delta_h[oc] = dh;
            }
        }
    }
    if (ovalid) {
        Xw[oc * D + od] = th0;
        Gw[oc * D + od] = g0;
    }
    if (owner && od == 0 && oc < C) {
        a.ws.logp[oc] = s.logp;
        a.ws.eps[oc] = s.eps;
        a.ws.da[oc] = s.da;
    }
}

static size_t logreg4_lds(int) {
    return (size_t)(128 + LR_NW * LR_PART) * sizeof(float) + LR_NW * 4 * sizeof(double);
}

bool fused_logreg_supported(const PlainArgs& a) {
    return !a.bf16_grad && a.tg.D <= 32 && a.tg.N <= (int64_t)LR_NW * 2 * 64;
}

template <int TPW, int QQ, typename XT>
static hipError_t launch_lr4(const PlainArgs& a, const FusedRun& r, hipStream_t s) {
    const size_t lds = logreg4_lds(TPW);
    const dim3 grid((unsigned)((a.C + 3) / 4));
    hipLaunchKernelGGL((k_fused_logreg4<TPW, QQ, XT>), grid, dim3(64 * LR_NW), lds, s, a, r);
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
