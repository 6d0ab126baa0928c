// k_logreg_bf16.hip -- mixed-precision gradient of Bayesian logistic
// regression for large data sets (X stored BF16): both contractions of each
// leapfrog step on v_mfma_f32_16x16x32_bf16 with FP32 accumulation,
//     S  = X theta              (M = rows, N = chains, K = dims)
//     G^T = R^T X,  R = y - sigmoid(S)   (M = chains, N = dims, K = rows)
// and an accurate-logit pass for the log-probability that enters dH: theta is
// split into three BF16 terms (hi + mid + lo), so X theta is formed from exact
// BF16 x BF16 products with FP32 accumulation, and the softplus terms are
// summed in FP64.  The gradient is a deterministic function of position, so
// the trajectory stays reversible and volume preserving; with dH taken from the
// accurate log-probability the accept test keeps detailed balance.
//
// Work decomposition: a workgroup (4 waves) owns 128 chains (32 per wave) and a
// chunk of rows; each wave computes S and G^T for its own 32 chains, so the R
// values never leave registers (K index 8 g + e of the second contraction is
// mapped to the rows the lane already holds: 4 g + e and 16 + 4 g + e - 4).
// 32-row sub-tiles of X (row-major) and X^T (pre-transposed copy) are staged
// in LDS, double buffered with a register prefetch, one barrier per sub-tile.
// Row chunks are mapped XCD-aware: blocks on the same XCD work on the same
// chunk, so the 32 CUs of an XCD stream X through their shared L2 together.
// Partials per chunk are summed in a fixed order by k_logreg_finish.
//
// Lane layouts (v_mfma_f32_16x16x32_bf16, checked on gfx950): A[i][k] at lane
// i + 16 (k / 8), element k % 8; B[k][j] at lane j + 16 (k / 8), element k % 8;
// D[i][j] in VGPR i % 4 of lane j + 16 (i / 4).
#include "hmc_internal.hpp"

namespace hmc {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));

constexpr int LB_NW = 4;      // waves per workgroup
constexpr int LB_CT = 128;    // chains per workgroup (32 per wave)
constexpr int LB_RS = 32;     // rows per sub-tile
constexpr int LB_XPAD = 8;    // bf16 padding of an LDS row of X
constexpr int LB_TPAD = 8;    // bf16 padding of an LDS row of X^T

__device__ __forceinline__ float sigmoid_hw(float s) {
    const float e = __builtin_amdgcn_exp2f(-1.4426950408889634f * s);
    return __builtin_amdgcn_rcpf(1.0f + e);
}

__device__ __forceinline__ float softplus_hw(float s) {
    const float e = __builtin_amdgcn_exp2f(-1.4426950408889634f * fabsf(s));
    const float l = e >= 0x1p-10f ? 0.69314718055994531f * __builtin_amdgcn_logf(1.0f + e)
                                  : e * (1.0f - e * (0.5f - e * 0.33333333f));
    return fmaxf(s, 0.f) + l;
}

__device__ __forceinline__ short bf16_bits(float f) { return (short)f32_to_bf16(f); }

// block -> (chain tile, row chunk): blocks b and b + 8k run on the same XCD
__device__ __forceinline__ void lb_map(int b, int ntile, int nsplit, int* tile, int* split) {
    if (nsplit <= 8 && (8 % nsplit) == 0 && ((ntile * nsplit) % 8) == 0) {
        const int xcd = b & 7, idx = b >> 3;
        *split = xcd % nsplit;
        *tile = idx * (8 / nsplit) + xcd / nsplit;
    } else {
        *split = b % nsplit;
        *tile = b / nsplit;
    }
}

// ---------------------------------------------------------------------------
// Gradient partials.  KS = ceil(D / 32) k-steps, NT = 2 KS dim tiles.
// ---------------------------------------------------------------------------
template <int KS>
__global__ __launch_bounds__(256) void k_lr16_grad(PlainArgs a, const float* __restrict__ xsrc,
                                                   const float* __restrict__ psrc, int drift, int64_t rows_per_split,
                                                   int nsplit, const uint16_t* __restrict__ Xt) {
    constexpr int NT = 2 * KS;
    constexpr int DP = 32 * KS;                 // padded dims
    constexpr int XS = DP + LB_XPAD;            // LDS row stride of X (bf16)
    constexpr int TS = LB_RS + LB_TPAD;         // LDS row stride of X^T (bf16)
    extern __shared__ __align__(16) uint16_t lds16[];
    uint16_t* xs = lds16;                                   // [2][32][XS]
    uint16_t* xts = xs + 2 * LB_RS * XS;                    // [2][DP][TS]
    float* ys = (float*)(xts + 2 * DP * TS);                // [2][32]

    const int64_t D = a.tg.D, N = a.tg.N, C = a.C;
    const int ntile = (int)((C + LB_CT - 1) / LB_CT);
    int tile, split;
    lb_map(blockIdx.x, ntile, nsplit, &tile, &split);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int l16 = lane & 15, g = lane >> 4;
    const int64_t cw = (int64_t)tile * LB_CT + 32 * w;   // first chain of this wave
    const uint16_t* X = (const uint16_t*)a.tg.X;

    // theta (drifted) as BF16 B operands: B[k][j] = theta[chain j][dim k]
    bf16x8 thb[2][KS];
#pragma unroll
    for (int cs = 0; cs < 2; ++cs) {
        const int64_t c = cw + 16 * cs + l16;
        const bool cok = c < C;
        const float eps = cok ? (float)a.ws.eps[c] : 0.f;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int64_t d = 32 * ks + 8 * g + e;
                float v = 0.f;
                if (cok && d < D) {
                    v = xsrc[c * D + d];
                    if (drift) v = fmaf(eps, psrc[c * D + d], v);
                }
                thb[cs][ks][e] = bf16_bits(v);
            }
        }
    }

    const int64_t r_begin = (int64_t)split * rows_per_split;
    int64_t r_end = r_begin + rows_per_split;
    if (r_end > N) r_end = N;
    const int nsub = r_begin < r_end ? (int)((r_end - r_begin + LB_RS - 1) / LB_RS) : 0;

    // staging: X rows (DP/8 chunks of 16 B per row) and X^T (4 chunks of 8 rows per dim)
    constexpr int XCH = LB_RS * DP / 8;     // 16-byte chunks of an X sub-tile
    constexpr int TCH = DP * LB_RS / 8;     // 16-byte chunks of an X^T sub-tile
    constexpr int XPT = (XCH + 255) / 256, TPT = (TCH + 255) / 256;
    uint4 pxs[2][XPT], pts[2][TPT];
    float pys[2] = {0.f, 0.f};
    auto fetch = [&](int sidx, uint4* px, uint4* pt, float& py) {
        const int64_t r0 = r_begin + (int64_t)sidx * LB_RS;
#pragma unroll
        for (int u = 0; u < XPT; ++u) {
            const int ch = threadIdx.x + 256 * u;
            const int row = ch / (DP / 8), c8 = ch % (DP / 8);
            const int64_t gr = r0 + row;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (ch < XCH && gr < r_end) {
                if (8 * c8 + 8 <= D && (D % 8) == 0) {
                    v = *(const uint4*)&X[gr * D + 8 * c8];
                } else {
                    uint16_t t[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) t[e] = (8 * c8 + e < D) ? X[gr * D + 8 * c8 + e] : (uint16_t)0;
                    v = make_uint4(t[0] | (t[1] << 16), t[2] | (t[3] << 16), t[4] | (t[5] << 16), t[6] | (t[7] << 16));
                }
            }
            px[u] = v;
        }
#pragma unroll
        for (int u = 0; u < TPT; ++u) {
            const int ch = threadIdx.x + 256 * u;
            const int dim = ch / (LB_RS / 8), rc = ch % (LB_RS / 8);
            const int64_t gr = r0 + 8 * rc;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (ch < TCH && dim < D && gr < r_end) {
                if (gr + 8 <= r_end && (N % 8) == 0) {
                    v = *(const uint4*)&Xt[(int64_t)dim * N + gr];
                } else {
                    uint16_t t[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) t[e] = (gr + e < r_end) ? Xt[(int64_t)dim * N + gr + e] : (uint16_t)0;
                    v = make_uint4(t[0] | (t[1] << 16), t[2] | (t[3] << 16), t[4] | (t[5] << 16), t[6] | (t[7] << 16));
                }
            }
            pt[u] = v;
        }
        if (threadIdx.x < LB_RS) {
            const int64_t gr = r0 + threadIdx.x;
            py = gr < r_end ? (float)a.tg.y[gr] : 0.f;
        }
    };
    auto stash = [&](int buf, const uint4* px, const uint4* pt, float py) {
#pragma unroll
        for (int u = 0; u < XPT; ++u) {
            const int ch = threadIdx.x + 256 * u;
            if (ch < XCH) {
                const int row = ch / (DP / 8), c8 = ch % (DP / 8);
                *(uint4*)&xs[(buf * LB_RS + row) * XS + 8 * c8] = px[u];
            }
        }
#pragma unroll
        for (int u = 0; u < TPT; ++u) {
            const int ch = threadIdx.x + 256 * u;
            if (ch < TCH) {
                const int dim = ch / (LB_RS / 8), rc = ch % (LB_RS / 8);
                *(uint4*)&xts[(buf * DP + dim) * TS + 8 * rc] = pt[u];
            }
        }
        if (threadIdx.x < LB_RS) ys[buf * LB_RS + threadIdx.x] = py;
    };

    floatx4 gacc[2][NT];
#pragma unroll
    for (int cs = 0; cs < 2; ++cs)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) gacc[cs][nt] = floatx4{0.f, 0.f, 0.f, 0.f};

    // pipeline: sub-tile s is in LDS buffer s % 2 while the loads of s + 1 and
    // s + 2 are in flight in the two register stages
    if (nsub > 0) {
        fetch(0, pxs[0], pts[0], pys[0]);
        stash(0, pxs[0], pts[0], pys[0]);
    }
    if (nsub > 1) fetch(1, pxs[1], pts[1], pys[1]);
    __syncthreads();
    auto body = [&](int sidx, uint4* pn, uint4* tn, float& yn, uint4* pf, uint4* tf, float& yf) {
        // pn/tn/yn: stage holding sub-tile sidx + 1; pf/tf/yf: stage to receive sidx + 2
        const int buf = sidx & 1;
        if (sidx + 2 < nsub) fetch(sidx + 2, pf, tf, yf);
        const uint16_t* xb = xs + buf * LB_RS * XS;
        const uint16_t* tb = xts + buf * DP * TS;
        const float* yb = ys + buf * LB_RS;
        // S for two 16-row tiles x two 16-chain tiles
        floatx4 sacc[2][2];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int cs = 0; cs < 2; ++cs) sacc[mt][cs] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                const bf16x8 ax = *(const bf16x8*)&xb[(mt * 16 + l16) * XS + 32 * ks + 8 * g];
#pragma unroll
                for (int cs = 0; cs < 2; ++cs)
                    sacc[mt][cs] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, thb[cs][ks], sacc[mt][cs], 0, 0, 0);
            }
        // R = y - sigmoid(S) (rows past the chunk contribute 0), packed as the A operand of G^T
        const int64_t r0 = r_begin + (int64_t)sidx * LB_RS;
        bf16x8 ra[2];
#pragma unroll
        for (int cs = 0; cs < 2; ++cs)
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = mt * 16 + 4 * g + v;
                    const float rv = (r0 + row < r_end) ? yb[row] - sigmoid_hw(sacc[mt][cs][v]) : 0.f;
                    ra[cs][4 * mt + v] = bf16_bits(rv);
                }
        // G^T += R^T X: B[k][j] = X[row(k)][dim 16 nt + j]
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const uint16_t* tr = &tb[(16 * nt + l16) * TS];
            const uint2 lo = *(const uint2*)&tr[4 * g];
            const uint2 hi = *(const uint2*)&tr[16 + 4 * g];
            bf16x8 bx;
            bx[0] = (short)(lo.x & 0xffff); bx[1] = (short)(lo.x >> 16);
            bx[2] = (short)(lo.y & 0xffff); bx[3] = (short)(lo.y >> 16);
            bx[4] = (short)(hi.x & 0xffff); bx[5] = (short)(hi.x >> 16);
            bx[6] = (short)(hi.y & 0xffff); bx[7] = (short)(hi.y >> 16);
#pragma unroll
            for (int cs = 0; cs < 2; ++cs)
                gacc[cs][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ra[cs], bx, gacc[cs][nt], 0, 0, 0);
        }
        if (sidx + 1 < nsub) stash(buf ^ 1, pn, tn, yn);
        __syncthreads();
    };
    for (int sidx = 0; sidx < nsub; sidx += 2) {
        // stage 1 holds sidx + 1; stage 0 receives sidx + 2
        body(sidx, pxs[1], pts[1], pys[1], pxs[0], pts[0], pys[0]);
        if (sidx + 1 < nsub) body(sidx + 1, pxs[0], pts[0], pys[0], pxs[1], pts[1], pys[1]);
    }
    // partial G[chain][dim] for this row chunk
#pragma unroll
    for (int cs = 0; cs < 2; ++cs)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t c = cw + 16 * cs + 4 * g + v;
                const int64_t d = 16 * nt + l16;
                if (c < C && d < D) a.ws.part_g[((int64_t)split * C + c) * D + d] = gacc[cs][nt][v];
            }
}

// ---------------------------------------------------------------------------
// Accurate log-probability partials: theta = hi + mid + lo (three BF16 terms),
// 64 chains per workgroup (16 per wave), softplus summed in FP64 per chain.
// ---------------------------------------------------------------------------
template <int KS>
__global__ __launch_bounds__(256) void k_lr16_logp(PlainArgs a, const float* __restrict__ xsrc,
                                                   int64_t rows_per_split, int nsplit) {
    constexpr int DP = 32 * KS;
    constexpr int XS = DP + LB_XPAD;
    constexpr int CT = 64;
    extern __shared__ __align__(16) uint16_t lds16[];
    uint16_t* xs = lds16;                                   // [2][32][XS]
    float* ys = (float*)(xs + 2 * LB_RS * XS);              // [2][32]
    const int64_t D = a.tg.D, N = a.tg.N, C = a.C;
    const int ntile = (int)((C + CT - 1) / CT);
    int tile, split;
    lb_map(blockIdx.x, ntile, nsplit, &tile, &split);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int l16 = lane & 15, g = lane >> 4;
    const int64_t c = (int64_t)tile * CT + 16 * w + l16;
    const bool cok = c < C;
    const uint16_t* X = (const uint16_t*)a.tg.X;

    bf16x8 th[3][KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int64_t d = 32 * ks + 8 * g + e;
            const float v = (cok && d < D) ? xsrc[c * D + d] : 0.f;
            const uint16_t h = f32_to_bf16(v);
            const float r1 = v - bf16_to_f32(h);
            const uint16_t m = f32_to_bf16(r1);
            const float r2 = r1 - bf16_to_f32(m);
            th[0][ks][e] = (short)h;
            th[1][ks][e] = (short)m;
            th[2][ks][e] = (short)f32_to_bf16(r2);
        }
    const int64_t r_begin = (int64_t)split * rows_per_split;
    int64_t r_end = r_begin + rows_per_split;
    if (r_end > N) r_end = N;
    const int nsub = r_begin < r_end ? (int)((r_end - r_begin + LB_RS - 1) / LB_RS) : 0;
    constexpr int XCH = LB_RS * DP / 8;
    constexpr int XPT = (XCH + 255) / 256;
    uint4 px[XPT];
    float py = 0.f;
    auto fetch = [&](int sidx) {
        const int64_t r0 = r_begin + (int64_t)sidx * LB_RS;
#pragma unroll
        for (int u = 0; u < XPT; ++u) {
            const int ch = threadIdx.x + 256 * u;
            const int row = ch / (DP / 8), c8 = ch % (DP / 8);
            const int64_t gr = r0 + row;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (ch < XCH && gr < r_end) {
                if (8 * c8 + 8 <= D && (D % 8) == 0) {
                    v = *(const uint4*)&X[gr * D + 8 * c8];
                } else {
                    uint16_t t[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) t[e] = (8 * c8 + e < D) ? X[gr * D + 8 * c8 + e] : (uint16_t)0;
                    v = make_uint4(t[0] | (t[1] << 16), t[2] | (t[3] << 16), t[4] | (t[5] << 16), t[6] | (t[7] << 16));
                }
            }
            px[u] = v;
        }
        if (threadIdx.x < LB_RS) {
            const int64_t gr = r0 + threadIdx.x;
            py = gr < r_end ? (float)a.tg.y[gr] : 0.f;
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int u = 0; u < XPT; ++u) {
            const int ch = threadIdx.x + 256 * u;
            if (ch < XCH) {
                const int row = ch / (DP / 8), c8 = ch % (DP / 8);
                *(uint4*)&xs[(buf * LB_RS + row) * XS + 8 * c8] = px[u];
            }
        }
        if (threadIdx.x < LB_RS) ys[buf * LB_RS + threadIdx.x] = py;
    };
    double lp = 0.0;
    if (nsub > 0) {
        fetch(0);
        stash(0);
    }
    __syncthreads();
    for (int sidx = 0; sidx < nsub; ++sidx) {
        const int buf = sidx & 1;
        if (sidx + 1 < nsub) fetch(sidx + 1);
        const uint16_t* xb = xs + buf * LB_RS * XS;
        const float* yb = ys + buf * LB_RS;
        floatx4 sacc[2] = {floatx4{0.f, 0.f, 0.f, 0.f}, floatx4{0.f, 0.f, 0.f, 0.f}};
        // smallest terms first
#pragma unroll
        for (int term = 2; term >= 0; --term)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) {
                    const bf16x8 ax = *(const bf16x8*)&xb[(mt * 16 + l16) * XS + 32 * ks + 8 * g];
                    sacc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, th[term][ks], sacc[mt], 0, 0, 0);
                }
        const int64_t r0 = r_begin + (int64_t)sidx * LB_RS;
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = mt * 16 + 4 * g + v;
                if (r0 + row < r_end) {
                    const float s = sacc[mt][v];
                    lp -= (double)softplus_hw(yb[row] > 0.5f ? -s : s);
                }
            }
        if (sidx + 1 < nsub) stash(buf ^ 1);
        __syncthreads();
    }
    // lanes holding chain l16: l16, l16 + 16, + 32, + 48
    lp += __shfl_xor(lp, 16, 64);
    lp += __shfl_xor(lp, 32, 64);
    if (g == 0 && cok) a.ws.part_lp[(int64_t)split * C + c] = lp;
}

__global__ __launch_bounds__(256) void k_lr16_lp_sum(PlainArgs a, int nsplit) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.C) return;
    double l = 0.0;
    for (int s = 0; s < nsplit; ++s) l += a.ws.part_lp[(int64_t)s * a.C + c];
    a.ws.lpq[c] = l;
}

__global__ __launch_bounds__(256) void k_transpose_bf16(const uint16_t* __restrict__ X, uint16_t* __restrict__ Xt,
                                                        int64_t N, int64_t D) {
    __shared__ uint16_t tile[32][33];
    const int64_t n0 = (int64_t)blockIdx.x * 32, d0 = (int64_t)blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int64_t n = n0 + r, d = d0 + tx;
        tile[r][tx] = (n < N && d < D) ? X[n * D + d] : (uint16_t)0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int64_t d = d0 + r, n = n0 + tx;
        if (n < N && d < D) Xt[d * N + n] = tile[tx][r];
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static int pow2_split(int ntile, int64_t N) {
    int s = 1;
    while (s < 8 && ntile * s < 256 && (N + 2 * s - 1) / (2 * s) >= 4 * LB_RS) s *= 2;
    return s;
}

int lb_grad_nsplit(int64_t N, int64_t C) { return pow2_split((int)((C + LB_CT - 1) / LB_CT), N); }
int lb_grad_nsplit_t(const PlainArgs& a) {
    return a.tune.lr16_nsplit > 0 ? a.tune.lr16_nsplit : lb_grad_nsplit(a.tg.N, a.C);
}
int lb_logp_nsplit(int64_t N, int64_t C) { return pow2_split((int)((C + 63) / 64), N); }

static int64_t rows_for(int64_t N, int nsplit) {
    const int64_t r = (N + nsplit - 1) / nsplit;
    return (r + LB_RS - 1) / LB_RS * LB_RS;
}

bool bf16_grad_supported(const TargetDev& tg) { return tg.kind == HMC_TGT_LOGREG && tg.x_bf16 && tg.D <= 256; }

hipError_t launch_transpose_bf16(const PlainArgs& a, void* Xt, hipStream_t s) {
    const dim3 grid((unsigned)((a.tg.N + 31) / 32), (unsigned)((a.tg.D + 31) / 32));
    hipLaunchKernelGGL(k_transpose_bf16, grid, dim3(256), 0, s, (const uint16_t*)a.tg.X, (uint16_t*)Xt, a.tg.N,
                       a.tg.D);
    return hipGetLastError();
}

template <int KS>
static hipError_t lb_grad_k(const PlainArgs& a, const float* x, const float* p, int drift, const void* Xt,
                            hipStream_t s) {
    const int ntile = (int)((a.C + LB_CT - 1) / LB_CT);
    const int nsplit = lb_grad_nsplit_t(a);
    const size_t lds = (size_t)(2 * LB_RS * (32 * KS + LB_XPAD) + 2 * 32 * KS * (LB_RS + LB_TPAD)) * 2 +
                       2 * LB_RS * sizeof(float);
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void*)k_lr16_grad<KS>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_lr16_grad<KS>, dim3((unsigned)(ntile * nsplit)), dim3(256), lds, s, a, x, p, drift,
                       rows_for(a.tg.N, nsplit), nsplit, (const uint16_t*)Xt);
    return hipGetLastError();
}

template <int KS>
static hipError_t lb_logp_k(const PlainArgs& a, const float* x, hipStream_t s) {
    const int ntile = (int)((a.C + 63) / 64);
    const int nsplit = lb_logp_nsplit(a.tg.N, a.C);
    const size_t lds = (size_t)(2 * LB_RS * (32 * KS + LB_XPAD)) * 2 + 2 * LB_RS * sizeof(float);
    hipLaunchKernelGGL(k_lr16_logp<KS>, dim3((unsigned)(ntile * nsplit)), dim3(256), lds, s, a, x,
                       rows_for(a.tg.N, nsplit), nsplit);
    hipLaunchKernelGGL(k_lr16_lp_sum, dim3((unsigned)((a.C + 255) / 256)), dim3(256), 0, s, a, nsplit);
    return hipGetLastError();
}

hipError_t launch_lr16_grad(const PlainArgs& a, const float* x, const float* p, int drift, const void* Xt,
                            hipStream_t s) {
    switch ((a.tg.D + 31) / 32) {
    case 1: return lb_grad_k<1>(a, x, p, drift, Xt, s);
    case 2: return lb_grad_k<2>(a, x, p, drift, Xt, s);
    case 3: case 4: return lb_grad_k<4>(a, x, p, drift, Xt, s);
    default: return lb_grad_k<8>(a, x, p, drift, Xt, s);
    }
}

hipError_t launch_lr16_logp(const PlainArgs& a, const float* x, hipStream_t s) {
    switch ((a.tg.D + 31) / 32) {
    case 1: return lb_logp_k<1>(a, x, s);
    case 2: return lb_logp_k<2>(a, x, s);
    case 3: case 4: return lb_logp_k<4>(a, x, s);
    default: return lb_logp_k<8>(a, x, s);
    }
}

}  // namespace hmc
