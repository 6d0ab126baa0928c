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
// Work decomposition: a workgroup (4 waves) owns 4 CW chains (CW = 64 per wave,
// four 16-chain tiles; 48 when D > 128, where 64 x D accumulators plus those of
// S would exceed the 256 AGPRs) and a chunk of rows; each wave computes S and G^T for its own
// chains, so the R values never leave registers (K index 8 g + e of the second
// contraction is mapped to the rows the lane already holds: 4 g + e and
// 16 + 4 g + e - 4).  theta stays in VGPRs as the B operands of the first
// contraction, the G^T accumulators (CW chains x D) in AGPRs; every LDS operand
// fragment feeds CW / 16 MFMAs.  32-row sub-tiles of X (row-major) and X^T
// (pre-transposed copy) are staged in LDS, double buffered, with the global
// loads of sub-tile s + 2 in flight while sub-tile s is multiplied.
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

typedef float floatx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));
// eight floats to BF16, round to nearest even (v_cvt_pk_bf16_f32)
__device__ __forceinline__ bf16x8 pack_bf16(floatx8 f) {
    return __builtin_bit_cast(bf16x8, __builtin_convertvector(f, bf16x8v));
}

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
// 16-chain tiles per wave for KS k-steps of 32 dims
__host__ __device__ constexpr int lb_cs(int KS) { return KS > 4 ? 3 : 4; }

template <int KS>
__global__ __launch_bounds__(256) void k_lr16_grad(PlainArgs a, const float* __restrict__ xsrc,
                                                   const float* __restrict__ psrc, int drift, int64_t rows_per_split,
                                                   int nsplit, const uint16_t* __restrict__ Xt) {
    constexpr int NT = 2 * KS;                  // 16-dim tiles of G
    constexpr int CS = lb_cs(KS);               // 16-chain tiles per wave
    constexpr int CW = 16 * CS, CT = LB_NW * CW;   // chains per wave / per workgroup
    constexpr int DP = 32 * KS;                 // padded dims
    constexpr int XS = DP + LB_XPAD;            // LDS row stride of X (bf16)
    constexpr int TS = LB_RS + LB_TPAD;         // LDS row stride of X^T (bf16)
    extern __shared__ __align__(16) uint16_t lds16[];
    uint16_t* xs = lds16;                                   // [2][32][XS]
    uint16_t* xts = xs + 2 * LB_RS * XS;                    // [2][DP][TS]
    float* ys = (float*)(xts + 2 * DP * TS);                // [2][32]

    const int64_t D = a.tg.D, N = a.tg.N, C = a.C;
    const int ntile = (int)((C + CT - 1) / CT);
    int tile, split;
    lb_map(blockIdx.x, ntile, nsplit, &tile, &split);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int l16 = lane & 15, g = lane >> 4;
    const int64_t cw = (int64_t)tile * CT + CW * w;     // first chain of this wave
    const uint16_t* X = (const uint16_t*)a.tg.X;

    // theta (drifted) as BF16 B operands: B[k][j] = theta[chain j][dim k]
    bf16x8 thb[CS][KS];
#pragma unroll
    for (int cs = 0; cs < CS; ++cs) {
        const int64_t c = cw + 16 * cs + l16;
        const bool cok = c < C;
        const float eps = cok ? (float)a.ws.eps[c] : 0.f;
        const float* xr = xsrc + (cok ? c : 0) * D;
        const float* pr = psrc + (cok ? c : 0) * D;
        const bool vec = (D % 4) == 0;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int d0 = 32 * ks + 8 * g;
            floatx8 v;
            if (vec && cok && d0 + 8 <= D) {
                const float4 x0 = *(const float4*)(xr + d0), x1 = *(const float4*)(xr + d0 + 4);
                v = floatx8{x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
                if (drift) {
                    const float4 p0 = *(const float4*)(pr + d0), p1 = *(const float4*)(pr + d0 + 4);
                    const floatx8 pv = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w};
#pragma unroll
                    for (int e = 0; e < 8; ++e) v[e] = fmaf(eps, pv[e], v[e]);
                }
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int d = d0 + e;
                    float t = 0.f;
                    if (cok && d < D) {
                        t = xr[d];
                        if (drift) t = fmaf(eps, pr[d], t);
                    }
                    v[e] = t;
                }
            }
            thb[cs][ks] = pack_bf16(v);
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
    uint4 px[XPT], pt[TPT];
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
    auto stash = [&](int buf) {
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

    floatx4 gacc[CS][NT];
#pragma unroll
    for (int cs = 0; cs < CS; ++cs)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) gacc[cs][nt] = floatx4{0.f, 0.f, 0.f, 0.f};

    // sub-tile s sits in LDS buffer s % 2; the loads of s + 1 are in flight in
    // registers while s is multiplied and are stored to the other buffer after it
    if (nsub > 0) {
        fetch(0);
        stash(0);
    }
    if (nsub > 1) fetch(1);
    __syncthreads();
    for (int sidx = 0; sidx < nsub; ++sidx) {
        const int buf = sidx & 1;
        const uint16_t* xb = xs + buf * LB_RS * XS;
        const uint16_t* tb = xts + buf * DP * TS;
        const float* yb = ys + buf * LB_RS;
        // S for two 16-row tiles x four 16-chain tiles; each X fragment feeds four MFMAs
        floatx4 sacc[2][CS];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int cs = 0; cs < CS; ++cs) sacc[mt][cs] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                const bf16x8 ax = *(const bf16x8*)&xb[(mt * 16 + l16) * XS + 32 * ks + 8 * g];
#pragma unroll
                for (int cs = 0; cs < CS; ++cs)
                    sacc[mt][cs] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, thb[cs][ks], sacc[mt][cs], 0, 0, 0);
            }
        // R = y - sigmoid(S) (rows past the chunk contribute 0), packed as the A operand of G^T
        const int64_t r0 = r_begin + (int64_t)sidx * LB_RS;
        bf16x8 ra[CS];
#pragma unroll
        for (int cs = 0; cs < CS; ++cs) {
            floatx8 rv;
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = mt * 16 + 4 * g + v;
                    rv[4 * mt + v] = (r0 + row < r_end) ? yb[row] - sigmoid_hw(sacc[mt][cs][v]) : 0.f;
                }
            ra[cs] = pack_bf16(rv);
        }
        // G^T += R^T X: B[k][j] = X[row(k)][dim 16 nt + j]; each X^T fragment feeds four MFMAs
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const uint16_t* tr = &tb[(16 * nt + l16) * TS];
            const uint2 lo = *(const uint2*)&tr[4 * g];
            const uint2 hi = *(const uint2*)&tr[16 + 4 * g];
            const bf16x8 bx = __builtin_bit_cast(bf16x8, make_uint4(lo.x, lo.y, hi.x, hi.y));
#pragma unroll
            for (int cs = 0; cs < CS; ++cs)
                gacc[cs][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ra[cs], bx, gacc[cs][nt], 0, 0, 0);
        }
        if (sidx + 1 < nsub) stash(buf ^ 1);
        __syncthreads();
        if (sidx + 2 < nsub) fetch(sidx + 2);
    }
    // partial G[chain][dim] for this row chunk
#pragma unroll
    for (int cs = 0; cs < CS; ++cs)
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
// Copy-staged kernels (D and N multiples of 8): the sub-tiles are copied global
// -> LDS by the load-to-LDS instructions (global_load_lds_dwordx4: lane i of an
// instruction writes bytes 16 i .. 16 i + 15 of a 1 KB block), so a ring of
// sub-tile buffers keeps several sub-tiles in flight without staging
// registers; the barrier between sub-tiles waits for LDS only, each wave first
// waiting (vmcnt) for its own copies of the sub-tile it is about to read.  The
// tiles use 16-byte slots XOR-swizzled by row so that the operand reads of the
// MFMAs spread over the LDS banks:
//   X   [32 rows][DP / 8 slots]: slot c of row r at position c ^ (r & XM)
//   X^T [DP dims][4 slots of 8 rows]: slot c of dim d at position c ^ ((d >> 1) & 3)
// ---------------------------------------------------------------------------
constexpr int LD_NB = 4;      // sub-tile buffers of the log-probability kernel
#ifndef LD_XM_MAX
#define LD_XM_MAX 8
#endif
#ifndef LD_TSHIFT
#define LD_TSHIFT 1
#endif
// X swizzle mask for SR slots per row; X^T slot swizzle of dim d
__host__ __device__ constexpr int ld_xmask(int SR) { return (SR < LD_XM_MAX ? SR : LD_XM_MAX) - 1; }
__device__ __forceinline__ int ld_tsw(int d) { return (d >> LD_TSHIFT) & 3; }
constexpr int LD_YB = 256;    // bytes reserved for the labels of a sub-tile (32 used)


// s_waitcnt vmcnt(n) leaving the other counters unconstrained (gfx9 encoding)
template <int n>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(n >= 0 && n < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8));
}

// workgroup barrier that orders LDS accesses only (in-flight global->LDS copies
// of later sub-tiles stay in flight)
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

typedef __attribute__((address_space(3))) void lds_void_t;

// shapes the load-to-LDS kernels take: 16-byte aligned rows of X and X^T, at
// least 64 rows, and X^T byte offsets within 32 bits
static bool ld_copy_ok(const TargetDev& tg) {
    return tg.D % 8 == 0 && tg.N % 8 == 0 && tg.N >= 64 && (uint64_t)tg.D * (uint64_t)tg.N * 2u < (1ull << 32);
}

// ---------------------------------------------------------------------------
// Gradient partials, software-pipelined (copy-staged): 64 chains per wave (four
// 16-chain tiles, so 256 chains per workgroup and, at 8192 chains, 32 chain
// tiles x 8 row splits = one workgroup per CU with each split on its own XCD).
// The residuals of one sub-tile are formed on the vector ALUs while the matrix
// cores run the other contraction, in three phases per sub-tile s:
//   1. the X fragments of rows 0..15 of s are read, the residuals of rows
//      16..31 of s - 1 computed while they arrive, then S of rows 0..15
//   2. the X fragments of rows 16..31 of s are read; G^T += R^T X^T of s - 1,
//      with the residuals of rows 0..15 of s computed between its MFMAs
//   3. S of rows 16..31 of s
// X^T of sub-tile s - 1 is still read in the iteration of s, so the X^T tiles
// (with their labels) sit in a ring of five buffers and the X tiles in a ring of
// four; the copies run three sub-tiles ahead.  Its X tiles use their own slot
// swizzle (see xsw) and row order within the S halves (see below).
// ---------------------------------------------------------------------------
typedef __bf16 bf16x4v __attribute__((ext_vector_type(4)));

// four floats to BF16 (round to nearest even), packed in two dwords
__device__ __forceinline__ uint2 pack4_bf16(floatx4 f) {
    return __builtin_bit_cast(uint2, __builtin_convertvector(f, bf16x4v));
}

constexpr int LP_NBX = 4;     // X sub-tile buffers of the pipelined kernel
constexpr int LP_NBT = 5;     // X^T sub-tile (+ labels) buffers

template <int KS>
__host__ __device__ constexpr int pipe_lds_bytes() {
    return LP_NBX * LB_RS * 32 * KS * 2 + LP_NBT * (32 * KS * LB_RS * 2 + LD_YB);
}

// FULL: D == 32 KS and every sub-tile whole (N a multiple of 32): the copies
// need no clamps and the residuals no row masks.
template <int KS, bool FULL>
__global__ __launch_bounds__(256) void k_lr16_grad_pipe(PlainArgs a, const float* __restrict__ xsrc,
                                                        const float* __restrict__ psrc, int drift,
                                                        int64_t rows_per_split, int nsplit,
                                                        const uint16_t* __restrict__ Xt) {
    constexpr int NT = 2 * KS;
    constexpr int CS = 4;
    constexpr int CW = 16 * CS, CT = LB_NW * CW;
    constexpr int DP = 32 * KS;
    constexpr int SR = DP / 8;
    // X slot swizzle of row r: (r & 3) | (bit 3 of r) << 2 (r & 3 with 4 slots), so
    // the rows one quarter-wave reads (8 q + 4 mt + (0..3)) fall on distinct slots
    auto xsw = [](int r) { return SR >= 8 ? ((r & 3) | (((r >> 3) & 1) << 2)) : (r & 3); };
    constexpr int XB = LB_RS * DP * 2;          // bytes of an X sub-tile
    constexpr int TB = DP * LB_RS * 2;          // bytes of an X^T sub-tile
    constexpr int TBY = TB + LD_YB;             // X^T sub-tile + labels
    constexpr int XI = XB / 1024, TI = TB / 1024;
    constexpr int JW = (XI + TI) / LB_NW;
    constexpr int J = JW + 1;
    static_assert((XI + TI) % LB_NW == 0, "copies must split evenly over the waves");
    extern __shared__ __align__(16) uint8_t ldsb[];
    uint8_t* xring = ldsb;                      // [LP_NBX][XB]
    uint8_t* tring = ldsb + LP_NBX * XB;        // [LP_NBT][TBY]

    const int64_t D = a.tg.D, N = a.tg.N, C = a.C;
    const int ntile = (int)((C + CT - 1) / CT);
    int tile, split;
    lb_map(blockIdx.x, ntile, nsplit, &tile, &split);
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int l16 = lane & 15, g = lane >> 4;
    const int64_t cw = (int64_t)tile * CT + CW * w;
    const uint16_t* X = (const uint16_t*)a.tg.X;
    const uint8_t* Y = a.tg.y;

    // theta (drifted) as BF16 B operands: B[k][j] = theta[chain j][dim k]
    bf16x8 thb[CS][KS];
#pragma unroll
    for (int cs = 0; cs < CS; ++cs) {
        const int64_t c = cw + 16 * cs + l16;
        const bool cok = c < C;
        const float eps = cok ? (float)a.ws.eps[c] : 0.f;
        const float* xr = xsrc + (cok ? c : 0) * D;
        const float* pr = psrc + (cok ? c : 0) * D;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int d0 = 32 * ks + 8 * g;
            floatx8 v = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (cok && d0 < D) {      // D % 8 == 0: the 8 dims are all in range
                const float4 x0 = *(const float4*)(xr + d0), x1 = *(const float4*)(xr + d0 + 4);
                v = floatx8{x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
                if (drift) {
                    const float4 p0 = *(const float4*)(pr + d0), p1 = *(const float4*)(pr + d0 + 4);
                    const floatx8 pv = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w};
#pragma unroll
                    for (int e = 0; e < 8; ++e) v[e] = fmaf(eps, pv[e], v[e]);
                }
            }
            thb[cs][ks] = pack_bf16(v);
        }
    }

    const int64_t r_begin = (int64_t)split * rows_per_split;
    int64_t r_end = r_begin + rows_per_split;
    if (r_end > N) r_end = N;
    const int nsub = r_begin < r_end ? (int)((r_end - r_begin + LB_RS - 1) / LB_RS) : 0;

    // copies of sub-tile sidx: X into xbase, X^T and the labels into tbase; in
    // the general case rows past the chunk and dims past D read in-range data
    // whose products are masked (residual 0) or discarded
    auto copy_in = [&](int sidx, uint8_t* __restrict__ xbase, uint8_t* __restrict__ tbase) {
        const int64_t r0 = r_begin + (int64_t)sidx * LB_RS;
        const char* xsrc_t = (const char*)(X + r0 * D);
        const char* tsrc_t = (const char*)(Xt + r0);
        // the lane index through an empty asm: the per-lane offsets below are
        // recomputed for every sub-tile instead of being hoisted out of the loop
        // (and spilled: a reload's wait would also wait for the copies in flight)
        int ln = lane;
        asm volatile("" : "+v"(ln));
        if constexpr (FULL) {
            // rows of exactly DP dims, X rows contiguous; the swizzle term of a wave's
            // copies does not depend on k (nor does that of X^T)
            // row of lane ln in copy k: A + (256 / SR) k with A below; its swizzle
            // depends on k only through bit 3 of the row, i.e. the parity of k when
            // SR = 32 (two offsets), not at all otherwise
            const int arow = (64 / SR) * w + ln / SR;
            uint32_t xoff[2];
#pragma unroll
            for (int par = 0; par < 2; ++par) {
                const int sw = SR >= 8 ? ((arow & 3) | ((((arow >> 3) & 1) ^ par) << 2)) : (arow & 3);
                xoff[par] = (uint32_t)(ln / SR) * (uint32_t)(DP * 2) + 16u * (uint32_t)((ln % SR) ^ sw);
            }
            const uint32_t toff = (uint32_t)(ln >> 2) * (uint32_t)N * 2u + 16u * (uint32_t)((ln & 3) ^ ((ln >> 3) & 3));
#pragma unroll
            for (int k = 0; k < JW; ++k) {
                const int i = w + LB_NW * k;
                const bool isx = (XI % LB_NW == 0) ? (k < XI / LB_NW) : (i < XI);
                if (isx) {
                    __builtin_amdgcn_global_load_lds((const void*)(xsrc_t + (uint32_t)i * 1024u +
                                                                   xoff[SR == 32 ? (k & 1) : 0]),
                                                     (lds_void_t*)(xbase + i * 1024), 16, 0, 0);
                } else {
                    const int ii = i - XI;
                    __builtin_amdgcn_global_load_lds((const void*)(tsrc_t + (uint32_t)(16 * ii) * (uint32_t)N * 2u + toff),
                                                     (lds_void_t*)(tbase + ii * 1024), 16, 0, 0);
                }
            }
            __builtin_amdgcn_global_load_lds((const void*)(Y + r0 + 4 * (ln & 7)), (lds_void_t*)(tbase + TB), 4, 0, 0);
        } else {
            const int nrow = (int)(r_end - r0 < LB_RS ? r_end - r0 : LB_RS);   // multiple of 8
#pragma unroll
            for (int k = 0; k < JW; ++k) {
                const int i = w + LB_NW * k;
                if (i < XI) {
                    const int q = i * 64 + ln;
                    const int row = q / SR, c = (q % SR) ^ xsw(row);
                    const int rowc = row < nrow ? row : nrow - 1;
                    const uint32_t off = (uint32_t)(rowc * (int)D + (8 * c < D ? 8 * c : 0)) * 2u;
                    __builtin_amdgcn_global_load_lds((const void*)(xsrc_t + off), (lds_void_t*)(xbase + i * 1024),
                                                     16, 0, 0);
                } else {
                    const int ii = i - XI;
                    const int q = ii * 64 + ln;
                    const int dim = q >> 2, c = (q & 3) ^ ld_tsw(dim);
                    const int rr = 8 * c + 8 <= nrow ? 8 * c : 0;
                    const uint32_t off = ((uint32_t)(dim < D ? dim : 0) * (uint32_t)N + (uint32_t)rr) * 2u;
                    __builtin_amdgcn_global_load_lds((const void*)(tsrc_t + off), (lds_void_t*)(tbase + ii * 1024),
                                                     16, 0, 0);
                }
            }
            // labels: dword (lane % 8) of the sub-tile's rows; the rows left in the chunk are a
            // multiple of 8, so a dword that starts in range ends in range (else row r0's is read)
            const int64_t yo = r0 + 4 * (ln & 7) < r_end ? r0 + 4 * (ln & 7) : r0;
            __builtin_amdgcn_global_load_lds((const void*)(Y + yo), (lds_void_t*)(tbase + TB), 4, 0, 0);
        }
    };
    auto xbuf = [&](int sidx) { return xring + (sidx % LP_NBX) * XB; };
    auto tbuf = [&](int sidx) { return tring + (sidx % LP_NBT) * TBY; };
    // Rows of the S halves: half mt, lane position i = 4 q + v holds sub-tile row
    // 8 q + 4 mt + v, so lane group g ends up with the residuals of rows 8 g .. 8 g + 7
    // (rows 8 g + v from half 0, 8 g + 4 + v from half 1), the K order of the second
    // contraction; its X^T operand is then the one 16-byte slot g of a dim.
    // Fragment addresses from a few per-lane offsets plus immediates.  X: row
    // rho = 8 (l16 >> 2) + 4 mt + (l16 & 3) has swizzle l16 & 7, and slot
    // (4 ks + g) ^ (l16 & 7) = 8 (ks >> 1) + 4 ((ks & 1) ^ rb) + (g ^ (l16 & 3)) with
    // rb = (l16 >> 2) & 1: two offsets (even / odd ks) per half.  X^T: the swizzle of
    // dim 16 nt + l16 is (l16 >> 1) & 3 for every nt.
    uint32_t xoff[2][2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        const int row = 8 * (l16 >> 2) + 4 * mt + (l16 & 3);
        const int sw = xsw(row);
        const int rb = (sw >> 2) & 1, gg = g ^ (sw & 3);
#pragma unroll
        for (int e = 0; e < 2; ++e) xoff[mt][e] = (uint32_t)(row * (DP * 2) + 16 * (4 * (e ^ rb) + gg));
    }
    const uint32_t toff = (uint32_t)(l16 * 64 + 16 * (g ^ ((l16 >> 1) & 3)));
    // a phase's base offsets pass through one empty asm at the phase's start, so
    // that a register per offset plus the instructions' immediate offsets address
    // its fragments (instead of one hoisted register per fragment)
    auto xfrag_o = [&](const uint8_t* xb, const uint32_t* o2, int ks) {
        return *(const bf16x8*)(xb + o2[ks & 1] + 128 * (ks >> 1));
    };
    auto xfrag = [&](const uint8_t* xb, int ks, int mt) { return xfrag_o(xb, xoff[mt], ks); };
    auto tfrag_o = [&](const uint8_t* tb, uint32_t o, int nt) { return *(const bf16x8*)(tb + o + 1024 * nt); };
    auto tfrag = [&](const uint8_t* tb, int nt) { return tfrag_o(tb, toff, nt); };
    // residuals of one 16-row half (rows row0 + v of the sub-tile, v = 0..3)
    auto resid = [&](floatx4 sv, uint32_t yw, int row0, int nvalid) {
        floatx4 r;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float y = (float)((yw >> (8 * v)) & 0xffu);
            const float t = y - sigmoid_hw(sv[v]);
            r[v] = (FULL || row0 + v < nvalid) ? t : 0.f;
        }
        return pack4_bf16(r);
    };
    // S of one 16-row half of the sub-tile in xb
    auto sphase = [&](const uint8_t* __restrict__ xb, int mt, floatx4* sacc) {
#pragma unroll
        for (int cs = 0; cs < CS; ++cs) sacc[cs] = floatx4{0.f, 0.f, 0.f, 0.f};
        bf16x8 xf0 = xfrag(xb, 0, mt), xf1 = KS > 1 ? xfrag(xb, 1, mt) : xf0;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const bf16x8 ax = xf0;
            xf0 = xf1;
            if (ks + 2 < KS) xf1 = xfrag(xb, ks + 2, mt);
#pragma unroll
            for (int cs = 0; cs < CS; ++cs)
                sacc[cs] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, thb[cs][ks], sacc[cs], 0, 0, 0);
        }
    };

    floatx4 gacc[CS][NT];
#pragma unroll
    for (int cs = 0; cs < CS; ++cs)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) gacc[cs][nt] = floatx4{0.f, 0.f, 0.f, 0.f};

    // G^T += R^T X^T of the sub-tile in tb with residual operands ra
    auto gphase = [&](const uint8_t* __restrict__ tb, const bf16x8* ra, uint32_t to) {
        auto tfrag = [&](const uint8_t* t, int nt) { return tfrag_o(t, to, nt); };
        bf16x8 tf0 = tfrag(tb, 0), tf1 = tfrag(tb, 1);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const bf16x8 bx = tf0;
            tf0 = tf1;
            if (nt + 2 < NT) tf1 = tfrag(tb, nt + 2);
#pragma unroll
            for (int cs = 0; cs < CS; ++cs)
                gacc[cs][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ra[cs], bx, gacc[cs][nt], 0, 0, 0);
        }
    };

    if (nsub > 0) copy_in(0, xbuf(0), tbuf(0));
    if (nsub > 1) copy_in(1, xbuf(1), tbuf(1));
    if (nsub > 2) copy_in(2, xbuf(2), tbuf(2));
    auto wait_tile = [&](int sidx) {
        if (sidx + 2 < nsub) wait_vmcnt<2 * J>();
        else if (sidx + 1 < nsub) wait_vmcnt<J>();
        else wait_vmcnt<0>();
        lds_barrier();
    };
    auto nvalid = [&](int sidx) {
        const int64_t r0 = r_begin + (int64_t)sidx * LB_RS;
        return (int)(r_end - r0 < LB_RS ? r_end - r0 : LB_RS);
    };

    // pipeline registers: S of rows 16..31 of the previous sub-tile, the packed
    // residuals of its rows 0..15, its labels and valid rows
    floatx4 s1p[CS];
    uint2 lo_p[CS];
    uint32_t yp1 = 0u;
    int nvp = 0;
    if (nsub > 0) {       // the first sub-tile: no G of a previous one
        wait_tile(0);
        if (3 < nsub) copy_in(3, xbuf(3), tbuf(3));
        const uint8_t* tb = tbuf(0);
        const uint2 yl = *(const uint2*)(tb + TB + 8 * g);
        const uint32_t y0 = yl.x;
        yp1 = yl.y;
        nvp = nvalid(0);
        floatx4 s0[CS];
        sphase(xbuf(0), 0, s0);
#pragma unroll
        for (int cs = 0; cs < CS; ++cs) lo_p[cs] = resid(s0[cs], y0, 8 * g, nvp);
        sphase(xbuf(0), 1, s1p);
    }
    // one sub-tile; the copy targets (xdst, tdst) and the buffers read (xb, tprev,
    // tcur) are distinct, which the restrict qualifiers tell the compiler, so the
    // LDS reads need not wait for the copies in flight (the explicit vmcnt waits
    // and the barrier order the sub-tiles)
    auto iter = [&](int sidx, uint8_t* __restrict__ xdst, uint8_t* __restrict__ tdst, const uint8_t* __restrict__ xb,
                    const uint8_t* __restrict__ tprev, const uint8_t* __restrict__ tcur) {
        if (sidx + 3 < nsub) copy_in(sidx + 3, xdst, tdst);
        const int nv = nvalid(sidx);
        // phase 1: the X fragments of rows 0..15 are read first, the residuals of
        // rows 16..31 of the previous sub-tile computed while they arrive, then S
        uint32_t o1[2] = {xoff[0][0], xoff[0][1]};
        asm volatile("" : "+v"(o1[0]), "+v"(o1[1]));
        bf16x8 xa[KS];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) xa[ks] = xfrag_o(xb, o1, ks);
        const uint2 yl = *(const uint2*)(tcur + TB + 8 * g);
        const uint32_t y0 = yl.x, y1 = yl.y;
        bf16x8 rp[CS];
#pragma unroll
        for (int cs = 0; cs < CS; ++cs) {
            const uint2 hi = resid(s1p[cs], yp1, 8 * g + 4, nvp);
            rp[cs] = __builtin_bit_cast(bf16x8, make_uint4(lo_p[cs].x, lo_p[cs].y, hi.x, hi.y));
        }
        floatx4 s0[CS];
#pragma unroll
        for (int cs = 0; cs < CS; ++cs) s0[cs] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int cs = 0; cs < CS; ++cs)
                s0[cs] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa[ks], thb[cs][ks], s0[cs], 0, 0, 0);
        // phase 2: the X fragments of rows 16..31 read for phase 3; G of the previous
        // sub-tile with the residuals of rows 0..15 of this one in between
        uint32_t o2[2] = {xoff[1][0], xoff[1][1]}, ot = toff;
        asm volatile("" : "+v"(o2[0]), "+v"(o2[1]), "+v"(ot));
        bf16x8 xb1[KS];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) xb1[ks] = xfrag_o(xb, o2, ks);
        gphase(tprev, rp, ot);
#pragma unroll
        for (int cs = 0; cs < CS; ++cs) lo_p[cs] = resid(s0[cs], y0, 8 * g, nv);
        // phase 3: S of rows 16..31
#pragma unroll
        for (int cs = 0; cs < CS; ++cs) s1p[cs] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int cs = 0; cs < CS; ++cs)
                s1p[cs] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xb1[ks], thb[cs][ks], s1p[cs], 0, 0, 0);
        yp1 = y1;
        nvp = nv;
    };
    for (int sidx = 1; sidx < nsub; ++sidx) {
        wait_tile(sidx);
        iter(sidx, xbuf(sidx + 3), tbuf(sidx + 3), xbuf(sidx), tbuf(sidx + LP_NBT - 1), tbuf(sidx));
    }
    if (nsub > 0) {
        bf16x8 rp[CS];
#pragma unroll
        for (int cs = 0; cs < CS; ++cs) {
            const uint2 hi = resid(s1p[cs], yp1, 8 * g + 4, nvp);
            rp[cs] = __builtin_bit_cast(bf16x8, make_uint4(lo_p[cs].x, lo_p[cs].y, hi.x, hi.y));
        }
        gphase(tbuf(nsub - 1), rp, toff);
    }
#pragma unroll
    for (int cs = 0; cs < CS; ++cs)
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

// The accurate log-probability partials with global -> LDS copies of X (D and
// N multiples of 8): 32 chains per wave (two 16-chain tiles), each X fragment
// feeding six MFMAs (three theta terms x two tiles); ring of LD_NB sub-tiles.
constexpr int LP_CW = 32;     // chains per wave

template <int KS>
__host__ __device__ constexpr int lp_buf_bytes() { return LB_RS * 32 * KS * 2 + LD_YB; }

template <int KS>
__global__ __launch_bounds__(256) void k_lr16_logp_dma(PlainArgs a, const float* __restrict__ xsrc,
                                                       int64_t rows_per_split, int nsplit) {
    constexpr int DP = 32 * KS;
    constexpr int SR = DP / 8;
    constexpr int XM = ld_xmask(SR);
    constexpr int XB = LB_RS * DP * 2;
    constexpr int BUF = lp_buf_bytes<KS>();
    constexpr int XI = XB / 1024;
    constexpr int JW = (XI + LB_NW - 1) / LB_NW;       // X copy instructions per wave (some waves may repeat one)
    constexpr int J = JW + 1;
    constexpr int CS = LP_CW / 16, CT = LB_NW * LP_CW;
    extern __shared__ __align__(16) uint8_t ldsb[];

    const int64_t D = a.tg.D, N = a.tg.N, C = a.C;
    const int ntile = (int)((C + CT - 1) / CT);
    int tile, split;
    lb_map(blockIdx.x, ntile, nsplit, &tile, &split);
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int l16 = lane & 15, g = lane >> 4;
    const int64_t cw = (int64_t)tile * CT + LP_CW * w;
    const uint16_t* X = (const uint16_t*)a.tg.X;
    const uint8_t* Y = a.tg.y;

    // theta = hi + mid + lo, three BF16 B operands per chain tile and k-step
    bf16x8 th[3][CS][KS];
#pragma unroll
    for (int cs = 0; cs < CS; ++cs) {
        const int64_t c = cw + 16 * cs + l16;
        const bool cok = c < C;
        const float* xr = xsrc + (cok ? c : 0) * D;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int d0 = 32 * ks + 8 * g;
            floatx8 v = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (cok && d0 < D) {
                const float4 x0 = *(const float4*)(xr + d0), x1 = *(const float4*)(xr + d0 + 4);
                v = floatx8{x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
            }
            floatx8 r1, r2;
            const bf16x8 h = pack_bf16(v);
#pragma unroll
            for (int e = 0; e < 8; ++e) r1[e] = v[e] - bf16_to_f32((uint16_t)h[e]);
            const bf16x8 m = pack_bf16(r1);
#pragma unroll
            for (int e = 0; e < 8; ++e) r2[e] = r1[e] - bf16_to_f32((uint16_t)m[e]);
            th[0][cs][ks] = h;
            th[1][cs][ks] = m;
            th[2][cs][ks] = pack_bf16(r2);
        }
    }
    const int64_t r_begin = (int64_t)split * rows_per_split;
    int64_t r_end = r_begin + rows_per_split;
    if (r_end > N) r_end = N;
    const int nsub = r_begin < r_end ? (int)((r_end - r_begin + LB_RS - 1) / LB_RS) : 0;

    auto copy_in = [&](int sidx, uint8_t* __restrict__ base) {
        const int64_t r0 = r_begin + (int64_t)sidx * LB_RS;
        const int nrow = (int)(r_end - r0 < LB_RS ? r_end - r0 : LB_RS);
        const char* xsrc_t = (const char*)(X + r0 * D);
#pragma unroll
        for (int k = 0; k < JW; ++k) {
            int i = w + LB_NW * k;
            if (i >= XI) i = XI - 1;          // a repeated copy keeps the count equal over the waves
            const int q = i * 64 + lane;
            const int row = q / SR, c = (q % SR) ^ (row & XM);
            const int rowc = row < nrow ? row : nrow - 1;
            const uint32_t off = (uint32_t)(rowc * (int)D + (8 * c < D ? 8 * c : 0)) * 2u;
            __builtin_amdgcn_global_load_lds((const void*)(xsrc_t + off), (lds_void_t*)(base + i * 1024), 16, 0, 0);
        }
        const int64_t yo = r0 + LB_RS <= r_end ? r0 + 4 * (lane & 7) : 0;
        __builtin_amdgcn_global_load_lds((const void*)(Y + yo), (lds_void_t*)(base + XB), 4, 0, 0);
    };
    double lp[CS] = {};
    if (nsub > 0) copy_in(0, ldsb);
    if (nsub > 1) copy_in(1, ldsb + BUF);
    if (nsub > 2) copy_in(2, ldsb + 2 * BUF);
    auto step = [&](int sidx, uint8_t* __restrict__ nxt, const uint8_t* __restrict__ base) {
        if (sidx + 3 < nsub) copy_in(sidx + 3, nxt);
        const int64_t r0 = r_begin + (int64_t)sidx * LB_RS;
        floatx4 sacc[2][CS];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int cs = 0; cs < CS; ++cs) sacc[mt][cs] = floatx4{0.f, 0.f, 0.f, 0.f};
        // smallest terms first; X fragments read two steps ahead of their MFMAs
        auto xfrag = [&](int idx) {
            const int ks = idx >> 1, row = (idx & 1) * 16 + l16;
            return *(const bf16x8*)(base + row * (DP * 2) + (((4 * ks + g) ^ (row & XM)) * 16));
        };
        bf16x8 xf0 = xfrag(0), xf1 = xfrag(1);
#pragma unroll
        for (int idx = 0; idx < 2 * KS; ++idx) {
            const bf16x8 ax = xf0;
            xf0 = xf1;
            if (idx + 2 < 2 * KS) xf1 = xfrag(idx + 2);
            const int ks = idx >> 1, mt = idx & 1;
#pragma unroll
            for (int term = 2; term >= 0; --term)
#pragma unroll
                for (int cs = 0; cs < CS; ++cs)
                    sacc[mt][cs] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, th[term][cs][ks], sacc[mt][cs], 0, 0, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
#pragma unroll
        for (int idx = 0; idx < 2 * KS; ++idx) {
            __builtin_amdgcn_sched_group_barrier(0x008, 3 * CS, 0);
            if (idx + 2 < 2 * KS) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
        uint32_t yw[2];
        if (r0 + LB_RS <= r_end) {
            yw[0] = *(const uint32_t*)(base + XB + 4 * g);
            yw[1] = *(const uint32_t*)(base + XB + 16 + 4 * g);
        } else {
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                uint32_t t = 0;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t gr = r0 + mt * 16 + 4 * g + v;
                    t |= (gr < r_end ? (uint32_t)Y[gr] : 0u) << (8 * v);
                }
                yw[mt] = t;
            }
        }
#pragma unroll
        for (int cs = 0; cs < CS; ++cs)
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = mt * 16 + 4 * g + v;
                    const float s = sacc[mt][cs][v];
                    const bool y1 = (yw[mt] >> (8 * v)) & 1u;
                    const float sp = softplus_hw(y1 ? -s : s);
                    lp[cs] -= (r0 + row < r_end) ? (double)sp : 0.0;
                }
    };
    for (int sidx = 0; sidx < nsub; ++sidx) {
        if (sidx + 2 < nsub) wait_vmcnt<2 * J>();
        else if (sidx + 1 < nsub) wait_vmcnt<J>();
        else wait_vmcnt<0>();
        lds_barrier();
        step(sidx, ldsb + ((sidx + 3) % LD_NB) * BUF, ldsb + (sidx % LD_NB) * BUF);
    }
    // lanes holding chain l16 of tile cs: l16, l16 + 16, + 32, + 48
#pragma unroll
    for (int cs = 0; cs < CS; ++cs) {
        double t = lp[cs];
        t += __shfl_xor(t, 16, 64);
        t += __shfl_xor(t, 32, 64);
        const int64_t c = cw + 16 * cs + l16;
        if (g == 0 && c < C) a.ws.part_lp[(int64_t)split * C + c] = t;
    }
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

// shapes the copy-staged kernels take (as ld_copy_ok, from the sizes alone)
static bool ld_copy_shape(int64_t N, int64_t D) {
    return D % 8 == 0 && N % 8 == 0 && N >= 64 && (uint64_t)D * (uint64_t)N * 2u < (1ull << 32);
}

// chains per workgroup of the gradient kernel for N rows and D dims: 256 for the
// pipelined kernel, else that of the register-staged one
static int lb_grad_ct(int64_t N, int64_t D) {
    return ld_copy_shape(N, D) ? LB_NW * 64 : LB_NW * 16 * lb_cs((int)((D + 31) / 32) > 4 ? 8 : 4);
}

// row splits: a power of two (so that blocks map to XCDs by split) filling the
// 256 CUs once, at most 8, at least 4 sub-tiles each
int lb_grad_nsplit(int64_t N, int64_t C, int64_t D) {
    const int ct = lb_grad_ct(N, D);
    const int ntile = (int)((C + ct - 1) / ct);
    int s = 1;
    while (s < 8 && ntile * 2 * s <= 256 && (N + 2 * s - 1) / (2 * s) >= 4 * LB_RS) s *= 2;
    return s;
}
int lb_grad_nsplit_t(const PlainArgs& a) {
    return a.tune.lr16_nsplit > 0 ? a.tune.lr16_nsplit : lb_grad_nsplit(a.tg.N, a.C, a.tg.D);
}
int lb_logp_nsplit(int64_t N, int64_t C) { return pow2_split((int)((C + 63) / 64), N); }
// row splits of the copy-staged log-probability kernel (128 chains per workgroup)
static int lp_dma_nsplit(int64_t N, int64_t C) {
    const int ntile = (int)((C + LB_NW * LP_CW - 1) / (LB_NW * LP_CW));
    int s = ntile >= 256 ? 1 : 256 / ntile;
    if (s > 8) s = 8;
    while (s > 1 && (N + s - 1) / s < 4 * LB_RS) --s;
    return s;
}

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
    constexpr int CT = LB_NW * 16 * lb_cs(KS);
    const int ntile = (int)((a.C + CT - 1) / CT);
    const int nsplit = lb_grad_nsplit_t(a);
    const size_t lds = (size_t)(2 * LB_RS * (32 * KS + LB_XPAD) + 2 * 32 * KS * (LB_RS + LB_TPAD)) * 2 +
                       2 * LB_RS * sizeof(float);
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void*)k_lr16_grad<KS>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (ld_copy_ok(a.tg)) {
        constexpr int PCT = LB_NW * 64;
        const int ptile = (int)((a.C + PCT - 1) / PCT);
        const size_t ldd = (size_t)pipe_lds_bytes<KS>();
        const bool full = a.tg.D == 32 * KS && a.tg.N % LB_RS == 0;
        auto kern = full ? k_lr16_grad_pipe<KS, true> : k_lr16_grad_pipe<KS, false>;
        if (ldd > 65536)
            (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)ldd);
        hipLaunchKernelGGL(kern, dim3((unsigned)(ptile * nsplit)), dim3(256), ldd, s, a, x, p, drift,
                           rows_for(a.tg.N, nsplit), nsplit, (const uint16_t*)Xt);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_lr16_grad<KS>, dim3((unsigned)(ntile * nsplit)), dim3(256), lds, s, a, x, p, drift,
                       rows_for(a.tg.N, nsplit), nsplit, (const uint16_t*)Xt);
    return hipGetLastError();
}

template <int KS>
static hipError_t lb_logp_k(const PlainArgs& a, const float* x, hipStream_t s) {
    if (ld_copy_ok(a.tg)) {
        constexpr int CT = LB_NW * LP_CW;
        const int ntile = (int)((a.C + CT - 1) / CT);
        const int nsplit = lp_dma_nsplit(a.tg.N, a.C);
        const size_t ldd = (size_t)LD_NB * lp_buf_bytes<KS>();
        if (ldd > 65536)
            (void)hipFuncSetAttribute((const void*)k_lr16_logp_dma<KS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)ldd);
        hipLaunchKernelGGL(k_lr16_logp_dma<KS>, dim3((unsigned)(ntile * nsplit)), dim3(256), ldd, s, a, x,
                           rows_for(a.tg.N, nsplit), nsplit);
        hipLaunchKernelGGL(k_lr16_lp_sum, dim3((unsigned)((a.C + 255) / 256)), dim3(256), 0, s, a, nsplit);
        return hipGetLastError();
    }
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
