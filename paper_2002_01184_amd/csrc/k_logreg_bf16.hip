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
// Data: at init the context builds zero-padded copies of the target in its
// workspace -- X as [NP, DP] and X^T as [DP, NP] (BF16), y as [NP] bytes, with
// NP = N rounded up to 32 rows and DP = 32 KS dims -- so every sub-tile of 32
// rows is whole and rows are 16-byte aligned.  Padded rows and dims are zero
// in X: they add nothing to S or G (their residuals multiply zeros), and the
// log-probability pass skips rows >= N.
//
// Work decomposition: a workgroup (NW waves) owns 16 NW CS chains and a chunk
// of rows; each wave computes S and G^T for its own 16 CS chains, so the
// residuals never leave registers.  theta (drifted) stays in registers as the B
// operands of the first contraction, beside the G^T accumulators; every LDS
// operand fragment feeds CS MFMAs.  32-row sub-tiles of X and X^T are copied global ->
// LDS by the load-to-LDS instructions (global_load_lds_dwordx4: lane i of an
// instruction writes bytes 16 i .. 16 i + 15 of a 1 KB block) into rings of
// buffers, a few sub-tiles ahead, with no staging registers; the barrier
// between sub-tiles waits for LDS only, each wave first waiting (vmcnt) for its
// own copies of the sub-tile it is about to read.  Row chunks are mapped
// XCD-aware: blocks on the same XCD work on the same chunk, so the 32 CUs of
// an XCD stream X through their shared L2 together.  Partials per chunk are
// summed in a fixed order by k_logreg_finish / k_lr16_lp_sum.
//
// Lane layouts (v_mfma_f32_16x16x32_bf16, checked on gfx950): A[i][k] at lane
// i + 16 (k / 8), element k % 8; B[k][j] at lane j + 16 (k / 8), element k % 8;
// D[i][j] in VGPR i % 4 of lane j + 16 (i / 4).
#include "hmc_internal.hpp"

namespace hmc {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx8 __attribute__((ext_vector_type(8)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4v __attribute__((ext_vector_type(4)));

constexpr int LB_NW = 4;      // waves per workgroup
constexpr int LB_RS = 32;     // rows per sub-tile
constexpr int LD_YB = 256;    // LDS bytes reserved for the labels of a sub-tile (32 used)

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

// eight floats to BF16, round to nearest even (v_cvt_pk_bf16_f32)
__device__ __forceinline__ bf16x8 pack_bf16(floatx8 f) {
    return __builtin_bit_cast(bf16x8, __builtin_convertvector(f, bf16x8v));
}
// four floats to BF16, packed in two dwords
__device__ __forceinline__ uint2 pack4_bf16(floatx4 f) {
    return __builtin_bit_cast(uint2, __builtin_convertvector(f, bf16x4v));
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

// ---------------------------------------------------------------------------
// Tile layouts in LDS (16-byte slots, XOR-swizzled so that the operand reads
// of the MFMAs spread over the LDS banks):
//   X   [32 rows][SR = DP / 8 slots]: slot c of row r at position c ^ xsw(r),
//       xsw(r) = (r & 3) | (bit 3 of r) << 2  (r & 3 when SR = 4)
//   X^T [DP dims][4 slots of 8 rows]: slot c of dim d at position c ^ ((d >> 1) & 3)
// The S halves take rows in the order 8 q + 4 mt + v (lane position i = 4 q + v
// of half mt), so lane group g holds the residuals of rows 8 g .. 8 g + 7 --
// rows 8 g + v from half 0, 8 g + 4 + v from half 1 -- which is the K order of
// the second contraction: its X^T operand is the one 16-byte slot g of a dim.
// ---------------------------------------------------------------------------
template <int SR>
__device__ __forceinline__ int lb_xsw(int r) {
    return SR >= 8 ? ((r & 3) | (((r >> 3) & 1) << 2)) : (r & 3);
}

// Copy of 1 KB block i of an X sub-tile (rows of the padded copy, stride DP)
// into xbase: lane ln writes position 64 i + ln of the tile's slot grid.
template <int KS>
__device__ __forceinline__ void lb_copy_x_block(const char* xsrc_t, uint8_t* __restrict__ xbase, int i, int ln) {
    constexpr int DP = 32 * KS, SR = DP / 8;
    const int q = i * 64 + ln;
    const int row = q / SR, c = (q % SR) ^ lb_xsw<SR>(row);
    const uint32_t off = (uint32_t)(row * (DP * 2) + 16 * c);
    __builtin_amdgcn_global_load_lds((const void*)(xsrc_t + off), (lds_void_t*)(xbase + i * 1024), 16, 0, 0);
}

// per-lane fragment offsets of the two S halves (even / odd k-step): row
// rho = 8 (l16 >> 2) + 4 mt + (l16 & 3), slot (4 ks + g) ^ xsw(rho) =
// 8 (ks >> 1) + 4 ((ks & 1) ^ rb) + (g ^ (sw & 3)) with sw = xsw(rho), rb = bit 2 of sw
template <int KS>
__device__ __forceinline__ void lb_xfrag_offsets(int l16, int g, uint32_t (&xoff)[2][2]) {
    constexpr int DP = 32 * KS, SR = DP / 8;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        const int row = 8 * (l16 >> 2) + 4 * mt + (l16 & 3);
        const int sw = lb_xsw<SR>(row);
        const int rb = (sw >> 2) & 1, gg = g ^ (sw & 3);
#pragma unroll
        for (int e = 0; e < 2; ++e) xoff[mt][e] = (uint32_t)(row * (DP * 2) + 16 * (4 * (e ^ rb) + gg));
    }
}

// theta (drifted when drift) of chain c as B operands B[k][j] = theta[j][k]:
// the 8 dims 32 ks + 8 g .. + 7 of k-step ks (zeros past D and for c >= C)
template <int KS>
__device__ __forceinline__ void lb_load_theta(const PlainArgs& a, const float* __restrict__ xsrc,
                                              const float* __restrict__ psrc, int drift, int64_t c, int g,
                                              floatx8 (&v)[KS]) {
    const int64_t D = a.tg.D;
    const bool cok = c < a.C;
    const float eps = cok ? (float)a.ws.eps[c] : 0.f;
    const float* xr = xsrc + (cok ? c : 0) * D;
    const float* pr = drift ? psrc + (cok ? c : 0) * D : nullptr;
    const bool vec = (D % 4) == 0;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int d0 = 32 * ks + 8 * g;
        floatx8 t = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (cok && vec && d0 + 8 <= D) {
            const float4 x0 = *(const float4*)(xr + d0), x1 = *(const float4*)(xr + d0 + 4);
            t = floatx8{x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
            if (drift) {
                const float4 p0 = *(const float4*)(pr + d0), p1 = *(const float4*)(pr + d0 + 4);
                const floatx8 pv = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w};
#pragma unroll
                for (int e = 0; e < 8; ++e) t[e] = fmaf(eps, pv[e], t[e]);
            }
        } else if (cok) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int d = d0 + e;
                float u = 0.f;
                if (d < D) {
                    u = xr[d];
                    if (drift) u = fmaf(eps, pr[d], u);
                }
                t[e] = u;
            }
        }
        v[ks] = t;
    }
}

// ---------------------------------------------------------------------------
// Gradient partials, software-pipelined: 16 CS chains per wave, NW waves per
// workgroup (LbGrad: 256 chains per workgroup up to D = 256, so at 8192 chains
// 32 chain tiles x 8 row splits = one workgroup per CU with each split on its
// own XCD; two waves per SIMD from D = 33 on).  The residuals of one sub-tile are
// formed on the vector ALUs while the matrix cores run the other contraction,
// in three phases per sub-tile s:
//   1. the X fragments of rows 0..15 of s are read, the residuals of rows
//      16..31 of s - 1 computed while they arrive, then S of rows 0..15
//   2. the X fragments of rows 16..31 of s are read; G^T += R^T X^T of s - 1,
//      with the residuals of rows 0..15 of s computed between its MFMAs
//   3. S of rows 16..31 of s
// X^T of sub-tile s - 1 is still read in the iteration of s, so the X^T tiles
// sit in a ring of NBX + 1 buffers and the X tiles in a ring of NBX (4, or 2
// beyond D = 256 where two X tiles and three X^T tiles of 32 KB fill the
// 160 KB); the copies run NBX - 1 sub-tiles ahead.  The labels of a sub-tile are
// copied beside its X^T tile, or (NBX = 2) read from global memory by each lane.
// ---------------------------------------------------------------------------
template <int KS>
struct LbGrad {
    // waves per workgroup and 16-chain tiles per wave: eight waves (two per SIMD, so that
    // one's residual work overlaps the other's MFMAs) of 32 chains from D = 33 to 256 and
    // of 16 beyond (theta and G^T of wider chains fill the registers); up to D = 32, whose
    // sub-tile has too few copies for eight waves, four of 64
    static constexpr int NW = KS >= 2 ? 8 : 4;
    static constexpr int CS = KS == 1 ? 4 : (KS <= 8 ? 2 : 1);
    static constexpr int CT = NW * 16 * CS;               // chains per workgroup
    static constexpr int NBX = KS <= 8 ? 4 : 2;           // X buffers
    static constexpr int NBT = NBX + 1;                   // X^T buffers
    static constexpr int PF = NBX - 1;                    // sub-tiles copied ahead
    static constexpr bool YLDS = NBX > 2;                 // labels copied to LDS
    static constexpr int DP = 32 * KS;
    static constexpr int XB = LB_RS * DP * 2;             // bytes of an X (or X^T) sub-tile
    static constexpr int TBY = XB + (YLDS ? LD_YB : 0);   // X^T sub-tile + labels
    static constexpr int XI = XB / 1024;                  // 1 KB copy blocks of a tile
    static constexpr int JW = (2 * XI) / NW;              // tile copies per wave
    static constexpr int J = JW + (YLDS ? 1 : 0);         // copy instructions per wave and sub-tile
    static constexpr int LDS = NBX * XB + NBT * TBY;
};

template <int KS>
__device__ __forceinline__ void lr16_grad_body(const PlainArgs& a, const float* __restrict__ xsrc,
                                               const float* __restrict__ psrc, int drift, int64_t rows_per_split,
                                               int nsplit, int blk) {
    using P = LbGrad<KS>;
    constexpr int CS = P::CS, CT = P::CT, NT = 2 * KS, DP = P::DP, XB = P::XB, TBY = P::TBY, XI = P::XI;
    constexpr int JW = P::JW, J = P::J, PF = P::PF, NBX = P::NBX, NBT = P::NBT, NW = P::NW;
    static_assert((2 * XI) % NW == 0, "copies must split evenly over the waves");
    static_assert(P::LDS <= 160 * 1024, "LDS");
    extern __shared__ __align__(16) uint8_t ldsb[];
    uint8_t* xring = ldsb;                      // [NBX][XB]
    uint8_t* tring = ldsb + NBX * XB;           // [NBT][TBY]

    const int64_t D = a.tg.D, C = a.C, NP = (a.tg.N + LB_RS - 1) / LB_RS * LB_RS;
    const int ntile = (int)((C + CT - 1) / CT);
    int tile, split;
    lb_map(blk, ntile, nsplit, &tile, &split);
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int l16 = lane & 15, g = lane >> 4;
    const int64_t cw = (int64_t)tile * CT + 16 * CS * w;
    const uint16_t* Xp = (const uint16_t*)a.ws.xp;
    const uint16_t* Xt = (const uint16_t*)a.ws.xt;
    const uint8_t* Yp = (const uint8_t*)a.ws.yp;

    bf16x8 thb[CS][KS];
#pragma unroll
    for (int cs = 0; cs < CS; ++cs) {
        floatx8 v[KS];
        lb_load_theta<KS>(a, xsrc, psrc, drift, cw + 16 * cs + l16, g, v);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) thb[cs][ks] = pack_bf16(v[ks]);
    }

    const int64_t r_begin = (int64_t)split * rows_per_split;
    int64_t r_end = r_begin + rows_per_split;
    if (r_end > NP) r_end = NP;
    const int nsub = r_begin < r_end ? (int)((r_end - r_begin) / LB_RS) : 0;

    // copies of sub-tile sidx: X into xbase, X^T (and the labels) into tbase
    auto copy_in = [&](int sidx, uint8_t* __restrict__ xbase, uint8_t* __restrict__ tbase) {
        const int64_t r0 = r_begin + (int64_t)sidx * LB_RS;
        const char* xsrc_t = (const char*)(Xp + r0 * DP);
        const char* tsrc_t = (const char*)(Xt + r0);
        // the lane index through an empty asm: the per-lane offsets are recomputed
        // for every sub-tile instead of being hoisted out of the loop (and spilled:
        // a reload's wait would also wait for the copies in flight)
        int ln = lane;
        asm volatile("" : "+v"(ln));
        const uint32_t toff = (uint32_t)(ln >> 2) * (uint32_t)NP * 2u + 16u * (uint32_t)((ln & 3) ^ ((ln >> 3) & 3));
        // with SR dividing 64 the row of lane ln in copy k is A + (64 NW / SR) k, A below,
        // with no carry from A's low bits into bit 3, so its swizzle depends on k only
        // through bit 3 of (64 NW / SR) k -- two offsets per sub-tile
        constexpr int SR = DP / 8;
        constexpr bool POW2 = (64 % SR) == 0;
        constexpr int KSTR = 64 * NW / SR;
        static_assert(!POW2 || KSTR % 8 == 0 || (KSTR == 4 && NW == 4), "row stride of the copies");
        uint32_t xo[2] = {0u, 0u};
        if constexpr (POW2) {
            const int arow = (64 / SR) * w + ln / SR;
#pragma unroll
            for (int par = 0; par < 2; ++par) {
                const int sw = SR >= 8 ? ((arow & 3) | ((((arow >> 3) & 1) ^ par) << 2)) : (arow & 3);
                xo[par] = (uint32_t)(ln / SR) * (uint32_t)(DP * 2) + 16u * (uint32_t)((ln % SR) ^ sw);
            }
        }
#pragma unroll
        for (int k = 0; k < JW; ++k) {
            const int i = w + NW * k;
            const bool isx = (XI % NW == 0) ? (k < XI / NW) : (i < XI);
            if (isx) {
                if constexpr (POW2)
                    __builtin_amdgcn_global_load_lds((const void*)(xsrc_t + (uint32_t)i * 1024u +
                                                                   xo[((KSTR * k) >> 3) & 1]),
                                                     (lds_void_t*)(xbase + i * 1024), 16, 0, 0);
                else
                    lb_copy_x_block<KS>(xsrc_t, xbase, i, ln);
            } else {
                const int ii = i - XI;
                __builtin_amdgcn_global_load_lds((const void*)(tsrc_t + (uint32_t)(16 * ii) * (uint32_t)NP * 2u + toff),
                                                 (lds_void_t*)(tbase + ii * 1024), 16, 0, 0);
            }
        }
        if constexpr (P::YLDS)
            __builtin_amdgcn_global_load_lds((const void*)(Yp + r0 + 4 * (ln & 7)), (lds_void_t*)(tbase + XB), 4, 0,
                                             0);
    };
    auto xbuf = [&](int sidx) { return xring + (sidx % NBX) * XB; };
    auto tbuf = [&](int sidx) { return tring + (sidx % NBT) * TBY; };
    // labels of the lane's rows 8 g .. 8 g + 7 of sub-tile sidx
    auto labels = [&](int sidx, const uint8_t* tb) {
        if constexpr (P::YLDS) return *(const uint2*)(tb + XB + 8 * g);
        else return *(const uint2*)(Yp + r_begin + (int64_t)sidx * LB_RS + 8 * g);
    };

    uint32_t xoff[2][2];
    lb_xfrag_offsets<KS>(l16, g, xoff);
    const uint32_t toff_f = (uint32_t)(l16 * 64 + 16 * (g ^ ((l16 >> 1) & 3)));
    auto xfrag = [&](const uint8_t* xb, const uint32_t* o2, int ks) {
        return *(const bf16x8*)(xb + o2[ks & 1] + 128 * (ks >> 1));
    };
    // residuals of one 16-row half (the lane's rows 8 g + 4 mt + v)
    auto resid = [&](floatx4 sv, uint32_t yw) {
        floatx4 r;
#pragma unroll
        for (int v = 0; v < 4; ++v) r[v] = (float)((yw >> (8 * v)) & 0xffu) - sigmoid_hw(sv[v]);
        return pack4_bf16(r);
    };
    // S of one half from fragments read ahead (all of them up to KS = 8, else
    // eight in flight)
    constexpr int FA = KS < 8 ? KS : 8;
    auto sphase = [&](const uint8_t* __restrict__ xb, const uint32_t* o2, floatx4* sacc) {
        bf16x8 xa[FA];
#pragma unroll
        for (int ks = 0; ks < FA; ++ks) xa[ks] = xfrag(xb, o2, ks);
#pragma unroll
        for (int cs = 0; cs < CS; ++cs) sacc[cs] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const bf16x8 ax = xa[ks % FA];
            if (ks + FA < KS) xa[ks % FA] = xfrag(xb, o2, ks + FA);
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
        auto tfrag = [&](int nt) { return *(const bf16x8*)(tb + to + 1024 * nt); };
        bf16x8 tf0 = tfrag(0), tf1 = tfrag(1);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const bf16x8 bx = tf0;
            tf0 = tf1;
            if (nt + 2 < NT) tf1 = tfrag(nt + 2);
#pragma unroll
            for (int cs = 0; cs < CS; ++cs)
                gacc[cs][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ra[cs], bx, gacc[cs][nt], 0, 0, 0);
        }
    };

#pragma unroll
    for (int t = 0; t < PF; ++t)
        if (t < nsub) copy_in(t, xbuf(t), tbuf(t));
    // sub-tile sidx complete: the copies of the following PF - 1 may stay outstanding
    auto wait_tile = [&](int sidx) {
        if constexpr (PF >= 3) {
            if (sidx + 2 < nsub) wait_vmcnt<2 * J>();
            else if (sidx + 1 < nsub) wait_vmcnt<J>();
            else wait_vmcnt<0>();
        } else if constexpr (PF == 2) {
            if (sidx + 1 < nsub) wait_vmcnt<J>();
            else wait_vmcnt<0>();
        } else {
            wait_vmcnt<0>();
        }
        lds_barrier();
    };

    // pipeline registers: S of rows 16..31 of the previous sub-tile, the packed
    // residuals of its rows 0..15 and its labels of rows 16..31
    floatx4 s1p[CS];
    uint2 lo_p[CS];
    uint32_t yp1 = 0u;
    if (nsub > 0) {       // the first sub-tile: no G of a previous one
        wait_tile(0);
        const uint2 yl = labels(0, tbuf(0));
        if (PF < nsub) copy_in(PF, xbuf(PF), tbuf(PF));
        yp1 = yl.y;
        floatx4 s0[CS];
        sphase(xbuf(0), xoff[0], s0);
#pragma unroll
        for (int cs = 0; cs < CS; ++cs) lo_p[cs] = resid(s0[cs], yl.x);
        sphase(xbuf(0), xoff[1], s1p);
    }
    // one sub-tile; the copy targets (xdst, tdst) and the buffers read (xb, tprev,
    // tcur) are distinct, which the restrict qualifiers tell the compiler, so the
    // LDS reads need not wait for the copies in flight (the explicit vmcnt waits
    // and the barrier order the sub-tiles)
    auto iter = [&](int sidx, uint8_t* __restrict__ xdst, uint8_t* __restrict__ tdst, const uint8_t* __restrict__ xb,
                    const uint8_t* __restrict__ tprev, const uint8_t* __restrict__ tcur) {
        // the labels first: a global read of them then waits only on older copies
        const uint2 yl = labels(sidx, tcur);
        if (sidx + PF < nsub) copy_in(sidx + PF, xdst, tdst);
        // phase 1; a phase's base offsets pass through one empty asm at its start, so
        // that a register per offset plus immediate offsets address its fragments
        uint32_t o1[2] = {xoff[0][0], xoff[0][1]};
        asm volatile("" : "+v"(o1[0]), "+v"(o1[1]));
        bf16x8 xa[FA];
#pragma unroll
        for (int ks = 0; ks < FA; ++ks) xa[ks] = xfrag(xb, o1, ks);
        bf16x8 rp[CS];
#pragma unroll
        for (int cs = 0; cs < CS; ++cs) {
            const uint2 hi = resid(s1p[cs], yp1);
            rp[cs] = __builtin_bit_cast(bf16x8, make_uint4(lo_p[cs].x, lo_p[cs].y, hi.x, hi.y));
        }
        floatx4 s0[CS];
#pragma unroll
        for (int cs = 0; cs < CS; ++cs) s0[cs] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const bf16x8 ax = xa[ks % FA];
            if (ks + FA < KS) xa[ks % FA] = xfrag(xb, o1, ks + FA);
#pragma unroll
            for (int cs = 0; cs < CS; ++cs)
                s0[cs] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, thb[cs][ks], s0[cs], 0, 0, 0);
        }
        // phase 2
        uint32_t o2[2] = {xoff[1][0], xoff[1][1]}, ot = toff_f;
        asm volatile("" : "+v"(o2[0]), "+v"(o2[1]), "+v"(ot));
        bf16x8 xb1[FA];
#pragma unroll
        for (int ks = 0; ks < FA; ++ks) xb1[ks] = xfrag(xb, o2, ks);
        gphase(tprev, rp, ot);
#pragma unroll
        for (int cs = 0; cs < CS; ++cs) lo_p[cs] = resid(s0[cs], yl.x);
        // phase 3
#pragma unroll
        for (int cs = 0; cs < CS; ++cs) s1p[cs] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const bf16x8 ax = xb1[ks % FA];
            if (ks + FA < KS) xb1[ks % FA] = xfrag(xb, o2, ks + FA);
#pragma unroll
            for (int cs = 0; cs < CS; ++cs)
                s1p[cs] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, thb[cs][ks], s1p[cs], 0, 0, 0);
        }
        yp1 = yl.y;
    };
    for (int sidx = 1; sidx < nsub; ++sidx) {
        wait_tile(sidx);
        iter(sidx, xbuf(sidx + PF), tbuf(sidx + PF), xbuf(sidx), tbuf(sidx + NBT - 1), tbuf(sidx));
    }
    if (nsub > 0) {
        bf16x8 rp[CS];
#pragma unroll
        for (int cs = 0; cs < CS; ++cs) {
            const uint2 hi = resid(s1p[cs], yp1);
            rp[cs] = __builtin_bit_cast(bf16x8, make_uint4(lo_p[cs].x, lo_p[cs].y, hi.x, hi.y));
        }
        gphase(tbuf(nsub - 1), rp, toff_f);
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
// Accurate log-probability partials: theta = hi + mid + lo (three BF16 terms,
// smallest first), 16 chains per wave, each X fragment feeding 3 MFMAs; the
// softplus terms summed per chain in FP64.  Pipelined
// like the gradient: the softplus of one 16-row half is computed while the
// fragments of the next half arrive and before its MFMAs.  X tiles (with their
// labels) in a ring of four buffers, copies three sub-tiles ahead.
// ---------------------------------------------------------------------------
template <int KS>
struct LbLogp {
    // eight waves of 16 chains (two waves per SIMD)
    static constexpr int NW = 8;
    static constexpr int CS = 1;
    static constexpr int CT = NW * 16 * CS;
    static constexpr int NB = 4;
    static constexpr int DP = 32 * KS;
    static constexpr int XB = LB_RS * DP * 2;
    static constexpr int BUF = XB + LD_YB;
    static constexpr int XI = XB / 1024;
    static constexpr int JW = (XI + NW - 1) / NW;         // X copy instructions per wave (a wave may repeat one)
    static constexpr int J = JW + 1;                      // plus the labels
    static constexpr int LDS = NB * BUF;
};

template <int KS>
__device__ __forceinline__ void lr16_logp_body(const PlainArgs& a, const float* __restrict__ xsrc,
                                               int64_t rows_per_split, int nsplit, int blk) {
    using P = LbLogp<KS>;
    constexpr int CS = P::CS, CT = P::CT, NB = P::NB, XB = P::XB, BUF = P::BUF, XI = P::XI, JW = P::JW, J = P::J;
    constexpr int DP = P::DP;
    static_assert(P::LDS <= 160 * 1024, "LDS");
    extern __shared__ __align__(16) uint8_t ldsb[];

    const int64_t N = a.tg.N, C = a.C, NP = (N + LB_RS - 1) / LB_RS * LB_RS;
    const int ntile = (int)((C + CT - 1) / CT);
    int tile, split;
    lb_map(blk, ntile, nsplit, &tile, &split);
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int l16 = lane & 15, g = lane >> 4;
    const int64_t cw = (int64_t)tile * CT + 16 * CS * w;
    const uint16_t* Xp = (const uint16_t*)a.ws.xp;
    const uint8_t* Yp = (const uint8_t*)a.ws.yp;

    // theta = hi + mid + lo, three BF16 B operands per chain tile and k-step
    bf16x8 th[3][CS][KS];
#pragma unroll
    for (int cs = 0; cs < CS; ++cs) {
        floatx8 v[KS];
        lb_load_theta<KS>(a, xsrc, nullptr, 0, cw + 16 * cs + l16, g, v);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            floatx8 r1, r2;
            const bf16x8 h = pack_bf16(v[ks]);
#pragma unroll
            for (int e = 0; e < 8; ++e) r1[e] = v[ks][e] - bf16_to_f32((uint16_t)h[e]);
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
    if (r_end > NP) r_end = NP;
    const int nsub = r_begin < r_end ? (int)((r_end - r_begin) / LB_RS) : 0;

    auto copy_in = [&](int sidx, uint8_t* __restrict__ base) {
        const int64_t r0 = r_begin + (int64_t)sidx * LB_RS;
        const char* xsrc_t = (const char*)(Xp + r0 * DP);
        int ln = lane;
        asm volatile("" : "+v"(ln));
#pragma unroll
        for (int k = 0; k < JW; ++k) {
            int i = w + P::NW * k;
            if (i >= XI) i = XI - 1;          // a repeated copy keeps the count equal over the waves
            lb_copy_x_block<KS>(xsrc_t, base, i, ln);
        }
        __builtin_amdgcn_global_load_lds((const void*)(Yp + r0 + 4 * (ln & 7)), (lds_void_t*)(base + XB), 4, 0, 0);
    };
    uint32_t xoff[2][2];
    lb_xfrag_offsets<KS>(l16, g, xoff);
    auto xfrag = [&](const uint8_t* xb, const uint32_t* o2, int ks) {
        return *(const bf16x8*)(xb + o2[ks & 1] + 128 * (ks >> 1));
    };
    // log-likelihood terms of one half, y s - softplus(s), for the lane's rows
    // row0 + v (rows at or past N skipped when the sub-tile reaches them); a
    // lane's four terms are added in FP32 before the FP64 sum (a rounding of
    // about 1e-7 of a few terms, far below what the accept test resolves)
    double lp[CS] = {};
    auto accum = [&](const floatx4* sv, uint32_t yw, int64_t row0) {
        const bool whole = row0 + 4 <= N;
#pragma unroll
        for (int cs = 0; cs < CS; ++cs) {
            float t4 = 0.f;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float s = sv[cs][v];
                const float y = (float)((yw >> (8 * v)) & 0xffu);
                const float t = fmaf(y, s, -softplus_hw(s));
                t4 += (whole || row0 + v < N) ? t : 0.f;
            }
            lp[cs] += (double)t4;
        }
    };
    constexpr int FA = KS < 8 ? KS : 8;
    auto shalf = [&](const uint8_t* __restrict__ xb, const uint32_t* o2, floatx4* sacc) {
#pragma unroll
        for (int cs = 0; cs < CS; ++cs) sacc[cs] = floatx4{0.f, 0.f, 0.f, 0.f};
        bf16x8 xa[FA];
#pragma unroll
        for (int ks = 0; ks < FA; ++ks) xa[ks] = xfrag(xb, o2, ks);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const bf16x8 ax = xa[ks % FA];
            if (ks + FA < KS) xa[ks % FA] = xfrag(xb, o2, ks + FA);
#pragma unroll
            for (int term = 2; term >= 0; --term)
#pragma unroll
                for (int cs = 0; cs < CS; ++cs)
                    sacc[cs] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, th[term][cs][ks], sacc[cs], 0, 0, 0);
        }
    };

#pragma unroll
    for (int t = 0; t < NB - 1; ++t)
        if (t < nsub) copy_in(t, ldsb + t * BUF);
    floatx4 sprev[CS];
    uint32_t yprev = 0u;
    int64_t rowprev = 0;
    bool have_prev = false;
    auto step = [&](int sidx, uint8_t* __restrict__ nxt, const uint8_t* __restrict__ base) {
        if (sidx + NB - 1 < nsub) copy_in(sidx + NB - 1, nxt);
        const int64_t r0 = r_begin + (int64_t)sidx * LB_RS;
        const uint2 yl = *(const uint2*)(base + XB + 8 * g);
        // half 0 of this sub-tile, with the previous half's softplus while its fragments arrive
        uint32_t o1[2] = {xoff[0][0], xoff[0][1]};
        asm volatile("" : "+v"(o1[0]), "+v"(o1[1]));
        floatx4 s0[CS];
        if (have_prev) accum(sprev, yprev, rowprev);
        shalf(base, o1, s0);
        // half 1, with half 0's softplus
        uint32_t o2[2] = {xoff[1][0], xoff[1][1]};
        asm volatile("" : "+v"(o2[0]), "+v"(o2[1]));
        accum(s0, yl.x, r0 + 8 * g);
        shalf(base, o2, sprev);
        yprev = yl.y;
        rowprev = r0 + 8 * g + 4;
        have_prev = true;
    };
    for (int sidx = 0; sidx < nsub; ++sidx) {
        if (sidx + 2 < nsub) wait_vmcnt<2 * J>();
        else if (sidx + 1 < nsub) wait_vmcnt<J>();
        else wait_vmcnt<0>();
        lds_barrier();
        step(sidx, ldsb + ((sidx + NB - 1) % NB) * BUF, ldsb + (sidx % NB) * BUF);
    }
    if (have_prev) accum(sprev, yprev, rowprev);
    // lanes holding chain l16: l16, l16 + 16, + 32, + 48
#pragma unroll
    for (int cs = 0; cs < CS; ++cs) {
        double v = lp[cs];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        const int64_t c = cw + 16 * cs + l16;
        if (g == 0 && c < C) a.ws.part_lp[(int64_t)split * C + c] = v;
    }
}

// lpq[c] = sum over splits (fixed order) of the log-probability partials
__device__ __forceinline__ void lr16_lp_sum_body(const PlainArgs& a, int nsplit, int blk) {
    const int64_t c = (int64_t)blk * blockDim.x + threadIdx.x;
    if (c >= a.C) return;
    double l = 0.0;
    for (int s = 0; s < nsplit; ++s) l += a.ws.part_lp[(int64_t)s * a.C + c];
    a.ws.lpq[c] = l;
}

template <int KS>
__global__ __launch_bounds__(64 * LbGrad<KS>::NW) void k_lr16_grad_pipe(PlainArgs a, const float* __restrict__ xsrc,
                                                        const float* __restrict__ psrc, int drift,
                                                        int64_t rows_per_split, int nsplit) {
    lr16_grad_body<KS>(a, xsrc, psrc, drift, rows_per_split, nsplit, blockIdx.x);
}

template <int KS>
__global__ __launch_bounds__(64 * LbLogp<KS>::NW) void k_lr16_logp_pipe(PlainArgs a, const float* __restrict__ xsrc,
                                                        int64_t rows_per_split, int nsplit) {
    lr16_logp_body<KS>(a, xsrc, rows_per_split, nsplit, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_lr16_lp_sum(PlainArgs a, int nsplit) { lr16_lp_sum_body(a, nsplit, blockIdx.x); }

// ---------------------------------------------------------------------------
// Several requests in one launch (the serving form): job j owns blocks
// begin[k] .. begin[k] + nblk[k] - 1 of the grid of kernel kind k; its
// arguments are copied out of the device job table into registers, and the
// body is the one-request kernel's with the job-local block index, so every
// request computes bitwise what it computes alone.
// ---------------------------------------------------------------------------
template <int KS>
__global__ __launch_bounds__(64 * LbGrad<KS>::NW) void k_lr16_grad_multi(const Lr16Job* __restrict__ jobs, int njobs) {
    int64_t lb;
    const int j = lr16_job_of(jobs, njobs, LR16_KIND_GRAD, blockIdx.x, &lb);
    if (j < 0) return;
    const PlainArgs a = jobs[j].a;
    lr16_grad_body<KS>(a, (const float*)a.ws.xq, (const float*)a.ws.pq, 1, jobs[j].rows_g, jobs[j].nsplit_g, (int)lb);
}

template <int KS>
__global__ __launch_bounds__(64 * LbLogp<KS>::NW) void k_lr16_logp_multi(const Lr16Job* __restrict__ jobs, int njobs) {
    int64_t lb;
    const int j = lr16_job_of(jobs, njobs, LR16_KIND_LOGP, blockIdx.x, &lb);
    if (j < 0) return;
    const PlainArgs a = jobs[j].a;
    lr16_logp_body<KS>(a, (const float*)a.ws.xq, jobs[j].rows_lp, jobs[j].nsplit_lp, (int)lb);
}

__global__ __launch_bounds__(256) void k_lr16_lp_sum_multi(const Lr16Job* __restrict__ jobs, int njobs) {
    int64_t lb;
    const int j = lr16_job_of(jobs, njobs, LR16_KIND_LPSUM, blockIdx.x, &lb);
    if (j < 0) return;
    const PlainArgs a = jobs[j].a;
    lr16_lp_sum_body(a, jobs[j].nsplit_lp, (int)lb);
}

// Padded copies: X [N, D] -> Xp [NP, DP] and Xt [DP, NP] (zeros outside), y -> yp
// [NP] (zeros past N); 32 x 32 tiles through LDS for the transpose.
__global__ __launch_bounds__(256) void k_pad_bf16(const uint16_t* __restrict__ X, const uint8_t* __restrict__ y,
                                                  uint16_t* __restrict__ Xp, uint16_t* __restrict__ Xt,
                                                  uint8_t* __restrict__ yp, int64_t N, int64_t D, int64_t NP,
                                                  int64_t DP) {
    __shared__ uint16_t tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int64_t n0 = (int64_t)blockIdx.x * 32, d0 = (int64_t)blockIdx.y * 32;
    for (int r = ty; r < 32; r += 8) {
        const int64_t n = n0 + r, d = d0 + tx;
        const uint16_t v = (n < N && d < D) ? X[n * D + d] : (uint16_t)0;
        tile[r][tx] = v;
        Xp[n * DP + d] = v;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) Xt[(d0 + r) * NP + n0 + tx] = tile[tx][r];
    if (blockIdx.y == 0 && threadIdx.x < 32) {
        const int64_t n = n0 + threadIdx.x;
        yp[n] = n < N ? y[n] : (uint8_t)0;
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
// 32-dim k-steps of the padded dims for D dims (0 beyond 512)
static int lb_ks(int64_t D) {
    const int64_t k = (D + 31) / 32;
    for (int v : {1, 2, 4, 6, 8, 12, 16})
        if (k <= v) return v;
    return 0;
}

bool bf16_grad_supported(const TargetDev& tg) { return tg.kind == HMC_TGT_LOGREG && tg.x_bf16 && lb_ks(tg.D) > 0; }

size_t lb_pad_bytes(int64_t N, int64_t D, int64_t* np, int64_t* dp) {
    const int64_t NP = (N + LB_RS - 1) / LB_RS * LB_RS, DP = 32 * (int64_t)lb_ks(D);
    if (np) *np = NP;
    if (dp) *dp = DP;
    return (size_t)NP * (size_t)DP * 2;
}

static int lb_grad_ct(int64_t D) { return lb_ks(D) <= 8 ? LbGrad<8>::CT : LbGrad<16>::CT; }
static int lb_logp_ct(int64_t D) { return lb_ks(D) <= 8 ? LbLogp<8>::CT : LbLogp<16>::CT; }

// row splits: a power of two (so that blocks map to XCDs by split) filling the
// 256 CUs once, at most 8, at least 4 sub-tiles each
static int lb_nsplit_for(int ntile, int64_t N) {
    int s = 1;
    while (s < 8 && ntile * 2 * s <= 256 && (N + 2 * s - 1) / (2 * s) >= 4 * LB_RS) s *= 2;
    return s;
}
int lb_grad_nsplit(int64_t N, int64_t C, int64_t D) {
    const int ct = lb_grad_ct(D);
    return lb_nsplit_for((int)((C + ct - 1) / ct), N);
}
int lb_grad_nsplit_t(const PlainArgs& a) {
    return a.tune.lr16_nsplit > 0 ? a.tune.lr16_nsplit : lb_grad_nsplit(a.tg.N, a.C, a.tg.D);
}
int lb_logp_nsplit(int64_t N, int64_t C, int64_t D) {
    const int ct = lb_logp_ct(D);
    return lb_nsplit_for((int)((C + ct - 1) / ct), N);
}

static int64_t rows_for(int64_t N, int nsplit) {
    const int64_t r = (N + nsplit - 1) / nsplit;
    return (r + LB_RS - 1) / LB_RS * LB_RS;
}

hipError_t launch_pad_bf16(const PlainArgs& a, hipStream_t s) {
    int64_t NP = 0, DP = 0;
    (void)lb_pad_bytes(a.tg.N, a.tg.D, &NP, &DP);
    const dim3 grid((unsigned)(NP / 32), (unsigned)(DP / 32));
    hipLaunchKernelGGL(k_pad_bf16, grid, dim3(256), 0, s, (const uint16_t*)a.tg.X, a.tg.y, (uint16_t*)a.ws.xp,
                       (uint16_t*)a.ws.xt, (uint8_t*)a.ws.yp, a.tg.N, a.tg.D, NP, DP);
    return hipGetLastError();
}

template <int KS>
static hipError_t lb_grad_k(const PlainArgs& a, const float* x, const float* p, int drift, hipStream_t s) {
    using P = LbGrad<KS>;
    const int ntile = (int)((a.C + P::CT - 1) / P::CT);
    const int nsplit = lb_grad_nsplit_t(a);
    const int64_t NP = (a.tg.N + LB_RS - 1) / LB_RS * LB_RS;
    const size_t lds = (size_t)P::LDS;
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void*)k_lr16_grad_pipe<KS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
    hipLaunchKernelGGL(k_lr16_grad_pipe<KS>, dim3((unsigned)(ntile * nsplit)), dim3(64 * P::NW), lds, s, a, x, p,
                       drift, rows_for(NP, nsplit), nsplit);
    return hipGetLastError();
}

template <int KS>
static hipError_t lb_logp_k(const PlainArgs& a, const float* x, hipStream_t s) {
    using P = LbLogp<KS>;
    const int ntile = (int)((a.C + P::CT - 1) / P::CT);
    const int nsplit = lb_logp_nsplit(a.tg.N, a.C, a.tg.D);
    const int64_t NP = (a.tg.N + LB_RS - 1) / LB_RS * LB_RS;
    const size_t lds = (size_t)P::LDS;
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void*)k_lr16_logp_pipe<KS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
    hipLaunchKernelGGL(k_lr16_logp_pipe<KS>, dim3((unsigned)(ntile * nsplit)), dim3(64 * P::NW), lds, s, a, x,
                       rows_for(NP, nsplit), nsplit);
    hipLaunchKernelGGL(k_lr16_lp_sum, dim3((unsigned)((a.C + 255) / 256)), dim3(256), 0, s, a, nsplit);
    return hipGetLastError();
}

int lr16_batch_class(const PlainArgs& a) {
    if (a.tg.kind != HMC_TGT_LOGREG || !a.bf16_grad || a.f64) return -1;
    const int ks = lb_ks(a.tg.D);
    return ks > 0 ? ks : -1;
}

void lr16_job_shape(const PlainArgs& a, Lr16Job* j) {
    const int64_t NP = (a.tg.N + LB_RS - 1) / LB_RS * LB_RS;
    j->nsplit_g = lb_grad_nsplit_t(a);
    j->nsplit_lp = lb_logp_nsplit(a.tg.N, a.C, a.tg.D);
    j->rows_g = rows_for(NP, j->nsplit_g);
    j->rows_lp = rows_for(NP, j->nsplit_lp);
    const int64_t ctg = lb_grad_ct(a.tg.D), ctl = lb_logp_ct(a.tg.D);
    j->nblk[LR16_KIND_GRAD] = (a.C + ctg - 1) / ctg * j->nsplit_g;
    j->nblk[LR16_KIND_LOGP] = (a.C + ctl - 1) / ctl * j->nsplit_lp;
    j->nblk[LR16_KIND_LPSUM] = (a.C + 255) / 256;
}

template <int KS>
static hipError_t lb_multi_k(int kind, const Lr16Job* jobs, int njobs, int64_t blocks, hipStream_t s) {
    const dim3 grid((unsigned)blocks);
    if (kind == LR16_KIND_GRAD) {
        const size_t lds = (size_t)LbGrad<KS>::LDS;
        if (lds > 65536)
            (void)hipFuncSetAttribute((const void*)k_lr16_grad_multi<KS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds);
        hipLaunchKernelGGL(k_lr16_grad_multi<KS>, grid, dim3(64 * LbGrad<KS>::NW), lds, s, jobs, njobs);
    } else if (kind == LR16_KIND_LOGP) {
        const size_t lds = (size_t)LbLogp<KS>::LDS;
        if (lds > 65536)
            (void)hipFuncSetAttribute((const void*)k_lr16_logp_multi<KS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds);
        hipLaunchKernelGGL(k_lr16_logp_multi<KS>, grid, dim3(64 * LbLogp<KS>::NW), lds, s, jobs, njobs);
    } else {
        hipLaunchKernelGGL(k_lr16_lp_sum_multi, grid, dim3(256), 0, s, jobs, njobs);
    }
    return hipGetLastError();
}

hipError_t launch_lr16_kind_multi(int kind, int64_t D, const Lr16Job* jobs_dev, int njobs, int64_t blocks,
                                  hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    switch (lb_ks(D)) {
    case 1: return lb_multi_k<1>(kind, jobs_dev, njobs, blocks, s);
    case 2: return lb_multi_k<2>(kind, jobs_dev, njobs, blocks, s);
    case 4: return lb_multi_k<4>(kind, jobs_dev, njobs, blocks, s);
    case 6: return lb_multi_k<6>(kind, jobs_dev, njobs, blocks, s);
    case 8: return lb_multi_k<8>(kind, jobs_dev, njobs, blocks, s);
    case 12: return lb_multi_k<12>(kind, jobs_dev, njobs, blocks, s);
    case 16: return lb_multi_k<16>(kind, jobs_dev, njobs, blocks, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_lr16_grad(const PlainArgs& a, const float* x, const float* p, int drift, hipStream_t s) {
    switch (lb_ks(a.tg.D)) {
    case 1: return lb_grad_k<1>(a, x, p, drift, s);
    case 2: return lb_grad_k<2>(a, x, p, drift, s);
    case 4: return lb_grad_k<4>(a, x, p, drift, s);
    case 6: return lb_grad_k<6>(a, x, p, drift, s);
    case 8: return lb_grad_k<8>(a, x, p, drift, s);
    case 12: return lb_grad_k<12>(a, x, p, drift, s);
    case 16: return lb_grad_k<16>(a, x, p, drift, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_lr16_logp(const PlainArgs& a, const float* x, hipStream_t s) {
    switch (lb_ks(a.tg.D)) {
    case 1: return lb_logp_k<1>(a, x, s);
    case 2: return lb_logp_k<2>(a, x, s);
    case 4: return lb_logp_k<4>(a, x, s);
    case 6: return lb_logp_k<6>(a, x, s);
    case 8: return lb_logp_k<8>(a, x, s);
    case 12: return lb_logp_k<12>(a, x, s);
    case 16: return lb_logp_k<16>(a, x, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hmc
