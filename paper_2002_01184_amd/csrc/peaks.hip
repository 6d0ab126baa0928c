// peaks.hip -- microbenchmarks of the achievable peaks that the roofline
// figures are set against: streaming read and copy bandwidth of a buffer
// (HBM, or the Infinity Cache / L2 when the buffer fits and is read several
// times per launch) and the issue rate of the matrix and vector instructions
// the sampler's kernels use.  Timed with HIP events on the caller's stream.
#include "hmc_internal.hpp"

namespace hmc {

// Written only when a sum equals an impossible pattern: keeps the loads and
// the arithmetic alive without a store per thread (external linkage, so that
// the stores, and what they depend on, are not removed as dead).
__device__ float g_peak_sink;
// Shader-clock and 100 MHz real-time counters of one wave at the start and end of a compute launch.
__device__ uint64_t g_peak_clk[4];

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr float kNever = -1.2345e-31f;

// one 16-byte load; NT: non-temporal (streamed data, not kept in the caches)
template <bool NT>
__device__ __forceinline__ floatx4 ld16(const floatx4* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// Grid-stride read of n4 16-byte vectors, `passes` times, eight loads in
// flight per thread (non-temporal for a single pass over a buffer larger than
// the caches, cached when the buffer is read again).
template <bool NT>
__global__ __launch_bounds__(256) void k_peak_read(const floatx4* __restrict__ src, int64_t n4, int passes) {
    constexpr int U = 8;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int ps = 0; ps < passes; ++ps) {
        int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        for (; i + (U - 1) * stride < n4; i += U * stride) {
            floatx4 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = ld16<NT>(src + i + u * stride);
#pragma unroll
            for (int u = 0; u < U; ++u) acc += v[u];
        }
        for (; i < n4; i += stride) acc += ld16<NT>(src + i);
    }
    const float s = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    if (s == kNever) g_peak_sink = s;
}

// Grid-stride copy of n4 16-byte vectors from src to dst, eight in flight per
// thread, non-temporal loads and stores.
__global__ __launch_bounds__(256) void k_peak_copy(const floatx4* __restrict__ src, floatx4* __restrict__ dst,
                                                   int64_t n4) {
    constexpr int U = 8;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (U - 1) * stride < n4; i += U * stride) {
        floatx4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = ld16<true>(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < U; ++u) __builtin_nontemporal_store(v[u], dst + i + u * stride);
    }
    for (; i < n4; i += stride) __builtin_nontemporal_store(ld16<true>(src + i), dst + i);
}

// KIND 0: v_mfma_f32_16x16x4f32; 1: v_mfma_f32_4x4x1f32 (16 blocks);
// 2: v_mfma_f32_16x16x32_bf16; 3: v_fma_f32 (vector ALU, no packed FP32);
// 4: v_mfma_f32_32x32x16_bf16.  Independent accumulators per wave: sixteen
// 4-register ones (a matrix pipe fed by fewer, eight, issued 16x16x32 BF16 at
// about 60% of its rate in measurements), four 16-register ones for 32x32x16.
template <int KIND>
__global__ __launch_bounds__(256) void k_peak_compute(int iters) {
    const float a = 1.0f + 1e-7f * (float)threadIdx.x, b = 1.0f - 1e-7f * (float)blockIdx.x;
    float s = 0.f;
    const bool clk = blockIdx.x == gridDim.x / 2 && threadIdx.x == 0;   // a wave in the middle of the launch
    uint64_t c0 = 0, r0 = 0;
    if (clk) {
        c0 = __builtin_amdgcn_s_memtime();
        r0 = __builtin_amdgcn_s_memrealtime();
    }
    constexpr int NA = KIND == 4 ? 4 : 16;
    if constexpr (KIND == 3) {
        float acc[NA];
#pragma unroll
        for (int k = 0; k < NA; ++k) acc[k] = 1e-3f * (float)k;
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int k = 0; k < NA; ++k) acc[k] = fmaf(acc[k], a, b);
#pragma unroll
        for (int k = 0; k < NA; ++k) s += acc[k];
    } else if constexpr (KIND == 4) {
        floatx16 acc[NA];
#pragma unroll
        for (int k = 0; k < NA; ++k)
#pragma unroll
            for (int j = 0; j < 16; ++j) acc[k][j] = 0.f;
        bf16x8 av, bv;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            av[e] = (__bf16)(a + (float)e);
            bv[e] = (__bf16)(b - (float)e);
        }
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int k = 0; k < NA; ++k) acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[k], 0, 0, 0);
#pragma unroll
        for (int k = 0; k < NA; ++k) s += acc[k][0] + acc[k][15];
    } else {
        floatx4 acc[NA];
#pragma unroll
        for (int k = 0; k < NA; ++k) acc[k] = floatx4{0.f, 0.f, 0.f, 0.f};
        if constexpr (KIND == 2) {
            bf16x8 av, bv;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                av[e] = (__bf16)(a + (float)e);
                bv[e] = (__bf16)(b - (float)e);
            }
            for (int it = 0; it < iters; ++it)
#pragma unroll
                for (int k = 0; k < NA; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[k], 0, 0, 0);
        } else {
            for (int it = 0; it < iters; ++it)
#pragma unroll
                for (int k = 0; k < NA; ++k) {
                    if constexpr (KIND == 0) acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[k], 0, 0, 0);
                    else acc[k] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, acc[k], 0, 0, 0);
                }
        }
#pragma unroll
        for (int k = 0; k < NA; ++k) s += (acc[k][0] + acc[k][1]) + (acc[k][2] + acc[k][3]);
    }
    if (s == kNever) g_peak_sink = s;
    if (clk) {
        const uint64_t c1 = __builtin_amdgcn_s_memtime(), r1 = __builtin_amdgcn_s_memrealtime();
        g_peak_clk[0] = c0;
        g_peak_clk[1] = c1;
        g_peak_clk[2] = r0;
        g_peak_clk[3] = r1;
    }
}

// independent accumulators per wave of each kind
int compute_accumulators(int kind) { return kind == 4 ? 4 : 16; }

// flops of one wave-level instruction of each kind
double compute_flops_per_instr(int kind) {
    switch (kind) {
    case 0: return 16.0 * 16 * 4 * 2;
    case 1: return 4.0 * 4 * 1 * 16 * 2;
    case 2: return 16.0 * 16 * 32 * 2;
    case 4: return 32.0 * 32 * 16 * 2;
    default: return 64.0 * 2;
    }
}

}  // namespace
}  // namespace hmc

using namespace hmc;

namespace {
// Times `reps` calls of launch() on s (after one untimed call); milliseconds.
template <typename F>
hmc_status time_launches(F launch, int reps, hipStream_t s, double* ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(HMC_E_DEVICE, "event creation failed");
    }
    launch();
    hipError_t e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
        launch();
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float f = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(HMC_E_DEVICE, hipGetErrorString(e));
    *ms = f;
    return HMC_OK;
}
}  // namespace

extern "C" {

hmc_status hmc_peak_memory(void* buf, size_t bytes, int32_t mode, int32_t passes, int32_t reps, void* hip_stream,
                           double* gbytes_per_s) {
    if (!buf || !gbytes_per_s) return fail(HMC_E_INVALID, "buf and gbytes_per_s must not be NULL");
    if (((uintptr_t)buf & 15) != 0) return fail(HMC_E_INVALID, "buf must be 16-byte aligned");
    if (mode != 0 && mode != 1) return fail(HMC_E_INVALID, "mode must be 0 (read) or 1 (copy)");
    if (reps < 1 || passes < 1 || (mode == 1 && passes != 1))
        return fail(HMC_E_INVALID, "reps >= 1; passes >= 1 for reads, 1 for copies");
    const int64_t n4 = (int64_t)(mode == 0 ? bytes / 16 : bytes / 32);
    if (n4 < 1) return fail(HMC_E_INVALID, "buffer too small");
    hipStream_t s = (hipStream_t)hip_stream;
    // beyond the L2s (32 MB over the 8 XCDs): 32 workgroups per CU queued; within them, 8 (one round of
    // 8 waves per SIMD), so that every thread has several vectors per pass
    const dim3 grid(bytes > (64u << 20) ? 256 * 32 : 256 * 8), block(256);
    const floatx4* src = (const floatx4*)buf;
    floatx4* dst = (floatx4*)buf + n4;
    double ms = 0.0;
    hmc_status st;
    if (mode == 1)
        st = time_launches([&] { hipLaunchKernelGGL(k_peak_copy, grid, block, 0, s, src, dst, n4); }, reps, s, &ms);
    else if (passes == 1)
        st = time_launches([&] { hipLaunchKernelGGL(k_peak_read<true>, grid, block, 0, s, src, n4, 1); }, reps, s,
                           &ms);
    else
        st = time_launches([&] { hipLaunchKernelGGL(k_peak_read<false>, grid, block, 0, s, src, n4, passes); }, reps,
                           s, &ms);
    if (st != HMC_OK) return st;
    const double moved = (double)n4 * 16.0 * (mode == 0 ? (double)passes : 2.0) * reps;
    *gbytes_per_s = moved / (ms * 1e-3) / 1e9;
    return HMC_OK;
}

hmc_status hmc_peak_compute(int32_t kind, int32_t waves_per_simd, int32_t iters, int32_t reps, void* hip_stream,
                            double* tflops, double* clock_mhz) {
    if (!tflops) return fail(HMC_E_INVALID, "tflops must not be NULL");
    if (kind < 0 || kind > 4) return fail(HMC_E_INVALID, "kind must be 0..4");
    if (waves_per_simd < 1 || waves_per_simd > 8) return fail(HMC_E_INVALID, "waves_per_simd must be 1..8");
    if (iters < 1 || reps < 1) return fail(HMC_E_INVALID, "iters and reps must be >= 1");
    hipStream_t s = (hipStream_t)hip_stream;
    const dim3 grid(256 * waves_per_simd), block(256);      // a workgroup of 4 waves per CU per wave per SIMD
    double ms = 0.0;
    hmc_status st;
    switch (kind) {
    case 0: st = time_launches([&] { hipLaunchKernelGGL(k_peak_compute<0>, grid, block, 0, s, iters); }, reps, s, &ms); break;
    case 1: st = time_launches([&] { hipLaunchKernelGGL(k_peak_compute<1>, grid, block, 0, s, iters); }, reps, s, &ms); break;
    case 2: st = time_launches([&] { hipLaunchKernelGGL(k_peak_compute<2>, grid, block, 0, s, iters); }, reps, s, &ms); break;
    case 3: st = time_launches([&] { hipLaunchKernelGGL(k_peak_compute<3>, grid, block, 0, s, iters); }, reps, s, &ms); break;
    default: st = time_launches([&] { hipLaunchKernelGGL(k_peak_compute<4>, grid, block, 0, s, iters); }, reps, s, &ms); break;
    }
    if (st != HMC_OK) return st;
    const double waves = (double)grid.x * (block.x / 64);
    const double flops = waves * iters * (double)compute_accumulators(kind) * compute_flops_per_instr(kind) * reps;
    *tflops = flops / (ms * 1e-3) / 1e12;
    if (clock_mhz) {
        uint64_t c[4] = {0, 0, 0, 0};
        const hipError_t e = hipMemcpyFromSymbol(c, HIP_SYMBOL(g_peak_clk), sizeof(c), 0, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return fail(HMC_E_DEVICE, hipGetErrorString(e));
        *clock_mhz = c[3] > c[2] ? 100.0 * (double)(c[1] - c[0]) / (double)(c[3] - c[2]) : 0.0;
    }
    return HMC_OK;
}

}  // extern "C"
