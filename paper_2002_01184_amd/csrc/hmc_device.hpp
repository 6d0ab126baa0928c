// hmc_device.hpp -- device-side building blocks shared by the HMC kernels.
//
// Counter-based random numbers (Philox4x32-10, Salmon et al., SC'11), the
// uniform and normal maps of the ABI (include/hmc.h), wavefront reductions,
// and the per-chain accept / dual-averaging step.  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hmc {

// ---------------------------------------------------------------------------
// Philox4x32-10: ten rounds of two 32x32->64 multiplies; round multipliers
// and Weyl key increments from the SC'11 paper (Sec. 3.2, Table 2).
// ---------------------------------------------------------------------------
struct Key {
    uint32_t k0, k1;
};

__host__ __device__ inline Key make_key(uint64_t seed) {
    return Key{(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
}

__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, Key key) {
    uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // each 32 x 32 -> 64-bit product as one v_mad_u64_u32 (instead of a
        // separate low and high multiply, both quarter-rate)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

enum : uint32_t { TAG_MOMENTUM = 0, TAG_ACCEPT = 1, TAG_SWAP = 2 };

// (k + 1/2) 2^-23 with k the top 23 bits: exact in binary32 and binary64.
__device__ __forceinline__ float u23_f32(uint32_t w) {
    return ((float)(w >> 9) + 0.5f) * 0x1p-23f;
}
__device__ __forceinline__ double u23_f64(uint32_t w) {
    return ((double)(w >> 9) + 0.5) * 0x1p-23;
}

// Box-Muller on one pair: r = sqrt(-2 log u1), angle = 2 pi u2 (sincospi of 2 u2,
// exact argument).
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, float& z0, float& z1) {
    const float r = sqrtf(-2.0f * logf(u23_f32(wa)));
    float s, c;
    sincospif(2.0f * u23_f32(wb), &s, &c);
    z0 = r * c;
    z1 = r * s;
}
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, double& z0, double& z1) {
    const double r = sqrt(-2.0 * log(u23_f64(wa)));
    double s, c;
    sincospi(2.0 * u23_f64(wb), &s, &c);
    z0 = r * c;
    z1 = r * s;
}

// Four momenta of chain c at transition t for dimensions 4*block .. 4*block+3.
// need_hi = false when dimensions 4*block+2 and +3 lie beyond D: the second
// Box-Muller pair is then not evaluated (its values would be discarded; the
// first pair does not depend on it) and z[2], z[3] are set to 0.
template <typename T>
__device__ __forceinline__ void momentum4(Key key, uint32_t chain, uint32_t t, uint32_t block, T z[4],
                                          bool need_hi = true) {
    const uint4 w = philox(chain, t, block, TAG_MOMENTUM, key);
    box_muller(w.x, w.y, z[0], z[1]);
    if (need_hi) {
        asm volatile("" ::: );   // keeps the pair behind the branch (not computed and selected)
        box_muller(w.z, w.w, z[2], z[3]);
    } else {
        z[2] = (T)0;
        z[3] = (T)0;
    }
}

// log of the uniform ((w0>>6) 2^26 + (w1>>6) + 1/2) 2^-52 of block
// (chain, t, 0, tag), in FP64: the Metropolis test (tag ACCEPT) and the
// replica-exchange test (tag SWAP).
__device__ __forceinline__ double log_uniform52(Key key, uint32_t chain, uint32_t t, uint32_t tag) {
    const uint4 w = philox(chain, t, 0u, tag, key);
    const double k = (double)(w.x >> 6) * 67108864.0 + (double)(w.y >> 6);
    return log((k + 0.5) * 0x1p-52);
}
__device__ __forceinline__ double log_accept_uniform(Key key, uint32_t chain, uint32_t t) {
    return log_uniform52(key, chain, t, TAG_ACCEPT);
}

// ---------------------------------------------------------------------------
// Reductions across a power-of-two group of G lanes (G <= 64) of a wavefront.
// ---------------------------------------------------------------------------
template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

template <typename T>
__device__ __forceinline__ T as_state(float v);
template <>
__device__ __forceinline__ float as_state<float>(float v) { return v; }
template <>
__device__ __forceinline__ double as_state<double>(float v) { return (double)v; }

// BF16 <-> FP32 (round to nearest even; inputs finite).
__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
    return __uint_as_float(((uint32_t)b) << 16);
}
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// ---------------------------------------------------------------------------
// Per-chain decision (Metropolis-Hastings on dH) and dual averaging
// (Hoffman & Gelman 2014, eq. 6).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double log_accept_ratio_of(double dh) {
    // -dH, with NaN and +inf dH mapped to -inf (reject)
    return (isnan(dh) || (isinf(dh) && dh > 0.0)) ? -INFINITY : -dh;
}

struct DualAvg {
    double hbar, log_eps_bar, mu;
};

// The factors of iteration m that do not depend on the chain: the averaging
// weight 1/(m + t0), the shrinkage sqrt(m)/gamma and the iterate weight m^-kappa.
struct DaConst {
    double w, k, eta;
};
__device__ __forceinline__ DaConst dual_avg_const(double m, double gamma, double t0, double kappa) {
    return DaConst{1.0 / (m + t0), sqrt(m) / gamma, pow(m, -kappa)};
}

// Iteration with accept statistic alpha; returns the new log step size.
__device__ __forceinline__ double dual_avg_apply(DualAvg& s, const DaConst& c, double alpha, double delta) {
    s.hbar = (1.0 - c.w) * s.hbar + c.w * (delta - alpha);
    const double log_eps = s.mu - c.k * s.hbar;
    s.log_eps_bar = c.eta * log_eps + (1.0 - c.eta) * s.log_eps_bar;
    return log_eps;
}

// Multiplicative rule (SimpleStepSizeAdaptation example of the wrapper
// pattern): grow after a transition whose accept statistic is above the
// target, shrink otherwise.
__device__ __forceinline__ double simple_adapt(double eps, double alpha, double target, double rate) {
    return alpha > target ? eps * (1.0 + rate) : eps / (1.0 + rate);
}

// Iteration m >= 1 with accept statistic alpha; returns the new log step size.
__device__ __forceinline__ double dual_avg_update(DualAvg& s, double m, double alpha, double delta,
                                                  double gamma, double t0, double kappa) {
    return dual_avg_apply(s, dual_avg_const(m, gamma, t0, kappa), alpha, delta);
}

// Control block of the plain/graph path (device resident, written by a
// one-thread kernel so that a captured graph can be replayed unchanged).
struct Ctrl {
    uint64_t t;               // current transition index
    uint64_t t_begin;         // first transition of the current sample_chain call
    int64_t n_burnin;
    int64_t n_results;
    int32_t adapt;
    int32_t adapt_kind;       // HMC_ADAPT_DUAL_AVERAGING or HMC_ADAPT_SIMPLE
    double target_accept, gamma, t0, kappa, rate;
    void* samples;            // [R, C, D] state dtype or null
    double* tr_step;
    uint8_t* tr_acc;
    double* tr_lar;
    double* tr_logp;
    uint8_t* out_acc;         // hmc_step outputs ([C] / [C, D]) or null
    double* out_lar;
    double* out_logp;
    void* out_xprop;
    void* out_pprop;
    double* out_dh;
};

}  // namespace hmc
