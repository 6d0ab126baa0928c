// exp_f64.hpp -- e^x in FP64 from a caller-held table of 1 / n!.
//
// The fused logistic kernel keeps the table in LDS, because the transition
// loop cannot afford the 14 registers; the host test of its accuracy builds
// the same table in memory.  Method: x = k ln2 + r with ln2 split in two
// parts (the high part has enough trailing zero bits that k ln2_hi is exact
// for |k| <= 1075) and |r| <= ln2 / 2; e^r from its Taylor series through
// r^13, whose remainder is below 2^-56 e^r, by Horner's rule with fused
// multiply-adds; then times 2^k.  x below -745.2 gives 0 (NaN stays NaN),
// above 709.8 gives +inf.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace hmc {

constexpr int EXP_NC = 14;

__host__ __device__ constexpr double exp_coef(int n) {   // 1 / n!
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= (double)i;
    return 1.0 / f;
}

__host__ __device__ __forceinline__ double exp_lds(double x, const double* cf) {
    if (!(x > -745.2)) return x != x ? x : 0.0;
    if (x > 709.8) return INFINITY;
    const double k = rint(x * 1.4426950408889634);
    const double r = fma(-k, 1.9082149292705877e-10, fma(-k, 0.6931471803691238, x));
    double s = cf[EXP_NC - 1];
#pragma unroll
    for (int n = EXP_NC - 2; n >= 0; --n) s = fma(s, r, cf[n]);
    return ldexp(s, (int)k);
}

}  // namespace hmc
