// FP64 exponential and log(1 + e) for the per-row maps, written out from
// textbook methods so that their cost is known and small:
//
//   exp(x):      Cody-Waite reduction x = k ln2 + r, |r| <= ln2 / 2, with ln2
//                split into a high part (trailing zero bits) and a low part,
//                then exp(r) by its Taylor polynomial to degree 13 (the
//                remainder |r|^14 / 14! < 2^-58) and a scale by 2^k;
//   log1p(e):    for 0 <= e <= 1 only (the softplus of the logistic map
//                needs log(1 + exp(-|u|))): 1 + e = 2^m z with z in
//                [sqrt(1/2), sqrt(2)), and log z = 2 atanh(s),
//                s = (z - 1) / (z + 1), |s| <= 0.1716, by the odd series
//                2 (s + s^3/3 + ... + s^21/21) (next term < 2^-58 relative).
//
//   log(x):      for positive normal x: x = 2^m z with z in [sqrt(1/2),
//                sqrt(2)) (z - 1 exact), log z = 2 atanh((z - 1) / (z + 1)) by
//                the same series, and m ln2 added with the split ln2 of exp;
//                near x = 1 (m = 0) the result keeps its relative accuracy.
//
//   1 / x:       for x in [1, 8] (the denominators above and of the
//                sigmoid): the hardware reciprocal estimate refined by two
//                Newton-Raphson steps r <- r + r (1 - x r), each of which
//                squares the relative error, instead of a full IEEE division
//                (which also scales and fixes up operands these values never
//                need).
//
// All are within a few units in the last place of the correctly rounded
// value; NaN in gives NaN out.
#pragma once

#include <hip/hip_runtime.h>

namespace glmk {

__device__ __forceinline__ double exp_f64(double x) {
    // beyond +-1100 the result is 0 or inf either way; clamping keeps k in
    // int range (NaN fails both comparisons and stays NaN)
    x = x < -1100.0 ? -1100.0 : (x > 1100.0 ? 1100.0 : x);
    const double k = rint(x * 1.4426950408889634074);          // x / ln2
    double r = fma(-k, 6.93147180369123816490e-01, x);          // ln2, high part
    r = fma(-k, 1.90821492927058770002e-10, r);                 // ln2, low part
    double p = 1.0 / 6227020800.0;                              // 1/13!
    p = fma(p, r, 1.0 / 479001600.0);                           // 1/12!
    p = fma(p, r, 1.0 / 39916800.0);
    p = fma(p, r, 1.0 / 3628800.0);
    p = fma(p, r, 1.0 / 362880.0);
    p = fma(p, r, 1.0 / 40320.0);
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)k);
}

// 1 / x for x in [1, 8].
__device__ __forceinline__ double recip_1_8(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// 2 atanh(zm1 / zp1) = log z for z = 1 + zm1 = zp1 - 1 in [sqrt(1/2), sqrt(2)).
__device__ __forceinline__ double log_series(double zm1, double zp1) {
    const double s = zm1 * recip_1_8(zp1);
    const double s2 = s * s;
    double q = 1.0 / 21.0;
    q = fma(q, s2, 1.0 / 19.0);
    q = fma(q, s2, 1.0 / 17.0);
    q = fma(q, s2, 1.0 / 15.0);
    q = fma(q, s2, 1.0 / 13.0);
    q = fma(q, s2, 1.0 / 11.0);
    q = fma(q, s2, 1.0 / 9.0);
    q = fma(q, s2, 1.0 / 7.0);
    q = fma(q, s2, 1.0 / 5.0);
    q = fma(q, s2, 1.0 / 3.0);
    const double s3 = s * s2;
    return fma(2.0 * s3, q, 2.0 * s);                           // 2 atanh(s)
}

// log(1 + e) for e in [0, 1].
__device__ __forceinline__ double log1p_unit(double e) {
    const bool up = e > 0.41421356237309504880;                 // sqrt(2) - 1
    const double zm1 = up ? (e - 1.0) * 0.5 : e;                // z - 1
    const double zp1 = up ? (e + 3.0) * 0.5 : e + 2.0;          // z + 1
    const double at = log_series(zm1, zp1);
    return up ? at + 6.93147180559945309417e-01 : at;           // + m ln2
}

// log(x) for positive normal x (the random-number transforms need it on
// (0, 1)).
__device__ __forceinline__ double log_f64(double x) {
    int ex = 0;
    double z = frexp(x, &ex);                                   // x = z 2^ex, z in [1/2, 1)
    if (z < 0.70710678118654752440) {                           // sqrt(1/2)
        z *= 2.0;
        --ex;
    }
    const double m = (double)ex;
    const double lz = log_series(z - 1.0, z + 1.0);             // z - 1 exact
    return fma(m, 6.93147180369123816490e-01, fma(m, 1.90821492927058770002e-10, lz));
}

}  // namespace glmk
