// FP64 natural logarithm and exponential for the scaling update
// u = (a / s)^fi = exp(fi (log a - log s)) of the batched solve.
//
// Written from the textbook reductions, for a caller that evaluates them
// once per row inside a register-bound loop (the library routines keep
// their coefficient tables in vector registers across such loops):
//  - log: x = m 2^e with m in [sqrt(1/2), sqrt(2)); log m = 2 atanh(s),
//    s = (m - 1) / (m + 1), |s| <= 0.1716, summed as the odd power series
//    2 (s + s^3/3 + ... + s^23/23) (truncation below 1e-19); then
//    log x = e ln2 + log m with ln2 split into a 32-bit head (e * head is
//    exact) and a tail.  Absolute error about one ulp of log x.
//  - exp: w = k ln2 + r with k = rint(w / ln2), |r| <= ln2 / 2 (same split
//    of ln2, so r carries no cancellation error); e^r by its Taylor series
//    to r^13 (truncation below 5e-18 relative); e^w = 2^k e^r.  Relative
//    error a few ulp.
// Compiled for the device by hipcc and for the host by a plain C++
// compiler (the CPU test of these functions against libm).
#pragma once

#include <cmath>

#ifdef __HIPCC__
#define UOT_SM_FN __host__ __device__ __forceinline__
#else
#define UOT_SM_FN inline
#endif

namespace uot {
namespace sm {

// A coefficient handed to the arithmetic from a scalar register at its
// point of use: the empty statement keeps the compiler from hoisting the
// coefficients of a loop body into vector registers for the whole loop.
UOT_SM_FN double kc(double c) {
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" : "+s"(c));
#endif
    return c;
}

constexpr double kLn2Hi = 0x1.62e42fee00000p-1;    // ln 2 to 32 significant bits
constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;   // ln 2 - kLn2Hi
constexpr double kInvLn2 = 0x1.71547652b82fep+0;
constexpr double kSqrtHalf = 0x1.6a09e667f3bcdp-1;

// log x for finite x > 0 (normal or subnormal).
UOT_SM_FN double log_pos(double x) {
    int e = 0;
    double m = std::frexp(x, &e);           // x = m 2^e, m in [1/2, 1)
    if (m < kc(kSqrtHalf)) {
        m *= 2.0;
        e -= 1;
    }
    const double s = (m - 1.0) / (m + 1.0);  // m - 1 is exact
    const double z = s * s;
    // P(z) = 1/3 + z/5 + ... + z^10/23
    double p = kc(0x1.642c8590b2164p-5);      // 1/23
    p = std::fma(p, z, kc(0x1.8618618618618p-5)); // 1/21
    p = std::fma(p, z, kc(0x1.af286bca1af28p-5)); // 1/19
    p = std::fma(p, z, kc(0x1.e1e1e1e1e1e1ep-5)); // 1/17
    p = std::fma(p, z, kc(0x1.1111111111111p-4)); // 1/15
    p = std::fma(p, z, kc(0x1.3b13b13b13b14p-4)); // 1/13
    p = std::fma(p, z, kc(0x1.745d1745d1746p-4)); // 1/11
    p = std::fma(p, z, kc(0x1.c71c71c71c71cp-4)); // 1/9
    p = std::fma(p, z, kc(0x1.2492492492492p-3)); // 1/7
    p = std::fma(p, z, kc(0x1.999999999999ap-3)); // 1/5
    p = std::fma(p, z, kc(0x1.5555555555555p-2)); // 1/3
    const double s2 = 2.0 * s;
    const double lm = std::fma(s2 * z, p, s2);
    const double ed = (double)e;
    return std::fma(ed, kc(kLn2Hi), std::fma(ed, kc(kLn2Lo), lm));
}

// e^w for any w (0 below -745.2, +inf above 709.79, NaN for NaN).
UOT_SM_FN double exp_any(double w) {
    if (w != w) return w;
    if (w > 709.79) return INFINITY;
    if (w < -745.2) return 0.0;
    const double k = std::rint(w * kc(kInvLn2));
    const double r = std::fma(-k, kc(kLn2Lo), std::fma(-k, kc(kLn2Hi), w));
    double p = kc(0x1.6124613a86d09p-33);      // 1/13!
    p = std::fma(p, r, kc(0x1.1eed8eff8d898p-29)); // 1/12!
    p = std::fma(p, r, kc(0x1.ae64567f544e4p-26)); // 1/11!
    p = std::fma(p, r, kc(0x1.27e4fb7789f5cp-22)); // 1/10!
    p = std::fma(p, r, kc(0x1.71de3a556c734p-19)); // 1/9!
    p = std::fma(p, r, kc(0x1.a01a01a01a01ap-16)); // 1/8!
    p = std::fma(p, r, kc(0x1.a01a01a01a01ap-13)); // 1/7!
    p = std::fma(p, r, kc(0x1.6c16c16c16c17p-10)); // 1/6!
    p = std::fma(p, r, kc(0x1.1111111111111p-7));  // 1/5!
    p = std::fma(p, r, kc(0x1.5555555555555p-5));  // 1/4!
    p = std::fma(p, r, kc(0x1.5555555555555p-3));  // 1/3!
    p = std::fma(p, r, 0.5);
    p = std::fma(p, r, 1.0);
    p = std::fma(p, r, 1.0);
    return std::ldexp(p, (int)k);
}

// Scaling factor (a / s)^fi from a > 0 given with log a, the row or column
// total s >= 0 and fi in (0, 1): special totals follow the plain formula
// (s = 0 gives +inf, s = +inf gives 0, NaN stays NaN).
UOT_SM_FN double scaling_pow(double log_a, double s, double fi) {
    if (s != s) return s;
    if (s == 0.0) return INFINITY;
    if (s == INFINITY) return 0.0;
    return exp_any(fi * (log_a - log_pos(s)));
}

}  // namespace sm
}  // namespace uot
