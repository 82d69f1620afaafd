// Accuracy of the library's FP64 log / exp / scaling power (the batched solve's factors)
// (paper_2412_11079_amd/csrc/scalemath.h, compiled here for the host)
// against long-double libm.  Prints one line of key=value pairs.
#include <cmath>
#include <cstdio>
#include <random>

#include "scalemath.h"

int main() {
    std::mt19937_64 rng(20241211);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    double log_err = 0.0, exp_err = 0.0, pow_err = 0.0;
    // log: x = 2^(uniform exponent) * mantissa over the normal and subnormal range;
    // error in units of max(|log x|, 1) * 2^-53.
    for (int k = 0; k < 2000000; ++k) {
        const double e = -1070.0 + 2090.0 * U(rng);
        const double x = std::ldexp(1.0 + U(rng), (int)std::floor(e));
        if (!(x > 0.0) || !std::isfinite(x)) continue;
        const long double ref = logl((long double)x);
        const double got = uot::sm::log_pos(x);
        const long double scale = fmaxl(fabsl(ref), 1.0L) * 0x1p-53L;
        log_err = std::fmax(log_err, (double)(fabsl((long double)got - ref) / scale));
    }
    // log near 1, where the result is small: relative error
    for (int k = 0; k < 1000000; ++k) {
        const double x = 1.0 + (U(rng) - 0.5) * std::ldexp(1.0, -(int)(40 * U(rng)));
        if (x == 1.0) continue;
        const long double ref = logl((long double)x);
        const double got = uot::sm::log_pos(x);
        log_err = std::fmax(log_err, (double)(fabsl(((long double)got - ref) / ref) / 0x1p-53L));
    }
    // exp over the range of normal results: relative error in units of 2^-53
    for (int k = 0; k < 2000000; ++k) {
        const double w = -708.0 + 1417.0 * U(rng);
        const long double ref = expl((long double)w);
        const double got = uot::sm::exp_any(w);
        exp_err = std::fmax(exp_err, (double)(fabsl(((long double)got - ref) / ref) / 0x1p-53L));
    }
    // (a / s)^fi with log a from libm, as the pass forms it (fi (log a -
    // log s), whose rounding scales with the size of the two logs):
    // relative error in units of (fi (|log a| + |log s|) + 1) 2^-53
    for (int k = 0; k < 1000000; ++k) {
        const double a = std::ldexp(1.0 + U(rng), -(int)(30 * U(rng)));
        const double s = std::ldexp(1.0 + U(rng), (int)(-300 + 600 * U(rng)));
        const double fi = 0.5 + 0.5 * U(rng);
        const long double w = (long double)fi * (logl((long double)a) - logl((long double)s));
        if (fabsl(w) > 700.0L) continue;
        const long double ref = expl(w);
        const double got = uot::sm::scaling_pow(std::log(a), s, fi);
        const long double cond = (long double)fi * (fabsl(logl((long double)a)) + fabsl(logl((long double)s))) + 1.0L;
        pow_err = std::fmax(pow_err, (double)(fabsl(((long double)got - ref) / ref) / (cond * 0x1p-53L)));
    }
    const bool specials = uot::sm::scaling_pow(0.0, 0.0, 0.9) == INFINITY &&
                          uot::sm::scaling_pow(0.0, INFINITY, 0.9) == 0.0 &&
                          std::isnan(uot::sm::scaling_pow(0.0, NAN, 0.9)) && uot::sm::exp_any(-800.0) == 0.0 &&
                          uot::sm::exp_any(710.0) == INFINITY && std::isnan(uot::sm::exp_any(NAN)) &&
                          uot::sm::exp_any(0.0) == 1.0 && uot::sm::log_pos(1.0) == 0.0;
    std::printf("log_ulps=%.3f exp_ulps=%.3f pow_units=%.3f specials=%d\n", log_err, exp_err, pow_err,
                specials ? 1 : 0);
    return 0;
}
