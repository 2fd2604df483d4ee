// log2 in double precision from a table of the mantissa's leading bits, to about
// 3e-13 absolute for every positive normal x: x = m 2^e with m in [1/2, 1), the
// mantissa's top kLog2TabBits bits pick the interval of width 2^-(kLog2TabBits + 1)
// that holds m, with centre T_j, and
//   log2 x = e + log2 T_j + log2(1 + t),  t = m / T_j - 1,  |t| <= 2^-(kLog2TabBits + 1),
// where t = fma(m, 1/T_j, -1) and log2(1 + t) is its Taylor series to t^4 (the first
// omitted term, t^5 / (5 ln 2), is below 3e-13).  The table holds 1/T_j and
// log2 T_j, evaluated at compile time (log2 T from the atanh series of ln T).  About
// twelve vector instructions and one table read; checked against log2l on the host
// (tests/test_exp2_f64.py).
#pragma once

#include <stdint.h>
#include <string.h>

#include "exp2_f64.hpp"

namespace qmc {

constexpr int kLog2TabBits = 7;
constexpr int kLog2Tab = 1 << kLog2TabBits;

struct Log2Entry {
    double inv;  // 1 / T_j
    double lg;   // log2 T_j
};

struct Log2Table {
    Log2Entry e[kLog2Tab];
};

// log2 T for T in [1/2, 1): ln T = 2 atanh(s) = 2 sum_k s^{2k+1} / (2k + 1) with
// s = (T - 1) / (T + 1) in [-1/3, 0); 40 terms leave less than 1e-38.  The terms are
// added smallest first.
constexpr double log2_of_mantissa(double T) {
    const double s = (T - 1.0) / (T + 1.0), s2 = s * s;
    double term[40] = {};
    double pw = s;
    for (int k = 0; k < 40; ++k) {
        term[k] = pw / (double)(2 * k + 1);
        pw *= s2;
    }
    double sum = 0.0;
    for (int k = 39; k >= 0; --k) sum += term[k];
    return 2.0 * sum * 1.44269504088896340736;  // log2(e)
}

constexpr Log2Table make_log2_table() {
    Log2Table t{};
    for (int j = 0; j < kLog2Tab; ++j) {
        const double T = 0.5 + ((double)j + 0.5) / (double)(2 * kLog2Tab);
        t.e[j].inv = 1.0 / T;
        t.e[j].lg = log2_of_mantissa(T);
    }
    return t;
}

// log2 x for finite x >= 2^-1022 (positive normal); the caller takes other x
// elsewhere.  `tab` is the table of make_log2_table().
QMC_HD inline double log2_tab(double x, const Log2Entry* tab) {
#if defined(__HIP_DEVICE_COMPILE__)
    const int e = __builtin_amdgcn_frexp_exp(x);  // x = m 2^e, m in [1/2, 1)
    const double m = __builtin_amdgcn_frexp_mant(x);
#else
    int e = 0;
    const double m = frexp(x, &e);
#endif
    uint64_t bits = 0;
    memcpy(&bits, &x, sizeof bits);
    const int j = (int)((bits >> (52 - kLog2TabBits)) & (uint64_t)(kLog2Tab - 1));
    const Log2Entry E = tab[j];
    const double t = fma(m, E.inv, -1.0);
    constexpr double l2e = 1.44269504088896340736;  // 1 / ln 2
    double q = fma(t, -l2e / 4.0, l2e / 3.0);
    q = horner_step(q, t, -l2e / 2.0);
    q = horner_step(q, t, l2e);
    return fma(t, q, (double)e + E.lg);
}

// log2 x as an unevaluated sum hi + lo, for finite x >= 2^-1022, to about 3e-16
// absolute: the same table, the series to t^6 (first omitted term below 3e-18), the
// fraction r = log2 T_j + log2(1 + t) in one double, and e + r split exactly into
// hi + lo (e is an integer with e = 0 or |e| >= 1 > |r| - 2^-7, so the
// subtraction below recovers the rounding of e + r).
QMC_HD inline void log2_tab_dd(double x, const Log2Entry* tab, double& hi, double& lo) {
#if defined(__HIP_DEVICE_COMPILE__)
    const int e = __builtin_amdgcn_frexp_exp(x);
    const double m = __builtin_amdgcn_frexp_mant(x);
#else
    int e = 0;
    const double m = frexp(x, &e);
#endif
    uint64_t bits = 0;
    memcpy(&bits, &x, sizeof bits);
    const int j = (int)((bits >> (52 - kLog2TabBits)) & (uint64_t)(kLog2Tab - 1));
    const Log2Entry E = tab[j];
    const double t = fma(m, E.inv, -1.0);
    constexpr double l2e = 1.44269504088896340736;  // 1 / ln 2
    double q = fma(t, -l2e / 6.0, l2e / 5.0);
    q = horner_step(q, t, -l2e / 4.0);
    q = horner_step(q, t, l2e / 3.0);
    q = horner_step(q, t, -l2e / 2.0);
    q = horner_step(q, t, l2e);
    const double r = fma(t, q, E.lg);
    const double de = (double)e;
    hi = de + r;
    lo = r - (hi - de);
}

}  // namespace qmc
