// 2^x in double precision for |x| <= 1000, written out so that it compiles both for
// the device and, with a plain C++ compiler, for the host check of its accuracy
// (tests/test_exp2_f64.py).  Used for the MDI-LR node-recurrence seeds and the
// per-point exponentials of the QMC_FP64 sums.
//
// x = i + f with i = rint(x) and |f| <= 1/2 (x - i is exact); 2^f = e^t with
// t = f ln 2, |t| <= 0.3466, by the Taylor series of e^t to degree 13 in Horner
// form (the first omitted term, t^14 / 14!, is below 5e-18 of the result), and the
// result scaled by 2^i exactly.  Within one unit in the last place of 2^x (0.94 at
// most over 10^7 points of [-1000, 1000] on the host); exact at integers.  Outside
// |x| <= 1000 the caller uses the library exp2.
#pragma once

#include <math.h>

#if defined(__HIPCC__)
#define QMC_HD __host__ __device__
#else
#define QMC_HD
#endif

namespace qmc {

constexpr double kLn2 = 0.69314718055994530942;

// p t + c for a series coefficient c (a compile-time constant, the same in every
// lane).  On the device one v_fma_f64 that reads c from a scalar register pair: left
// to itself the compiler may emit the two-address v_fmac_f64 with a copy of c into
// vector registers before each of them, and with c in vector registers a kernel keeps
// the thirteen coefficients in 26 of them (the plain sums' FP64 exp-sum and Gaussian
// kernels held 96 vector registers that way, 75 with the coefficients in scalar ones).
QMC_HD inline double horner_step(double p, double t, double c) {
#if defined(__HIP_DEVICE_COMPILE__)
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(p), "v"(t), "s"(c));
    return r;
#else
    return fma(p, t, c);
#endif
}

QMC_HD inline double exp2_f64(double x) {
    const double i = rint(x);
    const double t = (x - i) * kLn2;
    // Horner form of sum_k t^k / k!, k = 13 down to 0 (coefficients 1/k! rounded to
    // double: their errors are below 1e-16 of terms that are at most 0.35^k / k!).
    double p = 1.0 / 6227020800.0;                  // 1/13!
    p = horner_step(p, t, 1.0 / 479001600.0);       // 1/12!
    p = horner_step(p, t, 1.0 / 39916800.0);        // 1/11!
    p = horner_step(p, t, 1.0 / 3628800.0);         // 1/10!
    p = horner_step(p, t, 1.0 / 362880.0);          // 1/9!
    p = horner_step(p, t, 1.0 / 40320.0);           // 1/8!
    p = horner_step(p, t, 1.0 / 5040.0);            // 1/7!
    p = horner_step(p, t, 1.0 / 720.0);             // 1/6!
    p = horner_step(p, t, 1.0 / 120.0);             // 1/5!
    p = horner_step(p, t, 1.0 / 24.0);              // 1/4!
    p = horner_step(p, t, 1.0 / 6.0);               // 1/3!
    p = horner_step(p, t, 0.5);                     // 1/2!
    p = horner_step(p, t, 1.0);                     // 1/1!
    p = horner_step(p, t, 1.0);                     // 1/0!
    return ldexp(p, (int)i);
}

}  // namespace qmc
