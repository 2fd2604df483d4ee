// 2^x for the seeds of the MDI-LR node recurrences, |x| <= 1000, in double precision:
// the series of exp2_f64 (exp2_f64.hpp: x = i + f, i = rint(x), e^t with t = f ln 2 to
// degree 13, scaled by 2^i), here with every series coefficient read from a scalar
// register pair, and a short form without the reduction for small arguments:
// |x| <= 1/16 gives |t| <= 0.0434, and the series to degree 8 leaves a first omitted
// term below 1.5e-18 of the result.  Both forms are within one unit in the last place
// (checked on the host, tests/test_exp2_f64.py); exact at 0 and, in the reduced form,
// at integers.
//
// The MDI-LR kernel keeps its vector registers for occupancy: with the coefficients in
// vector registers its FP64 Gaussian kernel held about 90 of them (five waves per
// SIMD instead of eight) and copied the constants back before each series.  The
// per-point exponentials of the plain and batched sums keep exp2_f64 as it is: in the
// scalar-register form the batched FP64 kernel spills scalar registers and runs about
// 1 % slower.
#pragma once

#include "exp2_f64.hpp"

namespace qmc {

// p t + c for a series coefficient c (a compile-time constant, the same in every
// lane): on the device one v_fma_f64 that reads c from a scalar register pair.
QMC_HD inline double horner_step_sreg(double p, double t, double c) {
#if defined(__HIP_DEVICE_COMPILE__)
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(p), "v"(t), "s"(c));
    return r;
#else
    return fma(p, t, c);
#endif
}

// The reduced form, |x| <= 1000: the same reduction and coefficients as exp2_f64.
QMC_HD inline double exp2_seed_reduced(double x) {
    const double i = rint(x);
    const double t = (x - i) * kLn2;
    double p = 1.0 / 6227020800.0;                      // 1/13!
    p = horner_step_sreg(p, t, 1.0 / 479001600.0);      // 1/12!
    p = horner_step_sreg(p, t, 1.0 / 39916800.0);       // 1/11!
    p = horner_step_sreg(p, t, 1.0 / 3628800.0);        // 1/10!
    p = horner_step_sreg(p, t, 1.0 / 362880.0);         // 1/9!
    p = horner_step_sreg(p, t, 1.0 / 40320.0);          // 1/8!
    p = horner_step_sreg(p, t, 1.0 / 5040.0);           // 1/7!
    p = horner_step_sreg(p, t, 1.0 / 720.0);            // 1/6!
    p = horner_step_sreg(p, t, 1.0 / 120.0);            // 1/5!
    p = horner_step_sreg(p, t, 1.0 / 24.0);             // 1/4!
    p = horner_step_sreg(p, t, 1.0 / 6.0);              // 1/3!
    p = horner_step_sreg(p, t, 0.5);                    // 1/2!
    p = horner_step_sreg(p, t, 1.0);                    // 1/1!
    p = horner_step_sreg(p, t, 1.0);                    // 1/0!
    return ldexp(p, (int)i);
}

// The short form, |x| <= 1/16.
QMC_HD inline double exp2_seed_small(double x) {
    const double t = x * kLn2;
    double p = 1.0 / 40320.0;                           // 1/8!
    p = horner_step_sreg(p, t, 1.0 / 5040.0);           // 1/7!
    p = horner_step_sreg(p, t, 1.0 / 720.0);            // 1/6!
    p = horner_step_sreg(p, t, 1.0 / 120.0);            // 1/5!
    p = horner_step_sreg(p, t, 1.0 / 24.0);             // 1/4!
    p = horner_step_sreg(p, t, 1.0 / 6.0);              // 1/3!
    p = horner_step_sreg(p, t, 0.5);                    // 1/2!
    p = horner_step_sreg(p, t, 1.0);                    // 1/1!
    p = horner_step_sreg(p, t, 1.0);                    // 1/0!
    return p;
}

// The short form where it applies, else the reduced one.
QMC_HD inline double exp2_seed(double x) {
    return fabs(x) <= 0.0625 ? exp2_seed_small(x) : exp2_seed_reduced(x);
}

}  // namespace qmc
