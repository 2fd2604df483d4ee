// 2^x for the seeds of the MDI-LR node recurrences, |x| <= 1000, in double precision:
// exp2_f64 (exp2_f64.hpp), and for small arguments a short form without the
// reduction: |x| <= 1/16 gives |t| = |x ln 2| <= 0.0434, and the Taylor series of e^t
// to degree 8 leaves a first omitted term below 1.5e-18 of the result.  Both are within
// one unit in the last place (checked on the host, tests/test_exp2_f64.py); exact at 0.
#pragma once

#include "exp2_f64.hpp"

namespace qmc {

// The short form, |x| <= 1/16.
QMC_HD inline double exp2_seed_small(double x) {
    const double t = x * kLn2;
    double p = 1.0 / 40320.0;                      // 1/8!
    p = horner_step(p, t, 1.0 / 5040.0);           // 1/7!
    p = horner_step(p, t, 1.0 / 720.0);            // 1/6!
    p = horner_step(p, t, 1.0 / 120.0);            // 1/5!
    p = horner_step(p, t, 1.0 / 24.0);             // 1/4!
    p = horner_step(p, t, 1.0 / 6.0);              // 1/3!
    p = horner_step(p, t, 0.5);                    // 1/2!
    p = horner_step(p, t, 1.0);                    // 1/1!
    p = horner_step(p, t, 1.0);                    // 1/0!
    return p;
}

// e^t - 1 for |t| <= 0.0434 (the short form's range in t = x ln 2): the Taylor series to
// degree 9 in Horner form, without the leading 1, so that its relative error stays
// within a few units in the last place of the (small) result.
QMC_HD inline double expm1_small(double t) {
    double p = 1.0 / 362880.0;                     // 1/9!
    p = horner_step(p, t, 1.0 / 40320.0);          // 1/8!
    p = horner_step(p, t, 1.0 / 5040.0);           // 1/7!
    p = horner_step(p, t, 1.0 / 720.0);            // 1/6!
    p = horner_step(p, t, 1.0 / 120.0);            // 1/5!
    p = horner_step(p, t, 1.0 / 24.0);             // 1/4!
    p = horner_step(p, t, 1.0 / 6.0);              // 1/3!
    p = horner_step(p, t, 0.5);                    // 1/2!
    p = horner_step(p, t, 1.0);                    // 1/1!
    return p * t;
}

// The short form where it applies, else exp2_f64.
QMC_HD inline double exp2_seed(double x) {
    return fabs(x) <= 0.0625 ? exp2_seed_small(x) : exp2_f64(x);
}

}  // namespace qmc
