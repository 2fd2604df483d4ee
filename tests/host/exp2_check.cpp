// Host check of qmc::exp2_f64 (paper_2404_08867_amd/csrc/exp2_f64.hpp) and, with a
// fourth argument "small", "seed" or "expm1", of the MDI-LR seed forms
// qmc::exp2_seed_small and qmc::exp2_seed and of qmc::expm1_small (exp2_seed.hpp): the
// largest error, in units in the last place, against exp2l (expm1l for "expm1") over n
// pseudo-random points of [lo, hi] and the two end points; prints "<max ulp> <x at the
// max>".
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "exp2_seed.hpp"

static double ulp_error(double got, long double ref) {
    const double r = fabs((double)ref);
    const double ulp = nextafter(r, INFINITY) - r;
    return (double)(fabsl((long double)got - ref) / ulp);
}

static double eval(char which, double x) {
    switch (which) {
        case 's': return qmc::exp2_seed_small(x);
        case 'e': return qmc::exp2_seed(x);
        case 'm': return qmc::expm1_small(x);
        default: return qmc::exp2_f64(x);
    }
}

int main(int argc, char** argv) {
    if (argc != 4 && argc != 5) return 2;
    char which = 'f';  // exp2_f64
    if (argc == 5) {
        if (!strcmp(argv[4], "small")) which = 's';
        else if (!strcmp(argv[4], "seed")) which = 'e';
        else if (!strcmp(argv[4], "expm1")) which = 'm';
        else return 2;
    }
    const long n = atol(argv[1]);
    const double lo = atof(argv[2]), hi = atof(argv[3]);
    double worst = 0.0, worst_x = lo;
    uint64_t s = 88172645463325252ull;  // xorshift64
    for (long k = 0; k < n + 2; ++k) {
        double x;
        if (k == 0) x = lo;
        else if (k == 1) x = hi;
        else {
            s ^= s << 13;
            s ^= s >> 7;
            s ^= s << 17;
            x = lo + (hi - lo) * ((double)(s >> 11) * 0x1p-53);
        }
        const long double ref = which == 'm' ? expm1l((long double)x) : exp2l((long double)x);
        const double e = x == 0.0 && which == 'm' ? fabs(eval(which, x)) : ulp_error(eval(which, x), ref);
        if (e > worst) {
            worst = e;
            worst_x = x;
        }
    }
    printf("%.6f %.17g\n", worst, worst_x);
    return 0;
}
