// Host check of qmc::exp2_f64 (paper_2404_08867_amd/csrc/exp2_f64.hpp): the largest
// error, in units in the last place, against exp2l over n pseudo-random points of
// [lo, hi] and the two end points; prints "<max ulp> <x at the max>".
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "exp2_f64.hpp"

static double ulp_error(double got, long double ref) {
    const double r = fabs((double)ref);
    const double ulp = nextafter(r, INFINITY) - r;
    return (double)(fabsl((long double)got - ref) / ulp);
}

int main(int argc, char** argv) {
    if (argc != 4) return 2;
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
        const double e = ulp_error(qmc::exp2_f64(x), exp2l((long double)x));
        if (e > worst) {
            worst = e;
            worst_x = x;
        }
    }
    printf("%.6f %.17g\n", worst, worst_x);
    return 0;
}
