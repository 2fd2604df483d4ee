// Host check of qmc::log2_tab (paper_2404_08867_amd/csrc/log2_tab.hpp), or with a
// fourth argument "dd" of qmc::log2_tab_dd (hi + lo in long double): the largest
// absolute error against log2l over n points of [lo, hi] (uniform in log x) and the
// two end points, plus every interval edge of the table in [1/2, 1) scaled by 2^k for
// k in [-8, 8]; prints "<max abs error> <x at the max>".
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "log2_tab.hpp"

static constexpr qmc::Log2Table kTab = qmc::make_log2_table();

int main(int argc, char** argv) {
    if (argc < 4) {
        fprintf(stderr, "usage: log2_check n lo hi\n");
        return 2;
    }
    const long n = atol(argv[1]);
    const double lo = atof(argv[2]), hi = atof(argv[3]);
    const bool dd = argc > 4 && argv[4][0] == 'd';  // the two-part form log2_tab_dd
    double worst = 0.0, at = lo;
    auto value = [&](double x) -> long double {
        if (!dd) return (long double)qmc::log2_tab(x, kTab.e);
        double h = 0.0, l = 0.0;
        qmc::log2_tab_dd(x, kTab.e, h, l);
        return (long double)h + (long double)l;
    };
    auto check = [&](double x) {
        const double err = fabs((double)(value(x) - log2l((long double)x)));
        if (err > worst || err != err) {
            worst = err;
            at = x;
        }
    };
    check(lo);
    check(hi);
    uint64_t s = 0x9e3779b97f4a7c15ull;
    const double llo = log2(lo), lhi = log2(hi);
    for (long i = 0; i < n; ++i) {
        s = s * 6364136223846793005ull + 1442695040888963407ull;
        const double u = (double)(s >> 11) * 0x1p-53;
        check(exp2(llo + (lhi - llo) * u));
    }
    for (int k = -8; k <= 8; ++k)
        for (int j = 0; j <= 2 * qmc::kLog2Tab; ++j) {
            const double x = ldexp(0.5 + (double)j / (double)(4 * qmc::kLog2Tab), k);
            if (x >= lo && x <= hi) {
                check(x);
                check(nextafter(x, 0.0));
            }
        }
    printf("%.6e %.17g\n", worst, at);
    return 0;
}
