// Integrand families of the lattice sum, written for the dims-outer / points-inner
// loop of the sum kernels.  Each family is split into
//   Dim      constants of one direction j (computed once per workgroup, kept in LDS),
//   Acc      the running per-point state over directions (registers),
//   step     one direction's contribution for lattice index k in [0, n), given as
//            a 32-bit integer or, for n <= 2^24, as the same integer held exactly in
//            a float (the exact-float index step of common.hpp; (double)k is then a
//            conversion from float, and the FP32 factors take k with none),
//   finish   the per-point transcendental, returning f(x) / scale,
// and three workgroup-wide sums over directions (block_terms) that give the
// initial state and the final scale.  Coordinates are x_j = (k + sfrac_j) / n
// where sfrac_j is the fractional part of shift_j * n (the whole part is folded
// into the start index), so the shifted lattice of Sec. 2.1 costs nothing per point.
//
// Argument sums (exp-sum, Gaussian, oscillatory) are carried in double in both
// precisions: FP64 FMA issues at the same rate as FP32 on gfx950 when packed
// FP32 is not used, and it keeps the argument exact to ~1e-15 for d up to 1024.
// QMC_FP32_COMPENSATED evaluates the per-point transcendental (exp2, cos,
// reciprocal) and the product-peak factors in single precision.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "exp2_f64.hpp"

namespace qmc {

constexpr double kLog2e = 1.4426950408889634074;
constexpr double kSqrtLog2e = 1.2011224087864497918;
constexpr double kInv2Pi = 0.15915494309189533577;

enum FamilyId {
    kExpSum = 0,
    kProductPeak = 1,
    kGaussian = 2,
    kOscillatory = 3,
    kExpQuadratic = 4,
    // Internal: the Bernoulli product sums behind the lattice-quality criteria
    // (weights a_j; the S forms also multiply the sum by the parameter a_d).
    kBernoulli2 = 16,
    kBernoulli4 = 17,
    kBernoulli2S = 18,
    kBernoulli4S = 19,
};

// exp2 of a double argument: split off the nearest integer in double, take the
// fractional power in single precision (|fr| <= 1/2) and rescale exactly.
__device__ __forceinline__ double exp2_split_f32(double s) {
    const double r = rint(s);
    const float fr = (float)(s - r);
    return ldexp((double)__builtin_amdgcn_exp2f(fr), (int)r);
}

// exp2 in double precision: the local series (exp2_f64.hpp, within 1 ulp, about 20
// instructions) over its range, the library exp2 (overflow, underflow) beyond it.
__device__ __forceinline__ double exp2_double(double s) {
    return fabs(s) <= 1000.0 ? exp2_f64(s) : exp2(s);
}

// ------------------------------------------------------------------ exp-sum
// f = exp(sum_j c_j x_j) = 2^{sum_j a_j (k_j + sfrac_j)} with a_j = c_j log2(e) / n.
// The argument is centred by h = log2(e) sum_j c_j / 2 (folded into the scale).
template <bool FP32>
struct ExpSum {
    struct Dim {
        double a;
    };
    struct Acc {
        double s;
    };
    static constexpr int kRenorm = 0;
    static constexpr bool kBlockTerms = true;
    __device__ static void block_terms(const double* p, int d, int j, double inv_n, double sfrac,
                                       double& ds0, double& ds1, int& ie) {
        const double a = p[j] * kLog2e * inv_n;
        const double h = 0.5 * kLog2e * p[j];
        ds0 += a * sfrac - h;
        ds1 += h;
        (void)d;
        (void)ie;
    }
    __device__ static double extra(const double*) { return 0.0; }
    __device__ static Dim dim(const double* p, int d, int j, double inv_n, double sfrac) {
        (void)d;
        (void)sfrac;
        return Dim{p[j] * kLog2e * inv_n};
    }
    __device__ static Acc init(double s0) { return Acc{s0}; }
    template <class K>
    __device__ static void step(Acc& acc, K k, const Dim& c) {
        acc.s = fma((double)k, c.a, acc.s);
    }
    __device__ static void renorm(Acc&) {}
    __device__ static double finish(const Acc& acc) {
        if constexpr (FP32)
            return exp2_split_f32(acc.s);
        else
            return exp2_double(acc.s);
    }
    __device__ static double scale(double ds1, int ie) {
        (void)ie;
        return exp2(ds1);
    }
};

// ----------------------------------------------------------------- Gaussian
// f = exp(-sum_j c_j^2 (x_j - w_j)^2) = 2^{-sum_j y_j^2},
// y_j = c_j sqrt(log2 e) (x_j - w_j) = b_j k + g_j.
template <bool FP32>
struct Gaussian {
    struct Dim {
        double b, g;
    };
    struct Acc {
        double s;
    };
    static constexpr int kRenorm = 0;
    static constexpr bool kBlockTerms = false;
    __device__ static void block_terms(const double*, int, int, double, double, double&, double&,
                                       int&) {}
    __device__ static double extra(const double*) { return 0.0; }
    __device__ static Dim dim(const double* p, int d, int j, double inv_n, double sfrac) {
        const double c = p[j] * kSqrtLog2e, w = p[d + j];
        const double b = c * inv_n;
        return Dim{b, fma(b, sfrac, -c * w)};
    }
    __device__ static Acc init(double) { return Acc{0.0}; }
    template <class K>
    __device__ static void step(Acc& acc, K k, const Dim& c) {
        const double y = fma((double)k, c.b, c.g);
        acc.s = fma(y, y, acc.s);
    }
    __device__ static void renorm(Acc&) {}
    __device__ static double finish(const Acc& acc) {
        if constexpr (FP32)
            return exp2_split_f32(-acc.s);
        else
            return exp2_double(-acc.s);
    }
    __device__ static double scale(double, int) { return 1.0; }
};

// ------------------------------------------------------ exp of a quadratic
// f = exp(sum_j c_j (x_j - w_j)^2) with c_j of either sign = 2^{sum_j s_j y_j^2},
// y_j = sqrt(|c_j| log2(e)) (x_j - w_j), s_j = sign(c_j).  Per point and direction
// y and s_j y come from two FMAs on the same index (scaling by s_j = +-1 is exact),
// and one more FMA adds their product.  c_j = -g_j^2 is the Gaussian; alternating
// signs with w = 0 are Test 7's f_5.
template <bool FP32>
struct ExpQuadratic {
    struct Dim {
        double b, g, sb, sg;
    };
    struct Acc {
        double s;
    };
    static constexpr int kRenorm = 0;
    static constexpr bool kBlockTerms = false;
    __device__ static void block_terms(const double*, int, int, double, double, double&, double&,
                                       int&) {}
    __device__ static double extra(const double*) { return 0.0; }
    __device__ static Dim dim(const double* p, int d, int j, double inv_n, double sfrac) {
        const double c = p[j], w = p[d + j];
        const double m = sqrt(fabs(c) * kLog2e);
        const double b = m * inv_n, g = fma(b, sfrac, -m * w);
        const double sg = c < 0.0 ? -1.0 : 1.0;
        return Dim{b, g, sg * b, sg * g};
    }
    __device__ static Acc init(double) { return Acc{0.0}; }
    template <class K>
    __device__ static void step(Acc& acc, K k, const Dim& c) {
        const double kd = (double)k;
        const double y = fma(kd, c.b, c.g), ys = fma(kd, c.sb, c.sg);
        acc.s = fma(ys, y, acc.s);
    }
    __device__ static void renorm(Acc&) {}
    __device__ static double finish(const Acc& acc) {
        if constexpr (FP32)
            return exp2_split_f32(acc.s);
        else
            return exp2_double(acc.s);
    }
    __device__ static double scale(double, int) { return 1.0; }
};

// -------------------------------------------------------------- oscillatory
// f = cos(2 pi u + sum_j c_j x_j) = cos(2 pi T),  T = u + sum_j a_j (k_j + sfrac_j)
// in turns, a_j = c_j / (2 pi n).  Only the fractional part of T is needed.
template <bool FP32>
struct Oscillatory {
    struct Dim {
        double a;
    };
    struct Acc {
        double s;
    };
    static constexpr int kRenorm = 0;
    static constexpr bool kBlockTerms = true;
    __device__ static void block_terms(const double* p, int d, int j, double inv_n, double sfrac,
                                       double& ds0, double&, int&) {
        (void)d;
        ds0 += p[1 + j] * kInv2Pi * inv_n * sfrac;
    }
    __device__ static double extra(const double* p) { return p[0]; }
    __device__ static Dim dim(const double* p, int d, int j, double inv_n, double) {
        (void)d;
        return Dim{p[1 + j] * kInv2Pi * inv_n};
    }
    __device__ static Acc init(double s0) { return Acc{s0}; }
    template <class K>
    __device__ static void step(Acc& acc, K k, const Dim& c) {
        acc.s = fma((double)k, c.a, acc.s);
    }
    __device__ static void renorm(Acc&) {}
    __device__ static double finish(const Acc& acc) {
        const double fr = acc.s - rint(acc.s);  // in [-1/2, 1/2]
        if constexpr (FP32)
            return (double)__builtin_amdgcn_cosf((float)fr);  // cos(2 pi t), t in turns
        else
            return cospi(2.0 * fr);
    }
    __device__ static double scale(double, int) { return 1.0; }
};

// ------------------------------------------------------------- product peak
// f = prod_j 1 / (c_j^-2 + (x_j - w_j)^2).  Each factor is scaled by an exact
// power of four sigma_j = 4^-m_j that brings it near 1, so that the running
// product stays in range; the product is renormalised with frexp every kRenorm
// directions and the powers of two are restored exactly at the end.
//   q'_j = sigma_j q_j = y'^2 + g,  y' = 2^-m_j (x_j - w_j) = a k + b,  g = sigma_j c_j^-2.
// m = floor(e / 2) for q = c^-2 + 1/6 = mant 2^e, mant in [1/2, 1), puts q / 4^m in
// [1/2, 2); q needs only its exponent, so an approximate reciprocal serves.
__device__ __forceinline__ int peak_pow4(double c) {
    const double q = __builtin_amdgcn_rcp(c * c) + 1.0 / 6.0;
    return __builtin_amdgcn_frexp_exp(q) >> 1;
}

// FP32_DIMS: per-direction factors in single precision (6 VALU ops per point and
// direction with the exact-float index step).  Their constants a, b, g are rounded to
// FP32 once per direction: a bias that is the same for every point of the direction.
// Its first-order effect on the sum is computed in closed form from the three rounding
// errors (peak_fp32_bias) and divided out of the result; the per-point roundings of y,
// the factor and the product remain, up to a few 2^-24 per factor.  The single-
// precision factors are taken only where that leaves a result within the 1e-6 target:
// d <= kPeakF32MaxDims (launchers); every direction passes fp32_dim_ok, |c_j| <=
// kPeakF32MaxC and a factor range that keeps a run of kRenorm = 16 factors well inside
// the FP32 exponent range; the first-order bias is at most kPeakF32MaxBias; and the
// integrand is flat enough that the sum is not carried by a handful of points
// (n / prod_j (max f_j / mean f_j) >= kPeakF32MinPoints), where the per-point errors,
// which do not average out there, would show.  Other problems take the double-precision
// factors (same scale without the bias term).
// FP32_FINISH: the per-point reciprocal by v_rcp_f32 instead of an IEEE divide.
constexpr int kPeakF32MaxDims = 32;
constexpr double kPeakF32MaxC = 4.0;
constexpr double kPeakF32MaxBias = 1e-6;
constexpr double kPeakF32MinPoints = 16.0;

// Direction j of the single-precision product peak: the first-order relative change of
// the sum that rounding its constants a = s/n, b = s(sfrac/n - w), g = s^2/c^2 to FP32
// causes, and log(max f_j / mean f_j).  With u = x - w on [-w', 1 - w'] (w' = w -
// sfrac/n), q = c^-2 and the factor's denominator s^2 (u^2 + q), the rounding errors
// da, db, dg (relative) change the denominator by s^2 (2u(u + w') da - 2u w' db + q dg);
// weighted by f_j = 1/(u^2 + q) its mean relative effect on f_j is
//   -(2 da (Iu2 + w' Iu1) - 2 w' db Iu1 + q dg I1) / I0,
// I0 = int du/D, I1 = int du/D^2, Iu1 = int u du/D^2, Iu2 = int u^2 du/D^2, D = u^2 + q.
// What the bias of direction j needs: c, w' = w - sfrac/n, and the double-precision
// constants a, b, g that are rounded to FP32 (ProductPeak::dim computes the same).
struct PeakGuardIn {
    double c, wp, a, b, g;
};

__device__ __forceinline__ PeakGuardIn peak_guard_input(const double* p, int d, int j, double inv_n,
                                                        double sfrac) {
    const double c = p[j], w = p[d + j];
    const double s = ldexp(1.0, -peak_pow4(c));
    return PeakGuardIn{c, fma(-sfrac, inv_n, w), s * inv_n, s * fma(sfrac, inv_n, -w), s * s / (c * c)};
}

// The rounding errors are exact differences in double precision; the rest runs in
// single precision (a relative accuracy of 1e-6 is far more than a correction of a
// few 1e-8 needs), with no memory access.
__device__ inline void peak_fp32_bias(const PeakGuardIn& in, double& bias, double& log_ratio) {
    const double a = in.a, b = in.b, g = in.g;
    const float da = (float)((double)(float)a - a) * __builtin_amdgcn_rcpf((float)a);
    const float db = b != 0.0 ? (float)((double)(float)b - b) * __builtin_amdgcn_rcpf((float)b) : 0.0f;
    const float dg = (float)((double)(float)g - g) * __builtin_amdgcn_rcpf((float)g);
    const float ac = (float)fabs(in.c), q = __builtin_amdgcn_rcpf(ac * ac);
    const float wp = (float)in.wp;
    const float lo = -wp, hi = 1.0f - wp;
    const float dlo = lo * lo + q, dhi = hi * hi + q;
    // atan(hi ac) - atan(lo ac) as one arctangent: (x - y) / (1 + x y) with x = hi ac,
    // y = lo ac; x > y, so the difference lies in (0, pi) and takes pi when 1 + x y < 0
    // (1 + x y = 0 gives atan(+inf) = pi / 2)
    const float x = hi * ac, y = lo * ac, den = fmaf(x, y, 1.0f);
    const float t = atanf((x - y) * __builtin_amdgcn_rcpf(den));
    const float dt = den >= 0.0f ? t : t + 3.14159265f;
    const float rlo = __builtin_amdgcn_rcpf(dlo), rhi = __builtin_amdgcn_rcpf(dhi);
    const float I0 = ac * dt, c2 = ac * ac;  // c^2 = 1 / q
    const float I1 = 0.5f * c2 * (hi * rhi - lo * rlo) + 0.5f * c2 * ac * dt;
    const float Iu1 = 0.5f * (rlo - rhi);
    const float Iu2 = I0 - q * I1;
    bias = (double)(-(2.0f * da * (Iu2 + wp * Iu1) - 2.0f * wp * db * Iu1 + q * dg * I1) *
                    __builtin_amdgcn_rcpf(I0));
    const float umin = lo > 0.0f ? lo : (hi < 0.0f ? -hi : 0.0f);  // closest |u| to the peak
    log_ratio = (double)(-__logf((umin * umin + q) * I0));
}

template <bool FP32_DIMS, bool FP32_FINISH>
struct ProductPeak {
    using T = typename std::conditional<FP32_DIMS, float, double>::type;
    struct Dim {
        T a, b, g;
    };
    struct Acc {
        T D;
        int E;
    };
    static constexpr int kRenorm = FP32_DIMS ? 16 : 64;
    static constexpr bool kBlockTerms = true;
    // The FP32-factor form runs only where every direction passes fp32_dim_ok; the
    // double-precision factors serve the other problems (same scale, same constants).
    static constexpr bool kGuarded = FP32_DIMS;
    using Fallback = ProductPeak<false, FP32_FINISH>;
    __device__ static bool fp32_dim_ok(const double* p, int d, int j) {
        const double c = fabs(p[j]), w = p[d + j];
        if (!(c > 0.0 && c <= kPeakF32MaxC)) return false;
        const double s2 = ldexp(1.0, -2 * peak_pow4(c));
        const double ymax = fmax(fabs(w), fabs(1.0 - w));  // |x - w| for x in [0, 1]
        const double lo = s2 / (c * c), hi = s2 * (1.0 / (c * c) + ymax * ymax);
        // a factor in [2^-7, 2^7]: 16 of them stay within 2^+-112 of the renormalised
        // mantissa, inside FP32's normal range
        return lo >= 0x1p-7 && hi <= 0x1p7;
    }
    __device__ static void block_terms(const double* p, int d, int j, double, double, double&,
                                       double&, int& ie) {
        (void)d;
        ie += -2 * peak_pow4(p[j]);
    }
    // The problem-wide part of the guard: per direction log(max f_j / mean f_j) and the
    // first-order bias (summed over the directions by the setup), and the test on the
    // sums (NaN fails it).  The bias sum becomes ds1 of scale() when the test passes.
    using GuardIn = PeakGuardIn;
    __device__ static GuardIn guard_input(const double* p, int d, int j, double inv_n, double sfrac) {
        return peak_guard_input(p, d, j, inv_n, sfrac);
    }
    __device__ static void guard_terms(const GuardIn& in, double& log_ratio, double& bias) {
        peak_fp32_bias(in, bias, log_ratio);
    }
    __device__ static bool block_ok(double log_ratio, double bias, uint32_t n) {
        return log_ratio <= (double)__logf((float)n * (float)(1.0 / kPeakF32MinPoints)) &&
               fabs(bias) <= kPeakF32MaxBias;
    }
    __device__ static double extra(const double*) { return 0.0; }
    __device__ static Dim dim(const double* p, int d, int j, double inv_n, double sfrac) {
        const PeakGuardIn k = peak_guard_input(p, d, j, inv_n, sfrac);
        return Dim{(T)k.a, (T)k.b, (T)k.g};
    }
    __device__ static Acc init(double) { return Acc{(T)1, 0}; }
    template <class K>
    __device__ static void step(Acc& acc, K k, const Dim& c) {
        const T y = fma((T)k, c.a, c.b);
        acc.D *= fma(y, y, c.g);
    }
    __device__ static void renorm(Acc& acc) {
        if constexpr (FP32_DIMS) {
            acc.E += __builtin_amdgcn_frexp_expf(acc.D);
            acc.D = __builtin_amdgcn_frexp_mantf(acc.D);
        } else {
            acc.E += __builtin_amdgcn_frexp_exp(acc.D);
            acc.D = __builtin_amdgcn_frexp_mant(acc.D);
        }
    }
    __device__ static double finish(const Acc& acc) {
        if constexpr (FP32_DIMS) {
            return ldexp((double)__builtin_amdgcn_rcpf(acc.D), -acc.E);
        } else if constexpr (FP32_FINISH) {
            const int e = __builtin_amdgcn_frexp_exp(acc.D);
            const float m = (float)__builtin_amdgcn_frexp_mant(acc.D);
            return ldexp((double)__builtin_amdgcn_rcpf(m), -(acc.E + e));
        } else {
            return ldexp(1.0 / acc.D, -acc.E);
        }
    }
    __device__ static double scale(double ds1, int ie) {
        if constexpr (FP32_DIMS)
            return ldexp(1.0, ie) / (1.0 + ds1);
        else
            return ldexp(1.0, ie);
    }
};

// --------------------------------------------------- Bernoulli products (FP64)
// The product-form sums behind the lattice-quality criteria (eq. 2.4, eq. 2.12):
//   f(x) = prod_j (1 + a_j B_alpha(x_j)) - 1,   params a[d].
// With y = x (1 - x):  B_2(x) = 1/6 - y  and  B_4(x) = y^2 - 1/30, so a factor is
// one FMA on y: (1 + a/6) - a y, or (1 - a/30) + (a y) y.  Criteria are small
// differences of O(1) terms, so everything runs in FP64 in both precisions.
// SCALED (internal criteria): the parameter row holds a_0 .. a_{d-1} and then a
// positive constant C that multiplies the sum (eq. 2.12's prod_j (1 + gamma_j beta)).
template <int ALPHA, bool SCALED = false>
struct BernoulliProduct {
    struct Dim {
        double inv_n, off, a, c0;  // x = k inv_n + off; factor constant c0
    };
    struct Acc {
        double P;
    };
    static constexpr int kRenorm = 0;
    static constexpr bool kBlockTerms = false;
    // B_alpha(1 - x) = B_alpha(x) for even alpha.
    static constexpr bool kMirror = true;
    static constexpr bool kParamScale = SCALED;
    __device__ static void block_terms(const double*, int, int, double, double, double&, double&,
                                       int&) {}
    __device__ static double extra(const double*) { return 0.0; }
    __device__ static Dim dim(const double* p, int d, int j, double inv_n, double sfrac) {
        (void)d;
        const double a = p[j];
        return Dim{inv_n, sfrac * inv_n, a, ALPHA == 2 ? 1.0 + a / 6.0 : 1.0 - a / 30.0};
    }
    __device__ static Acc init(double) { return Acc{1.0}; }
    template <class K>
    __device__ static void step(Acc& acc, K k, const Dim& c) {
        const double x = fma((double)k, c.inv_n, c.off);
        const double y = fma(-x, x, x);
        double f;
        if constexpr (ALPHA == 2)
            f = fma(-c.a, y, c.c0);
        else
            f = fma(c.a * y, y, c.c0);
        acc.P *= f;
    }
    __device__ static void renorm(Acc&) {}
    __device__ static double finish(const Acc& acc) { return acc.P - 1.0; }
    __device__ static double scale(double, int) { return 1.0; }
};

}  // namespace qmc
