/*
 * qmc_oracle.c -- plain FP64 CPU oracle for the rank-1 lattice multi-summation
 * and its MDI-LR tensor-product form (Zhong & Feng, arXiv 2404.08867).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker, not the product: only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or constant with the HIP library; it is
 * deliberately slow and literal so that it can be read against the paper:
 *   - every lattice index k = (i * z_j) mod n is recomputed from scratch with
 *     exact 64-bit integer arithmetic (no incremental update);
 *   - every coordinate is an IEEE double division k / n (plus the shift, wrapped
 *     once into [0,1));
 *   - every sum is a Neumaier-compensated FP64 sum taken in index order.
 *
 * Integrand families (the parameter vector layout is part of the contract):
 *   0 EXP_SUM       f(x) = exp(sum_j c_j x_j)                      params c[d]
 *   1 PRODUCT_PEAK  f(x) = prod_j 1 / (c_j^-2 + (x_j - w_j)^2)     params c[d], w[d]
 *   2 GAUSSIAN      f(x) = exp(-sum_j c_j^2 (x_j - w_j)^2)         params c[d], w[d]
 *   3 OSCILLATORY   f(x) = cos(2 pi u + sum_j c_j x_j)             params u, c[d]
 *   4 EXP_QUADRATIC f(x) = exp(sum_j c_j (x_j - w_j)^2), c_j any sign  params c[d], w[d]
 * Oracle-only integrands used to pin the index map against the paper's tables:
 *   100 TEST1_F     f(x) = x_2 exp(x_1 x_2) / (e - 2)   (Test 1, d = 2)
 *   101 SIN_SQ      f(x) = sin(2 pi + sum_j x_j^2)       (Tests 1 and 2)
 *
 * Parity notes: nothing here is pinned by being retyped elsewhere; the pins live
 * in the test suite (printed table values, closed forms, the dual-lattice
 * character identity, brute force on tiny grids).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_EXP_SUM 0
#define OR_PRODUCT_PEAK 1
#define OR_GAUSSIAN 2
#define OR_OSCILLATORY 3
#define OR_EXP_QUADRATIC 4
#define OR_TEST1_F 100
#define OR_SIN_SQ 101

#define OR_OK 0
#define OR_BAD_ARG 1
#define OR_TOO_BIG 2

static const double OR_PI = 3.14159265358979323846264338327950288;

/* ------------------------------------------------------------------------- */
/* Neumaier (improved Kahan) compensated summation.                          */
/* ------------------------------------------------------------------------- */
typedef struct {
    double s, c;
} neu_t;

static void neu_add(neu_t* a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

static double neu_value(const neu_t* a) { return a->s + a->c; }

/* ------------------------------------------------------------------------- */
/* Korobov generating vector (Sec. 2.2, Korobov-lattice example):            */
/*   z(a) = (1, a, a^2, ..., a^{d-1}) mod n.                                  */
/* ------------------------------------------------------------------------- */
int oracle_korobov(int d, int64_t n, int64_t a, int64_t* z) {
    if (d < 1 || n < 1 || a < 0 || !z) return OR_BAD_ARG;
    if (n >= ((int64_t)1 << 31)) return OR_BAD_ARG;
    int64_t am = a % n;
    int64_t p = 1 % n;
    for (int j = 0; j < d; ++j) {
        z[j] = p;
        p = (p * am) % n; /* p, am < 2^31: the product fits in int64 */
    }
    return OR_OK;
}

/* Point indices of the rank-1 lattice (eq. 2.1): k_ij = (i z_j) mod n, for
 * i = i0 .. i0+count-1, written row-major [count][d]. */
int oracle_lattice_points(int d, int64_t n, const int64_t* z, int64_t i0, int64_t count,
                          int64_t* k_out) {
    if (d < 1 || n < 1 || !z || !k_out || i0 < 0 || count < 0) return OR_BAD_ARG;
    for (int64_t r = 0; r < count; ++r) {
        int64_t i = i0 + r;
        for (int j = 0; j < d; ++j) k_out[r * d + j] = (i % n) * z[j] % n;
    }
    return OR_OK;
}

/* Number of FP64 parameters of a family at dimension d. */
int oracle_param_count(int family, int d) {
    switch (family) {
        case OR_EXP_SUM: return d;
        case OR_PRODUCT_PEAK: return 2 * d;
        case OR_GAUSSIAN: return 2 * d;
        case OR_OSCILLATORY: return d + 1;
        case OR_EXP_QUADRATIC: return 2 * d;
        case OR_TEST1_F: return 0;
        case OR_SIN_SQ: return 0;
        default: return -1;
    }
}

/* The integrand itself, literally as defined above. */
double oracle_eval(int family, int d, const double* p, const double* x) {
    switch (family) {
        case OR_EXP_SUM: {
            double s = 0.0;
            for (int j = 0; j < d; ++j) s += p[j] * x[j];
            return exp(s);
        }
        case OR_PRODUCT_PEAK: {
            double f = 1.0;
            for (int j = 0; j < d; ++j) {
                double c = p[j], w = p[d + j];
                f *= 1.0 / (1.0 / (c * c) + (x[j] - w) * (x[j] - w));
            }
            return f;
        }
        case OR_GAUSSIAN: {
            double s = 0.0;
            for (int j = 0; j < d; ++j) {
                double c = p[j], w = p[d + j];
                s += c * c * (x[j] - w) * (x[j] - w);
            }
            return exp(-s);
        }
        case OR_OSCILLATORY: {
            double t = 2.0 * OR_PI * p[0];
            for (int j = 0; j < d; ++j) t += p[1 + j] * x[j];
            return cos(t);
        }
        case OR_EXP_QUADRATIC: {
            double s = 0.0;
            for (int j = 0; j < d; ++j) {
                double c = p[j], w = p[d + j];
                s += c * (x[j] - w) * (x[j] - w);
            }
            return exp(s);
        }
        case OR_TEST1_F:
            return x[1] * exp(x[0] * x[1]) / (exp(1.0) - 2.0);
        case OR_SIN_SQ: {
            double s = 2.0 * OR_PI;
            for (int j = 0; j < d; ++j) s += x[j] * x[j];
            return sin(s);
        }
        default:
            return NAN;
    }
}

/* Gradient of the integrand with respect to its parameter vector (same layout
 * as params), accumulated as g += scale * df/dp.  Only the five families. */
static void oracle_eval_grad(int family, int d, const double* p, const double* x, double scale,
                             double* g) {
    switch (family) {
        case OR_EXP_SUM: {
            double f = oracle_eval(family, d, p, x);
            for (int j = 0; j < d; ++j) g[j] += scale * x[j] * f;
            break;
        }
        case OR_PRODUCT_PEAK: {
            double f = oracle_eval(family, d, p, x);
            for (int j = 0; j < d; ++j) {
                double c = p[j], w = p[d + j];
                double q = 1.0 / (c * c) + (x[j] - w) * (x[j] - w);
                /* d(1/q)/dc = 2 c^-3 / q^2 ; d(1/q)/dw = 2 (x - w) / q^2 */
                g[j] += scale * f * (2.0 / (c * c * c)) / q;
                g[d + j] += scale * f * 2.0 * (x[j] - w) / q;
            }
            break;
        }
        case OR_GAUSSIAN: {
            double f = oracle_eval(family, d, p, x);
            for (int j = 0; j < d; ++j) {
                double c = p[j], w = p[d + j];
                g[j] += scale * f * (-2.0 * c * (x[j] - w) * (x[j] - w));
                g[d + j] += scale * f * (2.0 * c * c * (x[j] - w));
            }
            break;
        }
        case OR_EXP_QUADRATIC: {
            /* df/dc_j = f (x_j - w_j)^2 ; df/dw_j = -2 c_j (x_j - w_j) f */
            double f = oracle_eval(family, d, p, x);
            for (int j = 0; j < d; ++j) {
                double c = p[j], w = p[d + j];
                g[j] += scale * f * (x[j] - w) * (x[j] - w);
                g[d + j] += scale * f * (-2.0 * c * (x[j] - w));
            }
            break;
        }
        case OR_OSCILLATORY: {
            double t = 2.0 * OR_PI * p[0];
            for (int j = 0; j < d; ++j) t += p[1 + j] * x[j];
            double s = sin(t);
            g[0] += scale * (-2.0 * OR_PI * s);
            for (int j = 0; j < d; ++j) g[1 + j] += scale * (-x[j] * s);
            break;
        }
        default:
            break;
    }
}

/* Coordinates of lattice point i: x_j = {k_ij / n + shift_j} (eq. 2.1 and the
 * shifted lattice of Sec. 2.1), the fractional part taken by one subtraction. */
static void lattice_point(int d, int64_t n, const int64_t* z, const double* shift, int64_t i,
                          double* x) {
    for (int j = 0; j < d; ++j) {
        int64_t k = (i * z[j]) % n;
        double t = (double)k / (double)n;
        if (shift) {
            t += shift[j];
            if (t >= 1.0) t -= 1.0;
        }
        x[j] = t;
    }
}

static int check_lattice_args(int d, int64_t n, const int64_t* z, const double* shift) {
    if (d < 1 || d > 4096 || n < 1 || n >= ((int64_t)1 << 31) || !z) return OR_BAD_ARG;
    for (int j = 0; j < d; ++j)
        if (z[j] < 0 || z[j] >= n) return OR_BAD_ARG;
    if (shift)
        for (int j = 0; j < d; ++j)
            if (!(shift[j] >= 0.0 && shift[j] < 1.0)) return OR_BAD_ARG;
    return OR_OK;
}

/* Plain rank-1 lattice rule (eq. 1.2 with the points of eq. 2.1):
 *   Q = (1/n) sum_{i=0}^{n-1} f(x_i).
 * Also returns A = (1/n) sum |f(x_i)|, the scale used for relative errors of
 * mixed-sign results. */
int oracle_lattice_sum(int d, int64_t n, const int64_t* z, const double* shift, int family,
                       const double* params, double* q_out, double* absq_out) {
    if (check_lattice_args(d, n, z, shift) != OR_OK) return OR_BAD_ARG;
    if (oracle_param_count(family, d) < 0) return OR_BAD_ARG;
    double* x = (double*)malloc(sizeof(double) * (size_t)d);
    if (!x) return OR_TOO_BIG;
    neu_t acc = {0.0, 0.0}, aacc = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) {
        lattice_point(d, n, z, shift, i, x);
        double f = oracle_eval(family, d, params, x);
        neu_add(&acc, f);
        neu_add(&aacc, fabs(f));
    }
    free(x);
    if (q_out) *q_out = neu_value(&acc) / (double)n;
    if (absq_out) *absq_out = neu_value(&aacc) / (double)n;
    return OR_OK;
}

/* Same sum restricted to the index range [i0, i0 + count): the partial sum
 * (not divided by n).  Used to check sampled pieces of very large sums. */
int oracle_lattice_partial(int d, int64_t n, const int64_t* z, const double* shift, int family,
                           const double* params, int64_t i0, int64_t count, double* sum_out) {
    if (check_lattice_args(d, n, z, shift) != OR_OK) return OR_BAD_ARG;
    if (oracle_param_count(family, d) < 0 || i0 < 0 || count < 0 || i0 + count > n)
        return OR_BAD_ARG;
    double* x = (double*)malloc(sizeof(double) * (size_t)d);
    if (!x) return OR_TOO_BIG;
    neu_t acc = {0.0, 0.0};
    for (int64_t i = i0; i < i0 + count; ++i) {
        lattice_point(d, n, z, shift, i, x);
        neu_add(&acc, oracle_eval(family, d, params, x));
    }
    free(x);
    *sum_out = neu_value(&acc);
    return OR_OK;
}

/* Value and parameter gradient of the plain rule:
 *   q = (1/n) sum_i f(x_i),   grad_p = (1/n) sum_i df/dp (x_i).
 * Each gradient component is its own Neumaier sum in index order. */
int oracle_lattice_grad(int d, int64_t n, const int64_t* z, const double* shift, int family,
                        const double* params, double* q_out, double* grad_out) {
    if (check_lattice_args(d, n, z, shift) != OR_OK) return OR_BAD_ARG;
    int P = oracle_param_count(family, d);
    if (P < 0 || family >= 100) return OR_BAD_ARG;
    double* x = (double*)malloc(sizeof(double) * (size_t)d);
    double* g = (double*)malloc(sizeof(double) * (size_t)P);
    neu_t* gacc = (neu_t*)calloc((size_t)P, sizeof(neu_t));
    if (!x || !g || !gacc) {
        free(x);
        free(g);
        free(gacc);
        return OR_TOO_BIG;
    }
    neu_t acc = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) {
        lattice_point(d, n, z, shift, i, x);
        neu_add(&acc, oracle_eval(family, d, params, x));
        memset(g, 0, sizeof(double) * (size_t)P);
        oracle_eval_grad(family, d, params, x, 1.0, g);
        for (int p = 0; p < P; ++p) neu_add(&gacc[p], g[p]);
    }
    if (q_out) *q_out = neu_value(&acc) / (double)n;
    for (int p = 0; p < P; ++p) grad_out[p] = neu_value(&gacc[p]) / (double)n;
    free(x);
    free(g);
    free(gacc);
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Randomly shifted lattice rule (Sec. 2.1: the shifted lattice P + Delta and   */
/* the root-mean-square error over a shift drawn uniformly from [0,1]^d).      */
/* The R shifts are inputs (rows of `shifts`, drawn by the caller):            */
/*   Q_r  = (1/n) sum_i f({x_i + Delta_r}),        r = 0..R-1,                 */
/*   mean = (1/R) sum_r Q_r,                                                    */
/*   se   = sqrt( sum_r (Q_r - mean)^2 / (R (R - 1)) ),                         */
/* the standard error of the mean of R independent estimates (0 when R = 1).   */
/* Both sums are Neumaier sums in r order; the variance is taken in two passes. */
/* ------------------------------------------------------------------------- */
int oracle_shift_ensemble(int d, int64_t n, const int64_t* z, int family, const double* params,
                          const double* shifts, int R, double* q_out, double* mean_out,
                          double* se_out) {
    if (R < 1 || !shifts || !q_out) return OR_BAD_ARG;
    for (int r = 0; r < R; ++r) {
        int rc = oracle_lattice_sum(d, n, z, shifts + (size_t)r * (size_t)d, family, params,
                                    &q_out[r], NULL);
        if (rc != OR_OK) return rc;
    }
    neu_t sum = {0.0, 0.0};
    for (int r = 0; r < R; ++r) neu_add(&sum, q_out[r]);
    const double mean = neu_value(&sum) / (double)R;
    neu_t ss = {0.0, 0.0};
    for (int r = 0; r < R; ++r) neu_add(&ss, (q_out[r] - mean) * (q_out[r] - mean));
    if (mean_out) *mean_out = mean;
    if (se_out) *se_out = R > 1 ? sqrt(neu_value(&ss) / ((double)R * (double)(R - 1))) : 0.0;
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Lattice-quality criteria (Sec. 2.1, eq. 2.4 and eq. 2.12) and the two      */
/* constructions built on them (Sec. 2.2: Korobov search, CBC lattice).        */
/* ------------------------------------------------------------------------- */

static int64_t gcd64(int64_t a, int64_t b);

/* Bernoulli polynomials on [0,1] in their polynomial form; the paper defines
 * B_alpha by its Fourier series (Sec. 2.1), which the tests compare against. */
double oracle_bernoulli(int alpha, double x) {
    if (alpha == 2) return x * x - x + 1.0 / 6.0;
    if (alpha == 4) return x * x * x * x - 2.0 * x * x * x + x * x - 1.0 / 30.0;
    return NAN;
}

/* zeta(alpha) for the even orders used here. */
static double zeta_even(int alpha) {
    if (alpha == 2) return OR_PI * OR_PI / 6.0;
    return OR_PI * OR_PI * OR_PI * OR_PI / 90.0;
}

/* (-1)^{alpha/2 + 1} (2 pi)^alpha / alpha!, the factor in front of B_alpha in eq. 2.4. */
static double p_alpha_coeff(int alpha) {
    double f = 1.0;
    for (int i = 2; i <= alpha; ++i) f *= (double)i;
    return ((alpha / 2) % 2 == 1 ? 1.0 : -1.0) * pow(2.0 * OR_PI, (double)alpha) / f;
}

/* The fractional part {k z / n} by exact integer arithmetic. */
static double frac_kz(int64_t k, int64_t z, int64_t n) { return (double)((k * z) % n) / (double)n; }

/* Generic product-form lattice sum of the criteria:
 *   S = (1/n) sum_{k=0}^{n-1} [ prod_j (1 + a_j B_alpha({k z_j / n})) - 1 ].
 * Also returns A = (1/n) sum_k |prod_j (...) - 1|, the scale of this mixed-sign sum. */
int oracle_lattice_kernel_sum(int d, int64_t n, const int64_t* z, int alpha, const double* a,
                              double* s_out, double* abs_out) {
    if (check_lattice_args(d, n, z, NULL) != OR_OK || (alpha != 2 && alpha != 4) || !a)
        return OR_BAD_ARG;
    neu_t acc = {0.0, 0.0}, aacc = {0.0, 0.0};
    for (int64_t k = 0; k < n; ++k) {
        double prod = 1.0;
        for (int j = 0; j < d; ++j) prod *= 1.0 + a[j] * oracle_bernoulli(alpha, frac_kz(k, z[j], n));
        neu_add(&acc, prod - 1.0);
        neu_add(&aacc, fabs(prod - 1.0));
    }
    *s_out = neu_value(&acc) / (double)n;
    if (abs_out) *abs_out = neu_value(&aacc) / (double)n;
    return OR_OK;
}

/* eq. 2.4, second line, term by term: the k = 0 term (1 + 2 zeta(alpha))^d / n
 * separately, then the terms k = 1..n-1, then -1. */
int oracle_p_alpha(int d, int64_t n, const int64_t* z, int alpha, double* p_out) {
    if (check_lattice_args(d, n, z, NULL) != OR_OK || (alpha != 2 && alpha != 4)) return OR_BAD_ARG;
    const double c = p_alpha_coeff(alpha);
    neu_t acc = {0.0, 0.0};
    neu_add(&acc, -1.0);
    neu_add(&acc, pow(1.0 + 2.0 * zeta_even(alpha), (double)d) / (double)n);
    for (int64_t k = 1; k < n; ++k) {
        double prod = 1.0;
        for (int j = 0; j < d; ++j) prod *= 1.0 + c * oracle_bernoulli(alpha, frac_kz(k, z[j], n));
        neu_add(&acc, prod / (double)n);
    }
    *p_out = neu_value(&acc);
    return OR_OK;
}

/* eq. 2.12, second line (product weights gamma_nu = prod_{j in nu} gamma_j):
 *   e^2 = -prod_j (1 + gamma_j beta)
 *         + (1/n) sum_{k=0}^{n-1} prod_j (1 + gamma_j [B_2({k z_j / n}) + beta]),
 * beta = c^2 - c + 1/3 (anchored Sobolev space, anchor c) or 0 (unanchored). */
int oracle_shift_avg_wce2(int d, int64_t n, const int64_t* z, const double* gamma, double beta,
                          double* e2_out) {
    if (check_lattice_args(d, n, z, NULL) != OR_OK || !gamma) return OR_BAD_ARG;
    double c0 = 1.0;
    for (int j = 0; j < d; ++j) c0 *= 1.0 + gamma[j] * beta;
    neu_t acc = {0.0, 0.0};
    neu_add(&acc, -c0);
    for (int64_t k = 0; k < n; ++k) {
        double prod = 1.0;
        for (int j = 0; j < d; ++j)
            prod *= 1.0 + gamma[j] * (oracle_bernoulli(2, frac_kz(k, z[j], n)) + beta);
        neu_add(&acc, prod / (double)n);
    }
    *e2_out = neu_value(&acc);
    return OR_OK;
}

/* Candidates whose criteria agree to this relative tolerance count as tied:
 * mathematically equal criteria (a and n - a, or in two dimensions z and its
 * inverse mod n) come out of FP64 sums that differ in their last bits. */
#define OR_TIE_REL 1e-10

/* Index of the first value within OR_TIE_REL of the minimum of v[0..m), or -1. */
static int64_t first_near_min(const double* v, int64_t m) {
    double lo = INFINITY;
    for (int64_t i = 0; i < m; ++i)
        if (v[i] < lo) lo = v[i];
    if (!(lo < INFINITY)) return -1;
    for (int64_t i = 0; i < m; ++i)
        if (v[i] <= lo + OR_TIE_REL * fabs(lo)) return i;
    return -1;
}

/* Korobov search (Sec. 2.2): P_alpha(z(a)) for a = a0 .. a0 + count - 1, and the
 * smallest a whose value is within OR_TIE_REL of the smallest value.  Candidates
 * with gcd(a, n) != 1 are not generating vectors of the Korobov example; their
 * value is reported as +infinity and never chosen. */
int oracle_korobov_search(int d, int64_t n, int alpha, int64_t a0, int64_t count, double* p_out,
                          int64_t* best_a) {
    if (d < 1 || n < 2 || a0 < 1 || count < 1 || a0 + count > n || !p_out) return OR_BAD_ARG;
    int64_t* z = (int64_t*)malloc(sizeof(int64_t) * (size_t)d);
    if (!z) return OR_TOO_BIG;
    for (int64_t i = 0; i < count; ++i) {
        const int64_t a = a0 + i;
        if (gcd64(a, n) != 1) {
            p_out[i] = INFINITY;
            continue;
        }
        oracle_korobov(d, n, a, z);
        int rc = oracle_p_alpha(d, n, z, alpha, &p_out[i]);
        if (rc != OR_OK) {
            free(z);
            return rc;
        }
    }
    free(z);
    const int64_t i = first_near_min(p_out, count);
    if (best_a) *best_a = i < 0 ? -1 : a0 + i;
    return OR_OK;
}

/* CBC construction (Sec. 2.2, CBC-lattice example) with product weights:
 * z_1 = 1; for j = 2..d, with z_1..z_{j-1} fixed, z_j is the z in
 * N_n = {1 <= z <= n-1 : gcd(z, n) = 1} that minimises the j-dimensional e^2 of
 * eq. 2.12.  B_2(1 - x) = B_2(x) makes the criterion of z and n - z equal, so
 * the search takes the representatives z <= n/2.
 * Among candidates within OR_TIE_REL of the smallest criterion the smallest z is
 * taken.  e2_out[j-1] is the criterion of the chosen (z_1..z_j).  Every candidate
 * is evaluated by oracle_shift_avg_wce2. */
int oracle_cbc(int d, int64_t n, const double* gamma, double beta, int64_t* z_out, double* e2_out) {
    if (d < 1 || n < 2 || !gamma || !z_out) return OR_BAD_ARG;
    z_out[0] = 1;
    if (e2_out) {
        int rc = oracle_shift_avg_wce2(1, n, z_out, gamma, beta, &e2_out[0]);
        if (rc != OR_OK) return rc;
    }
    const int64_t half = n / 2;
    double* vals = (double*)malloc(sizeof(double) * (size_t)half);
    if (!vals) return OR_TOO_BIG;
    for (int j = 1; j < d; ++j) {
        for (int64_t c = 1; c <= half; ++c) {
            vals[c - 1] = INFINITY;
            if (gcd64(c, n) != 1) continue;
            z_out[j] = c;
            int rc = oracle_shift_avg_wce2(j + 1, n, z_out, gamma, beta, &vals[c - 1]);
            if (rc != OR_OK) {
                free(vals);
                return rc;
            }
        }
        const int64_t i = first_near_min(vals, half);
        if (i < 0) {
            free(vals);
            return OR_BAD_ARG;
        }
        z_out[j] = i + 1;
        if (e2_out) e2_out[j] = vals[i];
    }
    free(vals);
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* MDI-LR for integrands of the coordinate sum (Test 7's f_6 = (1 + sum x)^-(d+1)) */
/* on the improved tensor rule: N_k = N nodes (t + 1/2)/N for k < d and N_last   */
/* for the last direction,                                                      */
/*   Q = (1 / (N^{d-1} N_last)) sum_t g( sum_{k<d} (t_k + 1/2)/N + (t_d + 1/2)/N_last ).  */
/* Outer functions g (params):                                                  */
/*   0 SUM_POWER  g(s) = (b + c s)^(-p)          b, c, p                        */
/*   1 SUM_GAUSS  g(s) = exp(-c^2 (s - w)^2)     c, w                           */
/* ------------------------------------------------------------------------- */
static double sum_g(int gfam, const double* gp, double s) {
    if (gfam == 0) return pow(gp[0] + gp[1] * s, -gp[2]);
    return exp(-gp[0] * gp[0] * (s - gp[1]) * (s - gp[1]));
}

/* Brute force over the full grid (small d and N only). */
int oracle_mdi_sum_brute(int d, int64_t N, int64_t N_last, int gfam, const double* gp, double* q) {
    if (d < 1 || N < 1 || N_last < 1 || (gfam != 0 && gfam != 1) || !gp || !q) return OR_BAD_ARG;
    double total_pts = pow((double)N, (double)(d - 1)) * (double)N_last;
    if (total_pts > 5e7) return OR_TOO_BIG;
    int64_t* t = (int64_t*)calloc((size_t)d, sizeof(int64_t));
    if (!t) return OR_TOO_BIG;
    neu_t acc = {0.0, 0.0};
    for (;;) {
        double s = 0.0;
        for (int k = 0; k < d; ++k) {
            const int64_t Nk = k < d - 1 ? N : N_last;
            s += ((double)t[k] + 0.5) / (double)Nk;
        }
        neu_add(&acc, sum_g(gfam, gp, s));
        int k = 0;
        while (k < d) {
            const int64_t Nk = k < d - 1 ? N : N_last;
            if (++t[k] < Nk) break;
            t[k] = 0;
            ++k;
        }
        if (k == d) break;
    }
    free(t);
    *q = neu_value(&acc) / total_pts;
    return OR_OK;
}

/* Dimension iteration with merged states: after k equal directions the partial
 * sum is (T + k/2) / N for an integer T in [0, k (N - 1)], and c_k[T], the
 * fraction of the N^k index tuples with sum T, is the previous fraction averaged
 * over a window of N states (one step of the iteration of Algorithm 1, with the
 * terms that share a partial sum combined).  counts_out, if not NULL, receives
 * N^k c_k[T] (the number of tuples) for k = d - 1. */
int oracle_mdi_sum_sweep(int d, int64_t N, int64_t N_last, int gfam, const double* gp, double* q,
                         double* counts_out) {
    if (d < 1 || N < 1 || N_last < 1 || (gfam != 0 && gfam != 1) || !gp || !q) return OR_BAD_ARG;
    const int64_t L = (int64_t)(d - 1) * (N - 1) + 1;  /* states after d - 1 directions */
    if (L > ((int64_t)1 << 26)) return OR_TOO_BIG;
    double* c = (double*)calloc((size_t)L, sizeof(double));
    double* nc = (double*)calloc((size_t)L, sizeof(double));
    if (!c || !nc) {
        free(c);
        free(nc);
        return OR_TOO_BIG;
    }
    c[0] = 1.0;
    for (int k = 1; k < d; ++k) {
        const int64_t Lk = (int64_t)k * (N - 1) + 1;
        for (int64_t T = 0; T < Lk; ++T) {
            neu_t w = {0.0, 0.0};
            for (int64_t u = 0; u < N; ++u)
                if (T - u >= 0 && T - u < (int64_t)(k - 1) * (N - 1) + 1) neu_add(&w, c[T - u]);
            nc[T] = neu_value(&w) / (double)N;
        }
        double* tmp = c;
        c = nc;
        nc = tmp;
    }
    neu_t acc = {0.0, 0.0};
    for (int64_t T = 0; T < L; ++T) {
        const double s0 = ((double)T + 0.5 * (double)(d - 1)) / (double)N;
        neu_t inner = {0.0, 0.0};
        for (int64_t u = 0; u < N_last; ++u)
            neu_add(&inner, sum_g(gfam, gp, s0 + ((double)u + 0.5) / (double)N_last));
        neu_add(&acc, c[T] * neu_value(&inner) / (double)N_last);
    }
    *q = neu_value(&acc);
    if (counts_out) {
        const double scale = pow((double)N, (double)(d - 1));
        for (int64_t T = 0; T < L; ++T) counts_out[T] = c[T] * scale;
    }
    free(c);
    free(nc);
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* The affine transformation of Theorem 3.1 and the improved lattice rule's   */
/* point count (Sec. 3.2).  By the theorem's proof (its eq. 13) the transformed */
/* coordinates of lattice point j are                                          */
/*   y_{j,i} = | floor(j z_{i+1}/n)/z_{i+1} - floor(j z_i/n)/z_i |,  i < d,      */
/*   y_{j,d} = (z_d/n) floor(j - (n/z_d) floor(j z_d/n)),                       */
/* all rationals with a fixed denominator per direction: z_i z_{i+1} (i < d)   */
/* and n (i = d).  The oracle keeps the integer numerators                     */
/*   u_{j,i} = | floor(j z_{i+1}/n) z_i - floor(j z_i/n) z_{i+1} |,              */
/*   u_{j,d} = z_d floor(((j z_d) mod n) / z_d),                               */
/* so every comparison is exact.  The tensor grid of the improved rule is the   */
/* product of the per-direction value sets; n* is the number of its points that */
/* no lattice point reaches (the ghost points).                                 */
/* ------------------------------------------------------------------------- */
static void implr_point(int d, int64_t n, const int64_t* z, int64_t j, int64_t* u) {
    for (int i = 0; i + 1 < d; ++i) {
        const int64_t fi = (j * z[i]) / n, fi1 = (j * z[i + 1]) / n;
        const int64_t v = fi1 * z[i] - fi * z[i + 1];
        u[i] = v < 0 ? -v : v;
    }
    u[d - 1] = z[d - 1] * (((j * z[d - 1]) % n) / z[d - 1]);
}

static int implr_args_ok(int d, int64_t n, const int64_t* z) {
    if (d < 1 || n < 1 || n > ((int64_t)1 << 31) || !z) return 0;
    for (int i = 0; i < d; ++i)
        if (z[i] < 1 || z[i] >= n) return 0;
    return 1;
}

int oracle_implr_coords(int d, int64_t n, const int64_t* z, int64_t* u_out) {
    if (!implr_args_ok(d, n, z) || !u_out) return OR_BAD_ARG;
    for (int64_t j = 0; j < n; ++j) implr_point(d, n, z, j, u_out + j * d);
    return OR_OK;
}

/* The same numerators at m chosen lattice points js[0 .. m), 0 <= js[k] < n. */
int oracle_implr_coords_at(int d, int64_t n, const int64_t* z, int64_t m, const int64_t* js,
                           int64_t* u_out) {
    if (!implr_args_ok(d, n, z) || m < 0 || (m > 0 && (!js || !u_out))) return OR_BAD_ARG;
    for (int64_t k = 0; k < m; ++k) {
        if (js[k] < 0 || js[k] >= n) return OR_BAD_ARG;
        implr_point(d, n, z, js[k], u_out + k * d);
    }
    return OR_OK;
}

static int cmp_i64(const void* a, const void* b) {
    const int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static const int64_t* g_rows;  /* qsort context: rows of d numerators */
static int g_d;
static int cmp_row(const void* a, const void* b) {
    const int64_t ra = *(const int64_t*)a, rb = *(const int64_t*)b;
    for (int i = 0; i < g_d; ++i) {
        const int64_t x = g_rows[ra * g_d + i], y = g_rows[rb * g_d + i];
        if (x != y) return x < y ? -1 : 1;
    }
    return 0;
}

/* counts_out[i] = number of distinct values of direction i; *nstar = product of
 * the counts minus the number of distinct transformed points; *distinct = that
 * number (n when the transformation is one-to-one on the lattice). */
int oracle_implr_grid(int d, int64_t n, const int64_t* z, int64_t* counts_out, int64_t* nstar,
                      int64_t* distinct) {
    if (d < 1 || n < 1 || n > ((int64_t)1 << 24) || !z || !counts_out) return OR_BAD_ARG;
    int64_t* u = (int64_t*)malloc(sizeof(int64_t) * (size_t)n * (size_t)d);
    int64_t* col = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    if (!u || !col || !idx) {
        free(u);
        free(col);
        free(idx);
        return OR_TOO_BIG;
    }
    int rc = oracle_implr_coords(d, n, z, u);
    if (rc != OR_OK) {
        free(u);
        free(col);
        free(idx);
        return rc;
    }
    double grid = 1.0;
    for (int i = 0; i < d; ++i) {
        for (int64_t j = 0; j < n; ++j) col[j] = u[j * d + i];
        qsort(col, (size_t)n, sizeof(int64_t), cmp_i64);
        int64_t c = 1;
        for (int64_t j = 1; j < n; ++j) c += col[j] != col[j - 1];
        counts_out[i] = c;
        grid *= (double)c;
    }
    for (int64_t j = 0; j < n; ++j) idx[j] = j;
    g_rows = u;
    g_d = d;
    qsort(idx, (size_t)n, sizeof(int64_t), cmp_row);
    int64_t dist = 1;
    for (int64_t j = 1; j < n; ++j) dist += cmp_row(&idx[j], &idx[j - 1]) != 0;
    if (distinct) *distinct = dist;
    if (nstar) *nstar = grid < 9.0e18 ? (int64_t)grid - dist : -1;
    free(u);
    free(col);
    free(idx);
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Per-direction node counts of the transformed grid (eq. 3.5):              */
/*   n_i = lcm(z_i, z_{i+1}) / min(z_i, z_{i+1}),  i < d;   n_d = ceil(n / z_d). */
/* ------------------------------------------------------------------------- */
static int64_t gcd64(int64_t a, int64_t b) {
    while (b) {
        int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

int oracle_mdi_dims(int d, const int64_t* z, int64_t n, int64_t* N_out) {
    if (d < 1 || !z || !N_out || n < 1) return OR_BAD_ARG;
    for (int i = 0; i + 1 < d; ++i) {
        int64_t a = z[i], b = z[i + 1];
        if (a < 1 || b < 1) return OR_BAD_ARG;
        int64_t g = gcd64(a, b);
        int64_t mn = a < b ? a : b;
        /* lcm / min = (a / g) * b / min, computed without overflow for a, b < 2^31 */
        int64_t l = (a / g) * b;
        N_out[i] = l / mn;
    }
    if (z[d - 1] < 1) return OR_BAD_ARG;
    N_out[d - 1] = (n + z[d - 1] - 1) / z[d - 1];
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* MDI-LR value of the improved (tensor-product) rule.                       */
/* Reading used throughout: the transformed grid has N_k nodes in direction  */
/* k at the cell centres xi_{k,s} = (s + 1/2) / N_k, with the equal weight    */
/* 1 / prod_k N_k, i.e.                                                       */
/*   Qhat = (prod N_k)^-1 sum_{s in prod [0,N_k)} f(xi_{1,s_1}, ..., xi_{d,s_d}). */
/* ------------------------------------------------------------------------- */

/* Brute force over the whole grid (for tiny grids only). */
int oracle_mdi_lr_brute(int d, const int64_t* N, int family, const double* params, double* q_out) {
    if (d < 1 || !N || oracle_param_count(family, d) < 0) return OR_BAD_ARG;
    double total = 1.0;
    for (int k = 0; k < d; ++k) {
        if (N[k] < 1) return OR_BAD_ARG;
        total *= (double)N[k];
    }
    if (total > 67108864.0) return OR_TOO_BIG; /* 2^26 grid points */
    int64_t* s = (int64_t*)calloc((size_t)d, sizeof(int64_t));
    double* x = (double*)malloc(sizeof(double) * (size_t)d);
    if (!s || !x) {
        free(s);
        free(x);
        return OR_TOO_BIG;
    }
    neu_t acc = {0.0, 0.0};
    int64_t count = (int64_t)total;
    for (int64_t r = 0; r < count; ++r) {
        for (int k = 0; k < d; ++k) x[k] = ((double)s[k] + 0.5) / (double)N[k];
        neu_add(&acc, oracle_eval(family, d, params, x));
        /* mixed-radix increment of the multi-index s */
        for (int k = 0; k < d; ++k) {
            if (++s[k] < N[k]) break;
            s[k] = 0;
        }
    }
    free(s);
    free(x);
    *q_out = neu_value(&acc) / total;
    return OR_OK;
}

/* One factor phi_k(y) of a product-form integrand, as a complex number
 * (re, im).  EXP_SUM: e^{c y}; GAUSSIAN: e^{-c^2 (y-w)^2};
 * PRODUCT_PEAK: 1 / (c^-2 + (y-w)^2); OSCILLATORY: e^{i c y};
 * EXP_QUADRATIC: e^{c (y-w)^2}. */
static void factor(int family, int d, const double* p, int k, double y, double* re, double* im) {
    *im = 0.0;
    switch (family) {
        case OR_EXP_SUM: *re = exp(p[k] * y); break;
        case OR_GAUSSIAN: {
            double c = p[k], w = p[d + k];
            *re = exp(-c * c * (y - w) * (y - w));
            break;
        }
        case OR_PRODUCT_PEAK: {
            double c = p[k], w = p[d + k];
            *re = 1.0 / (1.0 / (c * c) + (y - w) * (y - w));
            break;
        }
        case OR_EXP_QUADRATIC: {
            double c = p[k], w = p[d + k];
            *re = exp(c * (y - w) * (y - w));
            break;
        }
        case OR_OSCILLATORY: {
            double a = p[1 + k] * y;
            *re = cos(a);
            *im = sin(a);
            break;
        }
        default: *re = NAN; break;
    }
}

/* MDI with m = 1 (Algorithm 1 driven by Algorithm 2) for product-form
 * integrands.  The "symbolic function" g_k that remains after the first
 * d - k coordinates have been summed out is carried as a coefficient C times
 * the product of the remaining factors; eq. 2.14c with m = 1 and weight 1/N_k
 * then turns g_k into g_{k-1} by multiplying C with the one-dimensional
 * weighted sum M = (1/N) sum_s phi(xi_s) of the coordinate being deleted.
 * For OSCILLATORY the function is Re(e^{2 pi i u} prod_k e^{i c_k y_k}) and C
 * is complex.  C is kept as a mantissa pair with a separate power-of-two
 * exponent so that d in the thousands cannot overflow. */
int oracle_mdi_lr_sweep(int d, const int64_t* N, int family, const double* params, double* q_out) {
    if (d < 1 || !N || family < 0 || family > 4) return OR_BAD_ARG;
    double cre = 1.0, cim = 0.0;
    int cexp = 0;
    if (family == OR_OSCILLATORY) {
        cre = cos(2.0 * OR_PI * params[0]);
        cim = sin(2.0 * OR_PI * params[0]);
    }
    for (int k = 0; k < d; ++k) { /* delete the first remaining coordinate */
        if (N[k] < 1) return OR_BAD_ARG;
        neu_t mre = {0.0, 0.0}, mim = {0.0, 0.0};
        for (int64_t s = 0; s < N[k]; ++s) {
            double y = ((double)s + 0.5) / (double)N[k];
            double re, im;
            factor(family, d, params, k, y, &re, &im);
            neu_add(&mre, re);
            neu_add(&mim, im);
        }
        double Mre = neu_value(&mre) / (double)N[k];
        double Mim = neu_value(&mim) / (double)N[k];
        double nre = cre * Mre - cim * Mim;
        double nim = cre * Mim + cim * Mre;
        double big = fabs(nre) > fabs(nim) ? fabs(nre) : fabs(nim);
        int e = 0;
        if (big > 0.0 && isfinite(big)) {
            frexp(big, &e);
            nre = ldexp(nre, -e);
            nim = ldexp(nim, -e);
            cexp += e;
        }
        cre = nre;
        cim = nim;
    }
    *q_out = ldexp(cre, cexp);
    return OR_OK;
}

/* The one-dimensional weighted sums M_k themselves (real part, imaginary part),
 * for diagnostics of the sweep. */
int oracle_mdi_lr_factors(int d, const int64_t* N, int family, const double* params, double* m_re,
                          double* m_im) {
    if (d < 1 || !N || family < 0 || family > 4) return OR_BAD_ARG;
    for (int k = 0; k < d; ++k) {
        if (N[k] < 1) return OR_BAD_ARG;
        neu_t mre = {0.0, 0.0}, mim = {0.0, 0.0};
        for (int64_t s = 0; s < N[k]; ++s) {
            double y = ((double)s + 0.5) / (double)N[k];
            double re, im;
            factor(family, d, params, k, y, &re, &im);
            neu_add(&mre, re);
            neu_add(&mim, im);
        }
        m_re[k] = neu_value(&mre) / (double)N[k];
        m_im[k] = neu_value(&mim) / (double)N[k];
    }
    return OR_OK;
}
