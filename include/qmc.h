/*
 * qmc.h -- C ABI of libqmc.so: rank-1 lattice multi-summation on MI355X (gfx950).
 *
 * The library evaluates the quasi-Monte Carlo lattice rule of Zhong & Feng,
 * "An efficient implementation algorithm for quasi-Monte Carlo approximations of
 * high-dimensional integrals" (arXiv 2404.08867):
 *
 *   plain form   Q = (1/n) sum_{i=0}^{n-1} f(x_i),  x_ij = { k_ij / n + Delta_j },
 *                k_ij = (i z_j) mod n                      (eq. 1.2, eq. 2.1, Sec. 2.1 shifted lattice)
 *   MDI-LR form  Qhat = (prod_k N_k)^-1 sum_{s} f((s_1 + 1/2)/N_1, ..., (s_d + 1/2)/N_d)
 *                evaluated by dimension sweeps           (Sec. 3.2 improved rule, eq. iQMC,
 *                                                          Algorithms 1 and 2 with m = 1)
 *
 * Integrand families (fixed parameter layout, FP64, device memory):
 *   QMC_EXP_SUM       f(x) = exp(sum_j c_j x_j)                    params: c[d]
 *   QMC_PRODUCT_PEAK  f(x) = prod_j 1 / (c_j^-2 + (x_j - w_j)^2)   params: c[d], w[d]
 *   QMC_GAUSSIAN      f(x) = exp(-sum_j c_j^2 (x_j - w_j)^2)       params: c[d], w[d]
 *   QMC_OSCILLATORY   f(x) = cos(2 pi u + sum_j c_j x_j)           params: u, c[d]
 *   QMC_EXP_QUADRATIC f(x) = exp(sum_j c_j (x_j - w_j)^2)         params: c[d], w[d]
 *                     (c_j of either sign; c_j = -g_j^2 is the Gaussian, alternating
 *                     signs with w = 0 are Test 7's f_5)
 * (the families of the paper's Tests 3-7: Gaussian, exp of a signed sum,
 *  product peak, cos of a sum, exp of a signed sum of squares -- with
 *  per-direction parameters).
 *
 * Conventions for every entry point:
 *   - Every call returns a qmc_status; no C++ exception crosses the ABI.  On an
 *     error nothing is launched and qmc_last_error() (thread-local) says why.
 *   - "device" arrays are caller-owned HIP device allocations; "host" arrays are
 *     ordinary host memory.  The library never frees caller memory.
 *   - Launches are asynchronous on `stream` (a hipStream_t; NULL = the default
 *     stream).  Results are valid once the stream has been synchronised.
 *   - No entry point that launches work allocates memory.  Scratch space comes
 *     (except for qmc_lattice_sum_noalloc) from the caller's workspace `ws` (device, 256-byte aligned, at least the
 *     size reported by the matching *_workspace_size query).  Its first 4 MiB
 *     hold completion counters and reduction slots: a workspace must be
 *     zero-filled once before its first use, and every call leaves that region at
 *     zero again, so one workspace serves any sequence of calls to any entry point
 *     without clearing.
 *     Calls that run concurrently need distinct workspaces.
 *   - Scalar arguments are validated before anything is launched:
 *       1 <= d <= 1024, 1 <= n < 2^31, 1 <= nsets <= 4096 (qmc_mdi_lr: 2^24),
 *       valid family and precision.  z_j in [0, n) and Delta_j in [0, 1) are the
 *       caller's contract for device arrays (not read back on the host).
 *   - Debug mode: with QMC_VALIDATE=1 in the environment, the entry points that take
 *     z, shift, gamma or N arrays (the plain sum, its shifts and adjoint, the criteria,
 *     the point export, batch plan creation, MDI-LR) read them back on their stream
 *     (synchronously, into host buffers) and return QMC_ERR_INVALID_ARG for an entry
 *     out of range, before launching anything.  While the stream is being captured
 *     into a graph the read-back is skipped.
 *   - Results are deterministic: every reduction runs in a fixed order, so a
 *     given call on given inputs returns bit-identical values on every run.
 */
#ifndef QMC_H
#define QMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QMC_OK = 0,
    QMC_ERR_INVALID_ARG = 1,   /* a scalar or pointer argument is out of its documented range */
    QMC_ERR_UNSUPPORTED = 2,   /* valid request the library does not implement */
    QMC_ERR_WORKSPACE = 3,     /* workspace missing, misaligned or smaller than required */
    QMC_ERR_OUT_OF_MEMORY = 4, /* a plan-creation allocation failed */
    QMC_ERR_DEVICE = 5         /* the HIP runtime reported an error */
} qmc_status;

typedef enum {
    QMC_EXP_SUM = 0,
    QMC_PRODUCT_PEAK = 1,
    QMC_GAUSSIAN = 2,
    QMC_OSCILLATORY = 3,
    QMC_EXP_QUADRATIC = 4
} qmc_family;

/* QMC_FP64: every arithmetic step in IEEE double precision.
 * QMC_FP32_COMPENSATED: exact integer indices; the index-to-coordinate map, the
 * argument sums and all accumulation in double; the per-point transcendental
 * (exp2, cos, reciprocal) and the product-peak factors in single precision
 * (up to 32 directions, with the first-order bias of their rounded constants divided
 * out; in double for a problem with |c_j| > 4, factors beyond [2^-7, 2^7], a bias
 * above 1e-6 or fewer than 16 effective lattice points).  Its relative error against the FP64 rule is reported by the tests and the
 * benchmark for every workload (target <= 1e-6).  In the MDI-LR product the FP32
 * error of one factor repeats in every direction with the same parameters, so for
 * inputs with many identical directions it can grow linearly in d.  The exp-sum,
 * Gaussian and signed-quadratic factors are summed by FP64 node recurrences, the
 * exp-sum and oscillatory node sums taken in closed form in FP64 and the product-peak
 * reciprocals refined in FP64; oscillatory factors with more than a quarter turn
 * between nodes and Gaussian factors too narrow for the recurrence keep FP32 node
 * values. */
typedef enum { QMC_FP64 = 0, QMC_FP32_COMPENSATED = 1 } qmc_precision;

/* How qmc_mdi_lr_dims obtains n for the Korobov lattice z(a) (Lemma 3.2, eq. 3.5). */
typedef enum {
    QMC_N_A_POW_D = 0,         /* n = a^d:      N_k = a for every k                     */
    QMC_N_ONE_PLUS_A_POW_D = 1,/* n = 1 + a^d:  N_k = a (k < d), N_d = a + 1             */
    QMC_N_EXPLICIT = 2         /* n given:      eq. 3.5 on z(a) = (1, a, ..) mod n        */
} qmc_n_mode;

/* ---- library information ------------------------------------------------- */
const char* qmc_version(void);
const char* qmc_status_string(qmc_status s);
/* Message of the last failing call on this thread ("" if none). */
const char* qmc_last_error(void);

/* ---- host helpers ------------------------------------------------------ */

/* Korobov generating vector (Sec. 2.2, Korobov-lattice example):
 *   z_out[j] = a^j mod n, j = 0..d-1, computed with exact 64-bit modular products.
 * z_out: host, d entries.  Requires 1 <= d <= 1024, 1 <= n < 2^31, 0 <= a.
 * gcd(a, n) = 1 is not enforced (the rule is defined for any z). */
qmc_status qmc_korobov(int32_t d, int64_t n, int64_t a, int64_t* z_out);

/* Node counts of the transformed tensor grid for the Korobov lattice (eq. 3.5):
 *   N_i = lcm(z_i, z_{i+1}) / min(z_i, z_{i+1}) for i < d,  N_d = ceil(n / z_d),
 * with n chosen by n_mode (n_explicit is used only by QMC_N_EXPLICIT).
 * N_out: host, d entries.  Fails with QMC_ERR_INVALID_ARG when a count would
 * exceed 2^20. */
qmc_status qmc_mdi_lr_dims(int32_t d, int64_t a, int32_t n_mode, int64_t n_explicit,
                           int32_t* N_out);

/* Number of FP64 parameters of `family` at dimension d (d, 2d, 2d or d + 1). */
qmc_status qmc_param_count(int32_t family, int32_t d, int32_t* count);

/* Workspace bytes sufficient for qmc_lattice_sum, qmc_lattice_sum_adjoint and
 * qmc_mdi_lr on problems with d <= max_d, n <= max_n and nsets <= max_sets. */
qmc_status qmc_workspace_size(int32_t max_d, int64_t max_n, int32_t max_sets, size_t* bytes);

/* ---- the plain rule ----------------------------------------------------- */

/* Plain rank-1 lattice rule, fused in one launch: exact integer point indices
 * generated in registers, coordinates, integrand, per-thread accumulation,
 * wavefront and workgroup reductions, and a fixed-order cross-workgroup sum.
 *   Q_s = (1/n) sum_{i=0}^{n-1} f_s(x_i),   s = 0..nsets-1,
 * with x_ij = {k_ij / n + shift_j}, k_ij = (i z_j) mod n (eq. 1.2, eq. 2.1; the
 * shifted lattice of Sec. 2.1).  All nsets parameter sets share z and shift.
 *   z       device int64[d], 0 <= z_j < n
 *   shift   device double[d] in [0,1), or NULL for the unshifted lattice
 *   params  device double[nsets][qmc_param_count(family, d)]
 *   q_out   device double[nsets]
 *   ws      device workspace of qmc_workspace_size(d, n, nsets) bytes */
qmc_status qmc_lattice_sum(int32_t d, int64_t n, const int64_t* z, const double* shift,
                           int32_t family, const double* params, int32_t nsets,
                           int32_t precision, double* q_out, void* ws, size_t ws_bytes,
                           void* stream);

/* qmc_lattice_sum without a workspace argument, for callers that cannot allocate
 * device memory (code under graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same kernels and the same result, bit for bit, with
 * their counters and reduction slots in a static device array of 4 MiB inside the
 * library (one per device, set up and cleared by the first call on that device
 * with the device current, held until the process ends).  The call allocates
 * nothing, on the device or the host.
 *   Arguments as qmc_lattice_sum (limits too: nsets <= 4096 fits the static
 *   scratch; a larger need returns QMC_ERR_WORKSPACE).
 * Every call on a device shares that device's array; a completed call leaves it
 * zero for the next one.  Calls that overlap on one device (other streams, other
 * threads) race and give wrong results: serialise them, or use qmc_lattice_sum
 * with distinct workspaces. */
qmc_status qmc_lattice_sum_noalloc(int32_t d, int64_t n, const int64_t* z, const double* shift,
                                   int32_t family, const double* params, int32_t nsets,
                                   int32_t precision, double* q_out, void* stream);

/* Randomly shifted lattice rule (Sec. 2.1: the shifted lattice P + Delta, whose
 * error averaged over a shift drawn uniformly from [0,1]^d is the quality measure
 * of randomly shifted rules).  For R = nshifts shifts sharing z and one parameter
 * set, in one launch:
 *   Q_r = (1/n) sum_{i=0}^{n-1} f({k_i / n + Delta_r}),   r = 0..R-1,
 * then, if stats_out is not NULL, a second small launch on the same stream writes
 *   stats_out[0] = mean = (1/R) sum_r Q_r,
 *   stats_out[1] = sqrt(sum_r (Q_r - mean)^2 / (R (R - 1)))   (0 for R = 1),
 * the standard error of the mean, both summed in a fixed order.  The shifts are
 * inputs: the caller draws them (e.g. i.i.d. uniform on [0,1)^d).
 *   z          device int64[d], 0 <= z_j < n
 *   shifts     device double[R][d], each in [0,1) (caller's contract)
 *   nshifts    R in [1, 4096]
 *   params     device double[qmc_param_count(family, d)], one set shared by all shifts
 *   q_out      device double[R]
 *   stats_out  device double[2], or NULL
 *   ws         device workspace of qmc_workspace_size(d, n, R) bytes */
qmc_status qmc_lattice_sum_shifts(int32_t d, int64_t n, const int64_t* z, const double* shifts,
                                  int32_t nshifts, int32_t family, const double* params,
                                  int32_t precision, double* q_out, double* stats_out, void* ws,
                                  size_t ws_bytes, void* stream);

/* ---- MDI-LR for integrands of the coordinate sum ---------------------------
 * f(x) = g(x_1 + ... + x_d), e.g. Test 7's f_6 = (1 + sum x)^-(d+1), on the
 * improved tensor midpoint rule with N nodes (t + 1/2)/N in each of the first
 * d - 1 directions and N_last in the last (eq. 3.5 gives N_last = a or
 * ceil(n / a^{d-1}) with N = a):
 *   Q = (1 / (N^{d-1} N_last)) sum_t g( sum_{k<d} (t_k + 1/2)/N + (t_d + 1/2)/N_last ).
 * Partial sums after k equal directions take k (N - 1) + 1 values, so the
 * dimension iteration merges terms and carries their weights (one window
 * average per direction); the result is evaluated for every parameter set of g.
 * Outer functions (params per set, FP64):
 *   QMC_SUM_POWER  g(s) = (b + c s)^(-p)         b, c, p   (b + c s > 0 on [0, d])
 *   QMC_SUM_GAUSS  g(s) = exp(-c^2 (s - w)^2)    c, w
 * QMC_FP32_COMPENSATED takes the exponent in FP64 and its fractional power in FP32. */
typedef enum { QMC_SUM_POWER = 0, QMC_SUM_GAUSS = 1 } qmc_sum_family;

/* Workspace bytes of qmc_mdi_lr_sum at d, N: the 4 MiB zero region shared by every
 * entry point (left untouched), then 35 vectors of d (N - 1) + 1 doubles (weights
 * and convolution partials; when N_last = N the last direction merges into the
 * states too). */
qmc_status qmc_mdi_lr_sum_workspace_size(int32_t d, int32_t N, size_t* bytes);

/* Q for nsets parameter sets of g (two launches on `stream`).
 *   d in [1, 1024]; N, N_last in [1, 2^20]; d (N - 1) + 1 <= 2^20
 *   params  device double[nsets][3] (power) or [nsets][2] (Gaussian)
 *   q_out   device double[nsets];  nsets in [1, 2^24]
 *   ws      device workspace of qmc_mdi_lr_sum_workspace_size(d, N) bytes */
qmc_status qmc_mdi_lr_sum(int32_t d, int32_t N, int32_t N_last, int32_t gfamily, const double* params,
                          int32_t nsets, int32_t precision, double* q_out, void* ws, size_t ws_bytes,
                          void* stream);

/* ---- the improved lattice rule's tensor grid (Theorem 3.1, Sec. 3.2) ------
 * For the Korobov lattice z = (1, a, ..., a^{d-1}) with a^{d-1} < n, the affine
 * transformation of Theorem 3.1 maps lattice point j to the grid ranks
 *   s_i = floor(j z_{i+1}/n) - a floor(j z_i/n) in [0, a)   (i < d),
 *   s_d = floor(((j z_d) mod n) / z_d) in [0, ceil(n / z_d)),
 * on a tensor grid of a^{d-1} ceil(n / a^{d-1}) points (eq. 3.5).  The improved
 * rule adds the grid points no lattice point reaches; their number n* is
 * computed exactly by one of two methods:
 *   QMC_IMPLR_AUTO    every point's grid index (s_1 most significant) is computed
 *                     and each consecutive pair is checked to increase strictly;
 *                     if all pass the n points are distinct and n* = grid - n,
 *                     otherwise the bitmap count runs (decided on the device);
 *   QMC_IMPLR_BITMAP  every point sets its grid point's bit in a bitmap of the
 *                     grid and n* = grid - set bits (no assumption on the order).
 * Six launches on `stream` (the unused ones exit at once).
 *   d in [1, 64]; n in [2, 2^31); 1 <= a < n with a^{d-1} < n.  gcd(a, n) = 1 is
 *   not required: the equal-count case n = a^d has gcd a.  n* always counts the
 *   points of eq. 3.5's grid, which contains every transformed point.
 *   counts_host_out  host int64[d]: the per-direction counts (eq. 3.5), or NULL
 *   nstar_out        device int64[1]
 *   ws               device workspace of qmc_implr_workspace_size(d, n, a) bytes: the
 *                    4 MiB zero region shared by every entry point (left untouched),
 *                    256 bytes of state and the grid's bitmap (no zero-fill needed)
 * Errors: QMC_ERR_INVALID_ARG for arguments outside these ranges, an unknown
 * method or a NULL nstar_out, QMC_ERR_WORKSPACE for a missing, misaligned or short
 * workspace; nothing is launched and counts_host_out is left untouched then. */
typedef enum { QMC_IMPLR_AUTO = 0, QMC_IMPLR_BITMAP = 1 } qmc_implr_method;
qmc_status qmc_implr_workspace_size(int32_t d, int64_t n, int64_t a, size_t* bytes);
qmc_status qmc_implr_grid(int32_t d, int64_t n, int64_t a, int32_t method, int64_t* counts_host_out,
                          int64_t* nstar_out, void* ws, size_t ws_bytes, void* stream);

/* The grid ranks of lattice points j = j0 .. j0 + count - 1 under the same
 * transformation (y_i = s_i / z_{i+1} for i < d, y_d = s_d z_d / n), direction-major:
 * s_out[i * ld + (j - j0)] = s_i(j).  One launch on `stream`; d, n, a as above,
 * 0 <= j0, j0 + count <= n, count <= ld <= 2^40.  Each lane writes four consecutive ranks
 * at once; rows that start on 16-byte boundaries (s_out and 4 ld multiples of 16)
 * are written fastest.
 *   s_out  device int32[d][ld], 4-byte aligned; may be NULL when count = 0 */
qmc_status qmc_implr_points(int32_t d, int64_t n, int64_t a, int64_t j0, int64_t count, int32_t* s_out,
                            int64_t ld, void* stream);

/* ---- lattice-quality criteria (Sec. 2.1) and constructions (Sec. 2.2) ----
 *
 * Both criteria of the paper are product-form lattice sums with Bernoulli factors,
 *   S(z) = (1/n) sum_{k=0}^{n-1} [ prod_j (1 + a_j B_alpha({k z_j / n})) - 1 ],
 * B_2(x) = x^2 - x + 1/6, B_4(x) = x^4 - 2x^3 + x^2 - 1/30 (alpha = 2 or 4):
 *   P_alpha(z) of eq. 2.4 is S with a_j = (-1)^{alpha/2+1} (2 pi)^alpha / alpha! for
 *   every j (2 pi^2 for alpha = 2, -2 pi^4 / 3 for alpha = 4);
 *   the squared shift-averaged worst-case error of eq. 2.12 with product weights
 *   gamma_j is prod_j (1 + gamma_j beta) * S with a_j = gamma_j / (1 + gamma_j beta)
 *   (beta = c^2 - c + 1/3 for the anchored space with anchor c, 0 unanchored).
 * The library derives the weights a_j and the factor prod_j (1 + gamma_j beta) on the
 * device: qmc_p_alpha, qmc_shift_avg_wce2, qmc_korobov_search and qmc_cbc return the
 * criteria themselves; qmc_bernoulli_sum returns S for weights the caller chooses.
 * Everything runs in FP64: criteria are small differences of O(1) terms.
 * The terms of k and n - k are equal (the points are mirror images and
 * B_alpha(1 - x) = B_alpha(x)), so the device evaluates k <= n/2 only, with
 * weight 2 except for k = 0 and, for even n, k = n/2: half the terms above.
 * Candidates whose values agree to 1e-10 relative count as tied; the smallest
 * candidate is chosen (the criteria of c and n - c are always equal).  Candidates
 * with gcd(c, n) != 1 get +infinity.  Values beyond the FP64 range (products that
 * overflow for large d and weights) come out as +-infinity or NaN. */

/* Which criterion a search or construction minimises. */
typedef enum {
    QMC_CRIT_P_ALPHA = 0, /* P_alpha of eq. 2.4 (alpha = 2 or 4; gamma and beta unused)      */
    QMC_CRIT_WCE2 = 1     /* e^2 of eq. 2.12 with product weights gamma_j and beta (alpha 2) */
} qmc_criterion_kind;

typedef struct {
    int32_t kind;          /* qmc_criterion_kind */
    int32_t alpha;         /* QMC_CRIT_P_ALPHA: 2 or 4; ignored by QMC_CRIT_WCE2 */
    const double* gamma;   /* QMC_CRIT_WCE2: device double[d], finite gamma_j >= 0 (caller's
                              contract; read back and checked under QMC_VALIDATE) */
    double beta;           /* QMC_CRIT_WCE2: finite beta >= 0 */
} qmc_criterion;

/* Workspace bytes of the criteria entry points (qmc_bernoulli_sum, qmc_p_alpha,
 * qmc_shift_avg_wce2, qmc_korobov_search, qmc_cbc) at d, n. */
qmc_status qmc_criteria_workspace_size(int32_t d, int64_t n, size_t* bytes);

/* P_alpha(z) of eq. 2.4 for nz generating vectors (rows of z), two launches.
 *   z      device int64[nz][d], 0 <= z_j < n;  nz in [1, 4096];  n in [2, 2^31)
 *   alpha  2 or 4
 *   p_out  device double[nz]
 *   ws     device workspace of qmc_criteria_workspace_size(d, n) bytes
 * Errors: QMC_ERR_INVALID_ARG (ranges, NULL pointers), QMC_ERR_WORKSPACE. */
qmc_status qmc_p_alpha(int32_t d, int64_t n, const int64_t* z, int32_t nz, int32_t alpha, double* p_out,
                       void* ws, size_t ws_bytes, void* stream);

/* e^2(z) of eq. 2.12 (squared worst-case error averaged over shifts, product
 * weights gamma_j, beta as above) for nz generating vectors, two launches.
 *   gamma   device double[d];  beta finite, >= 0;  other arguments as qmc_p_alpha */
qmc_status qmc_shift_avg_wce2(int32_t d, int64_t n, const int64_t* z, int32_t nz, const double* gamma,
                              double beta, double* e2_out, void* ws, size_t ws_bytes, void* stream);

/* S for nz generating vectors (rows of z) in one launch.
 *   z      device int64[nz][d], 0 <= z_j < n;  nz in [1, 4096];  n in [2, 2^31)
 *   a      device double[d]
 *   s_out  device double[nz]
 *   ws     device workspace of qmc_workspace_size(d, n, nz) bytes */
qmc_status qmc_bernoulli_sum(int32_t d, int64_t n, const int64_t* z, int32_t nz, int32_t alpha,
                             const double* a, double* s_out, void* ws, size_t ws_bytes,
                             void* stream);

/* Korobov search (Sec. 2.2): the criterion of the Korobov vectors
 * z(a) = (1, a, ..., a^{d-1}) mod n of a = a0 .. a0 + count - 1 (1 <= a0,
 * a0 + count <= n), and the best: best_out[0] = its criterion, best_out[1] = a (as a
 * double).  The search is O(count * n * d / 2) work; it is asynchronous like every launch.
 *   crit      host descriptor (copied at the call; gamma stays a device array)
 *   s_out     device double[count]: P_alpha or e^2 of each candidate
 *   best_out  device double[2]
 *   ws        device workspace of qmc_criteria_workspace_size(d, n) bytes */
qmc_status qmc_korobov_search(int32_t d, int64_t n, const qmc_criterion* crit, int64_t a0,
                              int32_t count, double* s_out, double* best_out, void* ws,
                              size_t ws_bytes, void* stream);

/* CBC construction (Sec. 2.2, CBC lattice): z_1 = 1, then for j = 2..d the z_j in
 * {1 <= c <= n/2 : gcd(c, n) = 1} minimising the criterion of (z_1..z_j) (e^2 of
 * eq. 2.12 with the weights gamma_1..gamma_j, or P_alpha of eq. 2.4).
 * s_out[j-1] is that criterion of the chosen (z_1..z_j).  O(d n^2 / 4) work,
 * 3 launches per component plus one, all on `stream`.
 *   crit    host descriptor, as qmc_korobov_search
 *   n       in [2, 2^26]
 *   z_out   device int64[d]
 *   s_out   device double[d]
 *   ws      device workspace of qmc_criteria_workspace_size(d, n) bytes */
qmc_status qmc_cbc(int32_t d, int64_t n, const qmc_criterion* crit, int64_t* z_out,
                   double* s_out, void* ws, size_t ws_bytes, void* stream);

/* Launch configuration of the plain-sum kernel.  Zero fields mean "choose
 * automatically".  points_per_thread must be 0, 4, 8 or 16 (the tile is
 * 1024 * points_per_thread consecutive points); max_blocks caps the persistent
 * grid of 1024-thread workgroups per parameter set (1 .. 512). */
typedef struct {
    int32_t points_per_thread;
    int32_t max_blocks;
} qmc_launch_config;

/* qmc_lattice_sum with an explicit launch configuration (cfg may be NULL).
 * The result does not depend on the configuration beyond rounding order. */
qmc_status qmc_lattice_sum_ex(int32_t d, int64_t n, const int64_t* z, const double* shift,
                              int32_t family, const double* params, int32_t nsets,
                              int32_t precision, double* q_out, void* ws, size_t ws_bytes,
                              void* stream, const qmc_launch_config* cfg);

/* Debug export of the point indices (eq. 2.1): k_out[r*d + j] = ((i0 + r) z_j) mod n
 * for r = 0..count-1, computed by the same device index generator as the sums.
 *   z      device int64[d];  k_out device int32[count*d];  0 <= i0, count <= 2^26. */
qmc_status qmc_lattice_points(int32_t d, int64_t n, const int64_t* z, int64_t i0, int64_t count,
                              int32_t* k_out, void* stream);

/* ---- the MDI-LR form ---------------------------------------------------- */

/* MDI-LR (Algorithm 2 driving Algorithm 1 with m = 1) for the improved rule:
 *   Qhat_s = prod_k M_{s,k},  M_{s,k} = (1/N_k) sum_{t=0}^{N_k-1} phi_{s,k}((t + 1/2)/N_k),
 * the dimension sweep of a product-form integrand (the oscillatory family is the
 * real part of a complex product with the factor e^{2 pi i u}).  Each sweep step
 * sums one direction out of the symbolic product, as eq. 2.14c does.
 *   N       device int32[d] node counts (e.g. from qmc_mdi_lr_dims, copied to the
 *           device).  1 <= N_k <= 2^20 is the caller's contract, like z_j in [0, n):
 *           with QMC_VALIDATE=1 the call reads N back and returns QMC_ERR_INVALID_ARG
 *           for an entry outside it; otherwise such an entry makes q_out NaN for
 *           every set (it is never clamped to a valid count).
 *   nsets   1 .. 2^24 parameter sets (one launch; no workspace is used)
 *   params  device double[nsets][qmc_param_count(family, d)]
 *   q_out   device double[nsets] */
qmc_status qmc_mdi_lr(int32_t d, const int32_t* N, int32_t family, const double* params,
                      int32_t nsets, int32_t precision, double* q_out, void* ws,
                      size_t ws_bytes, void* stream);

/* ---- adjoint of the plain rule ------------------------------------------- */

/* Values and parameter gradients of the plain rule for nsets parameter sets that
 * share the lattice (derivative of eq. 1.2 term by term):
 *   q_out[s]          = Q_s = (1/n) sum_i f_s(x_i)
 *   grad_out[s][p]    = gq[s] * dQ_s/dparams[s][p] = gq[s] * (1/n) sum_i df_s/dp (x_i)
 * with the parameter layout of the family (oscillatory: u first, then c_j).
 * Arguments as qmc_lattice_sum, plus
 *   gq        device double[nsets] (the incoming adjoint dL/dQ_s), or NULL for 1
 *   grad_out  device double[nsets][qmc_param_count(family, d)]
 *   ws        device workspace of qmc_workspace_size(d, n, nsets) bytes.
 * Supports d <= 512 (QMC_ERR_UNSUPPORTED above).  Deterministic. */
qmc_status qmc_lattice_sum_adjoint(int32_t d, int64_t n, const int64_t* z, const double* shift,
                                   int32_t family, const double* params, int32_t nsets,
                                   int32_t precision, const double* gq, double* q_out,
                                   double* grad_out, void* ws, size_t ws_bytes, void* stream);

/* ---- batched plain sums: many integrands in one persistent launch ----- */

/* One integrand of a batch: the plain rule of qmc_lattice_sum with its own
 * lattice and parameters (all pointers are device pointers, caller-owned and
 * read at every launch, so their contents may change between launches). */
typedef struct {
    int32_t family;        /* qmc_family */
    int32_t d;             /* 1 .. 1024 */
    int64_t n;             /* 1 .. 2^31 - 1 */
    const int64_t* z;      /* device int64[d], 0 <= z_j < n */
    const double* params;  /* device double[qmc_param_count(family, d)] */
    const double* shift;   /* device double[d] in [0,1), or NULL */
} qmc_problem;

/* Launch configuration of the batched kernel.  Zero fields mean the default. */
typedef struct {
    int32_t points_per_thread; /* 4, 8 or 16: tiles of 256 * points_per_thread points (default 8) */
    int32_t workgroups_per_cu; /* persistent workgroups per compute unit, 1 .. 8 (default 4) */
    int32_t order;             /* 0: longest problem (n * d) first, 1: input order */
} qmc_batch_config;

typedef struct qmc_batch_plan qmc_batch_plan; /* opaque */
typedef struct qmc_graph qmc_graph;           /* opaque */

/* Build the schedule of a batch: problems ordered by cost, tiles numbered
 * consecutively, and a device copy of the problem table (this call allocates
 * and uploads synchronously; it launches nothing).  `problems` is a host array
 * of `count` descriptors, 1 <= count <= 200000; it is copied.  cfg may be NULL. */
qmc_status qmc_batch_plan_create(int32_t count, const qmc_problem* problems, int32_t precision,
                                 const qmc_batch_config* cfg, qmc_batch_plan** plan);
qmc_status qmc_batch_plan_destroy(qmc_batch_plan* plan);
/* The configuration a plan uses (after qmc_batch_autotune: the tuned one). */
qmc_status qmc_batch_plan_config(const qmc_batch_plan* plan, qmc_batch_config* cfg);
/* Replace the configuration (rebuilds and re-uploads the problem table). */
qmc_status qmc_batch_plan_set_config(qmc_batch_plan* plan, const qmc_batch_config* cfg);
/* Workspace bytes for any configuration of this plan (1 MiB of counters plus one
 * double per tile of the smallest tile size). */
qmc_status qmc_batch_workspace_size(const qmc_batch_plan* plan, size_t* bytes);

/* All Q of a batch in one persistent launch: workgroups pop tiles from an atomic
 * queue in the workspace, evaluate them with the qmc_lattice_sum device code,
 * and the workgroup completing a problem sums its tile partials in tile order.
 *   q_out   device double[count], in the order of the descriptors given to the plan.
 * Results are bit-reproducible; the launch allocates nothing and uses no memset,
 * so it can be captured in a graph and replayed. */
qmc_status qmc_lattice_sum_batched(const qmc_batch_plan* plan, double* q_out, void* ws,
                                   size_t ws_bytes, void* stream);

/* Autotuner: times every candidate configuration (points per thread 4/8/16 x
 * workgroups per CU 1/2/4/8) on this batch, `reps` launches each, with HIP
 * events on `stream`, and keeps the fastest in the plan (best may be NULL).
 * Results are cached per batch signature in the process and in the file named by
 * the environment variable QMC_AUTOTUNE_CACHE, if set.  Synchronises `stream`. */
qmc_status qmc_batch_autotune(qmc_batch_plan* plan, double* q_out, void* ws, size_t ws_bytes,
                              void* stream, int32_t reps, qmc_batch_config* best);

/* Capture one qmc_lattice_sum_batched launch (plan, q_out and ws are bound) into
 * an instantiated HIP graph; qmc_graph_launch replays it on any stream. */
qmc_status qmc_batch_graph_create(const qmc_batch_plan* plan, double* q_out, void* ws,
                                  size_t ws_bytes, qmc_graph** graph);
qmc_status qmc_graph_launch(qmc_graph* graph, void* stream);
qmc_status qmc_graph_destroy(qmc_graph* graph);

#ifdef __cplusplus
}
#endif

#endif /* QMC_H */
