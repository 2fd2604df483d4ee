// Lattice-quality criteria and the constructions built on them (Sec. 2.1, eq. 2.4
// and eq. 2.12; Sec. 2.2: the Korobov search and the CBC lattice).
//
// All of them reduce to the product-form Bernoulli sum
//   S(z) = (1/n) sum_{k=0}^{n-1} [ prod_j (1 + a_j B_alpha({k z_j / n})) - 1 ],
// evaluated by the plain-sum kernel (family BernoulliProduct) for whole generating
// vectors, and by cbc_eval_kernel for the one-component-at-a-time search of CBC.
//
// Selection among candidates is deterministic: non-candidates (gcd(c, n) != 1) get
// +infinity; among the candidates whose S is within kTieRel of the smallest, the
// smallest candidate wins (the criteria of c and n - c are equal, and FP64 sums of
// equal criteria differ in their last bits).
#include "common.hpp"
#include "families.hpp"
#include "kernels.hpp"

namespace qmc {

constexpr double kTieRel = 1e-10;

__device__ __forceinline__ uint32_t gcd_u32(uint32_t a, uint32_t b) {
    while (b) {
        const uint32_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// --------------------------------------------------------------------------
// Korobov generating vectors z(a) = (1, a, a^2, ..., a^{d-1}) mod n (Sec. 2.2) for
// a = a0 + i, i < count: one thread per candidate, row i of the table, and
// coprime[i] = (gcd(a, n) == 1) for the selection.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void korobov_table_kernel(int d, uint32_t n, double inv_n,
                                                           int64_t a0, int count, int64_t* z,
                                                           uint8_t* coprime) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint64_t a = (uint64_t)(a0 + i) % n;
    coprime[i] = gcd_u32((uint32_t)a, n) == 1 ? 1 : 0;
    int64_t* row = z + (size_t)i * d;
    uint64_t v = 1 % n;
    for (int j = 0; j < d; ++j) {
        row[j] = (int64_t)v;
        v = mulmod(v, a, n, inv_n);
    }
}

// --------------------------------------------------------------------------
// Selection over v[0..count) for candidates c = c_first + i.  One workgroup.
// If `coprime` is not null, writes +infinity over the entries it marks 0; then
//   *best_value = v[i*] (times *value_scale if that is not null),
//   *best_cand_f64 = c_first + i*                        (if not null),
//   *best_cand_i64 = c_first + i*                        (if not null),
// i* the smallest index within kTieRel of the minimum (i* = 0 and +infinity when
// no candidate is coprime to n).  The coprimality test itself runs where the
// candidates are spread over many workgroups (the table and CBC kernels).
// --------------------------------------------------------------------------
constexpr int kSelectBlock = 1024;

__global__ __launch_bounds__(kSelectBlock) void select_kernel(double* v, int count, int64_t c_first,
                                                             const uint8_t* coprime,
                                                             double* best_value,
                                                             double* best_cand_f64,
                                                             int64_t* best_cand_i64,
                                                             const double* value_scale) {
    __shared__ double s_min[kSelectBlock / kWave];
    __shared__ int s_idx[kSelectBlock / kWave];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    constexpr int W = kSelectBlock / kWave;

    // Pass 1: filter and minimum (a minimum is exact, so its order does not matter).
    // Both passes are unrolled so that several loads are in flight per thread.
    double m = INFINITY;
#pragma unroll 8
    for (int i = tid; i < count; i += kSelectBlock) {
        double x = v[i];
        if (coprime && !coprime[i]) {
            x = INFINITY;
            v[i] = x;  // the same thread reads v[i] again in pass 2
        }
        m = fmin(m, x);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) m = fmin(m, __shfl_xor(m, off, kWave));
    if (lane == 0) s_min[wv] = m;
    __syncthreads();
    m = s_min[0];
#pragma unroll
    for (int w = 1; w < W; ++w) m = fmin(m, s_min[w]);
    const double thr = m + kTieRel * fabs(m);

    // Pass 2: the smallest index within the tolerance.
    int first = count;
#pragma unroll 8
    for (int i = tid; i < count; i += kSelectBlock) {
        if (v[i] <= thr) {
            first = i;
            break;
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) first = min(first, __shfl_xor(first, off, kWave));
    if (lane == 0) s_idx[wv] = first;
    __syncthreads();
    if (tid == 0) {
        int f = s_idx[0];
        for (int w = 1; w < W; ++w) f = min(f, s_idx[w]);
        if (f >= count) f = 0;
        *best_value = value_scale ? v[f] * *value_scale : v[f];
        if (best_cand_f64) *best_cand_f64 = (double)(c_first + f);
        if (best_cand_i64) *best_cand_i64 = c_first + f;
    }
}

// --------------------------------------------------------------------------
// Criterion weights.  Both criteria are S of the Bernoulli product sum with weights
//   P_alpha (eq. 2.4):  a_j = (-1)^{alpha/2+1} (2 pi)^alpha / alpha!  (2 pi^2 for
//                       alpha = 2, -2 pi^4 / 3 for alpha = 4), and P_alpha = S;
//   e^2 (eq. 2.12, product weights gamma_j, beta = c^2 - c + 1/3 for the anchored
//        space with anchor c, 0 unanchored, alpha = 2):  a_j = gamma_j / (1 + gamma_j beta)
//                       and e^2 = prod_j (1 + gamma_j beta) * S.
// One workgroup writes a[0..d) and a[d] = C_d, and cum[j] = C_{j+1} = prod_{i<=j}
// (1 + gamma_i beta) (all 1 for P_alpha), the products taken in index order.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void criterion_weights_kernel(int d, int kind, int alpha,
                                                               const double* gamma, double beta,
                                                               double* a, double* cum) {
    const double tp = 2.0 * 3.14159265358979323846;
    const double c_pa = alpha == 2 ? 0.5 * tp * tp : -(tp * tp) * (tp * tp) / 24.0;
    for (int j = threadIdx.x; j < d; j += blockDim.x)
        a[j] = kind == kCritPAlpha ? c_pa : gamma[j] / fma(gamma[j], beta, 1.0);
    if (threadIdx.x == 0) {
        double c = 1.0;
        for (int j = 0; j < d; ++j) {
            if (kind != kCritPAlpha) c *= fma(gamma[j], beta, 1.0);
            cum[j] = c;
        }
        a[d] = c;
    }
}

// --------------------------------------------------------------------------
// CBC (Sec. 2.2): with the running product p(k) = prod_{i<j} (1 + a_i B({k z_i/n}))
// in memory, the criterion of candidate c for component j is
//   S_j(c) = (1/n) sum_k [ p(k) (1 + a_j B_alpha({k c / n})) - 1 ].
// Index k and n - k give mirrored points ({(n - k) z / n} = 1 - {k z / n} or both
// 0) and B_alpha(1 - x) = B_alpha(x) for even alpha, so p and every term are equal
// at k and n - k: the sum is T(0) + 2 sum_{k=1}^{h} T(k) + [n even] T(n/2) with
// h = (n - 1) / 2, and p is kept for k <= n/2 only.
// A workgroup owns kCbcCand consecutive candidates and sweeps k = 1..h in chunks
// of kCbcBlock * kCbcM: each thread keeps kCbcM values of p and of k in registers
// and, from one candidate to the next, advances its residues k c mod n by k (one
// modular add).  Per candidate and chunk each wave adds its wave total to an LDS
// slot, in chunk order; thread c then adds T(0) and T(n/2) in a fixed order, so the
// result is reproducible.
// --------------------------------------------------------------------------
constexpr int kCbcBlock = 1024;
constexpr int kCbcM = 16;
constexpr int kCbcCand = 64;

// 1 + a B_alpha(x) from y = x (1 - x), with c0 = 1 + a B_alpha(0).
template <int ALPHA>
__device__ __forceinline__ double bernoulli_factor(double aj, double c0, double y) {
    if constexpr (ALPHA == 2)
        return fma(-aj, y, c0);  // 1 + a (1/6 - y) = 1 + a B_2(x)
    else
        return fma(aj * y, y, c0);  // 1 + a (y^2 - 1/30) = 1 + a B_4(x)
}

// FI: the residues stepped as exact floats (stepmod_f, n <= kFloatIndexMaxN), three
// FP32 operations per point in place of addmod's integer add, compare and select
// followed by a conversion; the same residues, so the same bits.
template <int ALPHA, bool FI>
__global__ __launch_bounds__(kCbcBlock) void cbc_eval_kernel(uint32_t n, double inv_n,
                                                            const double* a, int j,
                                                            const double* p, int64_t c_first,
                                                            int ncand, double* s_cand) {
    constexpr int W = kCbcBlock / kWave;
    __shared__ double s_acc[kCbcCand * W];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int g0 = blockIdx.x * kCbcCand;
    const int gc = min(kCbcCand, ncand - g0);
    const double aj = a[j];
    const double c0 = ALPHA == 2 ? 1.0 + aj / 6.0 : 1.0 - aj / 30.0;
    const uint32_t h = (n - 1) / 2;  // paired indices 1..h
    for (int i = tid; i < kCbcCand * W; i += kCbcBlock) s_acc[i] = 0.0;
    __syncthreads();
    const uint64_t cbeg = (uint64_t)(c_first + g0) % n;

    for (uint32_t k0 = 1; k0 <= h; k0 += kCbcBlock * kCbcM) {
        uint32_t r[kCbcM], kk[kCbcM];
        double pk[kCbcM];
        double bias = 0.0;  // +1 for each k > h, whose term below is exactly -1
#pragma unroll
        for (int m = 0; m < kCbcM; ++m) {
            const uint32_t k = k0 + (uint32_t)(m * kCbcBlock + tid);
            const bool ok = k <= h;
            kk[m] = ok ? k : 0u;
            pk[m] = ok ? p[k] : 0.0;
            bias += ok ? 0.0 : 1.0;
            r[m] = ok ? mulmod((uint64_t)k, cbeg, n, inv_n) : 0u;
        }
        float rf[kCbcM], kf[kCbcM], kmf[kCbcM];
        if constexpr (FI) {
#pragma unroll
            for (int m = 0; m < kCbcM; ++m) {
                rf[m] = (float)r[m];
                kf[m] = (float)kk[m];
                kmf[m] = (float)kk[m] - (float)n;
            }
        }
        for (int c = 0; c < gc; ++c) {
            double acc = bias;
#pragma unroll
            for (int m = 0; m < kCbcM; ++m) {
                const double x = (FI ? (double)rf[m] : (double)r[m]) * inv_n;
                const double y = fma(-x, x, x);  // x (1 - x)
                acc += fma(pk[m], bernoulli_factor<ALPHA>(aj, c0, y), -1.0);
                if constexpr (FI)
                    rf[m] = stepmod_f(rf[m], kf[m], kmf[m]);
                else
                    r[m] = addmod(r[m], kk[m], n);
            }
            const double w = wave_total(acc);
            if (lane == kWaveTotalLane) s_acc[c * W + wv] += w;
        }
    }
    __syncthreads();
    for (int c = tid; c < gc; c += kCbcBlock) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < W; ++w) t += s_acc[c * W + w];
        const uint32_t cand = (uint32_t)((cbeg + c) % n);
        // T(0): x = 0.  T(n/2) for even n: x = {c / 2}, 0 or 1/2.
        double total = fma(p[0], c0, -1.0) + 2.0 * t;
        if ((n & 1u) == 0) {
            const double y = (cand & 1u) ? 0.25 : 0.0;
            total += fma(p[n / 2], bernoulli_factor<ALPHA>(aj, c0, y), -1.0);
        }
        const bool ok = gcd_u32(cand, n) == 1;
        s_cand[g0 + c] = ok ? total * inv_n : INFINITY;
    }
}

// p(k) = 1 for k <= n/2.
__global__ __launch_bounds__(256) void cbc_init_kernel(uint32_t n, double* p) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k <= n / 2) p[k] = 1.0;
}

// p(k) *= 1 + a_j B_alpha({k z_j / n}) for k <= n/2, with the z_j just chosen (read
// from device memory).
template <int ALPHA>
__global__ __launch_bounds__(256) void cbc_update_kernel(uint32_t n, double inv_n, const double* a,
                                                        int j, const int64_t* z, double* p) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > n / 2) return;
    const double aj = a[j];
    const uint32_t r = mulmod((uint64_t)k, (uint64_t)z[j] % n, n, inv_n);
    const double x = (double)r * inv_n;
    const double y = fma(-x, x, x);
    p[k] *= bernoulli_factor<ALPHA>(aj, ALPHA == 2 ? 1.0 + aj / 6.0 : 1.0 - aj / 30.0, y);
}

// --------------------------------------------------------------------------
// Launchers
// --------------------------------------------------------------------------
// Criteria workspace: the zero region, the weights a[d + 1] and the cumulative
// scales cum[d] (criterion_weights_kernel), then either the search's table of
// kMaxSumSets vectors and one coprimality byte per candidate (< n), or CBC's
// running product and the candidates' values.
static size_t weights_bytes(int d) { return ((size_t)(2 * d + 1) * sizeof(double) + 255) / 256 * 256; }

size_t criteria_workspace_bytes(int d, int64_t n) {
    const size_t table = (size_t)kMaxSumSets * (size_t)d * sizeof(int64_t) + (size_t)n;
    const size_t cbc = ((size_t)n + (size_t)n / 2 + 2) * sizeof(double);
    return kZeroBytes + weights_bytes(d) + ((table > cbc ? table : cbc) + 255) / 256 * 256;
}

static double* weights_of(void* ws) { return (double*)((char*)ws + kZeroBytes); }
static void* after_weights(void* ws, int d) { return (char*)ws + kZeroBytes + weights_bytes(d); }

static hipError_t launch_weights(const CriterionSpec& c, int d, void* ws, hipStream_t stream) {
    double* a = weights_of(ws);
    hipLaunchKernelGGL(criterion_weights_kernel, dim3(1), dim3(256), 0, stream, d, c.kind, c.alpha,
                       c.gamma, c.beta, a, a + d + 1);
    return hipGetLastError();
}

// Bernoulli sums whose weights (and the scale a[d]) are in the workspace.
static hipError_t launch_scaled_sums(int d, uint32_t n, const int64_t* z, int nz, int alpha,
                                     const double* a, double* out, void* ws, hipStream_t stream) {
    PlainLaunch P{};
    P.d = d;
    P.n = n;
    P.z = z;
    P.shift = nullptr;
    P.family = alpha == 2 ? kBernoulli2S : kBernoulli4S;
    P.params = a;
    P.P = d + 1;
    P.nsets = nz;
    P.param_stride = 0;
    P.shift_stride = 0;
    P.z_stride = d;
    P.fp32 = false;
    P.q_out = out;
    P.ws = ws;
    return launch_lattice_sum(P, stream);
}

hipError_t launch_criterion(const CriterionLaunch& L, hipStream_t stream) {
    hipError_t e = launch_weights(L.crit, L.d, L.ws, stream);
    if (e != hipSuccess) return e;
    return launch_scaled_sums(L.d, L.n, L.z, L.nz, L.crit.alpha, weights_of(L.ws), L.out, L.ws, stream);
}

hipError_t launch_bernoulli_sum(const BernoulliLaunch& L, hipStream_t stream) {
    PlainLaunch P{};
    P.d = L.d;
    P.n = L.n;
    P.z = L.z;
    P.shift = nullptr;
    P.family = L.alpha == 2 ? kBernoulli2 : kBernoulli4;
    P.params = L.a;
    P.P = L.d;
    P.nsets = L.nz;
    P.param_stride = 0;
    P.shift_stride = 0;
    P.z_stride = L.d;
    P.fp32 = false;
    P.q_out = L.s_out;
    P.ws = L.ws;
    return launch_lattice_sum(P, stream);
}

hipError_t launch_korobov_search(const SearchLaunch& L, hipStream_t stream) {
    const double inv_n = 1.0 / (double)L.n;
    hipError_t e = launch_weights(L.crit, L.d, L.ws, stream);
    if (e != hipSuccess) return e;
    const double* a = weights_of(L.ws);
    int64_t* table = (int64_t*)after_weights(L.ws, L.d);
    uint8_t* coprime = (uint8_t*)(table + (size_t)kMaxSumSets * L.d);
    for (int64_t c0 = 0; c0 < L.count; c0 += kMaxSumSets) {
        const int cnt = (int)((L.count - c0) < kMaxSumSets ? (L.count - c0) : kMaxSumSets);
        hipLaunchKernelGGL(korobov_table_kernel, dim3((cnt + 255) / 256), dim3(256), 0, stream, L.d,
                           L.n, inv_n, L.a0 + c0, cnt, table, coprime + c0);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = launch_scaled_sums(L.d, L.n, table, cnt, L.crit.alpha, a, L.s_out + c0, L.ws, stream);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(select_kernel, dim3(1), dim3(kSelectBlock), 0, stream, L.s_out, L.count,
                       L.a0, (const uint8_t*)coprime, L.best_out, L.best_out + 1, (int64_t*)nullptr,
                       (const double*)nullptr);
    return hipGetLastError();
}

template <int ALPHA>
static hipError_t launch_cbc_a(const CbcLaunch& L, hipStream_t stream) {
    const double inv_n = 1.0 / (double)L.n;
    hipError_t e = launch_weights(L.crit, L.d, L.ws, stream);
    if (e != hipSuccess) return e;
    const double* a = weights_of(L.ws);
    const double* cum = a + L.d + 1;
    double* p = (double*)after_weights(L.ws, L.d);
    double* cand = p + L.n;
    const unsigned half_blocks = (unsigned)((L.n / 2 + 1 + 255) / 256);
    hipLaunchKernelGGL(cbc_init_kernel, dim3(half_blocks), dim3(256), 0, stream, L.n, p);
    e = hipGetLastError();
    for (int j = 0; j < L.d && e == hipSuccess; ++j) {
        // z_1 = 1; later components range over 1 <= c <= n/2 (c and n - c tie).  The
        // candidates are compared by S; the chosen one's criterion is C_{j+1} S.
        const int ncand = j == 0 ? 1 : (int)(L.n / 2);
        const dim3 eval_grid((ncand + kCbcCand - 1) / kCbcCand);
        if (L.n <= kFloatIndexMaxN)
            hipLaunchKernelGGL((cbc_eval_kernel<ALPHA, true>), eval_grid, dim3(kCbcBlock), 0, stream,
                               L.n, inv_n, a, j, p, (int64_t)1, ncand, cand);
        else
            hipLaunchKernelGGL((cbc_eval_kernel<ALPHA, false>), eval_grid, dim3(kCbcBlock), 0, stream,
                               L.n, inv_n, a, j, p, (int64_t)1, ncand, cand);
        hipLaunchKernelGGL(select_kernel, dim3(1), dim3(kSelectBlock), 0, stream, cand, ncand,
                           (int64_t)1, (const uint8_t*)nullptr, L.s_out + j, (double*)nullptr,
                           L.z_out + j, cum + j);
        hipLaunchKernelGGL((cbc_update_kernel<ALPHA>), dim3(half_blocks), dim3(256), 0, stream,
                           L.n, inv_n, a, j, L.z_out, p);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_cbc(const CbcLaunch& L, hipStream_t stream) {
    return L.crit.alpha == 2 ? launch_cbc_a<2>(L, stream) : launch_cbc_a<4>(L, stream);
}

}  // namespace qmc
