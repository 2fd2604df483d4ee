// MDI-LR for integrands of the coordinate sum, f(x) = g(x_1 + ... + x_d) (Test 7's
// f_6 = (1 + sum x)^-(d+1)), on the improved tensor midpoint rule with N nodes
// (t + 1/2)/N in each of the first d - 1 directions and N_last in the last.
//
// After k equal directions the partial sum is (T + k/2)/N for an integer T in
// [0, k (N - 1)]: the terms of the dimension iteration that share T merge, and
// the iteration carries c_k[T], the fraction of index tuples with sum T.  Each
// direction replaces c by its average over a window of N states (Algorithm 1's
// sweep with merged terms).  Then
//   Q = sum_T c_{d-1}[T] (1/N_last) sum_u g((T + (d-1)/2)/N + (u + 1/2)/N_last).
//
// When N_last = N the last direction's nodes lie on the same grid, so the pairs
// (T, u) merge into T + u as well: one more window step gives c_d, and
//   Q = sum_T c_d[T] g((T + d/2)/N)
// needs N times fewer evaluations of g.  The weights are built once for all
// parameter sets; then one workgroup per set evaluates Q.
#include "common.hpp"
#include "families.hpp"
#include "kernels.hpp"
#include "log2_tab.hpp"

namespace qmc {

// The weights after k equal directions are the k-fold self-convolution of the
// N-point window (each direction averages the previous weights over N states).
// Rather than k sequential window steps -- one short, serial pass per direction,
// a poor fit for 256 CUs -- the launcher forms them by repeated squaring:
// O(log k) convolutions, each parallel over its outputs, starting from powers of
// up to eight directions counted exactly (window_powers_kernel).  Each output adds
// positive terms in ascending order, so every state keeps full relative accuracy
// and the result does not depend on the schedule.
// A convolution out = a * b is split over (output tiles) x (segments of i):
// conv_partial_kernel stages a segment of a and the matching window of b in LDS,
// and each thread accumulates kConvR outputs kConvBlock apart (independent FMA
// chains, conflict-free LDS reads, a[i] broadcast); conv_reduce_kernel adds the
// segments in order.  Per output: i ascending within a segment, segments in order.
constexpr int kConvBlock = 256;
constexpr int kConvR = 4;
constexpr int kConvOut = kConvBlock * kConvR;  // outputs per workgroup
constexpr int kConvChunk = 1024;               // i values staged in LDS at once
constexpr int kConvMaxSeg = 32;

// partial[s][T] = sum over i in segment s of a[i] b[T - i], T < Lo = La + Lb - 1.
__global__ __launch_bounds__(kConvBlock) void conv_partial_kernel(const double* a, int La,
                                                                 const double* b, int Lb,
                                                                 int seg_len, double* partial) {
    __shared__ double sa[kConvChunk];
    __shared__ double sb[kConvOut + kConvChunk - 1];
    const int tid = threadIdx.x;
    const int Lo = La + Lb - 1;
    const int TB = blockIdx.x * kConvOut;
    const int seg = blockIdx.y;
    const int s0 = seg * seg_len, s1 = min(La, s0 + seg_len);
    double acc[kConvR];
#pragma unroll
    for (int r = 0; r < kConvR; ++r) acc[r] = 0.0;
    for (int c0 = s0; c0 < s1; c0 += kConvChunk) {
        const int ni = min(kConvChunk, s1 - c0);
        // a[c0 .. c0 + ni) and b[TB - (c0 + ni - 1) .. TB + kConvOut - 1 - c0]
        const int blo = TB - (c0 + ni - 1);
        const int nb = kConvOut + ni - 1;
        __syncthreads();  // the previous chunk's reads are done
        for (int k = tid; k < ni; k += kConvBlock) sa[k] = a[c0 + k];
        for (int k = tid; k < nb; k += kConvBlock) {
            const int idx = blo + k;
            sb[k] = (idx >= 0 && idx < Lb) ? b[idx] : 0.0;
        }
        __syncthreads();
        // output T = TB + tid + r kConvBlock needs b[T - i] = sb[tid + r kConvBlock + ni - 1 - k]
        for (int k = 0; k < ni; ++k) {
            const double ai = sa[k];
#pragma unroll
            for (int r = 0; r < kConvR; ++r)
                acc[r] = fma(ai, sb[tid + r * kConvBlock + ni - 1 - k], acc[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < kConvR; ++r) {
        const int T = TB + tid + r * kConvBlock;
        if (T < Lo) partial[(size_t)seg * Lo + T] = acc[r];
    }
}

// out[T] = sum_s partial[s][T], s ascending.  Unrolled by eight so that the loads
// of eight segments are in flight together (the additions keep their order).
__global__ __launch_bounds__(kConvBlock) void conv_reduce_kernel(const double* partial, int nseg,
                                                                int Lo, double* out) {
    const int T = blockIdx.x * kConvBlock + threadIdx.x;
    if (T >= Lo) return;
    double t = 0.0;
#pragma unroll 8
    for (int s = 0; s < nseg; ++s) t += partial[(size_t)s * Lo + T];
    out[T] = t;
}

// r = (1) and w = the window (1/N, ..., 1/N).
__global__ __launch_bounds__(kConvBlock) void states_init_kernel(int N, double* r, double* w) {
    const int t = blockIdx.x * kConvBlock + threadIdx.x;
    if (t == 0) r[0] = 1.0;
    if (t < N) w[t] = 1.0 / (double)N;
}

// The table of log2_tab (log2_tab.hpp), copied into LDS by the kernels that use it.
__constant__ Log2Table kLog2TableDev = make_log2_table();

// log2 x for x > 0 to about 3e-13 absolute: the table form for positive normal x,
// the library log2 for anything else.
__device__ __forceinline__ double log2_fast(double x, const Log2Entry* tab) {
    if (!(x >= 0x1p-1022 && x < __builtin_huge_val())) return log2(x);
    return log2_tab(x, tab);
}

// g of the sum: power (b + c s)^-p, or Gaussian exp(-c^2 (s - w)^2).
template <int GFAM, bool FP32>
__device__ __forceinline__ double sum_g(const double* gp, double s, const Log2Entry* tab) {
    if constexpr (GFAM == 0) {
        if constexpr (FP32) {
            // 2^{-p log2(b + c s)}: the exponent in FP64, its fractional power in FP32
            return exp2_split_f32(-gp[2] * log2_fast(fma(gp[1], s, gp[0]), tab));
        } else {
            // 2^{-p log2 x} with log2 x = hi + lo from the table (2.2e-16 absolute) and
            // y = -p log2 x as yh + yl (the product's rounding by an FMA): the exp2 of
            // yh within one unit in the last place, times 1 + yl ln 2.
            const double x = fma(gp[1], s, gp[0]), p = gp[2];
            if (!(x >= 0x1p-1022 && x < __builtin_huge_val())) return pow(x, -p);
            double hi, lo;
            log2_tab_dd(x, tab, hi, lo);
            const double yh = -p * hi;
            const double yl = fma(-p, lo, fma(-p, hi, -yh));
            if (!(fabs(yh) <= 1000.0)) return pow(x, -p);
            return exp2_f64(yh) * fma(yl, kLn2, 1.0);
        }
    } else {
        const double y = gp[0] * (s - gp[1]);
        if constexpr (FP32)
            return exp2_split_f32(-kLog2e * y * y);
        else
            return exp(-y * y);
    }
}

constexpr int kSumEvalBlock = 256;

// Q of set blockIdx.x over `states` states and `nl` remaining nodes per state:
//   Q = (1/nl) sum_T c[T] sum_{u < nl} g(T/N + off + u/nl).
// Thread t owns the states T = t, t + kSumEvalBlock, ...; for each it sums g over
// the nodes in order, weights by c[T], and the workgroup adds the thread sums in
// the fixed order of block_sum.
template <int GFAM, bool FP32>
__global__ __launch_bounds__(kSumEvalBlock) void sum_eval_kernel(int states, int N, int nl, double off,
                                                                const double* c,
                                                                const double* params, int P,
                                                                double* q_out) {
    __shared__ double s_red[kSumEvalBlock / kWave];
    __shared__ Log2Entry s_tab[kLog2Tab];
    constexpr bool kTable = GFAM == 0;  // the power's log2 in the table form
    if constexpr (kTable) {
        for (int k = threadIdx.x; k < kLog2Tab; k += kSumEvalBlock) s_tab[k] = kLog2TableDev.e[k];
        __syncthreads();
    }
    const double* gp = params + (size_t)blockIdx.x * P;
    const double invN = 1.0 / (double)N, invNl = 1.0 / (double)nl;
    double acc = 0.0;
    for (int T = threadIdx.x; T < states; T += kSumEvalBlock) {
        const double s0 = fma((double)T, invN, off);
        double inner = 0.0;
        for (int u = 0; u < nl; ++u) inner += sum_g<GFAM, FP32>(gp, fma((double)u, invNl, s0), s_tab);
        acc = fma(c[T], inner, acc);
    }
    const double t = block_sum(acc, s_red);
    if (threadIdx.x == 0) q_out[blockIdx.x] = t * invNl;
}

size_t mdi_sum_workspace_bytes(int d, int N) {
    const size_t L = (size_t)d * (size_t)(N - 1) + 1;  // enough for both forms
    // the shared zero region, then three rotating weight vectors and the
    // convolution's segment partials
    return kZeroBytes + ((3 + kConvMaxSeg) * L * sizeof(double) + 255) / 256 * 256;
}

template <int GFAM, bool FP32>
static hipError_t launch_eval(const MdiSumLaunch& L, int states, int nl, double off, const double* c,
                              hipStream_t stream) {
    hipLaunchKernelGGL((sum_eval_kernel<GFAM, FP32>), dim3((unsigned)L.nsets), dim3(kSumEvalBlock), 0,
                       stream, states, L.N, nl, off, c, L.params, L.P, L.q_out);
    return hipGetLastError();
}

// The k-fold self-convolution of the N-point window for small k, exactly.  The number
// of k-tuples of nodes in [0, N) with index sum T is, by inclusion and exclusion over
// the coordinates that exceed N - 1,
//   c_k[T] = sum_{i >= 0, i N <= T} (-1)^i C(k, i) C(T - i N + k - 1, k - 1),
// computed here in 64-bit integers (direct_k checks that every term and every partial
// product of the binomials fits), and w_k[T] = c_k[T] / N^k with one rounding.  It
// stands for the first log2 k squarings of the window, and it is exact where they
// round.
constexpr int kDirectMaxK = 8;

template <int K>
__device__ __forceinline__ uint64_t window_count(uint64_t N, uint64_t T) {
    int64_t total = 0;
    uint64_t cki = 1;  // C(K, i)
#pragma unroll
    for (int i = 0; i <= K; ++i) {
        if ((uint64_t)i * N > T) break;
        const uint64_t m = T - (uint64_t)i * N + (K - 1);
        uint64_t c = 1;  // C(m, r), r = 0 .. K - 1: C(m, r) = C(m, r - 1) (m - r + 1) / r exactly
#pragma unroll
        for (int r = 1; r < K; ++r) c = c * (m - r + 1) / r;
        const int64_t term = (int64_t)(cki * c);
        total += (i & 1) ? -term : term;
        cki = cki * (K - i) / (i + 1);
    }
    return (uint64_t)total;
}

template <int K>
__device__ __forceinline__ void window_power(int N, double NK, int T, double* w) {
    if (T <= K * (N - 1)) w[T] = (double)window_count<K>((uint64_t)N, (uint64_t)T) / NK;
}

__device__ __forceinline__ void window_power_k(int k, int N, double NK, int T, double* w) {
    switch (k) {
        case 1: window_power<1>(N, NK, T, w); break;
        case 2: window_power<2>(N, NK, T, w); break;
        case 3: window_power<3>(N, NK, T, w); break;
        case 4: window_power<4>(N, NK, T, w); break;
        case 5: window_power<5>(N, NK, T, w); break;
        case 6: window_power<6>(N, NK, T, w); break;
        case 7: window_power<7>(N, NK, T, w); break;
        case 8: window_power<8>(N, NK, T, w); break;
        default: break;  // k = 0: nothing to write
    }
}

// w1 = w_{k1} (if k1 > 0) and w2 = w_{k2}, N^k as doubles in nk1 and nk2.
__global__ __launch_bounds__(kConvBlock) void window_powers_kernel(int N, int k1, double nk1, double* w1,
                                                                  int k2, double nk2, double* w2) {
    const int T = blockIdx.x * kConvBlock + threadIdx.x;
    window_power_k(k1, N, nk1, T, w1);
    window_power_k(k2, N, nk2, T, w2);
}

// The largest power of two k <= min(kDirectMaxK, steps) for which window_count stays in
// 64-bit integers at every T: N^k, every term C(k, i) C(m, k - 1) (m <= k N - 1, and
// C(k, i) <= 2^k) with the sum of their magnitudes, and every partial product
// r C(m, r) <= (k - 1) C(k N - 1, k - 1) below 2^62.  1 if none is.
static int direct_k(int N, int steps) {
    int best = 1;
    for (int k = 2; k <= kDirectMaxK && k <= steps; k *= 2) {
        long double c = 1.0L;  // C(k N - 1, k - 1)
        for (int r = 1; r < k; ++r) c = c * (long double)((int64_t)k * N - r) / (long double)r;
        const long double nk = powl((long double)N, (long double)k);
        const long double lim = 0x1p62L;
        if (nk > lim || c * (long double)(1 << k) > lim || c * (long double)(k - 1) > lim) break;
        best = k;
    }
    return best;
}

// out = a * b through `partial` (kConvMaxSeg * (La + Lb - 1) doubles).  An operand a
// of at most kConvOneSeg states is one segment: its partial sums are the output and
// no reduction launch follows.  (Longer single segments make each thread's FMA chain
// long enough to cost more than the reduction launch saves.)
constexpr int kConvOneSeg = 64;

static hipError_t launch_conv(const double* a, int La, const double* b, int Lb, double* out,
                              double* partial, hipStream_t stream) {
    const int Lo = La + Lb - 1;
    int nseg = La <= kConvOneSeg ? 1 : (La + 63) / 64;
    if (nseg > kConvMaxSeg) nseg = kConvMaxSeg;
    const int seg_len = (La + nseg - 1) / nseg;
    nseg = (La + seg_len - 1) / seg_len;
    if (nseg == 1) {
        hipLaunchKernelGGL(conv_partial_kernel, dim3((Lo + kConvOut - 1) / kConvOut, 1), dim3(kConvBlock), 0,
                           stream, a, La, b, Lb, seg_len, out);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(conv_partial_kernel, dim3((Lo + kConvOut - 1) / kConvOut, nseg), dim3(kConvBlock),
                       0, stream, a, La, b, Lb, seg_len, partial);
    hipLaunchKernelGGL(conv_reduce_kernel, dim3((Lo + kConvBlock - 1) / kConvBlock), dim3(kConvBlock), 0,
                       stream, partial, nseg, Lo, out);
    return hipGetLastError();
}

hipError_t launch_mdi_sum(const MdiSumLaunch& L, hipStream_t stream) {
    // Equal node counts merge the last direction too.
    const bool merge = L.N_last == L.N;
    const int steps = merge ? L.d : L.d - 1;
    const int nl = merge ? 1 : L.N_last;
    const double off = merge ? 0.5 * (double)L.d / (double)L.N
                             : 0.5 * (double)(L.d - 1) / (double)L.N + 0.5 / (double)L.N_last;
    // Three buffers of d (N - 1) + 1 doubles hold the running result R, the running
    // square B and the output of each convolution; R and B may share one (R = B after
    // the first factor).
    const size_t cap = (size_t)L.d * (size_t)(L.N - 1) + 1;
    double* const base = (double*)((char*)L.ws + kZeroBytes);  // past the shared zero region
    double* buf[3] = {base, base + cap, base + 2 * cap};
    double* partial = base + 3 * cap;
    int iR = 0, iB = 1;
    auto free_buf = [&]() {
        for (int i = 0; i < 3; ++i)
            if (i != iR && i != iB) return i;
        return 2;
    };
    // R = w_r0 and B = w_kd from the exact counts, then R * B^(steps / kd) by repeated
    // squaring; without them (kd = 1) R = (1), B = the window and R * B^steps.
    const int kd = direct_k(L.N, steps);
    int LR, LB, bits;
    bool r_one;  // R is the empty product (1)
    hipError_t e;
    if (kd >= 2) {
        const int r0 = steps % kd;
        LB = kd * (L.N - 1) + 1;
        LR = r0 * (L.N - 1) + 1;
        r_one = r0 == 0;
        bits = steps / kd;
        const double nk0 = pow((double)L.N, (double)r0), nkd = pow((double)L.N, (double)kd);
        hipLaunchKernelGGL(window_powers_kernel, dim3((LB + kConvBlock - 1) / kConvBlock), dim3(kConvBlock), 0,
                           stream, L.N, r0, nk0, buf[iR], kd, nkd, buf[iB]);
    } else {
        LR = 1;
        LB = L.N;
        r_one = true;
        bits = steps;
        hipLaunchKernelGGL(states_init_kernel, dim3((L.N + kConvBlock - 1) / kConvBlock), dim3(kConvBlock),
                           0, stream, L.N, buf[iR], buf[iB]);
    }
    e = hipGetLastError();
    for (; bits > 0 && e == hipSuccess; bits >>= 1) {
        if (bits & 1) {
            if (r_one) {
                iR = iB;  // R = 1 * B: share B's buffer
                LR = LB;
                r_one = false;
            } else {
                // the shorter operand is staged as a (the convolution is symmetric)
                const int iT = free_buf();
                e = LR <= LB ? launch_conv(buf[iR], LR, buf[iB], LB, buf[iT], partial, stream)
                             : launch_conv(buf[iB], LB, buf[iR], LR, buf[iT], partial, stream);
                iR = iT;
                LR += LB - 1;
            }
        }
        if ((bits >> 1) > 0 && e == hipSuccess) {
            const int iT = free_buf();
            e = launch_conv(buf[iB], LB, buf[iB], LB, buf[iT], partial, stream);
            iB = iT;
            LB = 2 * LB - 1;
        }
    }
    double* R = buf[iR];
    if (e != hipSuccess) return e;
    // LR = steps (N - 1) + 1 states.
    if (L.gfamily == 0)
        return L.fp32 ? launch_eval<0, true>(L, LR, nl, off, R, stream)
                      : launch_eval<0, false>(L, LR, nl, off, R, stream);
    return L.fp32 ? launch_eval<1, true>(L, LR, nl, off, R, stream)
                  : launch_eval<1, false>(L, LR, nl, off, R, stream);
}

}  // namespace qmc
