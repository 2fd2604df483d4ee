// Adjoint of the plain lattice rule: Q_s and gq_s * dQ_s/d(params_s) for every
// parameter set s sharing the lattice (derivative of eq. 1.2):
//   dQ/dp = (1/n) sum_i df/dp (x_i).
// For the product- or sum-form families df/dp_j = w(x) * h_j(x_j): a per-point
// weight w times a function of one coordinate,
//   exp-sum      w = f,        dc_j: h = x_j
//   oscillatory  w = -sin(th), dc_j: h = x_j,  du: 2 pi w (per point)
//   Gaussian     w = f,        dc_j: h = -2 c_j (x_j - w_j)^2,  dw_j: h = 2 c_j^2 (x_j - w_j)
//   exp of a quadratic  w = f, dc_j: h = (x_j - w_j)^2,         dw_j: h = -2 c_j (x_j - w_j)
//   product peak w = f,        dc_j: h = 2 c_j^-3 / q_j,        dw_j: h = 2 (x_j - w_j) / q_j
// so a tile is processed in two sweeps over the directions: the first is the
// forward accumulation of the sum kernel (giving f and w per point), the second
// regenerates each direction's indices from the same LDS tables and adds
// w * h_j(x) of the thread's points; a wave64 sum per direction goes into a
// per-wave LDS slot.  Per-workgroup vectors are combined by the two-level
// fixed-order grid sum (vector form), so the gradients are bit-reproducible.
#include "common.hpp"
#include "families.hpp"
#include "kernels.hpp"
#include "tile.hpp"

namespace qmc {

struct AdjArgs {
    int d;
    uint32_t n;
    double inv_n;  // 1.0 / n
    const int64_t* z;
    const double* shift;
    const double* params;
    int P;
    uint32_t tiles;
    const double* gq;  // may be null (= 1)
    double* q_out;
    double* grad_out;
    uint32_t* tickets;
    double* scratch;
    size_t scratch_stride;  // doubles per set
};

struct AdjDim {
    double c, w, soff;  // c_j, w_j (or 0), shift fraction / n
};

constexpr double kTwoPi = 6.283185307179586477;

template <int FAM, bool FP32>
struct AdjFam;

template <bool FP32>
struct AdjFam<kExpSum, FP32> {
    using F = ExpSum<FP32>;
    static constexpr bool kTwo = false;
    __device__ static void point(const typename F::Acc& acc, double& val, double& wt, double& gu) {
        val = F::finish(acc);
        wt = val;
        gu = 0.0;
    }
    __device__ static void dir(double x, const AdjDim&, double wt, double& ga, double&) { ga = fma(wt, x, ga); }
    __device__ static int ia(int j, int) { return j; }
    __device__ static int ib(int j, int) { return j; }
};

template <bool FP32>
struct AdjFam<kOscillatory, FP32> {
    using F = Oscillatory<FP32>;
    static constexpr bool kTwo = false;
    __device__ static void point(const typename F::Acc& acc, double& val, double& wt, double& gu) {
        const double fr = acc.s - rint(acc.s);
        if constexpr (FP32) {
            val = (double)__builtin_amdgcn_cosf((float)fr);
            wt = -(double)__builtin_amdgcn_sinf((float)fr);
        } else {
            double sn, cs;
            sincospi(2.0 * fr, &sn, &cs);
            val = cs;
            wt = -sn;
        }
        gu = kTwoPi * wt;
    }
    __device__ static void dir(double x, const AdjDim&, double wt, double& ga, double&) { ga = fma(wt, x, ga); }
    __device__ static int ia(int j, int) { return 1 + j; }
    __device__ static int ib(int j, int) { return 1 + j; }
};

template <bool FP32>
struct AdjFam<kGaussian, FP32> {
    using F = Gaussian<FP32>;
    static constexpr bool kTwo = true;
    __device__ static void point(const typename F::Acc& acc, double& val, double& wt, double& gu) {
        val = F::finish(acc);
        wt = val;
        gu = 0.0;
    }
    __device__ static void dir(double x, const AdjDim& c, double wt, double& ga, double& gb) {
        const double y = x - c.w;
        ga = fma(wt, -2.0 * c.c * y * y, ga);
        gb = fma(wt, 2.0 * c.c * c.c * y, gb);
    }
    __device__ static int ia(int j, int) { return j; }
    __device__ static int ib(int j, int d) { return d + j; }
};

template <bool FP32>
struct AdjFam<kExpQuadratic, FP32> {
    using F = ExpQuadratic<FP32>;
    static constexpr bool kTwo = true;
    __device__ static void point(const typename F::Acc& acc, double& val, double& wt, double& gu) {
        val = F::finish(acc);
        wt = val;
        gu = 0.0;
    }
    __device__ static void dir(double x, const AdjDim& c, double wt, double& ga, double& gb) {
        const double y = x - c.w;
        ga = fma(wt, y * y, ga);
        gb = fma(wt, -2.0 * c.c * y, gb);
    }
    __device__ static int ia(int j, int) { return j; }
    __device__ static int ib(int j, int d) { return d + j; }
};

template <class PF>
struct AdjPeak {
    using F = PF;
    static constexpr bool kTwo = true;
    __device__ static void point(const typename F::Acc& acc, double& val, double& wt, double& gu) {
        val = F::finish(acc);
        wt = val;
        gu = 0.0;
    }
    __device__ static void dir(double x, const AdjDim& c, double wt, double& ga, double& gb) {
        const double y = x - c.w;
        const double r = 1.0 / fma(y, y, 1.0 / (c.c * c.c));
        ga = fma(wt, 2.0 * r / (c.c * c.c * c.c), ga);
        gb = fma(wt, 2.0 * y * r, gb);
    }
    __device__ static int ia(int j, int) { return j; }
    __device__ static int ib(int j, int d) { return d + j; }
};

// Vector grid sum (two levels, grouped as in grid_sum_wave0): every workgroup
// holds L values in LDS `v`; returns true in exactly one workgroup, whose `v` then
// holds the totals over all workgroups.  Partials are stored and waited for
// before each ticket.
__device__ __forceinline__ bool grid_sum_vec(double* v, int L, int b, int G, double* partials,
                                             double* group_partials, uint32_t* tickets, int* flag) {
    const int NG = G < kReduceGroups ? G : kReduceGroups;
    const int g = b % NG;
    const int members = (G - g + NG - 1) / NG;
    for (int p = threadIdx.x; p < L; p += kBlock) publish_partial(&partials[(size_t)b * L + p], v[p]);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) *flag = take_ticket(&tickets[g], (uint32_t)members) ? 1 : 0;
    __syncthreads();
    if (!*flag) return false;
    for (int p = threadIdx.x; p < L; p += kBlock) {
        double t = 0.0;
        for (int i = 0; i < members; ++i) t += read_partial(&partials[(size_t)(g + i * NG) * L + p]);
        publish_partial(&group_partials[(size_t)g * L + p], t);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) *flag = take_ticket(&tickets[kReduceGroups], (uint32_t)NG) ? 1 : 0;
    __syncthreads();
    if (!*flag) return false;
    for (int p = threadIdx.x; p < L; p += kBlock) {
        double t = 0.0;
        for (int i = 0; i < NG; ++i) t += read_partial(&group_partials[(size_t)i * L + p]);
        v[p] = t;
    }
    __syncthreads();
    return true;
}

template <int FAM, bool FP32, class A, int M>
__global__ __launch_bounds__(kBlock) void adjoint_kernel(const AdjArgs a) {
    using F = typename A::F;
    using Acc = typename F::Acc;
    using Dim = typename F::Dim;
    constexpr uint32_t kTile = kBlock * M;
    extern __shared__ double s_g[];  // [kWaves][L] per-wave sums, then [L] block totals
    __shared__ TileShared<F> s;
    __shared__ AdjDim s_adj[kDimChunk];
    __shared__ double s_red[3 * kWaves];
    __shared__ int s_flag;

    const int set = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int P = a.P, L = P + 1;  // slot P holds the sum of f / scale
    const double* p = a.params + (size_t)set * P;
    const ProblemView v = make_view(a.d, a.n, a.inv_n, a.z, a.shift, p);
    double init0, ds1;
    int ie;
    block_constants<F>(v, s_red, init0, ds1, ie);
    for (int i = tid; i < kWaves * L; i += kBlock) s_g[i] = 0.0;

    auto fill_adj = [&](int j0, int dc) {
        for (int e = tid; e < dc; e += kBlock) {
            const int j = j0 + e;
            uint32_t whole;
            double frac;
            split_shift(v.shift, j, v.n, whole, frac);
            AdjDim t;
            if constexpr (FAM == kOscillatory) {
                t.c = p[1 + j];
                t.w = 0.0;
            } else if constexpr (FAM == kExpSum) {
                t.c = p[j];
                t.w = 0.0;
            } else {
                t.c = p[j];
                t.w = p[v.d + j];
            }
            t.soff = frac * v.inv_n;
            s_adj[e] = t;
        }
    };
    const bool one_chunk = v.d <= kDimChunk;
    if (one_chunk) {
        fill_dims<F>(v, s, 0, v.d);
        fill_adj(0, v.d);
    }

    double tval = 0.0, tgu = 0.0;
    for (uint32_t tile = blockIdx.x; tile < a.tiles; tile += gridDim.x) {
        const uint32_t tile_base = tile * kTile;
        const uint32_t i0 = tile_base + (uint32_t)wv * (kWave * M) + (uint32_t)lane;
        // ---- sweep 1: forward state of the thread's points
        Acc acc[M];
#pragma unroll
        for (int m = 0; m < M; ++m) acc[m] = F::init(init0);
        for (int j0 = 0; j0 < v.d; j0 += kDimChunk) {
            const int dc = min(kDimChunk, v.d - j0);
            __syncthreads();
            if (!one_chunk) {
                fill_dims<F>(v, s, j0, dc);
                __syncthreads();
            }
            fill_tile<F, M>(v, s, j0, dc, tile_base);
            __syncthreads();
            for (int jj = 0; jj < dc; ++jj) {
                uint32_t k = addmod(s.kw[jj * kWaves + wv], s.lz[jj * kWave + lane], v.n);
                const uint2 stp = s.st[jj];
                const Dim c = s.c[jj];
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    F::step(acc[m], k, c);
                    k = stepmod(k, stp.x, stp.y);
                }
                if constexpr (F::kRenorm > 0) {
                    if ((j0 + jj + 1) % F::kRenorm == 0) {
#pragma unroll
                        for (int m = 0; m < M; ++m) F::renorm(acc[m]);
                    }
                }
            }
        }
        double wt[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            double val, w, gu;
            A::point(acc[m], val, w, gu);
            const bool ok = i0 + (uint32_t)(kWave * m) < v.n;
            wt[m] = ok ? w : 0.0;
            tval += ok ? val : 0.0;
            tgu += ok ? gu : 0.0;
        }
        // ---- sweep 2: per-direction derivative terms
        for (int j0 = 0; j0 < v.d; j0 += kDimChunk) {
            const int dc = min(kDimChunk, v.d - j0);
            if (!one_chunk) {
                __syncthreads();
                fill_dims<F>(v, s, j0, dc);
                fill_adj(j0, dc);
                __syncthreads();
                fill_tile<F, M>(v, s, j0, dc, tile_base);
                __syncthreads();
            }
            for (int jj = 0; jj < dc; ++jj) {
                uint32_t k = addmod(s.kw[jj * kWaves + wv], s.lz[jj * kWave + lane], v.n);
                const uint2 stp = s.st[jj];
                const AdjDim c = s_adj[jj];
                double ga = 0.0, gb = 0.0;
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    const double x = fma((double)k, v.inv_n, c.soff);
                    A::dir(x, c, wt[m], ga, gb);
                    k = stepmod(k, stp.x, stp.y);
                }
                ga = wave_total(ga);
                if constexpr (A::kTwo) gb = wave_total(gb);
                if (lane == kWaveTotalLane) {
                    s_g[wv * L + A::ia(j0 + jj, v.d)] += ga;
                    if constexpr (A::kTwo) s_g[wv * L + A::ib(j0 + jj, v.d)] += gb;
                }
            }
        }
    }
    // Workgroup vector: waves in order, then the per-point terms.
    tval = block_sum(tval, s_red);
    tgu = block_sum(tgu, s_red);
    double* tot = s_g + kWaves * L;
    for (int i = tid; i < L; i += kBlock) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) t += s_g[w * L + i];
        if (i == P) t = tval;
        if (FAM == kOscillatory && i == 0) t = tgu;
        tot[i] = t;
    }
    __syncthreads();
    const int G = (int)gridDim.x;
    double* part = a.scratch + (size_t)set * a.scratch_stride;
    if (!grid_sum_vec(tot, L, (int)blockIdx.x, G, part, part + (size_t)G * L,
                      a.tickets + (size_t)set * kTicketsPerReduction, &s_flag))
        return;
    const double scale = F::scale(ds1, ie) / v.dn;
    const double g = a.gq ? a.gq[set] : 1.0;
    for (int i = tid; i < P; i += kBlock) a.grad_out[(size_t)set * P + i] = g * scale * tot[i];
    if (tid == 0) a.q_out[set] = scale * tot[P];
}

// --------------------------------------------------------------------------
// Set-batched form for the linear-argument families (exp-sum, oscillatory) with
// d <= kSetsMaxDims and many parameter sets sharing the lattice.  With
// x_j = (k_j + phi_j) / n (k_j the shifted index, phi_j the shift's fraction times
// n) the argument of set s at point i is
//   t_is = t0_s + sum_j k_ij a_js   (a_js = c_sj / (2 pi n) in turns, or c_sj log2(e) / n)
// and the derivative sums need only
//   K_js = sum_i k_ij w_is,   W_s = sum_i w_is,   sum_i x_ij w_is = (K_js + phi_j W_s) / n.
// Both are dense contractions over the lattice indices, T = k A and K = k^T W, done
// with the FP64 matrix instruction v_mfma_f64_16x16x4f64 (D[m][n] += sum_q
// A[m][q] B[q][n] over a 16 x 4 by 4 x 16 block; lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16] and holds D[4 r + l / 16][l % 16] in register r -- the
// layout as measured on gfx950).
//
// A wave serves the kSetsPerWave = 32 sets of group blockIdx.y (two blocks of 16)
// over a contiguous range of points, 16 points at a time:
//  1. T[16 points][32 sets] = t0 + k[16][4 DQ] A[4 DQ][32]: the A operand is the
//     lane's own index k(point c0 + l % 16, direction 4 q + l / 16), stepped by
//     16 z_j mod n per block (exact integers, converted to double); the B operand
//     is the coefficient a(direction 4 q + l / 16, set 16 b + l % 16), held in
//     registers.
//  2. the lane holds T for points c0 + 4 r + l / 16 (r < 4) of set 16 b + l % 16
//     and evaluates f and the weight w there;
//  3. K[16 e + m][16 b + n] += sum over the block's points of k(point, direction)
//     w(point, set), with reduction step u pairing the lanes' register r = u with
//     points c0 + 4 u + l / 16: the weights are already where the B operand needs
//     them; the A operand is the lane's index k(point c0 + 4 u + l / 16,
//     direction 16 e + l % 16), stepped like the first.
// Partial points of the last block get w = 0 and f = 0.  The K accumulators (one
// 16 x 16 block per 16 directions and 16 sets) stay in registers over the wave's
// points; then waves are added in order and workgroups by the vector grid sum, so
// the result is bit-reproducible.
// Two blocks of 16 sets per wave keep the state at about 230 registers (two
// waves per SIMD); four needed 476 and one wave per SIMD, and moved accumulators
// between the register files every block.
constexpr int kSetsMaxDims = kAdjSetsMaxParams - 1;
constexpr int kSetBlocks = 2;                    // blocks of 16 sets per wave
constexpr int kSetsPerWave = 16 * kSetBlocks;
constexpr int kMfmaPoints = 16;      // points per block

typedef double v4d __attribute__((ext_vector_type(4)));

struct AdjSetsArgs {
    int d;
    uint32_t n;
    double inv_n;
    const int64_t* z;
    const double* shift;
    const double* params;
    int P;
    int nsets;
    uint64_t points_per_wave;  // a multiple of kMfmaPoints
    const double* gq;
    double* q_out;
    double* grad_out;
    uint32_t* tickets;
    double* scratch;
    size_t scratch_stride;  // doubles per group of kSetsPerWave sets
};

// LDS doubles: the coefficient table [DM][kSetsPerWave] during the sweep, then the block
// totals (per set K_0 .. K_{DM-1}, W, Q) and per-lane partials of W, Q.
__host__ __device__ constexpr int sets_lds_doubles(int DM) {
    return DM * kSetsPerWave > kSetsPerWave * (DM + 2) + 2 * kWave ? DM * kSetsPerWave
                                                                    : kSetsPerWave * (DM + 2) + 2 * kWave;
}

__device__ __forceinline__ uint32_t index_of(uint64_t i, uint32_t z, uint32_t whole, uint32_t n, double inv_n) {
    return addmod(mulmod(i, (uint64_t)z, n, inv_n), whole, n);
}

template <int FAM, bool FP32, int DQ>
__global__ __launch_bounds__(kBlock) void adjoint_sets_kernel(const AdjSetsArgs a) {
    constexpr int NE = (DQ + 3) / 4;  // blocks of 16 directions in K
    constexpr int DM = 4 * DQ;        // directions covered (>= d)
    extern __shared__ double s_tot[];  // [DM][sets] coefficients; later [sets][DM + 2] totals, [2][64] partials
    __shared__ double s_phi[DM];        // shift fraction * n per direction
    __shared__ uint32_t s_whole[DM];    // shift whole part per direction
    __shared__ uint32_t s_step[DM];     // 16 z_j mod n
    __shared__ uint32_t s_z[DM];
    __shared__ int s_flag;

    const int tid = threadIdx.x, l = tid & (kWave - 1), wv = tid / kWave;
    const int lr = l % 16, lq = l / 16;
    const int d = a.d;
    const int pc = FAM == kOscillatory ? 1 : 0;  // parameter offset of c_0
    const double dn = (double)a.n;

    for (int j = tid; j < DM; j += kBlock) {
        uint32_t whole = 0;
        double frac = 0.0;
        if (j < d) split_shift(a.shift, j, a.n, whole, frac);
        s_phi[j] = frac;
        s_whole[j] = whole;
        s_z[j] = j < d ? (uint32_t)a.z[j] : 0u;
        s_step[j] = j < d ? mulmod_small((uint32_t)kMfmaPoints, (uint32_t)a.z[j], dn, a.inv_n) : 0u;
    }
    __syncthreads();

    // coefficient table: s_coef[j * kSetsPerWave + s] = a_js of set s of the group (0 beyond d
    // and past the last set); the B operand of step 1 reads a(4 q + lq, 16 b + lr)
    double* s_coef = s_tot;
    for (int e = tid; e < DM * kSetsPerWave; e += kBlock) {
        const int j = e / kSetsPerWave, set = blockIdx.y * kSetsPerWave + e % kSetsPerWave;
        double c = 0.0;
        if (j < d && set < a.nsets) c = a.params[(size_t)set * a.P + pc + j];
        s_coef[e] = FAM == kOscillatory ? c * kInv2Pi * a.inv_n : c * kLog2e * a.inv_n;
    }
    // t0 of set 16 b + lr
    double t0[kSetBlocks];
#pragma unroll
    for (int b = 0; b < kSetBlocks; ++b) {
        const int set = blockIdx.y * kSetsPerWave + 16 * b + lr;
        const double* p = a.params + (size_t)(set < a.nsets ? set : 0) * a.P;
        double c0 = FAM == kOscillatory ? p[0] : 0.0;
        for (int j = 0; j < d; ++j) {
            const double c = p[pc + j];
            const double aj = FAM == kOscillatory ? c * kInv2Pi * a.inv_n : c * kLog2e * a.inv_n;
            // exp-sum: centred by sum_j c_j log2(e) / 2 (restored by the final scale)
            c0 += aj * s_phi[j] - (FAM == kExpSum ? 0.5 * kLog2e * c : 0.0);
        }
        t0[b] = c0;
    }
    __syncthreads();

    const uint64_t p0 = ((uint64_t)blockIdx.x * kWaves + wv) * a.points_per_wave;
    const uint64_t p1 = min(p0 + a.points_per_wave, (uint64_t)a.n);
    // index states: step 1 (point p + lr, direction 4 q + lq), step 3 (point p + 4 u + lq, direction 16 e + lr)
    uint32_t kt[DQ], kk[4][NE], st_t[DQ], st_k[NE];
#pragma unroll
    for (int q = 0; q < DQ; ++q) {
        const int j = 4 * q + lq;
        st_t[q] = s_step[j];
        kt[q] = j < d ? index_of(p0 + lr, s_z[j], s_whole[j], a.n, a.inv_n) : 0u;
    }
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        const int j = 16 * e + lr;
        st_k[e] = j < DM ? s_step[j] : 0u;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            kk[u][e] = j < d ? index_of(p0 + 4 * u + lq, s_z[j], s_whole[j], a.n, a.inv_n) : 0u;
    }
    v4d acc[NE][kSetBlocks];
#pragma unroll
    for (int e = 0; e < NE; ++e)
#pragma unroll
        for (int b = 0; b < kSetBlocks; ++b) acc[e][b] = v4d{0.0, 0.0, 0.0, 0.0};
    double qs[kSetBlocks] = {}, ws[kSetBlocks] = {};

    for (uint64_t c0 = p0; c0 < p1; c0 += kMfmaPoints) {
        // 1. arguments of the block's 16 points for the wave's sets
        v4d t[kSetBlocks];
#pragma unroll
        for (int b = 0; b < kSetBlocks; ++b) t[b] = v4d{t0[b], t0[b], t0[b], t0[b]};
#pragma unroll
        for (int q = 0; q < DQ; ++q) {
            const double av = (double)kt[q];
            const double* cr = s_coef + (4 * q + lq) * kSetsPerWave + lr;
#pragma unroll
            for (int b = 0; b < kSetBlocks; ++b)
                t[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, cr[16 * b], t[b], 0, 0, 0);
            // at most 4 kSetBlocks coefficient loads in flight: keeps them from all
            // being hoisted into registers ahead of the matrix instructions
            if ((q & 3) == 3) asm volatile("" ::: "memory");
        }
        // 2. f and its weight at points c0 + 4 r + lq
        double w[kSetBlocks][4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const bool live = c0 + (uint64_t)(4 * r + lq) < p1;
#pragma unroll
            for (int b = 0; b < kSetBlocks; ++b) {
                const double tt = t[b][r];
                double val, wt;
                if constexpr (FAM == kOscillatory) {
                    const double fr = tt - rint(tt);
                    if constexpr (FP32) {
                        val = (double)__builtin_amdgcn_cosf((float)fr);
                        wt = -(double)__builtin_amdgcn_sinf((float)fr);
                    } else {
                        double sn, cs;
                        sincospi(2.0 * fr, &sn, &cs);
                        val = cs;
                        wt = -sn;
                    }
                } else {
                    val = FP32 ? exp2_split_f32(tt) : exp2_double(tt);
                    wt = val;
                }
                val = live ? val : 0.0;
                wt = live ? wt : 0.0;
                qs[b] += val;
                ws[b] += wt;
                w[b][r] = wt;
            }
        }
        // 3. K += k^T w over the block's points
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                const double av = (double)kk[u][e];
#pragma unroll
                for (int b = 0; b < kSetBlocks; ++b)
                    acc[e][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, w[b][u], acc[e][b], 0, 0, 0);
            }
        }
        // next block: 16 points on
#pragma unroll
        for (int q = 0; q < DQ; ++q) kt[q] = addmod(kt[q], st_t[q], a.n);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int e = 0; e < NE; ++e) kk[u][e] = addmod(kk[u][e], st_k[e], a.n);
    }

    // block totals, waves in order: K from the accumulators (register r of block
    // (e, b) is direction 16 e + 4 r + lq of set 16 b + lr); W and Q summed over lq
    constexpr int L = DM + 2;
    double* part = s_tot + kSetsPerWave * L;  // [2][64]: per-lane W, Q partials of one wave
    __syncthreads();  // every wave is past the coefficient table
    for (int w = 0; w < kWaves; ++w) {
        if (wv == w) {
#pragma unroll
            for (int e = 0; e < NE; ++e)
#pragma unroll
                for (int b = 0; b < kSetBlocks; ++b)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int j = 16 * e + 4 * r + lq;
                        if (j < DM) {
                            double* slot = &s_tot[(16 * b + lr) * L + j];
                            *slot = (w == 0 ? 0.0 : *slot) + acc[e][b][r];
                        }
                    }
        }
        __syncthreads();
        for (int b = 0; b < kSetBlocks; ++b) {
            if (wv == w) {
                part[l] = ws[b];
                part[kWave + l] = qs[b];
            }
            __syncthreads();
            if (wv == w && lq == 0) {
                const double wsum = ((part[lr] + part[16 + lr]) + part[32 + lr]) + part[48 + lr];
                const double qsum = ((part[kWave + lr] + part[kWave + 16 + lr]) + part[kWave + 32 + lr]) +
                                    part[kWave + 48 + lr];
                double* row = &s_tot[(16 * b + lr) * L];
                row[DM] = (w == 0 ? 0.0 : row[DM]) + wsum;
                row[DM + 1] = (w == 0 ? 0.0 : row[DM + 1]) + qsum;
            }
            __syncthreads();
        }
    }
    const int G = (int)gridDim.x;
    double* gpart = a.scratch + (size_t)blockIdx.y * a.scratch_stride;
    if (!grid_sum_vec(s_tot, kSetsPerWave * L, (int)blockIdx.x, G, gpart, gpart + (size_t)G * kSetsPerWave * L,
                      a.tickets + (size_t)blockIdx.y * kTicketsPerReduction, &s_flag))
        return;
    // one thread per (set, output)
    const double inv_n2 = a.inv_n * a.inv_n;
    for (int e = tid; e < kSetsPerWave * (a.P + 1); e += kBlock) {
        const int es = e / (a.P + 1), o = e % (a.P + 1);
        const int st = blockIdx.y * kSetsPerWave + es;
        if (st >= a.nsets) continue;
        const double* ps = a.params + (size_t)st * a.P;
        double scale = 1.0;
        if constexpr (FAM == kExpSum) {
            double h = 0.0;
            for (int j = 0; j < d; ++j) h += 0.5 * kLog2e * ps[j];
            scale = exp2(h);
        }
        const double g = a.gq ? a.gq[st] : 1.0;
        const double* v = s_tot + es * L;
        if (o == a.P) {
            a.q_out[st] = scale * v[DM + 1] * a.inv_n;
        } else if (FAM == kOscillatory && o == 0) {
            a.grad_out[(size_t)st * a.P] = g * kTwoPi * v[DM] * a.inv_n;
        } else {
            const int j = o - pc;
            a.grad_out[(size_t)st * a.P + o] = g * scale * (v[j] + s_phi[j] * v[DM]) * inv_n2;
        }
    }
}

static int sets_blocks(int groups) {
    int g = 512 / groups;
    return g < 1 ? 1 : g;
}

// Doubles per group of kSetsPerWave sets: one vector of kSetsPerWave (DM + 2) per
// workgroup and per group.
static size_t sets_group_stride(int DM, int groups) {
    const size_t G = (size_t)sets_blocks(groups);
    return (G + (G < (size_t)kReduceGroups ? G : (size_t)kReduceGroups)) * (size_t)kSetsPerWave *
           (size_t)(DM + 2);
}

static int sets_dims(int d) {
    return d <= 16 ? 16 : d <= 32 ? 32 : d <= 48 ? 48 : d <= 52 ? 52 : d <= 56 ? 56 : 64;
}

static size_t sets_workspace_bytes(int d, int nsets) {
    const int groups = (nsets + kSetsPerWave - 1) / kSetsPerWave;
    const int DM = sets_dims(d);
    return kZeroBytes + ((size_t)groups * sets_group_stride(DM, groups) * sizeof(double) + 255) / 256 * 256;
}

static bool use_sets_kernel(const AdjLaunch& L) {
    return (L.family == kExpSum || L.family == kOscillatory) && L.d <= kSetsMaxDims && L.nsets >= 16;
}

template <int FAM, bool FP32, int DQ>
static hipError_t launch_sets_dq(const AdjLaunch& L, hipStream_t stream) {
    constexpr int DM = 4 * DQ;
    AdjSetsArgs a;
    a.d = L.d;
    a.n = L.n;
    a.inv_n = 1.0 / (double)L.n;
    a.z = L.z;
    a.shift = L.shift;
    a.params = L.params;
    a.P = L.P;
    a.nsets = L.nsets;
    const int groups = (L.nsets + kSetsPerWave - 1) / kSetsPerWave;
    int G = sets_blocks(groups);
    const uint64_t waves_min = ((uint64_t)L.n + kMfmaPoints - 1) / kMfmaPoints;  // at least one block per wave
    if ((uint64_t)G * kWaves > waves_min) G = (int)((waves_min + kWaves - 1) / kWaves);
    a.points_per_wave = (((uint64_t)L.n + (uint64_t)G * kWaves - 1) / ((uint64_t)G * kWaves) + kMfmaPoints - 1) /
                        kMfmaPoints * kMfmaPoints;
    a.gq = L.gq;
    a.q_out = L.q_out;
    a.grad_out = L.grad_out;
    a.tickets = (uint32_t*)L.ws;
    a.scratch = (double*)((char*)L.ws + kZeroBytes);
    a.scratch_stride = sets_group_stride(DM, groups);
    const size_t lds = (size_t)sets_lds_doubles(DM) * sizeof(double);
    hipLaunchKernelGGL((adjoint_sets_kernel<FAM, FP32, DQ>), dim3((unsigned)G, (unsigned)groups), dim3(kBlock), lds,
                       stream, a);
    return hipGetLastError();
}

template <int FAM, bool FP32>
static hipError_t launch_sets(const AdjLaunch& L, hipStream_t stream) {
    switch (sets_dims(L.d)) {
        case 16: return launch_sets_dq<FAM, FP32, 4>(L, stream);
        case 32: return launch_sets_dq<FAM, FP32, 8>(L, stream);
        case 48: return launch_sets_dq<FAM, FP32, 12>(L, stream);
        case 52: return launch_sets_dq<FAM, FP32, 13>(L, stream);
        case 56: return launch_sets_dq<FAM, FP32, 14>(L, stream);
        default: return launch_sets_dq<FAM, FP32, 16>(L, stream);
    }
}

// --------------------------------------------------------------------------
int adjoint_blocks_per_set(int nsets) {
    int g = kMaxAdjBlocks / (nsets > 0 ? nsets : 1);
    if (g < 1) g = 1;
    return g;
}

// Scratch doubles per set: one vector of P + 1 per workgroup and per group.
static size_t adjoint_set_stride(int P, int nsets) {
    const size_t G = (size_t)adjoint_blocks_per_set(nsets);
    return (G + (G < (size_t)kReduceGroups ? G : (size_t)kReduceGroups)) * (size_t)(P + 1);
}

size_t adjoint_workspace_bytes(int P, int nsets) {
    const size_t per_set =
        kZeroBytes + ((size_t)nsets * adjoint_set_stride(P, nsets) * sizeof(double) + 255) / 256 * 256;
    // the set-batched form (d = P or P - 1 <= kSetsMaxDims) lays its scratch out per
    // group of kSetsPerWave sets; d <= min(P, kSetsMaxDims) bounds its size
    const size_t batched = P <= kSetsMaxDims + 1 ? sets_workspace_bytes(P < kSetsMaxDims ? P : kSetsMaxDims, nsets)
                                                 : 0;
    return per_set > batched ? per_set : batched;
}

template <int FAM, bool FP32, class A, int M>
static hipError_t launch_adj_m(const AdjLaunch& L, hipStream_t stream) {
    AdjArgs a;
    a.d = L.d;
    a.n = L.n;
    a.inv_n = 1.0 / (double)L.n;
    a.z = L.z;
    a.shift = L.shift;
    a.params = L.params;
    a.P = L.P;
    const uint64_t tile = (uint64_t)kBlock * M;
    a.tiles = (uint32_t)(((uint64_t)L.n + tile - 1) / tile);
    a.gq = L.gq;
    a.q_out = L.q_out;
    a.grad_out = L.grad_out;
    a.tickets = (uint32_t*)L.ws;
    a.scratch = (double*)((char*)L.ws + kZeroBytes);
    int g = adjoint_blocks_per_set(L.nsets);
    if ((uint32_t)g > a.tiles) g = (int)a.tiles;
    a.scratch_stride = adjoint_set_stride(L.P, L.nsets);
    const size_t lds = (size_t)(kWaves + 1) * (L.P + 1) * sizeof(double);
    hipLaunchKernelGGL((adjoint_kernel<FAM, FP32, A, M>), dim3((unsigned)g, (unsigned)L.nsets),
                       dim3(kBlock), lds, stream, a);
    return hipGetLastError();
}

template <int FAM, bool FP32, class A>
static hipError_t launch_adj_f(const AdjLaunch& L, hipStream_t stream) {
    const uint64_t want_tiles = 3ull * device_cu_count() / 2;
    const uint64_t per_set = (want_tiles + L.nsets - 1) / L.nsets;
    int M = 16;
    while (M > 4 && ((uint64_t)L.n + kBlock * M - 1) / ((uint64_t)kBlock * M) < per_set) M /= 2;
    if (M == 16) return launch_adj_m<FAM, FP32, A, 16>(L, stream);
    if (M == 8) return launch_adj_m<FAM, FP32, A, 8>(L, stream);
    return launch_adj_m<FAM, FP32, A, 4>(L, stream);
}

hipError_t launch_adjoint(const AdjLaunch& L, hipStream_t stream) {
    if (use_sets_kernel(L)) {
        if (L.family == kExpSum)
            return L.fp32 ? launch_sets<kExpSum, true>(L, stream) : launch_sets<kExpSum, false>(L, stream);
        return L.fp32 ? launch_sets<kOscillatory, true>(L, stream) : launch_sets<kOscillatory, false>(L, stream);
    }
    if (L.fp32) {
        switch (L.family) {
            case kExpSum: return launch_adj_f<kExpSum, true, AdjFam<kExpSum, true>>(L, stream);
            case kOscillatory: return launch_adj_f<kOscillatory, true, AdjFam<kOscillatory, true>>(L, stream);
            case kGaussian: return launch_adj_f<kGaussian, true, AdjFam<kGaussian, true>>(L, stream);
            case kExpQuadratic:
                return launch_adj_f<kExpQuadratic, true, AdjFam<kExpQuadratic, true>>(L, stream);
            case kProductPeak:
                // double-precision factors (FP32 reciprocal per point): the FP32 factors'
                // per-direction rounding would bias the gradient sums as it biases Q
                return launch_adj_f<kProductPeak, true, AdjPeak<ProductPeak<false, true>>>(L, stream);
        }
    } else {
        switch (L.family) {
            case kExpSum: return launch_adj_f<kExpSum, false, AdjFam<kExpSum, false>>(L, stream);
            case kOscillatory: return launch_adj_f<kOscillatory, false, AdjFam<kOscillatory, false>>(L, stream);
            case kGaussian: return launch_adj_f<kGaussian, false, AdjFam<kGaussian, false>>(L, stream);
            case kExpQuadratic:
                return launch_adj_f<kExpQuadratic, false, AdjFam<kExpQuadratic, false>>(L, stream);
            case kProductPeak:
                return launch_adj_f<kProductPeak, false, AdjPeak<ProductPeak<false, false>>>(L, stream);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace qmc
