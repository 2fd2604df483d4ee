// Adjoint of the plain lattice rule: Q_s and gq_s * dQ_s/d(params_s) for every
// parameter set s sharing the lattice (derivative of eq. 1.2):
//   dQ/dp = (1/n) sum_i df/dp (x_i).
// For the four product- or sum-form families df/dp_j = w(x) * h_j(x_j): a per-point
// weight w times a function of one coordinate,
//   exp-sum      w = f,        dc_j: h = x_j
//   oscillatory  w = -sin(th), dc_j: h = x_j,  du: 2 pi w (per point)
//   Gaussian     w = f,        dc_j: h = -2 c_j (x_j - w_j)^2,  dw_j: h = 2 c_j^2 (x_j - w_j)
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
    return kZeroBytes + ((size_t)nsets * adjoint_set_stride(P, nsets) * sizeof(double) + 255) / 256 * 256;
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
    if (L.fp32) {
        switch (L.family) {
            case kExpSum: return launch_adj_f<kExpSum, true, AdjFam<kExpSum, true>>(L, stream);
            case kOscillatory: return launch_adj_f<kOscillatory, true, AdjFam<kOscillatory, true>>(L, stream);
            case kGaussian: return launch_adj_f<kGaussian, true, AdjFam<kGaussian, true>>(L, stream);
            case kProductPeak:
                if (L.d <= kPeakF32MaxDims)
                    return launch_adj_f<kProductPeak, true, AdjPeak<ProductPeak<true, true>>>(L, stream);
                return launch_adj_f<kProductPeak, true, AdjPeak<ProductPeak<false, true>>>(L, stream);
        }
    } else {
        switch (L.family) {
            case kExpSum: return launch_adj_f<kExpSum, false, AdjFam<kExpSum, false>>(L, stream);
            case kOscillatory: return launch_adj_f<kOscillatory, false, AdjFam<kOscillatory, false>>(L, stream);
            case kGaussian: return launch_adj_f<kGaussian, false, AdjFam<kGaussian, false>>(L, stream);
            case kProductPeak:
                return launch_adj_f<kProductPeak, false, AdjPeak<ProductPeak<false, false>>>(L, stream);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace qmc
