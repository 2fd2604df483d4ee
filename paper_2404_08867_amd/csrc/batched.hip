// Batched plain lattice rule: many integrands with their own d, n, z, family and
// parameters in one persistent launch (eq. 1.2 for each problem).
//
// The plan (host) orders the problems longest-first (cost n * d) and numbers
// their tiles consecutively.  Persistent workgroups pop tile numbers from an
// atomic queue in the workspace's counter region, find the tile's problem by a
// binary search over the tile offsets, evaluate the tile with the same device
// code as the single-problem kernel (tile.hpp) and publish one FP64 partial per
// tile.  The workgroup that completes a problem's last tile sums that problem's
// partials in tile order and writes its Q -- a fixed order, so the results are
// bit-reproducible whatever the schedule was.  The last workgroup to leave resets
// the queue, so the launch can be replayed (e.g. from a captured graph) without
// any memset.  When every problem has n <= 2^24 the indices are stepped as exact
// floats (tile.hpp).
#include "batched.hpp"
#include "tile.hpp"

namespace qmc {

struct BatchArgs {
    const DevProblem* probs;  // [count], in schedule order
    int count;
    uint32_t total_tiles;
    double* q_out;            // [count], indexed by DevProblem::out_index
    uint32_t* counters;       // [0] queue, [1] exit, [2 + p] tickets of problem p
    double* partials;         // [total_tiles]
};

template <bool FP32>
struct BatchFamilies {
    using E = ExpSum<FP32>;
    using PS = ProductPeak<FP32, FP32>;   // FP32 factors (d <= kPeakF32MaxDims when FP32)
    using PD = ProductPeak<false, FP32>;  // FP64 factors
    using G = Gaussian<FP32>;
    using O = Oscillatory<FP32>;
    using Q = ExpQuadratic<FP32>;
};

template <bool FP32>
union BatchShared {
    TileShared<typename BatchFamilies<FP32>::E> e;
    TileShared<typename BatchFamilies<FP32>::PS> ps;
    TileShared<typename BatchFamilies<FP32>::PD> pd;
    TileShared<typename BatchFamilies<FP32>::G> g;
    TileShared<typename BatchFamilies<FP32>::O> o;
    TileShared<typename BatchFamilies<FP32>::Q> q;
};

template <class F, int M, bool FI>
__device__ __forceinline__ void run_tile(const BatchArgs& a, int pi, const DevProblem& pr,
                                         uint32_t local_tile, TileShared<F>& s, double* red,
                                         int* flag) {
    constexpr uint32_t kTile = kBlock * M;
    const ProblemView v = make_view(pr.d, pr.n, pr.inv_n, pr.z, pr.shift, pr.params);
    double init0, ds1;
    int ie;
    double t;
    if (v.d <= kDimChunk) {
        guard_in_t<F> gin{};
        setup_one_chunk<F, M>(v, s, red, local_tile * kTile, init0, ds1, ie, gin);
        guard_check<F, kBlock>(v, s, gin);
        t = tile_points_one_chunk<F, M, kBlock, FI>(v, s, local_tile * kTile, init0, true);
    } else {
        block_constants<F>(v, red, init0, ds1, ie);
        t = tile_points<F, M, kBlock, FI>(v, s, local_tile * kTile, init0);
    }
    double bsum = block_sum(t, red);
    if (v.d <= kDimChunk && guard_redo(s, ds1))
        bsum = block_sum(redo_tiles<F, M, kBlock, FI, false>(v, s, local_tile, 1, local_tile + 1, init0), red);
    if (threadIdx.x == 0) {
        publish_partial(&a.partials[pr.tile_begin + local_tile], bsum);
        *flag = take_ticket(&a.counters[2 + pi], pr.tiles) ? 1 : 0;
    }
    __syncthreads();
    if (*flag) {
        double u = 0.0;
        for (uint32_t i = threadIdx.x; i < pr.tiles; i += kBlock)
            u += read_partial(&a.partials[pr.tile_begin + i]);
        u = block_sum(u, red);
        if (threadIdx.x == 0) a.q_out[pr.out_index] = (u / v.dn) * F::scale(ds1, ie);
    }
}

template <bool FP32, int M, bool FI>
__global__ __launch_bounds__(kBlock) void batched_kernel(const BatchArgs a) {
    using Fam = BatchFamilies<FP32>;
    __shared__ BatchShared<FP32> s;
    __shared__ double red[3 * kWaves];
    __shared__ int flag;
    __shared__ uint32_t s_tile;

    for (;;) {
        if (threadIdx.x == 0)
            s_tile = __hip_atomic_fetch_add(&a.counters[0], 1u, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const uint32_t tile = s_tile;
        __syncthreads();  // every thread has read s_tile before it is written again
        if (tile >= a.total_tiles) break;
        // The problem whose tiles [tile_begin, tile_begin + tiles) contain `tile`.
        int lo = 0, hi = a.count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.probs[mid].tile_begin <= tile) lo = mid;
            else hi = mid - 1;
        }
        const DevProblem pr = a.probs[lo];
        const uint32_t local = tile - pr.tile_begin;
        switch (pr.family) {
            case kExpSum: run_tile<typename Fam::E, M, FI>(a, lo, pr, local, s.e, red, &flag); break;
            case kProductPeak:
                if (!FP32 || pr.d <= kPeakF32MaxDims)
                    run_tile<typename Fam::PS, M, FI>(a, lo, pr, local, s.ps, red, &flag);
                else
                    run_tile<typename Fam::PD, M, FI>(a, lo, pr, local, s.pd, red, &flag);
                break;
            case kGaussian: run_tile<typename Fam::G, M, FI>(a, lo, pr, local, s.g, red, &flag); break;
            case kExpQuadratic: run_tile<typename Fam::Q, M, FI>(a, lo, pr, local, s.q, red, &flag); break;
            default: run_tile<typename Fam::O, M, FI>(a, lo, pr, local, s.o, red, &flag); break;
        }
        __syncthreads();  // shared tables and flag are free for the next tile
    }
    // The last workgroup to leave resets the queue for the next launch.
    if (threadIdx.x == 0 && take_ticket(&a.counters[1], gridDim.x))
        __hip_atomic_store(&a.counters[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool FP32, int M, bool FI>
static hipError_t launch_batched_m(const BatchLaunch& L, hipStream_t stream) {
    BatchArgs a;
    a.probs = L.probs;
    a.count = L.count;
    a.total_tiles = L.total_tiles;
    a.q_out = L.q_out;
    a.counters = (uint32_t*)L.ws;
    a.partials = (double*)((char*)L.ws + kZeroBytes);
    hipLaunchKernelGGL((batched_kernel<FP32, M, FI>), dim3((unsigned)L.grid), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

template <int M, bool FI>
static hipError_t launch_batched_mf(const BatchLaunch& L, hipStream_t stream) {
    return L.fp32 ? launch_batched_m<true, M, FI>(L, stream) : launch_batched_m<false, M, FI>(L, stream);
}

template <int M>
static hipError_t launch_batched_mm(const BatchLaunch& L, hipStream_t stream) {
    return L.float_index ? launch_batched_mf<M, true>(L, stream) : launch_batched_mf<M, false>(L, stream);
}

hipError_t launch_batched(const BatchLaunch& L, hipStream_t stream) {
    switch (L.points_per_thread) {
        case 4: return launch_batched_mm<4>(L, stream);
        case 8: return launch_batched_mm<8>(L, stream);
        case 16: return launch_batched_mm<16>(L, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace qmc
