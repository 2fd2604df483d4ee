// Plain rank-1 lattice rule, fused into one persistent launch (eq. 1.2, eq. 2.1):
//   Q = (1/n) sum_{i=0}^{n-1} f(x_i),  x_ij = {(k_ij + shift_j n) / n},  k_ij = (i z_j) mod n.
//
// Work decomposition: tiles of kSumBlock * M consecutive indices (tile.hpp), the
// workgroups of a set looping over tiles (persistent grid).  The loop runs over
// directions outside and over a thread's M points inside, so that each
// direction's constants are loaded once per M points and the per-point state is M
// registers whatever d is; no 64-bit arithmetic runs per point.
//
// The Bernoulli products behind the lattice-quality criteria satisfy
// f(x) = f(1 - x) in every coordinate; on an unshifted lattice point n - i mirrors
// point i, so those sums evaluate i <= n/2 only (finish_points).
//
// Reduction: per-thread FP64 sums, a DPP wave reduction, waves in order, one
// FP64 partial per workgroup, then the two-level fixed-order grid sum of
// common.hpp, run by wave 0 (tickets and tagged slots in the workspace's zero
// region, left zero by their last user).
#include "common.hpp"
#include "families.hpp"
#include "kernels.hpp"
#include "tile.hpp"

namespace qmc {

// Kernel arguments: the ones the prologue needs come first, so that a build with
// kernel-argument preloading has them in scalar registers at wave start instead
// of behind a load from the argument segment.
struct SumArgs {
    const int64_t* z;
    const double* params;
    const double* shift;  // may be null
    double inv_n;         // 1.0 / n
    uint32_t n;
    int d;
    int param_stride;     // doubles between the parameter rows of two sets (0: shared)
    int shift_stride;     // doubles between the shift rows of two sets (0: shared)
    int z_stride;         // int64 between the generating vectors of two sets (0: shared)
    uint32_t tiles;
    double* q_out;
    uint32_t* tickets;    // counter region of the workspace
    double* scratch;      // tagged slots, `scratch_stride` doubles per set
    uint32_t scratch_stride;
    int slot_stride;      // doubles between two slots of a set
};

// Set `set` owns slots [set * scratch_stride, ...) and the tickets
// set, set + kMaxSumSets, ..., one per 16 KiB line of the counter region.
__device__ __forceinline__ GridSlots set_slots(double* scratch, uint32_t scratch_stride,
                                               int slot_stride, uint32_t* tickets, int set, int G) {
    GridSlots s;
    s.partials = scratch + (size_t)set * scratch_stride;
    s.group_partials = s.partials + (size_t)G * slot_stride;
    s.tickets = tickets + set;
    s.slot_stride = slot_stride;
    s.ticket_stride = kMaxSumSets;
    return s;
}

template <class F, int M, int B, bool FI, bool MIRROR>
__global__ __launch_bounds__(B) void lattice_sum_kernel(
    const int64_t* z, const double* params, const double* shift, double inv_n, uint32_t n, int d,
    int param_stride, int shift_stride, int z_stride, uint32_t tiles, double* q_out,
    uint32_t* tickets, double* scratch, uint32_t scratch_stride, int slot_stride) {
    constexpr uint32_t kTile = B * M;
    __shared__ TileShared<F, B> s;
    __shared__ double s_red[3 * (B / kWave)];

    const int set = blockIdx.y;
    const ProblemView v =
        make_view(d, n, inv_n, z + (size_t)set * z_stride,
                  shift ? shift + (size_t)set * shift_stride : nullptr,
                  params + (size_t)set * param_stride);
    double init0, ds1;
    int ie;
    double tacc = 0.0;
    if (v.d <= kDimChunk) {
        // One set of direction tables serves every tile; the first tile's start
        // residues are built with them.
        guard_in_t<F> gin{};
        setup_one_chunk<F, M, B>(v, s, s_red, blockIdx.x * kTile, init0, ds1, ie, gin);
        guard_check<F, B>(v, s, gin);
        for (uint32_t tile = blockIdx.x; tile < tiles; tile += gridDim.x)
            tacc += tile_points_one_chunk<F, M, B, FI, MIRROR>(v, s, tile * kTile, init0, tile == blockIdx.x);
    } else {
        block_constants<F, B>(v, s_red, init0, ds1, ie);
        for (uint32_t tile = blockIdx.x; tile < tiles; tile += gridDim.x)
            tacc += tile_points<F, M, B, FI, MIRROR>(v, s, tile * kTile, init0);
    }

    // Workgroup total to wave 0 (red[B / kWave ..) is untouched by the setup), then
    // the grid sum by wave 0 alone; the other waves are done.
    double bsum = block_sum_wave0<B>(tacc, s_red);
    if (v.d <= kDimChunk && guard_redo(s, ds1))
        bsum = block_sum_wave0<B>(redo_tiles<F, M, B, FI, MIRROR>(v, s, blockIdx.x, gridDim.x, tiles, init0), s_red);
    if (threadIdx.x >= kWave) return;
    const GridSlots slots =
        set_slots(scratch, scratch_stride, slot_stride, tickets, set, (int)gridDim.x);
    double total;
    if (grid_sum_wave0(bsum, (int)blockIdx.x, (int)gridDim.x, slots, total) && threadIdx.x == 0) {
        double q = (total / v.dn) * F::scale(ds1, ie);
        if constexpr (param_scaled<F>::value) q *= v.p[v.d];
        q_out[set] = q;
    }
}

static_assert((kMaxSumBlocksPerSet + kReduceGroups - 1) / kReduceGroups <= kWave &&
                  kReduceGroups <= kWave,
              "grid_sum_wave0 puts one group member, and one group, per lane");

// --------------------------------------------------------------------------
// Randomly shifted rule (Sec. 2.1): after the R shifted sums, their mean and the
// standard error of the mean, sqrt(sum_r (Q_r - mean)^2 / (R (R - 1))) (0 for
// R = 1).  One wave; lane l owns r = l, l + 64, ... and the lanes are combined by
// the fixed-order wave reduction, so the result is reproducible.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(kWave) void shift_stats_kernel(const double* q, int R, double* stats) {
    const int lane = threadIdx.x;
    double s = 0.0;
    for (int r = lane; r < R; r += kWave) s += q[r];
    const double mean = lane_value(wave_total(s), kWaveTotalLane) / (double)R;
    double v = 0.0;
    for (int r = lane; r < R; r += kWave) {
        const double e = q[r] - mean;
        v = fma(e, e, v);
    }
    const double ss = lane_value(wave_total(v), kWaveTotalLane);
    if (lane == 0) {
        stats[0] = mean;
        stats[1] = R > 1 ? sqrt(ss / ((double)R * (double)(R - 1))) : 0.0;
    }
}

hipError_t launch_shift_stats(const double* q, int R, double* stats, hipStream_t stream) {
    hipLaunchKernelGGL(shift_stats_kernel, dim3(1), dim3(kWave), 0, stream, q, R, stats);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Debug export of the indices, through the same start/step decomposition.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void lattice_points_kernel(int d, uint32_t n, double inv_n,
                                                                const int64_t* z, uint64_t i0,
                                                                uint64_t count, int32_t* k_out) {
    constexpr int M = 4;
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    const uint64_t base = i0 + (uint64_t)blockIdx.x * (kBlock * M) + (uint64_t)wv * (kWave * M);
    for (int j = 0; j < d; ++j) {
        const uint32_t zj = (uint32_t)z[j];
        const uint32_t kw = mulmod(base % n, zj, n, inv_n);
        uint32_t k = addmod(kw, mulmod((uint64_t)lane, zj, n, inv_n), n);
        const uint32_t st = mulmod((uint64_t)kWave, zj, n, inv_n), stm = st - n;
        for (int m = 0; m < M; ++m) {
            const uint64_t r = base - i0 + (uint64_t)lane + (uint64_t)(kWave * m);
            if (r < count) k_out[r * d + j] = (int32_t)k;
            k = stepmod(k, st, stm);
        }
    }
}

// --------------------------------------------------------------------------
// Launchers
// --------------------------------------------------------------------------
int sum_blocks_per_set(int nsets) {
    int g = kMaxSumBlocks / (nsets > 0 ? nsets : 1);
    if (g < 1) g = 1;
    if (g > kMaxSumBlocksPerSet) g = kMaxSumBlocksPerSet;
    return g;
}

// Slot spacing: one 128-byte line per slot when every set's slots fit the slot
// region that way, else packed.  Packed, nsets * set_stride <= 2048 + 64 * nsets
// doubles (<= 2.1 MiB for nsets <= kMaxSumSets) fits in kSlotBytes.
static int slot_stride(int nsets) {
    const size_t lined = (size_t)nsets * grid_scratch_doubles(sum_blocks_per_set(nsets)) * 16;
    return lined * sizeof(double) <= kSlotBytes ? 16 : 1;
}

// Slot doubles per set, rounded to 256 bytes.
static size_t set_stride(int nsets) {
    return (grid_scratch_doubles(sum_blocks_per_set(nsets)) * slot_stride(nsets) + 31) / 32 * 32;
}

size_t plain_workspace_bytes(int nsets) {
    // Tickets and tagged slots both live in the zero region.
    (void)nsets;
    return kZeroBytes;
}

int device_cu_count() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            cus = prop.multiProcessorCount;
        if (cus <= 0) cus = 256;
    }
    return cus;
}

// Points a launch evaluates: n, or n/2 + 1 for a mirrored sum (finish_points).
static uint64_t evaluated_points(const PlainLaunch& L, bool mirror) {
    return mirror ? (uint64_t)L.n / 2 + 1 : (uint64_t)L.n;
}

template <class F, int M, bool FI, bool MIRROR>
static hipError_t launch_fm(const PlainLaunch& L, hipStream_t stream) {
    SumArgs a;
    a.z = L.z;
    a.params = L.params;
    a.shift = L.shift;
    a.inv_n = 1.0 / (double)L.n;
    a.n = L.n;
    a.d = L.d;
    a.param_stride = L.param_stride;
    a.shift_stride = L.shift_stride;
    a.z_stride = L.z_stride;
    const uint64_t tile = (uint64_t)kSumBlock * M;
    a.tiles = (uint32_t)((evaluated_points(L, MIRROR) + tile - 1) / tile);
    a.q_out = L.q_out;
    a.tickets = (uint32_t*)L.ws;
    a.scratch = (double*)((char*)L.ws + kTicketBytes);  // tagged-slot part of the zero region
    a.scratch_stride = (uint32_t)set_stride(L.nsets);
    a.slot_stride = slot_stride(L.nsets);
    int g = sum_blocks_per_set(L.nsets);
    if (L.max_blocks > 0 && L.max_blocks < g) g = L.max_blocks;
    if ((uint32_t)g > a.tiles) g = (int)a.tiles;
    dim3 grid((unsigned)g, (unsigned)L.nsets);
    hipLaunchKernelGGL((lattice_sum_kernel<F, M, kSumBlock, FI, MIRROR>), grid, dim3(kSumBlock), 0, stream,
                       a.z, a.params, a.shift, a.inv_n, a.n, a.d, a.param_stride, a.shift_stride,
                       a.z_stride, a.tiles, a.q_out, a.tickets, a.scratch, a.scratch_stride,
                       a.slot_stride);
    return hipGetLastError();
}

// The exact-float index step whenever n allows; mirror-symmetric families on an
// unshifted lattice sum half of the points.
template <class F, int M>
static hipError_t launch_fi(const PlainLaunch& L, hipStream_t stream) {
    const bool fi = L.n <= kFloatIndexMaxN;
    if constexpr (mirror_family<F>::value) {
        if (!L.shift) return fi ? launch_fm<F, M, true, true>(L, stream) : launch_fm<F, M, false, true>(L, stream);
    }
    return fi ? launch_fm<F, M, true, false>(L, stream) : launch_fm<F, M, false, false>(L, stream);
}

template <class F>
static hipError_t launch_f(const PlainLaunch& L, hipStream_t stream) {
    int M = L.points_per_thread;
    if (M == 0) {
        // As many points per thread as still leaves >= 1.5 tiles per CU over all the
        // launch's sets (the per-direction setup is amortised over M points, the
        // latency over the workgroups resident on a CU).
        const uint64_t want_tiles = 3ull * device_cu_count() / 2;
        const uint64_t pts = evaluated_points(L, mirror_family<F>::value && !L.shift);
        M = 16;
        while (M > 4 &&
               (uint64_t)L.nsets * ((pts + kSumBlock * M - 1) / ((uint64_t)kSumBlock * M)) < want_tiles)
            M /= 2;
    }
    switch (M) {
        case 4: return launch_fi<F, 4>(L, stream);
        case 8: return launch_fi<F, 8>(L, stream);
        case 16: return launch_fi<F, 16>(L, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_lattice_sum(const PlainLaunch& L, hipStream_t stream) {
    // The Bernoulli products behind the criteria run in FP64 in both precisions.
    if (L.family == kBernoulli2) return launch_f<BernoulliProduct<2>>(L, stream);
    if (L.family == kBernoulli4) return launch_f<BernoulliProduct<4>>(L, stream);
    if (L.family == kBernoulli2S) return launch_f<BernoulliProduct<2, true>>(L, stream);
    if (L.family == kBernoulli4S) return launch_f<BernoulliProduct<4, true>>(L, stream);
    if (L.fp32) {
        switch (L.family) {
            case kExpSum: return launch_f<ExpSum<true>>(L, stream);
            case kProductPeak:
                if (L.d <= kPeakF32MaxDims) return launch_f<ProductPeak<true, true>>(L, stream);
                return launch_f<ProductPeak<false, true>>(L, stream);
            case kGaussian: return launch_f<Gaussian<true>>(L, stream);
            case kOscillatory: return launch_f<Oscillatory<true>>(L, stream);
            case kExpQuadratic: return launch_f<ExpQuadratic<true>>(L, stream);
        }
    } else {
        switch (L.family) {
            case kExpSum: return launch_f<ExpSum<false>>(L, stream);
            case kProductPeak: return launch_f<ProductPeak<false, false>>(L, stream);
            case kGaussian: return launch_f<Gaussian<false>>(L, stream);
            case kOscillatory: return launch_f<Oscillatory<false>>(L, stream);
            case kExpQuadratic: return launch_f<ExpQuadratic<false>>(L, stream);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_lattice_points(int d, uint32_t n, const int64_t* z, int64_t i0, int64_t count,
                                 int32_t* k_out, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    const uint64_t per_block = (uint64_t)kBlock * 4;
    const unsigned grid = (unsigned)(((uint64_t)count + per_block - 1) / per_block);
    hipLaunchKernelGGL(lattice_points_kernel, dim3(grid), dim3(kBlock), 0, stream, d, n,
                       1.0 / (double)n, z, (uint64_t)i0, (uint64_t)count, k_out);
    return hipGetLastError();
}

}  // namespace qmc
