// Phase timeline of the plain-sum launch: the body of the single-problem kernel of
// csrc/lattice_sum.hip for a problem with d <= 64 directions (one set of direction
// tables), built from the same device code (tile.hpp, common.hpp, families.hpp), with
// the constant 100 MHz clock read at the boundaries of its phases.  Not part of
// libqmc.so; built into libqmc_probe.so and called by bench.py (--workload
// timeline_d20_peak), which also checks that it returns the library's bits.
//
// Marks of workgroup b, marks[b * kMarks + m] (clock ticks, written by one lane):
//   0      first instruction of wave 0
//   1      direction tables and first start residues built (after setup's barrier)
//   2..17  end of wave w's tiles (w = 0..15)
//   18     workgroup total in wave 0 (after block_sum_wave0's barrier)
//   19     wave 0 returned from the grid sum
//   20     1 in the workgroup that produced the total, else 0
// Modes: 0 the whole kernel; 1 an empty kernel on the same grid (marks 0 and 19);
// 2 the fixed part alone: setup, workgroup total and grid sum, without the tiles.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"
#include "families.hpp"
#include "kernels.hpp"
#include "tile.hpp"

namespace {

using namespace qmc;

constexpr int kMarks = 24;
constexpr int kM = 4;  // points per thread: the library's choice for n near 2^20

__device__ __forceinline__ void put_mark(unsigned long long* marks, int m) {
    marks[(size_t)blockIdx.x * kMarks + m] = (unsigned long long)wall_clock64();
}

template <class F, int M, int B, bool FI, int MODE>
__global__ __launch_bounds__(B) void plain_timeline_kernel(const int64_t* z, const double* params,
                                                           double inv_n, uint32_t n, int d, uint32_t tiles,
                                                           double* q_out, uint32_t* tickets, double* slots_base,
                                                           int slot_stride, unsigned long long* marks) {
    constexpr uint32_t kTile = B * M;
    __shared__ TileShared<F, B> s;
    __shared__ double s_red[3 * (B / kWave)];
    const bool lead = threadIdx.x == 0;
    if (lead) put_mark(marks, 0);
    if constexpr (MODE == 1) {
        if (lead) put_mark(marks, 19);
        return;
    } else {
        const ProblemView v = make_view(d, n, inv_n, z, nullptr, params);
        double init0, ds1;
        int ie;
        double tacc = 0.0;
        guard_in_t<F> gin{};
        setup_one_chunk<F, M, B>(v, s, s_red, blockIdx.x * kTile, init0, ds1, ie, gin);
        if (lead) put_mark(marks, 1);
        guard_check<F, B>(v, s, gin);
        if constexpr (MODE == 0) {
            for (uint32_t tile = blockIdx.x; tile < tiles; tile += gridDim.x)
                tacc += tile_points_one_chunk<F, M, B, FI, false>(v, s, tile * kTile, init0, tile == blockIdx.x);
        }
        if ((threadIdx.x & (kWave - 1)) == 0) put_mark(marks, 2 + (int)(threadIdx.x / kWave));
        double bsum = block_sum_wave0<B>(tacc, s_red);
        if (guard_redo(s, ds1))
            bsum = block_sum_wave0<B>(redo_tiles<F, M, B, FI, false>(v, s, blockIdx.x, gridDim.x, MODE == 0 ? tiles : 0u, init0), s_red);
        if (threadIdx.x >= kWave) return;
        if (lead) put_mark(marks, 18);
        GridSlots gs;
        gs.partials = slots_base;
        gs.group_partials = slots_base + (size_t)gridDim.x * slot_stride;
        gs.tickets = tickets;
        gs.slot_stride = slot_stride;
        gs.ticket_stride = kMaxSumSets;
        double total;
        const bool last = grid_sum_wave0(bsum, (int)blockIdx.x, (int)gridDim.x, gs, total);
        if (lead) {
            put_mark(marks, 19);
            marks[(size_t)blockIdx.x * kMarks + 20] = last ? 1ull : 0ull;
            if (last) {
                double q = (total / v.dn) * F::scale(ds1, ie);
                if constexpr (param_scaled<F>::value) q *= v.p[v.d];
                q_out[0] = q;
            }
        }
    }
}

template <int MODE>
hipError_t launch_mode(unsigned g, const int64_t* z, const double* params, double inv_n, uint32_t n, int d,
                       uint32_t tiles, double* q_out, uint32_t* tickets, double* slots, int slot_stride,
                       unsigned long long* marks, hipStream_t stream) {
    using F = ProductPeak<true, true>;
    hipLaunchKernelGGL((plain_timeline_kernel<F, kM, kSumBlock, true, MODE>), dim3(g), dim3(kSumBlock), 0,
                       stream, z, params, inv_n, n, d, tiles, q_out, tickets, slots, slot_stride, marks);
    return hipGetLastError();
}

}  // namespace

extern "C" {

// Marks per workgroup.
int qmc_probe_timeline_marks(void) { return kMarks; }

// One launch of the product-peak plain sum with FP32 factors (QMC_FP32_COMPENSATED,
// d <= 32 directions, n <= 2^24, no shift), laid out as the library lays it out for
// one problem: kSumBlock threads per workgroup, kM points per thread, one workgroup
// per tile up to the library's limit per problem.  z (d int64), params (2d + 1
// doubles, the family's layout), q_out (1 double) and marks (at least
// qmc_probe_timeline_workgroups(n) * qmc_probe_timeline_marks() uint64) are device
// arrays; ws is a library workspace whose zero region is zero (the launch leaves it
// zero).  Returns the number of workgroups launched, -1 for bad arguments, or
// -(1000 + HIP error).
int qmc_probe_timeline_workgroups(uint32_t n) {
    if (n < 1) return -1;
    const uint64_t tiles = ((uint64_t)n + (uint64_t)kSumBlock * kM - 1) / ((uint64_t)kSumBlock * kM);
    return (int)(tiles < (uint64_t)kMaxSumBlocksPerSet ? tiles : (uint64_t)kMaxSumBlocksPerSet);
}

int qmc_probe_plain_timeline(int mode, int d, uint32_t n, const int64_t* z, const double* params, double* q_out,
                             unsigned long long* marks, void* ws, void* stream) {
    if (mode < 0 || mode > 2 || d < 1 || d > kPeakF32MaxDims || n < 1 || n > kFloatIndexMaxN || !z || !params ||
        !q_out || !marks || !ws)
        return -1;
    const uint32_t tiles = (uint32_t)(((uint64_t)n + (uint64_t)kSumBlock * kM - 1) / ((uint64_t)kSumBlock * kM));
    const unsigned g = (unsigned)qmc_probe_timeline_workgroups(n);
    // The library's layout for one problem: tickets at the start of the zero region,
    // the tagged slots after them, one 128-byte line per slot.
    uint32_t* tickets = (uint32_t*)ws;
    double* slots = (double*)((char*)ws + kTicketBytes);
    const int slot_stride = 16;
    static_assert(grid_scratch_doubles(kMaxSumBlocksPerSet) * 16 * sizeof(double) <= kSlotBytes,
                  "one problem's slots fit the slot region a line apart");
    const double inv_n = 1.0 / (double)n;
    hipError_t e;
    switch (mode) {
        case 0: e = launch_mode<0>(g, z, params, inv_n, n, d, tiles, q_out, tickets, slots, slot_stride, marks, (hipStream_t)stream); break;
        case 1: e = launch_mode<1>(g, z, params, inv_n, n, d, tiles, q_out, tickets, slots, slot_stride, marks, (hipStream_t)stream); break;
        default: e = launch_mode<2>(g, z, params, inv_n, n, d, tiles, q_out, tickets, slots, slot_stride, marks, (hipStream_t)stream); break;
    }
    return e == hipSuccess ? (int)g : -(1000 + (int)e);
}

}  // extern "C"
