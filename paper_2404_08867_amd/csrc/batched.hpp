// Batched lattice sums: the device-side problem table and the launcher (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace qmc {

// One problem of a batch as the kernel reads it (schedule order).
struct DevProblem {
    const int64_t* z;
    const double* params;
    const double* shift;   // may be null
    double inv_n;          // 1.0 / n
    uint32_t n;
    int32_t d;
    int32_t family;
    int32_t out_index;     // position of this problem's Q in the caller's output
    uint32_t tile_begin;   // first global tile number of the problem
    uint32_t tiles;        // number of tiles
};

struct BatchLaunch {
    const DevProblem* probs;
    int count;
    uint32_t total_tiles;
    int points_per_thread;  // 4, 8 or 16
    int grid;               // persistent workgroups
    bool fp32;
    bool float_index;       // every problem has n <= kFloatIndexMaxN: exact-float index step
    double* q_out;
    void* ws;
};

hipError_t launch_batched(const BatchLaunch& L, hipStream_t stream);

// Counter words and scratch doubles of the batched launch: a queue, an exit
// counter and one completion counter per problem; one partial per tile.
inline size_t batched_counter_words(int count) { return 2 + (size_t)count; }

}  // namespace qmc
