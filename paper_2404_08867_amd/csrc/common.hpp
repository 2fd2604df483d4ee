// Device-side building blocks shared by the lattice-sum kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qmc {

constexpr int kWave = 64;         // CDNA wavefront width
constexpr int kBlock = 256;       // threads per workgroup of the sum kernels
constexpr int kWaves = kBlock / kWave;
constexpr int kDimChunk = 64;     // dimensions whose index tables sit in LDS at once

// ---------------------------------------------------------------------------
// Exact modular arithmetic on lattice indices (eq. 2.1: k = (i z) mod n).
// Indices are residues in [0, n) with n < 2^31, so sums of two residues fit in
// 32 bits and products of two residues fit in 62 bits.
// ---------------------------------------------------------------------------

// (a * b) mod n for 0 <= a, b < n < 2^31.  The quotient is estimated in double
// precision -- off by at most 2 because a*b < n^2 < 2^62 -- and the remainder is
// corrected exactly in 64-bit integers with a fixed number of conditional steps
// (arguments outside the contract give a wrong residue, never a long loop).
__device__ __forceinline__ uint32_t mulmod(uint64_t a, uint64_t b, uint32_t n, double inv_n) {
    const uint64_t p = a * b;
    const uint64_t q = (uint64_t)floor((double)p * inv_n);
    int64_t r = (int64_t)(p - q * (uint64_t)n);
    const int64_t nn = (int64_t)n;
    r = r < 0 ? r + nn : r;
    r = r < 0 ? r + nn : r;
    r = r < 0 ? r + nn : r;
    r = r >= nn ? r - nn : r;
    r = r >= nn ? r - nn : r;
    r = r >= nn ? r - nn : r;
    return (uint32_t)r;
}

// (a * b) mod n when a * b < 2^52: the product and the remainder are exact in
// double precision, and the floor of the rounded quotient is off by at most one.
__device__ __forceinline__ uint32_t mulmod_small(uint32_t a, uint32_t b, double dn, double inv_n) {
    const double p = (double)a * (double)b;
    const double q = floor(p * inv_n);
    double r = fma(-q, dn, p);
    r = r < 0.0 ? r + dn : r;
    r = r >= dn ? r - dn : r;
    return (uint32_t)r;
}

// (a + b) mod n for residues a, b in [0, n): if a + b < n the subtraction wraps
// to a huge unsigned value and the minimum picks a + b.
__device__ __forceinline__ uint32_t addmod(uint32_t a, uint32_t b, uint32_t n) {
    const uint32_t t = a + b;
    return min(t, t - n);
}

// One step k <- (k + st) mod n with stm = st - n precomputed (mod 2^32):
// two independent adds and a min (three VALU operations).
__device__ __forceinline__ uint32_t stepmod(uint32_t k, uint32_t st, uint32_t stm) {
    return min(k + st, k + stm);
}

// The same step on an index held as a float, for n <= kFloatIndexMaxN = 2^24:
// k < n, st and stm = st - n are exact in single precision.  If k + st < n, that
// sum is exact and the other one negative, and a negative float's sign bit makes
// its bit pattern the larger one.  Otherwise k + st - n lies in [0, n) and is
// exact, and k + st (rounded when above 2^24) is not smaller; non-negative floats
// order like their patterns (an exact zero is +0.0, pattern 0).  Either way the
// unsigned minimum of the two patterns is the residue, as a float: three VALU
// operations and no integer-to-float conversion per point.
constexpr uint32_t kFloatIndexMaxN = 1u << 24;

__device__ __forceinline__ float stepmod_f(float k, float st, float stm) {
    return __uint_as_float(min(__float_as_uint(k + st), __float_as_uint(k + stm)));
}

// ---------------------------------------------------------------------------
// Deterministic reductions (fixed order within the wave, waves in index order
// across the workgroup).
// ---------------------------------------------------------------------------

// A double moved across lanes by one DPP pattern (both 32-bit halves); lanes of
// rows outside ROW_MASK receive 0.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_move(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over the wave's 64 lanes with DPP lane moves (no LDS traffic): pairs and
// quads by quad permutations, rows of 8 and 16 by the half-row and row mirrors,
// then rows 0+1 and 2+3 by a broadcast of lane 15, and all four rows by a
// broadcast of lane 31.  The total lands in lane kWave - 1; other lanes hold
// partial sums.  The order of the additions is fixed.
constexpr int kWaveTotalLane = kWave - 1;
__device__ __forceinline__ double wave_total(double v) {
    v += dpp_move<0xB1>(v);        // quad_perm [1,0,3,2]
    v += dpp_move<0x4E>(v);        // quad_perm [2,3,0,1]
    v += dpp_move<0x141>(v);       // row_half_mirror
    v += dpp_move<0x140>(v);       // row_mirror
    v += dpp_move<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// Sum over the workgroup; every thread receives the total.  `red` is an LDS
// scratch array of at least B / kWave doubles.  Ends with a barrier.
template <int B = kBlock>
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_total(v);
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    __syncthreads();
    if (lane == kWaveTotalLane) red[wv] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < (B / kWave); ++w) t += red[w];
    __syncthreads();
    return t;
}

// Three sums at once (two doubles and a small int carried as a double); every
// thread receives the totals.  `red` holds 3 * B / kWave doubles.
template <int B = kBlock>
__device__ __forceinline__ void block_sum3(double& a, double& b, int& c, double* red) {
    const double x = wave_total(a), y = wave_total(b), w = wave_total((double)c);
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    __syncthreads();
    if (lane == kWaveTotalLane) {
        red[wv] = x;
        red[(B / kWave) + wv] = y;
        red[2 * (B / kWave) + wv] = w;
    }
    __syncthreads();
    double tx = 0.0, ty = 0.0, tw = 0.0;
#pragma unroll
    for (int i = 0; i < (B / kWave); ++i) {
        tx += red[i];
        ty += red[(B / kWave) + i];
        tw += red[2 * (B / kWave) + i];
    }
    __syncthreads();
    a = tx;
    b = ty;
    c = (int)tw;
}

// ---------------------------------------------------------------------------
// Cross-workgroup completion: each workgroup publishes its partial and takes a
// ticket; the workgroup that draws the last ticket reads every partial and
// resets the ticket to zero for the next call.
//
// Only device-scope atomic accesses carry data between workgroups: partials are
// written with device-scope stores (write-through past the per-XCD L2) and read
// with device-scope loads, and every store is waited for before the ticket is
// taken.  This avoids the whole-L2 write-back and invalidate that an agent-scope
// release/acquire fence costs on a multi-XCD device.
//
// Two levels keep every counter lightly contended: workgroup b of G belongs to
// group g = b % NG (NG = min(G, kReduceGroups)); the last workgroup of a group sums
// the group's partials in index order and takes a ticket on the top counter; the
// last group sums the NG group partials in order.  The order of every addition is
// fixed, so results are bit-reproducible.
// ---------------------------------------------------------------------------
constexpr int kReduceGroups = 32;

__device__ __forceinline__ void publish_partial(double* slot, double v) {
    __hip_atomic_store(slot, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double read_partial(const double* slot) {
    return __hip_atomic_load(const_cast<double*>(slot), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One thread: wait until this wave's device-scope stores are complete, then take
// a ticket; the caller that draws the last of `expected` tickets resets it.
__device__ __forceinline__ bool take_ticket(uint32_t* ticket, uint32_t expected) {
    __builtin_amdgcn_s_waitcnt(0);
    const uint32_t t = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (t + 1 == expected) {
        __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return true;
    }
    return false;
}

// Workspace layout shared by every entry point: the first kTicketBytes hold
// counters that are zero between calls (each call returns the ones it used to
// zero); everything after is scratch that needs no initialisation.  Keeping the
// counters at fixed offsets means that no call can find another call's scratch
// data where it expects a zero counter, whatever sizes the two calls had.
constexpr size_t kTicketBytes = size_t(1) << 20;
// Then kSlotBytes of tagged slots (plain-sum grid reduction), also zero between
// calls; scratch that needs no initialisation starts at kZeroBytes.
constexpr size_t kSlotBytes = size_t(3) << 20;
constexpr size_t kZeroBytes = kTicketBytes + kSlotBytes;
constexpr int kTicketsPerReduction = kReduceGroups + 1;

// Workspace slots of one reduction over G workgroups.  Slot i sits at
// partials[i * slot_stride] (group slots likewise), ticket g at
// tickets[g * ticket_stride]: strides of a cache line or more keep the writers of
// different slots, and the atomics on different tickets, off each other's lines.
struct GridSlots {
    double* partials;        // [G] slots
    double* group_partials;  // [kReduceGroups] slots
    uint32_t* tickets;       // [kReduceGroups + 1] counters: per group, then the top one
    int slot_stride;         // doubles between consecutive slots
    int ticket_stride;       // counters between consecutive tickets
};

// Slots of one reduction over G workgroups.
__host__ __device__ constexpr size_t grid_scratch_doubles(int G) { return (size_t)G + kReduceGroups; }

// Scalar grid sum with tagged slots.  A slot holds the bits of a double XOR
// kSlotTag, so a zero slot means "not written yet" (the workspace is zero-filled
// and every reader clears the slots it consumed).  A writer publishes its slot
// and takes its ticket without waiting for the store to land; the reader that
// drew the last ticket waits on each slot until it is non-zero.  That wait ends:
// every slot it waits on belongs to a workgroup that issued the store before
// taking its ticket.  This keeps two store-completion round trips off the
// critical path of the last workgroup.
constexpr uint64_t kSlotTag = 0x7ff8dead5eedbeefull;  // a NaN pattern no partial takes

__device__ __forceinline__ void put_slot(double* slot, double v) {
    uint64_t e = (uint64_t)__double_as_longlong(v) ^ kSlotTag;
    if (e == 0) e = 0x7ff8000000000000ull ^ kSlotTag;  // the tag pattern itself: store a quiet NaN
    __hip_atomic_store(reinterpret_cast<uint64_t*>(slot), e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double take_slot(double* slot) {
    uint64_t* p = reinterpret_cast<uint64_t*>(slot);
    uint64_t x;
    while ((x = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == 0) {
        __builtin_amdgcn_s_sleep(1);
    }
    __hip_atomic_store(p, (uint64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double((long long)(x ^ kSlotTag));
}

// One thread: take a ticket without waiting for earlier stores (their readers
// wait on the tagged slots instead).
__device__ __forceinline__ bool take_ticket_nowait(uint32_t* ticket, uint32_t expected) {
    const uint32_t t = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (t + 1 == expected) {
        __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return true;
    }
    return false;
}

// A double of one lane, delivered to every lane of the wave.
__device__ __forceinline__ double lane_value(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Workgroup sum delivered to wave 0: the total of wave w (of W = B / kWave) goes
// to red[W + w] and, one barrier later, wave 0 adds them in wave order.  Lanes of
// wave 0 return the total, the other waves 0 (they need not take part in what
// follows).  red[W .. 2 W) must be free: no thread may still read them.
template <int B = kBlock>
__device__ __forceinline__ double block_sum_wave0(double v, double* red) {
    constexpr int W = B / kWave;
    v = wave_total(v);
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    if (lane == kWaveTotalLane) red[W + wv] = v;
    __syncthreads();
    double t = 0.0;
    if (wv == 0) {
#pragma unroll
        for (int w = 0; w < W; ++w) t += red[W + w];
    }
    return t;
}

// Grid sum run by wave 0 alone, with no workgroup barrier.  Called by the 64
// lanes of wave 0 of workgroup b of G, all holding the workgroup total v.
// Returns true in exactly one workgroup, whose wave-0 lanes then hold the grand
// total.  Member i of a group is lane i and group i is lane i of the top level,
// so the order of every addition is fixed whoever arrives last.
// Needs ceil(G / kReduceGroups) <= kWave and kReduceGroups <= kWave.
__device__ __forceinline__ bool grid_sum_wave0(double v, int b, int G, const GridSlots& s,
                                               double& total) {
    const int lane = threadIdx.x;
    const int NG = G < kReduceGroups ? G : kReduceGroups;
    const int g = b % NG;
    const int members = (G - g + NG - 1) / NG;
    const int me = b / NG;  // this workgroup's position in its group
    const size_t ss = (size_t)s.slot_stride;
    int last = 0;
    if (lane == 0) {
        if (members > 1) put_slot(&s.partials[b * ss], v);
        last = (members == 1 ||
                take_ticket_nowait(&s.tickets[(size_t)g * s.ticket_stride], (uint32_t)members))
                   ? 1
                   : 0;
    }
    if (!__builtin_amdgcn_readlane(last, 0)) return false;
    double t = 0.0;
    if (lane < members) t = (lane == me) ? v : take_slot(&s.partials[(g + (size_t)lane * NG) * ss]);
    if (members > 1 && lane == 0) {
        // Own slot: cleared by the lane that wrote it, so the clear follows the store.
        __hip_atomic_store(reinterpret_cast<uint64_t*>(&s.partials[b * ss]), (uint64_t)0,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    t = lane_value(wave_total(t), kWaveTotalLane);
    if (lane == 0) {
        if (NG > 1) put_slot(&s.group_partials[g * ss], t);
        last = (NG == 1 || take_ticket_nowait(&s.tickets[(size_t)kReduceGroups * s.ticket_stride],
                                              (uint32_t)NG))
                   ? 1
                   : 0;
    }
    if (!__builtin_amdgcn_readlane(last, 0)) return false;
    double u = 0.0;
    if (lane < NG) u = (lane == g) ? t : take_slot(&s.group_partials[lane * ss]);
    if (NG > 1 && lane == 0) {
        __hip_atomic_store(reinterpret_cast<uint64_t*>(&s.group_partials[g * ss]), (uint64_t)0,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    total = lane_value(wave_total(u), kWaveTotalLane);
    return true;
}

}  // namespace qmc
