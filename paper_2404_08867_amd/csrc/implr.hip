// The affine transformation of Theorem 3.1 on a Korobov lattice and the improved
// lattice rule's tensor grid (Sec. 3.2, Lemma 3.2).
//
// For z = (1, a, ..., a^{d-1}) with a^{d-1} < n (so z_{i+1} = a z_i exactly), the
// transformed coordinates of lattice point j are grid ranks
//   s_i = | floor(j z_{i+1} / n) - a floor(j z_i / n) | = floor(a {j z_i / n})  in [0, a),  i < d,
//   s_d = floor(((j z_d) mod n) / z_d)                  in [0, n_d = ceil(n / z_d)),
// i.e. y_i = s_i / z_{i+1} and y_d = s_d z_d / n.  The grid has
// a^{d-1} ceil(n / a^{d-1}) points (eq. 3.5); n* is the number of them that no
// lattice point reaches -- the points the improved rule adds.  Integer work only:
// every result is exact and independent of the schedule.
//
// Two exact ways to count the reached grid points:
//  * order check: with s_1 most significant the grid index idx(j) of the Korobov
//    lattice grows strictly with j (within equal leading ranks the next fractional
//    part grows with j, and s_d grows by one per step).  The order kernel verifies
//    idx(j) < idx(j + 1) for every j with exact integer arithmetic (between two
//    residue wraps the recurrences fix the increment at one, so it computes idx
//    at the wraps only); when all pass, the n indices are n distinct grid points
//    and n* = grid - n;
//  * bitmap: every point sets its grid point's bit; n* = grid - set bits.  Runs
//    when the order check reports a violation (never, for inputs the entry point
//    accepts) or when the caller asks for it; it assumes nothing about the order.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace qmc {

constexpr int kImplrBlock = 256;

// floor(j z / n) for j, z < n < 2^31: the FP64 quotient is off by at most one.
__device__ __forceinline__ uint64_t floor_div(uint64_t j, uint64_t z, uint64_t n, double inv_n) {
    const uint64_t p = j * z;
    uint64_t q = (uint64_t)((double)p * inv_n);
    if (q * n > p) --q;
    if ((q + 1) * n <= p) ++q;
    return q;
}

// Workspace header: the set-bit counter and the order-violation flag.
struct ImplrState {
    unsigned long long set_count;
    uint32_t violation;
};

// The bitmap kernels run only when `force` is set or the order check failed.
__device__ __forceinline__ bool bitmap_needed(const ImplrState* st, int force) {
    return force || __hip_atomic_load(&st->violation, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
}

constexpr int kImplrGrid = 2048;  // workgroups of the grid-stride bitmap kernels

__global__ void implr_init_kernel(ImplrState* st) {
    if (threadIdx.x == 0) {
        st->set_count = 0ull;
        st->violation = 0u;
    }
}

__global__ __launch_bounds__(kImplrBlock) void implr_clear_kernel(uint32_t* bits, uint64_t words,
                                                                 const ImplrState* st, int force) {
    if (!bitmap_needed(st, force)) return;
    for (uint64_t i = (uint64_t)blockIdx.x * kImplrBlock + threadIdx.x; i < words;
         i += (uint64_t)gridDim.x * kImplrBlock)
        bits[i] = 0u;
}

// Residue and grid digit of direction i < d at lattice point j: r = (j z_i) mod n
// and s_i = floor(a r / n); e = (a r) mod n is the residue of direction i + 1.
__device__ __forceinline__ void implr_digit(uint64_t j, uint64_t z, uint32_t n, double inv_n, uint32_t a,
                                            uint32_t& r, uint32_t& s, uint32_t& e) {
    r = (uint32_t)(j * z - floor_div(j, z, n, inv_n) * n);
    s = (uint32_t)floor_div(r, a, n, inv_n);
    e = (uint32_t)((uint64_t)r * a - (uint64_t)s * n);
}

// The grid index with s_1 most significant: idx = ((s_1 a + s_2) a + ...) n_d + s_d.
// In this order the map j -> idx is strictly increasing (within a run of equal
// s_1 .. s_{i-1}, {j z_i / n} grows with j, and s_d grows by one per step), so a
// run of consecutive j covers an ascending, nearly contiguous range of bits.
//
// Each thread takes kImplrRun consecutive j.  Per direction it computes the
// residue once and then steps it (r += z_i, minus n on a wrap); the digit follows
// from the wraps: s_i(j + 1) = s_i(j) + w_{i+1} - a w_i.  The last digit steps its
// quotient and remainder by z_d (a wrap subtracts n = Q z_d + R).  The bits of one
// 32-bit word are gathered before one atomic OR; neighbouring lanes write
// neighbouring words, so a wave's atomics fall in a few cache lines.
constexpr int kImplrRun = 32;

__device__ __forceinline__ void implr_mark_run(uint64_t j0, int d, uint32_t n, double inv_n, uint32_t a,
                                               uint32_t zd, uint32_t nd, uint32_t Q, uint32_t R,
                                               uint32_t* bits) {
    const int cnt = (int)min((uint64_t)kImplrRun, (uint64_t)n - j0);
    uint64_t idx[kImplrRun];
#pragma unroll
    for (int t = 0; t < kImplrRun; ++t) idx[t] = 0;
    uint32_t z = 1;
    for (int i = 0; i + 1 < d; ++i) {
        const uint32_t zn = z * a;  // z_{i+1} = a z_i < n
        uint32_t r, s, e;
        implr_digit(j0, z, n, inv_n, a, r, s, e);
#pragma unroll
        for (int t = 0; t < kImplrRun; ++t) {
            idx[t] = idx[t] * a + s;
            r += z;
            const bool wi = r >= n;
            r = wi ? r - n : r;
            e += zn;
            const bool wn = e >= n;
            e = wn ? e - n : e;
            s = s + (uint32_t)wn - (wi ? a : 0u);
        }
        z = zn;
    }
    // last direction: r_d = (j z_d) mod n = q z_d + m
    uint32_t r = (uint32_t)(j0 * zd - floor_div(j0, zd, n, inv_n) * n);
    uint32_t q = r / zd, m = r - q * zd;
#pragma unroll
    for (int t = 0; t < kImplrRun; ++t) {
        idx[t] = idx[t] * nd + q;
        r += zd;
        const bool w = r >= n;
        const bool borrow = w && m < R;
        r = w ? r - n : r;
        q = q + 1u - (w ? Q : 0u) - (borrow ? 1u : 0u);
        m = m + (borrow ? zd : 0u) - (w ? R : 0u);
    }
    uint64_t word = idx[0] >> 5;
    uint32_t mask = 0;
#pragma unroll
    for (int t = 0; t < kImplrRun; ++t) {
        if (t < cnt) {
            if ((idx[t] >> 5) != word) {
                __hip_atomic_fetch_or(&bits[word], mask, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                word = idx[t] >> 5;
                mask = 0;
            }
            mask |= 1u << (idx[t] & 31);
        }
    }
    __hip_atomic_fetch_or(&bits[word], mask, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(kImplrBlock) void implr_mark_kernel(int d, uint32_t n, double inv_n,
                                                                uint32_t a, uint32_t zd, uint32_t nd,
                                                                uint32_t Q, uint32_t R, uint32_t* bits,
                                                                const ImplrState* st, int force) {
    if (!bitmap_needed(st, force)) return;
    for (uint64_t j0 = ((uint64_t)blockIdx.x * kImplrBlock + threadIdx.x) * kImplrRun; j0 < n;
         j0 += (uint64_t)gridDim.x * kImplrBlock * kImplrRun)
        implr_mark_run(j0, d, n, inv_n, a, zd, nd, Q, R, bits);
}

// The generator.  Wave w of the launch owns the 256 kImplrWalkK consecutive points
// from j0 + w * 256 kImplrWalkK; at step k lane l writes the four consecutive
// points j = base + 256 k + 4 l + t (t < 4) of each direction with one 16-byte
// store, so each store of a wave covers 1 KiB of one direction's row.  A lane
// keeps four independent steppers (one per t), each advancing by 256 points.
// Directions run last to first.  Per direction a stepper computes its first
// residue r = (j z_i) mod n and digit once, then steps both:
// r += D_i (D_i = 256 z_i mod n, minus n on a wrap w_i) and
//   s_i += c_i + w_{i+1} - a w_i,   c_i = floor(a D_i / n),
// because a r_i = s_i n + r_{i+1} and a D_i = c_i n + D_{i+1}; the wraps of
// direction i + 1 come from the previous pass.  The last digit steps its
// quotient and remainder by z_d (D_d = Q_d z_d + R_d; a wrap subtracts
// n = Q z_d + R).
constexpr int kImplrWalkK = 16;
constexpr int kImplrQuad = 4;
constexpr int kImplrWavePoints = kWave * kImplrQuad * kImplrWalkK;
constexpr int kImplrWalkWaves = kImplrBlock / kWave;

// Four ranks of one direction at rows row .. row + 3 (one 16-byte store when no
// guard is needed; rows need only 4-byte alignment).
template <bool GUARD>
__device__ __forceinline__ void implr_store4(int32_t* p, const uint32_t (&v)[kImplrQuad], uint64_t row,
                                             uint64_t count) {
#pragma unroll
    for (int t = 0; t < kImplrQuad; ++t)
        if (!GUARD || row + t < count) p[t] = (int32_t)v[t];
}

// One wave's 256 kImplrWalkK points; GUARD for the wave that reaches past count.
template <bool GUARD>
__device__ __forceinline__ void implr_points_wave(int d, uint32_t n, double inv_n, uint32_t a, uint32_t zd,
                                                  uint32_t Q, uint32_t R, uint64_t j0, uint64_t count,
                                                  uint64_t ld, int32_t* s_out, uint64_t row0) {
    const uint64_t jl = j0 + row0;
    constexpr uint32_t kStride = kWave * kImplrQuad;  // points between a stepper's steps
    uint32_t wnext[kImplrQuad] = {0u, 0u, 0u, 0u};
    // last direction: s = floor(r / z_d)
    {
        int32_t* out = s_out + (uint64_t)(d - 1) * ld + row0;
        uint32_t r[kImplrQuad], q[kImplrQuad], m[kImplrQuad];
#pragma unroll
        for (int t = 0; t < kImplrQuad; ++t) {
            r[t] = (uint32_t)((jl + t) * zd - floor_div(jl + t, zd, n, inv_n) * n);
            q[t] = r[t] / zd;
            m[t] = r[t] - q[t] * zd;
        }
        const uint32_t D = (uint32_t)((uint64_t)kStride * zd % n);
        const uint32_t Qd = D / zd, Rd = D - Qd * zd;
#pragma unroll
        for (int k = 0; k < kImplrWalkK; ++k) {
            implr_store4<GUARD>(out + (uint64_t)kStride * k, q, row0 + (uint64_t)kStride * k, count);
#pragma unroll
            for (int t = 0; t < kImplrQuad; ++t) {
                r[t] += D;
                const bool w = r[t] >= n;
                r[t] = w ? r[t] - n : r[t];
                m[t] += Rd;
                const bool c1 = m[t] >= zd;
                m[t] = c1 ? m[t] - zd : m[t];
                q[t] += Qd + (c1 ? 1u : 0u);
                const bool b = w && m[t] < R;
                q[t] = q[t] - (w ? Q : 0u) - (b ? 1u : 0u);
                m[t] = m[t] + (b ? zd : 0u) - (w ? R : 0u);
                wnext[t] |= (w ? 1u : 0u) << k;
            }
        }
    }
    uint32_t z = zd;
    for (int i = d - 2; i >= 0; --i) {
        z /= a;  // z_i = a^i
        int32_t* out = s_out + (uint64_t)i * ld + row0;
        uint32_t r[kImplrQuad], sd[kImplrQuad], wcur[kImplrQuad];
#pragma unroll
        for (int t = 0; t < kImplrQuad; ++t) {
            uint32_t e;
            implr_digit(jl + t, z, n, inv_n, a, r[t], sd[t], e);
            wcur[t] = 0u;
        }
        const uint32_t D = (uint32_t)((uint64_t)kStride * z % n);
        const uint32_t c = (uint32_t)floor_div(D, a, n, inv_n);
#pragma unroll
        for (int k = 0; k < kImplrWalkK; ++k) {
            implr_store4<GUARD>(out + (uint64_t)kStride * k, sd, row0 + (uint64_t)kStride * k, count);
#pragma unroll
            for (int t = 0; t < kImplrQuad; ++t) {
                r[t] += D;
                const bool w = r[t] >= n;
                r[t] = w ? r[t] - n : r[t];
                sd[t] = sd[t] + c + ((wnext[t] >> k) & 1u) - (w ? a : 0u);
                wcur[t] |= (w ? 1u : 0u) << k;
            }
        }
#pragma unroll
        for (int t = 0; t < kImplrQuad; ++t) wnext[t] = wcur[t];
    }
}

__global__ __launch_bounds__(kImplrBlock) void implr_points_kernel(int d, uint32_t n, double inv_n, uint32_t a,
                                                                  uint32_t zd, uint32_t Q, uint32_t R,
                                                                  uint64_t j0, uint64_t count, uint64_t ld,
                                                                  int32_t* s_out) {
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t wbase =
        ((uint64_t)blockIdx.x * kImplrWalkWaves + (threadIdx.x >> 6)) * (uint64_t)kImplrWavePoints;
    if (wbase >= count) return;  // wave-uniform
    const uint64_t row0 = wbase + (uint64_t)(kImplrQuad * lane);
    if (wbase + (uint64_t)kImplrWavePoints <= count)
        implr_points_wave<false>(d, n, inv_n, a, zd, Q, R, j0, count, ld, s_out, row0);
    else
        implr_points_wave<true>(d, n, inv_n, a, zd, Q, R, j0, count, ld, s_out, row0);
}

// The order check.  Lane l of the launch takes the kImplrOrderRun consecutive
// points starting at l * kImplrOrderRun.  Stepping j -> j + 1 adds z_i to every
// residue r_i = (j z_i) mod n; while no residue wraps, every digit but the last
// stays fixed (s_i changes only by w_{i+1} - a w_i) and the last grows by one, so
// idx grows by exactly one per step.  The lane therefore jumps from one wrap to
// the next: t = min_i ceil((n - r_i) / z_i) steps reach the next wrap of any
// direction; the t - 1 steps before it add t - 1 to idx and z_i (t - 1) to each
// residue; the step with the wrap is taken exactly (digits from the wraps, last
// digit from its residue) and idx is recomputed from the digits and must exceed
// the previous value.  The lane's first index is computed directly and must
// exceed the index of the point before it (the lane below's last, or, for lane 0
// of a wave, that point computed directly); every index must be below the grid
// size.  Exact integer work, about d divisions per wrap: a wrap of the last
// direction comes every n / z_d steps.
constexpr int kImplrOrderRun = 4096;
constexpr int kImplrMaxDims = 64;

__device__ __forceinline__ uint32_t implr_index_direct(uint64_t j, int d, uint32_t n, double inv_n,
                                                       uint32_t a, uint32_t zd, uint32_t nd) {
    uint32_t idx = 0, z = 1;
    for (int i = 0; i + 1 < d; ++i) {
        uint32_t r, s, e;
        implr_digit(j, z, n, inv_n, a, r, s, e);
        idx = idx * a + s;
        z *= a;
    }
    const uint32_t r = (uint32_t)(j * zd - floor_div(j, zd, n, inv_n) * n);
    return idx * nd + r / zd;
}

__global__ __launch_bounds__(kImplrBlock) void implr_order_kernel(int d, uint32_t n, double inv_n, uint32_t a,
                                                                 uint32_t zd, uint32_t nd, uint64_t grid,
                                                                 ImplrState* st) {
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t j0 = ((uint64_t)blockIdx.x * kImplrBlock + threadIdx.x) * kImplrOrderRun;
    const uint64_t wave_j0 = ((uint64_t)blockIdx.x * kImplrBlock + (threadIdx.x & ~(kWave - 1))) * kImplrOrderRun;
    if (wave_j0 >= n) return;  // wave-uniform
    bool bad = false;
    uint32_t first = 0, last = 0;
    const bool active = j0 < n;
    if (active) {
        const uint32_t steps = (uint32_t)min((uint64_t)kImplrOrderRun, (uint64_t)n - j0) - 1;
        uint32_t r[kImplrMaxDims], s[kImplrMaxDims], z[kImplrMaxDims];
        uint32_t zi = 1;
        for (int i = 0; i < d; ++i) {
            z[i] = zi;
            r[i] = (uint32_t)(j0 * zi - floor_div(j0, zi, n, inv_n) * n);
            s[i] = i + 1 < d ? (uint32_t)floor_div(r[i], a, n, inv_n) : r[i] / zd;
            if (i + 1 < d) zi *= a;
        }
        auto index = [&]() {
            uint32_t v = 0;
            for (int i = 0; i + 1 < d; ++i) v = v * a + s[i];
            return v * nd + s[d - 1];
        };
        uint32_t idx = index();
        first = idx;
        bad = (uint64_t)idx >= grid;
        uint32_t pos = 0;
        while (pos < steps) {
            // steps to the next wrap of any direction, capped at the run's end
            uint32_t t = steps - pos;
            for (int i = 0; i < d; ++i) {
                const uint32_t ti = (n - r[i] + z[i] - 1) / z[i];
                t = ti < t ? ti : t;
            }
            // t - 1 steps without a wrap: residues advance, the last digit and idx grow by t - 1
            const uint32_t adv = t - 1;
            for (int i = 0; i < d; ++i) r[i] += adv * z[i];
            s[d - 1] += adv;
            idx += adv;
            pos += adv;
            // one exact step (it holds the wrap unless the run ends first)
            uint64_t w = 0;  // bit i: residue i wrapped
            for (int i = 0; i < d; ++i) {
                r[i] += z[i];
                if (r[i] >= n) {
                    r[i] -= n;
                    w |= 1ull << i;
                }
            }
            for (int i = 0; i + 1 < d; ++i)
                s[i] = s[i] + (uint32_t)((w >> (i + 1)) & 1u) - (((w >> i) & 1u) ? a : 0u);
            s[d - 1] = r[d - 1] / zd;
            const uint32_t next = index();
            bad = bad || next <= idx || (uint64_t)next >= grid;
            idx = next;
            pos += 1;
        }
        last = idx;
    }
    // the point before the lane's first: the lane below's last, or directly
    const uint32_t below = (uint32_t)__shfl_up((int)last, 1, kWave);
    uint32_t prev = below;
    if (lane == 0) prev = j0 > 0 ? implr_index_direct(j0 - 1, d, n, inv_n, a, zd, nd) : 0u;
    if (active && j0 > 0 && first <= prev) bad = true;
    if (bad) __hip_atomic_fetch_or(&st->violation, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(kImplrBlock) void implr_count_kernel(const uint32_t* bits, uint64_t words,
                                                                 ImplrState* st, int force) {
    if (!bitmap_needed(st, force)) return;
    unsigned long long c = 0ull;
    for (uint64_t i = (uint64_t)blockIdx.x * kImplrBlock + threadIdx.x; i < words;
         i += (uint64_t)gridDim.x * kImplrBlock)
        c += (unsigned long long)__popc(bits[i]);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0 && c)
        __hip_atomic_fetch_add(&st->set_count, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// n* = grid - reached points: n when the order check passed, else the set bits.
__global__ void implr_finish_kernel(const ImplrState* st, uint64_t grid, uint64_t n, int force,
                                    int64_t* nstar_out) {
    if (threadIdx.x == 0) {
        const uint64_t reached = bitmap_needed(st, force) ? st->set_count : n;
        *nstar_out = (int64_t)(grid - reached);
    }
}

size_t implr_workspace_bytes(uint64_t grid) {
    const uint64_t words = (grid + 31) / 32;
    return kZeroBytes + 256 + (words * 4 + 255) / 256 * 256;
}

static unsigned blocks_for(uint64_t count, uint64_t per_block) {
    return (unsigned)((count + per_block - 1) / per_block);
}

hipError_t launch_implr(const ImplrLaunch& L, hipStream_t stream) {
    // Workspace: the shared zero region (untouched here), 256 bytes of state, then
    // the bitmap of the grid.
    ImplrState* st = (ImplrState*)((char*)L.ws + kZeroBytes);
    uint32_t* bits = (uint32_t*)((char*)L.ws + kZeroBytes + 256);
    const uint64_t words = (L.grid + 31) / 32;
    const double inv_n = 1.0 / (double)L.n;
    const uint32_t Q = L.n / L.zd, R = L.n % L.zd;
    const int force = L.bitmap ? 1 : 0;
    hipLaunchKernelGGL(implr_init_kernel, dim3(1), dim3(kWave), 0, stream, st);
    if (!L.bitmap)
        hipLaunchKernelGGL(implr_order_kernel, dim3(blocks_for(L.n, (uint64_t)kImplrBlock * kImplrOrderRun)),
                           dim3(kImplrBlock), 0, stream, L.d, L.n, inv_n, L.a, L.zd, L.nd, L.grid, st);
    const uint64_t clear_blocks = std::min<uint64_t>(kImplrGrid, (words + kImplrBlock - 1) / kImplrBlock);
    const uint64_t runs = ((uint64_t)L.n + kImplrRun - 1) / kImplrRun;
    const uint64_t mark_blocks = std::min<uint64_t>(kImplrGrid, (runs + kImplrBlock - 1) / kImplrBlock);
    hipLaunchKernelGGL(implr_clear_kernel, dim3((unsigned)clear_blocks), dim3(kImplrBlock), 0, stream, bits,
                       words, st, force);
    hipLaunchKernelGGL(implr_mark_kernel, dim3((unsigned)mark_blocks), dim3(kImplrBlock), 0, stream, L.d, L.n,
                       inv_n, L.a, L.zd, L.nd, Q, R, bits, st, force);
    hipLaunchKernelGGL(implr_count_kernel, dim3((unsigned)clear_blocks), dim3(kImplrBlock), 0, stream, bits,
                       words, st, force);
    hipLaunchKernelGGL(implr_finish_kernel, dim3(1), dim3(kWave), 0, stream, st, L.grid, (uint64_t)L.n, force,
                       L.nstar_out);
    return hipGetLastError();
}

hipError_t launch_implr_points(const ImplrPointsLaunch& L, hipStream_t stream) {
    if (L.count == 0) return hipSuccess;
    const dim3 grid(blocks_for(L.count, (uint64_t)kImplrWalkWaves * kImplrWavePoints));
    hipLaunchKernelGGL(implr_points_kernel, grid, dim3(kImplrBlock), 0, stream, L.d, L.n, 1.0 / (double)L.n, L.a,
                       L.zd, L.n / L.zd, L.n % L.zd, L.j0, L.count, L.ld, L.s_out);
    return hipGetLastError();
}

}  // namespace qmc
