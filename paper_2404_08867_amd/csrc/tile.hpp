// One tile of the plain rank-1 lattice rule: the device code shared by the
// single-problem kernel (lattice_sum.hip) and the batched kernel (batched.hip).
//
// A tile is B * M consecutive point indices (B threads per workgroup, a
// template parameter of every function here, kBlock by default); wave w owns
//   i = tile_base + w*64*M + lane + 64*m,   m = 0..M-1,
// and the loop runs over directions outside and over the thread's M points inside:
//   start:  k = (Kw_j + Lz_j[lane]) mod n,  Kw_j = (wave_base * z_j + shift_whole_j) mod n,
//                                           Lz_j[l] = (l * z_j) mod n,
//   step:   k <- (k + D_j) mod n,           D_j = (64 z_j) mod n           (eq. 2.1)
// with the per-direction tables built cooperatively in LDS, kDimChunk directions
// at a time.  One step is two 32-bit adds and a min.
#pragma once

#include <type_traits>

#include "common.hpp"
#include "families.hpp"

namespace qmc {

// Families with f(x) = f(1 - x) in every coordinate (F::kMirror): on an unshifted
// lattice their sum needs only the points i <= n/2 (finish_points).
template <class F, class = void>
struct mirror_family : std::false_type {};
template <class F>
struct mirror_family<F, std::void_t<decltype(F::kMirror)>> : std::bool_constant<F::kMirror> {};

// Families whose result is multiplied by the parameter after the d weights
// (F::kParamScale): p[d] scales the sum.
template <class F, class = void>
struct param_scaled : std::false_type {};
template <class F>
struct param_scaled<F, std::void_t<decltype(F::kParamScale)>> : std::bool_constant<F::kParamScale> {};

// Families whose single-precision form is valid only for some parameters
// (F::kGuarded): F::fp32_dim_ok decides per direction and F::block_ok on the sums of
// the block terms; a problem that fails either is evaluated by F::Fallback (same
// constants, and the same scale once the form's own block term ds1 is dropped).
template <class F, class = void>
struct guarded_family : std::false_type {
    using fallback_dim = char;
};
template <class F>
struct guarded_family<F, std::void_t<decltype(F::kGuarded)>> : std::bool_constant<F::kGuarded> {
    using fallback_dim = typename F::Fallback::Dim;
};

// What a guarded family's problem-wide test needs from a direction (F::GuardIn), kept in
// the registers of the wave-0 lane that loaded it during the setup.
template <class F, class = void>
struct guard_input_of {
    using type = char;
};
template <class F>
struct guard_input_of<F, std::void_t<typename F::GuardIn>> {
    using type = typename F::GuardIn;
};
template <class F>
using guard_in_t = typename guard_input_of<F>::type;

// A problem as seen by the device: lattice, shift and one parameter row.
struct ProblemView {
    int d;
    uint32_t n;
    double inv_n;
    double dn;
    const int64_t* z;
    const double* shift;  // may be null
    const double* p;      // parameter row
};

// inv_n is 1.0 / n rounded to double (the host passes it, so that no workgroup
// spends a divide on it).
__device__ __forceinline__ ProblemView make_view(int d, uint32_t n, double inv_n, const int64_t* z,
                                                 const double* shift, const double* p) {
    ProblemView v;
    v.d = d;
    v.n = n;
    v.dn = (double)n;
    v.inv_n = inv_n;
    v.z = z;
    v.shift = shift;
    v.p = p;
    return v;
}

// Fractional shift in index units: shift_j * n = whole + frac, whole in [0, n).
__device__ __forceinline__ void split_shift(const double* shift, int j, uint32_t n, uint32_t& whole,
                                            double& frac) {
    if (!shift) {
        whole = 0;
        frac = 0.0;
        return;
    }
    const double t = shift[j] * (double)n;
    const double w = floor(t);
    frac = t - w;
    const uint32_t wi = (uint32_t)w;
    whole = wi >= n ? wi - n : wi;
}

// B: threads per workgroup (a multiple of kWave).
template <class F, int B = kBlock>
struct TileShared {
    uint32_t lz[kDimChunk * kWave];   // [j][lane]
    uint32_t kw[kDimChunk * (B / kWave)];  // [j][wave]
    uint2 st[kDimChunk];              // (D_j, D_j - n)
    float2 stf[kDimChunk];            // the same as exact floats (used when n <= kFloatIndexMaxN)
    uint32_t sh[kDimChunk];           // whole part of the shift
    typename F::Dim c[kDimChunk];     // family constants
    // guarded families: the fallback's constants and whether the problem needs them
    typename guarded_family<F>::fallback_dim c2[guarded_family<F>::value ? kDimChunk : 1];
    int use_fallback;   // a direction fails the family's per-direction check
    int guard_fail;     // the problem fails the family's problem-wide check (guard_check)
    double guard_bias;  // the single-precision form's ds1 (guard_check)
};

// Workgroup constants of a problem: sums over all directions in a fixed order.
// Every thread receives init0 (initial accumulator), ds1 and ie (final scale).
template <class F, int B = kBlock>
__device__ __forceinline__ void block_constants(const ProblemView& v, double* red, double& init0,
                                                double& ds1, int& ie) {
    double ds0 = 0.0;
    ds1 = 0.0;
    ie = 0;
    if constexpr (F::kBlockTerms) {
        for (int j = threadIdx.x; j < v.d; j += B) {
            uint32_t whole;
            double frac;
            split_shift(v.shift, j, v.n, whole, frac);
            F::block_terms(v.p, v.d, j, v.inv_n, frac, ds0, ds1, ie);
        }
        block_sum3<B>(ds0, ds1, ie, red);
    }
    init0 = ds0 + F::extra(v.p);
}

// Lz_j[l] = (l z_j) mod n for directions [j0, j0 + dc), dc <= kDimChunk.
// l * z_j < 2^37, so the exact double-precision mulmod applies.  When a thread
// owns at most four rows (B >= 1024), thread (wave w, lane l) fills rows
// j = w, w + B / kWave, ... and issues all of its loads of z before the first is
// used, so the table costs one memory round trip; otherwise a plain strided
// loop keeps the register count (and the occupancy) of smaller workgroups.
template <class F, int B>
__device__ __forceinline__ void fill_lz(const ProblemView& v, TileShared<F, B>& s, int j0, int dc) {
    constexpr int kRows = kDimChunk / (B / kWave);
    if constexpr (kRows <= 4) {
        const int l = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
        // z_j < 2^31: its low 32-bit word (little-endian) is the value.
        const uint32_t* z32 = reinterpret_cast<const uint32_t*>(v.z + j0);
        uint32_t zr[kRows];
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            // Rows past dc load the last direction again: an unconditional,
            // in-bounds load lets every load issue before the first wait.
            const int j = min(wv + r * (B / kWave), dc - 1);
            zr[r] = z32[2 * j];
        }
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            const int j = wv + r * (B / kWave);
            if (j < dc) s.lz[j * kWave + l] = mulmod_small((uint32_t)l, zr[r], v.dn, v.inv_n);
        }
    } else {
        for (int e = threadIdx.x; e < dc * kWave; e += B) {
            const int j = e / kWave, l = e % kWave;
            s.lz[e] = mulmod_small((uint32_t)l, (uint32_t)v.z[j0 + j], v.dn, v.inv_n);
        }
    }
}

// Tables that do not depend on the tile for directions [j0, j0 + dc).
// 64 * z_j < 2^37, so the exact double-precision mulmod applies.
template <class F, int B>
__device__ __forceinline__ void fill_dims(const ProblemView& v, TileShared<F, B>& s, int j0, int dc) {
    const int tid = threadIdx.x;
    fill_lz<F, B>(v, s, j0, dc);
    for (int e = tid; e < dc; e += B) {
        const int j = j0 + e;
        uint32_t whole;
        double frac;
        split_shift(v.shift, j, v.n, whole, frac);
        const uint32_t st = mulmod_small((uint32_t)kWave, (uint32_t)v.z[j], v.dn, v.inv_n);
        s.st[e] = make_uint2(st, st - v.n);
        s.stf[e] = make_float2((float)st, (float)st - (float)v.n);
        s.sh[e] = whole;
        s.c[e] = F::dim(v.p, v.d, j, v.inv_n, frac);
    }
}

// Per-wave start residues of one tile (general 62-bit products).
template <class F, int M, int B>
__device__ __forceinline__ void fill_tile(const ProblemView& v, TileShared<F, B>& s, int j0, int dc,
                                          uint32_t tile_base) {
    for (int e = threadIdx.x; e < dc * (B / kWave); e += B) {
        const int j = e / (B / kWave), w = e % (B / kWave);
        const uint32_t b = (tile_base + (uint32_t)w * (kWave * M)) % v.n;
        s.kw[e] = addmod(mulmod((uint64_t)b, (uint64_t)v.z[j0 + j], v.n, v.inv_n), s.sh[j], v.n);
    }
}

// Accumulates directions [j0, j0 + dc) into the thread's M point states, from
// the direction tables (fill_dims) and the tile's start residues (fill_tile) in s.
// FI (n <= kFloatIndexMaxN): the thread's M indices of a direction are stepped as
// exact floats (stepmod_f: two FP32 adds and a minimum, which gfx950 issues at
// about twice the rate of the integer step's two 32-bit adds and minimum), and the
// family takes the float (a float-to-double conversion where it needs a double).
// `dims` holds F's constants of the chunk's directions (the tables' own c, or the
// fallback constants c2 of a guarded family).
// M0 > 0: the accumulators hold the thread's points M0 .. M0 + M - 1 (each index
// is first stepped M0 times).
template <class F, int M, int B, bool FI = false, int M0 = 0, class S>
__device__ __forceinline__ void chunk_points(typename F::Acc (&acc)[M], const S& s,
                                             const typename F::Dim* dims, int j0, int dc, uint32_t n) {
    using Dim = typename F::Dim;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    for (int jj = 0; jj < dc; ++jj) {
        uint32_t k = addmod(s.kw[jj * (B / kWave) + wv], s.lz[jj * kWave + lane], n);
        const Dim c = dims[jj];
        if constexpr (M0 > 0) {
            const uint2 stp = s.st[jj];
#pragma unroll
            for (int m = 0; m < M0; ++m) k = stepmod(k, stp.x, stp.y);
        }
        if constexpr (FI) {
            const float2 stp = s.stf[jj];
            float kf = (float)k;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                F::step(acc[m], kf, c);
                kf = stepmod_f(kf, stp.x, stp.y);
            }
        } else {
            const uint2 stp = s.st[jj];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                F::step(acc[m], k, c);
                k = stepmod(k, stp.x, stp.y);
            }
        }
        if constexpr (F::kRenorm > 0) {
            if ((j0 + jj + 1) % F::kRenorm == 0) {
#pragma unroll
                for (int m = 0; m < M; ++m) F::renorm(acc[m]);
            }
        }
    }
}

// The thread's sum of f / scale over its M points (points >= n contribute zero).
// MIRROR (unshifted lattices, integrands with f(x) = f(1 - x) in every coordinate):
// point n - i is the mirror image of point i, so only i <= n/2 is evaluated, with
// weight 2 except for i = 0 and, for even n, i = n/2 (their own mirrors).
// MT is the thread's number of points in the tile and M0 the first of them that acc
// holds (chunk_points with the same M0).
template <class F, int M, bool MIRROR = false, int MT = M, int M0 = 0>
__device__ __forceinline__ double finish_points(const typename F::Acc (&acc)[M], uint32_t tile_base,
                                                uint32_t n) {
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const uint32_t i0 = tile_base + (uint32_t)wv * (kWave * MT) + (uint32_t)(kWave * M0) + (uint32_t)lane;
    double t = 0.0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const double f = F::finish(acc[m]);
        const uint32_t i = i0 + (uint32_t)(kWave * m);
        if constexpr (MIRROR) {
            const double w = (i == 0 || 2 * i == n) ? 1.0 : 2.0;
            t += (i <= n / 2) ? w * f : 0.0;
        } else {
            t += (i < n) ? f : 0.0;
        }
    }
    return t;
}

// The thread's sum of f / scale over its M points of the tile, any d: the
// tables are rebuilt chunk by chunk.  Begins with a barrier; the caller may
// reuse s afterwards only after another barrier.
template <class F, int M, int B, bool FI = false, bool MIRROR = false>
__device__ __forceinline__ double tile_points(const ProblemView& v, TileShared<F, B>& s,
                                              uint32_t tile_base, double init0) {
    typename F::Acc acc[M];
#pragma unroll
    for (int m = 0; m < M; ++m) acc[m] = F::init(init0);
    for (int j0 = 0; j0 < v.d; j0 += kDimChunk) {
        const int dc = min(kDimChunk, v.d - j0);
        __syncthreads();  // every read of the previous tables is done
        fill_dims<F, B>(v, s, j0, dc);
        __syncthreads();
        fill_tile<F, M, B>(v, s, j0, dc, tile_base);
        __syncthreads();
        chunk_points<F, M, B, FI>(acc, s, s.c, j0, dc, v.n);
    }
    return finish_points<F, M, MIRROR>(acc, tile_base, v.n);
}

// ---------------------------------------------------------------------------
// Problems with d <= kDimChunk keep one set of direction tables for every tile.
// setup_one_chunk builds all of them in one pass with one barrier: the index
// table Lz by every thread, the direction constants and the workgroup sums by
// wave 0 (lane j owns direction j), and the start residues of the workgroup's
// first tile (at first_base) by the other waves.
// ---------------------------------------------------------------------------
template <class F, int M, int B>
__device__ __forceinline__ void setup_one_chunk(const ProblemView& v, TileShared<F, B>& s, double* red,
                                                uint32_t first_base, double& init0, double& ds1,
                                                int& ie, guard_in_t<F>& gin) {
    const int tid = threadIdx.x, d = v.d;
    fill_lz<F, B>(v, s, 0, d);
    if (tid < kWave) {
        double t0 = 0.0, t1 = 0.0;
        int te = 0;
        bool bad = false;  // a direction the guarded family's FP32 form cannot take
        (void)bad;

        if (tid < d) {
            const int j = tid;
            uint32_t whole;
            double frac;
            split_shift(v.shift, j, v.n, whole, frac);
            if constexpr (F::kBlockTerms) F::block_terms(v.p, d, j, v.inv_n, frac, t0, t1, te);
            const uint32_t st = mulmod_small((uint32_t)kWave, (uint32_t)v.z[j], v.dn, v.inv_n);
            s.st[j] = make_uint2(st, st - v.n);
            s.stf[j] = make_float2((float)st, (float)st - (float)v.n);
            s.sh[j] = whole;
            s.c[j] = F::dim(v.p, d, j, v.inv_n, frac);
            if constexpr (guarded_family<F>::value) {
                s.c2[j] = F::Fallback::dim(v.p, d, j, v.inv_n, frac);
                bad = !F::fp32_dim_ok(v.p, d, j);
                gin = F::guard_input(v.p, d, j, v.inv_n, frac);
            }
        }
        if constexpr (guarded_family<F>::value) {
            const bool any_bad = __builtin_amdgcn_ballot_w64(bad) != 0;
            if (tid == 0) s.use_fallback = any_bad ? 1 : 0;
        }
        if constexpr (F::kBlockTerms) {
            const double x = wave_total(t0), y = wave_total(t1), w = wave_total((double)te);
            if (tid == kWaveTotalLane) {
                red[0] = x;
                red[1] = y;
                red[2] = w;
            }
        }
    } else {
        for (int e = tid - kWave; e < d * (B / kWave); e += B - kWave) {
            const int j = e / (B / kWave), w = e % (B / kWave);
            uint32_t whole;
            double frac;
            split_shift(v.shift, j, v.n, whole, frac);
            const uint32_t b = (first_base + (uint32_t)w * (kWave * M)) % v.n;
            s.kw[e] = addmod(mulmod((uint64_t)b, (uint64_t)v.z[j], v.n, v.inv_n), whole, v.n);
        }
    }
    __syncthreads();
    double ds0 = 0.0;
    ds1 = 0.0;
    ie = 0;
    if constexpr (F::kBlockTerms) {
        ds0 = red[0];
        ds1 = red[1];
        ie = (int)red[2];
    }
    init0 = ds0 + F::extra(v.p);
}

// Guarded families, problem-wide part of the test (F::guard_terms summed over the
// directions, F::block_ok on the sums): run by wave 0 right after setup_one_chunk,
// while the other waves start on their points, so that it adds nothing to the setup.
// The tiles take the single-precision form unless a direction failed (use_fallback);
// after the workgroup sum, guard_redo tells whether to redo them with the fallback
// (redo_tiles) because the problem-wide test failed.
template <class F, int B>
__device__ __forceinline__ void guard_check(const ProblemView& v, TileShared<F, B>& s,
                                            const guard_in_t<F>& gin) {
    if constexpr (guarded_family<F>::value) {
        if (threadIdx.x < kWave) {
            const int j = threadIdx.x;
            double g0 = 0.0, g1 = 0.0;
            if (j < v.d) F::guard_terms(gin, g0, g1);
            const double x = wave_total(g0), y = wave_total(g1);
            if (j == kWaveTotalLane) {
                s.guard_fail = F::block_ok(x, y, v.n) ? 0 : 1;
                s.guard_bias = y;
            }
        }
    }
}

// Points M0 .. M0 + M - 1 of the thread's MT points of a tile, with the fallback
// constants c2 of a guarded family (F is the fallback).
template <class F, int M, int MT, int M0, int B, bool FI, bool MIRROR, class S>
__device__ __forceinline__ double fallback_points(const ProblemView& v, const S& s, uint32_t tile_base,
                                                  double init0) {
    typename F::Acc acc[M];
#pragma unroll
    for (int m = 0; m < M; ++m) acc[m] = F::init(init0);
    chunk_points<F, M, B, FI, M0>(acc, s, s.c2, 0, v.d, v.n);
    return finish_points<F, M, MIRROR, MT, M0>(acc, tile_base, v.n);
}

// One tile of a problem set up by setup_one_chunk.  With `kw_ready` the start
// residues of this tile are already in s; otherwise they are rebuilt between two
// barriers.  The caller may overwrite s afterwards only after a barrier.
template <class F, int M, int B, bool FI = false, bool MIRROR = false>
__device__ __forceinline__ double tile_points_one_chunk(const ProblemView& v, TileShared<F, B>& s,
                                                        uint32_t tile_base, double init0,
                                                        bool kw_ready, bool force_fallback = false) {
    if (!kw_ready) {
        __syncthreads();  // every read of the previous tile's residues is done
        fill_tile<F, M, B>(v, s, 0, v.d, tile_base);
        __syncthreads();
    }
    if constexpr (guarded_family<F>::value) {
        if (s.use_fallback || force_fallback) {
            // The double-precision factors take twice the registers of the single-
            // precision ones; for M >= 8 they run over the thread's points in two
            // halves, so that this rarely taken branch does not set the register
            // count (and the occupancy) of the whole kernel.
            using FB = typename F::Fallback;
            if constexpr (M >= 8) {
                return fallback_points<FB, M / 2, M, 0, B, FI, MIRROR>(v, s, tile_base, init0) +
                       fallback_points<FB, M / 2, M, M / 2, B, FI, MIRROR>(v, s, tile_base, init0);
            } else {
                return fallback_points<FB, M, M, 0, B, FI, MIRROR>(v, s, tile_base, init0);
            }
        }
    }
    typename F::Acc acc[M];
#pragma unroll
    for (int m = 0; m < M; ++m) acc[m] = F::init(init0);
    chunk_points<F, M, B, FI>(acc, s, s.c, 0, v.d, v.n);
    return finish_points<F, M, MIRROR>(acc, tile_base, v.n);
}

// After the workgroup sum of a problem's tiles (setup_one_chunk, guard_check): that
// sum's barrier has made guard_check's results visible.  Sets ds1 for F::scale (the
// single-precision form's bias correction, none for the fallback) and returns whether
// the tiles must be redone with the fallback (the problem-wide test failed); the same
// answer in every thread of the workgroup.
template <class F, int B>
__device__ __forceinline__ bool guard_redo(const TileShared<F, B>& s, double& ds1) {
    if constexpr (guarded_family<F>::value) {
        const bool fb = s.use_fallback != 0, redo = !fb && s.guard_fail != 0;
        ds1 = (fb || redo) ? 0.0 : s.guard_bias;
        return redo;
    } else {
        (void)s;
        (void)ds1;
        return false;
    }
}

// The workgroup's tiles first, first + stride, ... < tiles with the fallback (after
// guard_redo).  Begins with a barrier.
template <class F, int M, int B, bool FI, bool MIRROR>
__device__ __forceinline__ double redo_tiles(const ProblemView& v, TileShared<F, B>& s, uint32_t first,
                                             uint32_t stride, uint32_t tiles, double init0) {
    constexpr uint32_t kTile = B * M;
    double t = 0.0;
    for (uint32_t tile = first; tile < tiles; tile += stride)
        t += tile_points_one_chunk<F, M, B, FI, MIRROR>(v, s, tile * kTile, init0, false, true);
    return t;
}

}  // namespace qmc
