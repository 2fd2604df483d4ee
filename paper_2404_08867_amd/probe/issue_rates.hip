// Issue-rate probe behind the benchmark's ALU roofline: how many lane-operations per
// second gfx950 completes for each instruction type on the lattice path, alone and
// mixed with other types.  Not part of libqmc.so; built into libqmc_probe.so and
// called by bench.py (--workload rates).
//
// Every thread runs kChains independent dependency chains (enough to cover the
// pipeline latency), each advanced by one step of the measured kind, kUnroll steps
// per loop iteration.  An empty asm statement with a "+v" operand after an integer
// step keeps the compiler from folding a chain of integer operations (a chain of adds
// into a multiply, a repeated minimum into one); it emits no instruction.
// Floating-point chains cannot be folded and need none.  The transcendentals are the
// compiler builtins that map to v_exp_f32, v_rcp_f32, v_cos_f32 and v_log_f32.  At
// the end each thread stores one value derived from every chain, so no chain is dead.
// Loop overhead (one scalar add, compare and branch per kUnroll * kChains steps) is
// not counted.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kChains = 8;
constexpr int kUnroll = 16;
constexpr int kBlock = 256;

#define KEEP(x) asm volatile("" : "+v"(x))

enum Kind : int {
    kU32Add = 0,       // v_add_u32
    kIndexStep = 1,    // the integer modular step min(k + st, k + st - n): v_add_u32 x2, v_min_u32
    kF32Fma = 2,       // v_fma_f32 (non-packed: packed-FP32 forms are disabled)
    kF64Fma = 3,       // v_fma_f64
    kF64Add = 4,       // v_add_f64
    kCvtF64U32 = 5,    // v_cvt_f64_u32
    kCvtF32U32 = 6,    // v_cvt_f32_u32
    kExp2F32 = 7,      // v_exp_f32
    kRcpF32 = 8,       // v_rcp_f32
    kCosF32 = 9,       // v_cos_f32
    kLog2F32 = 10,     // v_log_f32
    kF64FmaExp = 11,   // 4 v_fma_f64 and 1 v_exp_f32 per step (5 ops)
    kU32F64Fma = 12,   // v_add_u32 and v_fma_f64 per step (2 ops)
    kPointDim = 13,    // exp-sum work of one point and direction (5 ops): the integer
                       // index step, v_cvt_f64_u32 and the argument's v_fma_f64
    kU32Min = 14,      // v_min_u32
    kU32Sub = 15,      // v_sub_u32
    kCmpSel = 16,      // v_sub_u32, v_cmp_gt_u32 and v_cndmask_b32 per step (3 ops)
    kF32Add = 17,      // v_add_f32
    kF32Mul = 18,      // v_mul_f32
    kFloatStep = 19,   // the exact-float index step: v_add_f32 x2, v_min_u32 on the patterns
    kU32F32Fma = 20,   // v_add_u32 and v_fma_f32 per step (2 ops)
    kF32F64Fma = 21,   // v_fma_f32 and v_fma_f64 per step (2 ops)
    kF32FmaExp = 22,   // 4 v_fma_f32 and 1 v_exp_f32 per step (5 ops)
    kPeakDim = 23,     // product-peak work of one point and direction in FP32 (6 ops): the
                       // exact-float index step, y = k b + g, y^2 + h, product
    kCvtF64F32 = 24,   // v_cvt_f64_f32
    kPointDimF = 25,   // exp-sum work of one point and direction with the exact-float step
                       // (5 ops): float step, v_cvt_f64_f32, v_fma_f64
    kGaussDim = 26,    // Gaussian (FP64) work of one point and direction (6 ops): integer
                       // step, v_cvt_f64_u32, y = k b + g, s += y y
    kGaussDimF = 27,   // the same with the exact-float step and v_cvt_f64_f32 (6 ops)
    kF64Mul = 28,      // v_mul_f64
    kHorner = 29,      // the MDI-LR node step h = r h + 1, r = r q (v_fma_f64, v_mul_f64)
    kHorner2 = 30,     // the same step in only two of the chains (two directions' sums, as
                       // the MDI-LR kernel runs them per lane): latency exposed
    kNumKinds = 31
};

// Lane-operations one step of one chain performs (on average over the chains).
__host__ __device__ constexpr double ops_per_step(int kind) {
    switch (kind) {
        case kHorner: return 2;
        case kHorner2: return 2.0 * 2 / kChains;
        case kIndexStep: case kFloatStep: return 3;
        case kF64FmaExp: case kPointDim: case kF32FmaExp: case kPointDimF: return 5;
        case kGaussDim: case kGaussDimF: return 6;
        case kU32F64Fma: case kU32F32Fma: case kF32F64Fma: return 2;
        case kCmpSel: return 3;
        case kPeakDim: return 6;
        default: return 1;
    }
}

template <int K>
__global__ __launch_bounds__(kBlock) void rate_kernel(int iters, uint32_t seed, double* out) {
    const uint32_t tid = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t s = seed ^ (tid * 2654435761u);
    const uint32_t n = 1000003u, dlt = (s & 0xffffu) + 1u, dm = dlt - n;
    const float a = 0.999f + (float)(s & 15) * 1e-6f, b = 1e-3f;
    const double ad = 0.999 + (double)(s & 15) * 1e-9, bd = 1e-3;
    uint32_t r[kChains];
    float x[kChains];
    double y[kChains], h[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        r[c] = (s >> (c & 15)) % n;
        x[c] = (float)r[c];  // an exact integer below 2^24 for the float step
        y[c] = 0.25 + (double)c * 0.01 + (double)(s & 7) * 1e-3;
        h[c] = 1.0;
    }
    const float stf = (float)dlt, stmf = (float)dlt - (float)n;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) {
                if constexpr (K == kU32Add) {
                    r[c] = r[c] + dlt;
                    KEEP(r[c]);
                } else if constexpr (K == kIndexStep) {
                    const uint32_t t1 = r[c] + dlt, t2 = r[c] + dm;
                    r[c] = t1 < t2 ? t1 : t2;
                } else if constexpr (K == kF32Fma) {
                    x[c] = __builtin_fmaf(x[c], a, b);
                } else if constexpr (K == kF64Fma) {
                    y[c] = __builtin_fma(y[c], ad, bd);
                } else if constexpr (K == kF64Add) {
                    y[c] = y[c] + bd;
                } else if constexpr (K == kCvtF64U32) {
                    // the chain runs through the result's bits (a free reinterpretation)
                    y[c] = (double)r[c];
                    r[c] = (uint32_t)__double_as_longlong(y[c]);
                } else if constexpr (K == kCvtF32U32) {
                    x[c] = (float)r[c];
                    r[c] = __float_as_uint(x[c]);
                } else if constexpr (K == kExp2F32) {
                    x[c] = __builtin_amdgcn_exp2f(x[c]);
                } else if constexpr (K == kRcpF32) {
                    x[c] = __builtin_amdgcn_rcpf(x[c]);
                } else if constexpr (K == kCosF32) {
                    x[c] = __builtin_amdgcn_cosf(x[c]);
                } else if constexpr (K == kLog2F32) {
                    x[c] = __builtin_amdgcn_logf(x[c]);
                } else if constexpr (K == kF64FmaExp) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) y[c] = __builtin_fma(y[c], ad, bd);
                    x[c] = __builtin_amdgcn_exp2f(x[c]);
                } else if constexpr (K == kU32F64Fma) {
                    r[c] = r[c] + dlt;
                    KEEP(r[c]);
                    y[c] = __builtin_fma(y[c], ad, bd);
                } else if constexpr (K == kPointDim) {
                    const uint32_t t1 = r[c] + dlt, t2 = r[c] + dm;
                    r[c] = t1 < t2 ? t1 : t2;
                    y[c] = __builtin_fma((double)r[c], bd, y[c]);
                } else if constexpr (K == kU32Min) {
                    r[c] = r[c] < dm ? r[c] : dm;
                    KEEP(r[c]);
                } else if constexpr (K == kU32Sub) {
                    r[c] = r[c] - dlt;
                    KEEP(r[c]);
                } else if constexpr (K == kCmpSel) {
                    r[c] = r[c] > dm ? r[c] - dlt : dlt;
                    KEEP(r[c]);
                } else if constexpr (K == kF32Add) {
                    x[c] = x[c] + b;
                } else if constexpr (K == kF32Mul) {
                    x[c] = x[c] * a;
                } else if constexpr (K == kFloatStep) {
                    const uint32_t p1 = __float_as_uint(x[c] + stf), p2 = __float_as_uint(x[c] + stmf);
                    x[c] = __uint_as_float(p1 < p2 ? p1 : p2);
                } else if constexpr (K == kU32F32Fma) {
                    r[c] = r[c] + dlt;
                    KEEP(r[c]);
                    x[c] = __builtin_fmaf(x[c], a, b);
                } else if constexpr (K == kF32F64Fma) {
                    x[c] = __builtin_fmaf(x[c], a, b);
                    y[c] = __builtin_fma(y[c], ad, bd);
                } else if constexpr (K == kF32FmaExp) {
                    float w = x[c];
#pragma unroll
                    for (int q = 0; q < 4; ++q) w = __builtin_fmaf(w, a, b);
                    x[c] = w;
                    // the exponential's chain lives in r's bits (free reinterpretations)
                    r[c] = __float_as_uint(__builtin_amdgcn_exp2f(__uint_as_float(r[c])));
                } else if constexpr (K == kPeakDim) {
                    // chain c: the float index k (x), and a product p kept in y's low word
                    const uint32_t p1 = __float_as_uint(x[c] + stf), p2 = __float_as_uint(x[c] + stmf);
                    x[c] = __uint_as_float(p1 < p2 ? p1 : p2);
                    const float yy = __builtin_fmaf(x[c], 1e-6f, -0.5f);
                    const float g = __builtin_fmaf(yy, yy, 0.3f);
                    const float pr = __uint_as_float((uint32_t)__double_as_longlong(y[c])) * g;
                    y[c] = __longlong_as_double((long long)__float_as_uint(pr));
                } else if constexpr (K == kCvtF64F32) {
                    y[c] = (double)x[c];
                    x[c] = __uint_as_float((uint32_t)__double_as_longlong(y[c]));
                } else if constexpr (K == kPointDimF) {
                    const uint32_t p1 = __float_as_uint(x[c] + stf), p2 = __float_as_uint(x[c] + stmf);
                    x[c] = __uint_as_float(p1 < p2 ? p1 : p2);
                    y[c] = __builtin_fma((double)x[c], bd, y[c]);
                } else if constexpr (K == kGaussDim) {
                    const uint32_t t1 = r[c] + dlt, t2 = r[c] + dm;
                    r[c] = t1 < t2 ? t1 : t2;
                    const double g = __builtin_fma((double)r[c], bd, -0.5);
                    y[c] = __builtin_fma(g, g, y[c]);
                } else if constexpr (K == kGaussDimF) {
                    const uint32_t p1 = __float_as_uint(x[c] + stf), p2 = __float_as_uint(x[c] + stmf);
                    x[c] = __uint_as_float(p1 < p2 ? p1 : p2);
                    const double g = __builtin_fma((double)x[c], bd, -0.5);
                    y[c] = __builtin_fma(g, g, y[c]);
                } else if constexpr (K == kF64Mul) {
                    y[c] = y[c] * ad;
                } else if constexpr (K == kHorner || K == kHorner2) {
                    if (K == kHorner || c < 2) {
                        h[c] = __builtin_fma(y[c], h[c], 1.0);
                        y[c] = y[c] * ad;
                    }
                }
            }
        }
    }
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc += (double)r[c] + (double)x[c] + y[c] + h[c];
    out[tid] = acc;
}

template <int K>
hipError_t launch_kind(int blocks, int iters, double* out, hipStream_t stream) {
    hipLaunchKernelGGL(rate_kernel<K>, dim3(blocks), dim3(kBlock), 0, stream, iters, 1u, out);
    return hipGetLastError();
}

template <int K>
hipError_t launch_from(int kind, int blocks, int iters, double* out, hipStream_t stream) {
    if constexpr (K >= kNumKinds) {
        return hipErrorInvalidValue;
    } else {
        if (kind == K) return launch_kind<K>(blocks, iters, out, stream);
        return launch_from<K + 1>(kind, blocks, iters, out, stream);
    }
}

}  // namespace

extern "C" {

// Number of probe kinds.
int qmc_probe_kinds(void) { return kNumKinds; }

// Lane-operations of one probe launch of `kind` with `blocks` workgroups of 256
// threads and `iters` loop iterations (-1 for bad arguments).
double qmc_probe_lane_ops(int kind, int blocks, int iters) {
    if (kind < 0 || kind >= kNumKinds || blocks < 1 || iters < 1) return -1.0;
    return (double)blocks * kBlock * (double)iters * kUnroll * kChains * ops_per_step(kind);
}

// Launches one probe of `kind` on `stream`; `out` is a device array of blocks * 256
// doubles.  Returns 0, -1 for bad arguments, or the HIP error code.
int qmc_probe_launch(int kind, int blocks, int iters, double* out, void* stream) {
    if (kind < 0 || kind >= kNumKinds || blocks < 1 || blocks > (1 << 20) || iters < 1 || !out) return -1;
    const hipError_t e = launch_from<0>(kind, blocks, iters, out, (hipStream_t)stream);
    return e == hipSuccess ? 0 : (int)e;
}

}  // extern "C"
