// MDI-LR: the improved (tensor-product) lattice rule evaluated by dimension
// sweeps (Algorithm 2 driving Algorithm 1 with m = 1; eq. 2.14c).
//
// For a product-form integrand g(y) = C prod_k phi_k(y_k) each sweep step sums
// the first remaining coordinate out of the symbolic product with the rule's
// weights 1/N_k, which multiplies the coefficient C by
//   M_k = (1/N_k) sum_{t=0}^{N_k-1} phi_k((t + 1/2) / N_k),
// so Qhat = C_0 prod_k M_k (C_0 = 1, or e^{2 pi i u} for the oscillatory family,
// whose factors e^{i c_k y} are complex).  The d sweeps are independent of one
// another, so a workgroup evaluates the M_k of G parameter sets in parallel --
// one (set, direction) pair per thread, N_k nodes each -- keeps them in LDS, and
// then multiplies each set's d factors in direction order with exact
// power-of-two renormalisation (no overflow or underflow of the running product
// for d in the thousands).
#include "common.hpp"
#include "families.hpp"
#include "kernels.hpp"

namespace qmc {

struct MdiArgs {
    int d;
    const int32_t* N;
    const double* params;
    int P;
    int nsets;
    int G;  // sets per workgroup
    double* q_out;
};

// Sum over t = 0..Nk-1 of 2^{s y_t^2}, y_t = A t + B, s = -1 (a Gaussian) or +1 (a
// growing factor of the signed quadratic), by the exact recurrence on equispaced
// nodes: phi_{t+1} = phi_t r_t and r_{t+1} = r_t q with r_t = 2^{s A (2 y_t + A)},
// q = 2^{2 s A^2} -- two FP64 multiplies and one add per node.  phi and r are
// recomputed with exp2 at every S-th node, which bounds the compounded rounding of a
// run to S^2/2 units in the last place: S = 8 for QMC_FP64 (< 1e-15 per factor, so
// that a thousand identical directions stay within 1e-12), 64 for
// QMC_FP32_COMPENSATED (one run for N = 64).  The recurrence is used only while
// every node value, every ratio and q stay within 2^-1000..2^1000 (max y^2 over the
// nodes, taken at an end point, and 2 A^2 at most 1000), so no intermediate value
// underflows or overflows; otherwise each node is evaluated directly (FP32: FP64
// argument, split FP32 exp2).
template <bool FP32>
__device__ __forceinline__ double quad_node_sum(double A, double B, int Nk, double s) {
    constexpr int kSeed = FP32 ? 64 : 8;
    const double y_last = fma((double)(Nk - 1), A, B);
    double sr = 0.0;
    if (fmax(fmax(B * B, y_last * y_last), 2.0 * A * A) <= 1000.0) {
        const double q = exp2(2.0 * s * A * A);
        for (int t0 = 0; t0 < Nk; t0 += kSeed) {
            const double y = fma((double)t0, A, B);
            double f = exp2(s * y * y), r = exp2(s * A * fma(2.0, y, A));
            const int n1 = min(kSeed, Nk - t0);
            sr += f;
#pragma unroll 4
            for (int t = 1; t < n1; ++t) {
                f *= r;
                r *= q;
                sr += f;
            }
        }
    } else if constexpr (FP32) {
        for (int t = 0; t < Nk; ++t) {
            const double y = fma((double)t, A, B);
            sr += exp2_split_f32(s * y * y);
        }
    } else {
        for (int t = 0; t < Nk; ++t) {
            const double y = fma((double)t, A, B);
            sr += exp2(s * y * y);
        }
    }
    return sr;
}

// One direction's weighted node sum.  FP32 evaluates the factor in single
// precision (argument, exp2 / reciprocal / cos-sin) and accumulates in double.
template <int FAM, bool FP32>
__device__ __forceinline__ void direction_sum(const double* p, int d, int k, int Nk, double& re,
                                              double& im) {
    const double invN = 1.0 / (double)Nk;
    double sr = 0.0, si = 0.0;
    if constexpr (FAM == kExpSum) {
        // phi = 2^{c log2e (t + 1/2)/N} = 2^{A t + B}: a geometric sequence, phi_{t+1} =
        // phi_t 2^A, one FP64 multiply and one add per node in both precisions; phi is
        // reseeded with exp2 every 64 nodes (the rounding of a run grows linearly).
        const double c = p[k] * kLog2e;
        const double A = c * invN, B = 0.5 * c * invN;
        const double R = exp2(A);
        for (int t0 = 0; t0 < Nk; t0 += 64) {
            double f = exp2(fma((double)t0, A, B));
            const int n1 = min(64, Nk - t0);
            sr += f;
#pragma unroll 4
            for (int t = 1; t < n1; ++t) {
                f *= R;
                sr += f;
            }
        }
    } else if constexpr (FAM == kGaussian) {
        // phi = 2^{-y^2}, y = c sqrt(log2 e) ((t + 1/2)/N - w) = A t + B
        const double c = p[k] * kSqrtLog2e, w = p[d + k];
        const double A = c * invN, B = c * fma(0.5, invN, -w);
        sr = quad_node_sum<FP32>(A, B, Nk, -1.0);
    } else if constexpr (FAM == kExpQuadratic) {
        // phi = 2^{s y^2}, y = sqrt(|c| log2 e) ((t + 1/2)/N - w) = A t + B, s = sign(c)
        const double cq = p[k], w = p[d + k];
        const double m = sqrt(fabs(cq) * kLog2e);
        const double A = m * invN, B = m * fma(0.5, invN, -w);
        sr = quad_node_sum<FP32>(A, B, Nk, cq < 0.0 ? -1.0 : 1.0);
    } else if constexpr (FAM == kProductPeak) {
        // phi = 1 / (c^-2 + y^2), y = (t + 1/2)/N - w = A t + B
        const double c = p[k], w = p[d + k];
        const double g = 1.0 / (c * c), A = invN, B = fma(0.5, invN, -w);
        // v = g + y^2 lies in [g, g + max(B^2, y_last^2)] (y^2 is largest at an end node)
        const double y_last = fma((double)(Nk - 1), A, B);
        const bool f32_range = g >= 1e-36 && g + fmax(B * B, y_last * y_last) <= 1e36;
        if (FP32 && f32_range) {
            // FP32 reciprocal refined by one Newton step in FP64 (relative error ~1e-15):
            // an FP32 factor's rounding would repeat in every direction with the same
            // parameters and grow linearly in d (3.4e-6 at d = 1000 for Table 2-3).  Only
            // where every denominator is a normal FP32 number.
            double td = 0.0;
#pragma unroll 4
            for (int t = 0; t < Nk; ++t, td += 1.0) {
                const double y = fma(td, A, B), v = fma(y, y, g);
                const double r = (double)__builtin_amdgcn_rcpf((float)v);
                sr += fma(r, fma(-v, r, 1.0), r);
            }
        } else {
            for (int t = 0; t < Nk; ++t) {
                const double y = fma((double)t, A, B);
                sr += 1.0 / fma(y, y, g);
            }
        }
    } else {  // kOscillatory: phi = e^{i c y}, angle in turns a = c/(2 pi) y = A t + B
        const double c = p[1 + k] * kInv2Pi;
        const double A = c * invN, B = 0.5 * c * invN;
        if constexpr (FP32) {
            // The few nodes per direction do not average the hardware sin/cos error
            // away, so the factor uses the correctly reduced single-precision sincospi.
            for (int t = 0; t < Nk; ++t) {
                const double a = fma((double)t, A, B);
                const float fr = (float)(a - rint(a));
                float s, co;
                sincospif(2.0f * fr, &s, &co);
                sr += (double)co;
                si += (double)s;
            }
        } else {
            for (int t = 0; t < Nk; ++t) {
                const double a = fma((double)t, A, B);
                const double fr = a - rint(a);
                double s, co;
                sincospi(2.0 * fr, &s, &co);
                sr += co;
                si += s;
            }
        }
    }
    re = sr * invN;
    im = si * invN;
}

template <int FAM, bool FP32>
__global__ __launch_bounds__(kBlock) void mdi_lr_kernel(const MdiArgs a) {
    extern __shared__ double s_m[];  // [G*d] real parts, then [G*d] imaginary parts (oscillatory)
    constexpr bool kComplex = FAM == kOscillatory;
    const int set0 = blockIdx.x * a.G;
    const int g_here = min(a.G, a.nsets - set0);
    const int pairs = g_here * a.d;
    double* s_im = s_m + (size_t)a.G * a.d;

    for (int q = threadIdx.x; q < pairs; q += kBlock) {
        const int sl = q / a.d, k = q % a.d;
        const double* p = a.params + (size_t)(set0 + sl) * a.P;
        double re, im;
        // N_k in [1, 2^20] is the caller's contract; clamp so that a bad value
        // cannot turn into an unbounded loop.
        const int Nk = min(max(a.N[k], 1), 1 << 20);
        direction_sum<FAM, FP32>(p, a.d, k, Nk, re, im);
        s_m[q] = re;
        if constexpr (kComplex) s_im[q] = im;
    }
    __syncthreads();

    // Product over directions in order: the coefficient of the symbolic function
    // after each sweep step, kept as mantissa pair times 2^E.
    for (int sl = threadIdx.x; sl < g_here; sl += kBlock) {
        const double* p = a.params + (size_t)(set0 + sl) * a.P;
        double cr = 1.0, ci = 0.0;
        int E = 0;
        if constexpr (kComplex) sincospi(2.0 * p[0], &ci, &cr);
        for (int k = 0; k < a.d; ++k) {
            const double mr = s_m[sl * a.d + k];
            double nr, ni = 0.0;
            if constexpr (kComplex) {
                const double mi = s_im[sl * a.d + k];
                nr = cr * mr - ci * mi;
                ni = cr * mi + ci * mr;
            } else {
                nr = cr * mr;
            }
            const double big = kComplex ? fmax(fabs(nr), fabs(ni)) : fabs(nr);
            if (big > 0.0 && big < INFINITY) {
                const int e = __builtin_amdgcn_frexp_exp(big);
                nr = ldexp(nr, -e);
                ni = ldexp(ni, -e);
                E += e;
            }
            cr = nr;
            ci = ni;
        }
        a.q_out[set0 + sl] = ldexp(cr, E);
    }
}

template <int FAM, bool FP32>
static hipError_t launch_mdi_t(const MdiLaunch& L, hipStream_t stream) {
    MdiArgs a;
    a.d = L.d;
    a.N = L.N;
    a.params = L.params;
    a.P = L.P;
    a.nsets = L.nsets;
    // About 4096 (set, direction) pairs per workgroup (16 per thread); 32 KB of LDS.
    int G = (FAM == kOscillatory ? 2048 : 4096) / L.d;
    if (G < 1) G = 1;
    if (G > L.nsets) G = L.nsets;
    a.G = G;
    a.q_out = L.q_out;
    const size_t lds = (size_t)G * L.d * sizeof(double) * (FAM == kOscillatory ? 2 : 1);
    const unsigned grid = (unsigned)((L.nsets + G - 1) / G);
    hipLaunchKernelGGL((mdi_lr_kernel<FAM, FP32>), dim3(grid), dim3(kBlock), lds, stream, a);
    return hipGetLastError();
}

hipError_t launch_mdi_lr(const MdiLaunch& L, hipStream_t stream) {
    switch (L.family * 2 + (L.fp32 ? 1 : 0)) {
        case kExpSum * 2: return launch_mdi_t<kExpSum, false>(L, stream);
        case kExpSum * 2 + 1: return launch_mdi_t<kExpSum, true>(L, stream);
        case kProductPeak * 2: return launch_mdi_t<kProductPeak, false>(L, stream);
        case kProductPeak * 2 + 1: return launch_mdi_t<kProductPeak, true>(L, stream);
        case kGaussian * 2: return launch_mdi_t<kGaussian, false>(L, stream);
        case kGaussian * 2 + 1: return launch_mdi_t<kGaussian, true>(L, stream);
        case kOscillatory * 2: return launch_mdi_t<kOscillatory, false>(L, stream);
        case kOscillatory * 2 + 1: return launch_mdi_t<kOscillatory, true>(L, stream);
        case kExpQuadratic * 2: return launch_mdi_t<kExpQuadratic, false>(L, stream);
        case kExpQuadratic * 2 + 1: return launch_mdi_t<kExpQuadratic, true>(L, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace qmc
