// MDI-LR: the improved (tensor-product) lattice rule evaluated by dimension
// sweeps (Algorithm 2 driving Algorithm 1 with m = 1; eq. 2.14c).
//
// For a product-form integrand g(y) = C prod_k phi_k(y_k) each sweep step sums
// the first remaining coordinate out of the symbolic product with the rule's
// weights 1/N_k, which multiplies the coefficient C by
//   M_k = (1/N_k) sum_{t=0}^{N_k-1} phi_k((t + 1/2) / N_k),
// so Qhat = C_0 prod_k M_k (C_0 = 1, or e^{2 pi i u} for the oscillatory family,
// whose factors e^{i c_k y} are complex).  The d sweeps are independent of one
// another: L lanes of a wave serve one parameter set (L a power of two chosen so
// that the grid fills the GPU), lane l takes directions k = l, l + L, l + 2L, ...,
// multiplies their M_k into a running product kept as mantissa times 2^E (exact
// power-of-two renormalisation, so d in the thousands cannot overflow or
// underflow), and the L partial products are combined by a fixed butterfly of
// lane exchanges (every lane of the group ends with the same bits).
#include "common.hpp"
#include "exp2_seed.hpp"
#include "families.hpp"
#include "kernels.hpp"

namespace qmc {

struct MdiArgs {
    int d;
    const int32_t* N;
    const double* params;
    int P;
    int nsets;
    int lanes_log2;  // L = 2^lanes_log2 lanes per set, L <= kWave
    double* q_out;
};

constexpr int kMdiBlock = 256;
constexpr int kMaxNodesPerDim = 1 << 20;

// Sum over t = 0..Nk-1 of 2^{s y_t^2} by direct evaluation of every node (the
// fallback of quad_node_sums; FP32: FP64 argument, split FP32 exp2).
template <bool FP32>
__device__ __forceinline__ double quad_node_direct(double A, double B, int Nk, double s) {
    double sr = 0.0;
    for (int t = 0; t < Nk; ++t) {
        const double y = fma((double)t, A, B);
        if constexpr (FP32)
            sr += exp2_split_f32(s * y * y);
        else
            sr += exp2(s * y * y);
    }
    return sr;
}

// For each of J directions (J = 1 or 2, summed together so that their two dependent
// chains interleave): the sum over t = 0..Nk-1 of 2^{s y_t^2}, y_t = A t + B, s = -1
// (a Gaussian) or +1 (a growing factor of the signed quadratic).  Consecutive nodes
// differ by the ratio r_t = phi_{t+1} / phi_t = 2^{s A (2 y_t + A)}, and
// r_{t-1} = r_t / q with q = 2^{2 s A^2}, so a run of nodes t0 .. t0 + m - 1 sums in
// Horner form,
//   phi_{t0} (1 + r_{t0} (1 + r_{t0+1} (1 + ... (1 + r_{t0+m-2})))),
// from its last ratio down: one FP64 multiply (the ratio) and one FP64 FMA (the
// partial sum) per node.  phi_{t0} and the run's last ratio come from exp2: every
// S-th node (S = 8 for QMC_FP64, which keeps the compounded rounding of a run below
// ~1e-15 so that a thousand identical directions stay within 1e-12; 64 for
// QMC_FP32_COMPENSATED).  In QMC_FP64 the ratio's step q^-1 is carried as an unevaluated
// sum of two doubles where |2 s A^2| <= 1/16: q^-1 = 1 + u with u = expm1(-2 s A^2 ln 2)
// from its series, the rounding of 1 + u kept as the low part, and r <- r q^-1 as
// fma(r, hi, r lo).  Its rounding otherwise compounds along the run, the same in every
// direction with the same parameters: a factor's error drops from up to 1.7e-15 to
// 2.5e-16 (host emulation against a 50-digit sum; c = 1/sqrt(2), N = 64: 1.1e-15 to
// 4e-17).  The recurrence is used only while every node value, ratio
// and q stay within 2^-1000..2^1000 (max y^2 over the nodes, taken at an end point,
// and 2 A^2 at most 1000; a ratio's exponent is a difference of two node exponents),
// so every exp2 argument lies in [-1000, 1000] and no partial sum or ratio leaves the
// FP64 range; otherwise the nodes are evaluated directly.  A direction's sum does
// not depend on J or on the other direction: where one of two directions fails the
// range test, each is summed on its own.  The loops' trip counts depend only on Nk,
// which is the same in every lane where the caller has checked that (the loops then
// run on the scalar unit).
template <bool FP32, int J>
__device__ __forceinline__ void quad_node_sums(const double (&A)[J], const double (&B)[J],
                                               const double (&s)[J], int Nk, double (&out)[J]) {
    constexpr int kSeed = FP32 ? 64 : 8;
    bool ok[J], all = true;
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const double y_last = fma((double)(Nk - 1), A[j], B[j]);
        ok[j] = fmax(fmax(B[j] * B[j], y_last * y_last), 2.0 * A[j] * A[j]) <= 1000.0;
        all = all && ok[j];
    }
    if (all) {
        double qinv[J], qlo[J], sr[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const double x = -2.0 * s[j] * A[j] * A[j];
            qlo[j] = 0.0;
            if (!FP32 && fabs(x) <= 0.0625) {
                const double u = expm1_small(x * kLn2);
                qinv[j] = 1.0 + u;
                qlo[j] = u - (qinv[j] - 1.0);  // exact: qinv - 1 is exact near 1
            } else {
                qinv[j] = exp2_seed(x);
            }
            sr[j] = 0.0;
        }
        for (int t0 = 0; t0 < Nk; t0 += kSeed) {
            const int m = min(kSeed, Nk - t0);
            double phi0[J], r[J], h[J];
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const double y0 = fma((double)t0, A[j], B[j]);
                phi0[j] = exp2_f64(s[j] * y0 * y0);
                const double yl = fma((double)(t0 + m - 2), A[j], B[j]);  // the run's last ratio r_{t0+m-2}
                r[j] = exp2_seed(s[j] * A[j] * fma(2.0, yl, A[j]));
                h[j] = 1.0;
            }
#pragma unroll 8
            for (int t = m - 2; t >= 0; --t) {
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    h[j] = fma(r[j], h[j], 1.0);
                    if constexpr (FP32)
                        r[j] *= qinv[j];
                    else
                        r[j] = fma(r[j], qinv[j], r[j] * qlo[j]);
                }
            }
#pragma unroll
            for (int j = 0; j < J; ++j) sr[j] = fma(phi0[j], h[j], sr[j]);
        }
#pragma unroll
        for (int j = 0; j < J; ++j) out[j] = sr[j];
    } else if constexpr (J == 1) {
        out[0] = quad_node_direct<FP32>(A[0], B[0], Nk, s[0]);
    } else {
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const double Aj[1] = {A[j]}, Bj[1] = {B[j]}, sj[1] = {s[j]};
            double oj[1];
            quad_node_sums<FP32, 1>(Aj, Bj, sj, Nk, oj);
            out[j] = oj[0];
        }
    }
}

// The inputs of one direction's factor: its node count and the family's one or two
// parameters (c, w), read one direction ahead of their use so that the loads'
// latency overlaps the previous direction's sum.
struct DirIn {
    double c, w;
    int Nk;
};

template <int FAM>
__device__ __forceinline__ DirIn load_dir(const double* p, int d, const int32_t* N, int k) {
    DirIn in;
    in.Nk = N[k];
    if constexpr (FAM == kOscillatory) {
        in.c = p[1 + k];
        in.w = 0.0;
    } else if constexpr (FAM == kExpSum) {
        in.c = p[k];
        in.w = 0.0;
    } else {
        in.c = p[k];
        in.w = p[d + k];
    }
    return in;
}

// The factors M_k = (1/N_k) sum_t phi_k((t + 1/2)/N_k) (real and imaginary parts) of
// J directions with the same node count Nk, 1 <= Nk <= 2^20, invN = 1/Nk.
template <int FAM, bool FP32, int J>
__device__ __forceinline__ void direction_sums(const DirIn (&in)[J], int Nk, double invN,
                                               double (&re)[J], double (&im)[J]) {
    double sr[J], si[J];
#pragma unroll
    for (int j = 0; j < J; ++j) sr[j] = si[j] = 0.0;
    if constexpr (FAM == kGaussian || FAM == kExpQuadratic) {
        // Gaussian: phi = 2^{-y^2}, y = c sqrt(log2 e) ((t + 1/2)/N - w) = A t + B.
        // Signed quadratic: phi = 2^{s y^2}, y = sqrt(|c| log2 e) ((t + 1/2)/N - w),
        // s = sign(c).
        double A[J], B[J], sg[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const double m = FAM == kGaussian ? in[j].c * kSqrtLog2e : sqrt(fabs(in[j].c) * kLog2e);
            A[j] = m * invN;
            B[j] = m * fma(0.5, invN, -in[j].w);
            sg[j] = FAM == kGaussian || in[j].c < 0.0 ? -1.0 : 1.0;
        }
        quad_node_sums<FP32, J>(A, B, sg, Nk, sr);
    } else {
#pragma unroll
        for (int j = 0; j < J; ++j) {
            if constexpr (FAM == kExpSum) {
                // phi = e^{c (t + 1/2)/N}: a geometric sequence, whose sum over the N nodes
                // is e^{c/(2N)} (e^c - 1) / (e^{c/N} - 1) = expm1(c) / (2 sinh(c / (2N)))
                // (c != 0; every term 1 for c = 0), evaluated in FP64 in both precisions.
                const double c = in[j].c;
                sr[j] = c == 0.0 ? (double)Nk : expm1(c) / (2.0 * sinh(0.5 * c * invN));
            } else if constexpr (FAM == kProductPeak) {
                // phi = 1 / (c^-2 + y^2), y = (t + 1/2)/N - w = A t + B
                const double c = in[j].c, w = in[j].w;
                const double g = 1.0 / (c * c), A = invN, B = fma(0.5, invN, -w);
                // v = g + y^2 lies in [g, g + max(B^2, y_last^2)] (y^2 is largest at an end node)
                const double y_last = fma((double)(Nk - 1), A, B);
                const bool f32_range = g >= 1e-36 && g + fmax(B * B, y_last * y_last) <= 1e36;
                double acc = 0.0;
                if (FP32 && f32_range) {
                    // FP32 reciprocal refined by one Newton step in FP64 (relative error
                    // ~1e-15): an FP32 factor's rounding would repeat in every direction
                    // with the same parameters and grow linearly in d (3.4e-6 at d = 1000
                    // for Table 2-3).  Only where every denominator is a normal FP32 number.
                    double td = 0.0;
#pragma unroll 4
                    for (int t = 0; t < Nk; ++t, td += 1.0) {
                        const double y = fma(td, A, B), v = fma(y, y, g);
                        const double r = (double)__builtin_amdgcn_rcpf((float)v);
                        acc += fma(r, fma(-v, r, 1.0), r);
                    }
                } else {
                    for (int t = 0; t < Nk; ++t) {
                        const double y = fma((double)t, A, B);
                        acc += 1.0 / fma(y, y, g);
                    }
                }
                sr[j] = acc;
            } else {  // kOscillatory: phi = e^{i c y}, angle in turns a = c/(2 pi) y = A t + B
                // Also a geometric sequence: with x = c / (2N), the node sum is
                //   sum_t e^{i c (t + 1/2)/N} = e^{i c/2} sin(c/2) / sin(x),
                // evaluated in FP64 in both precisions for 0 < |x| <= pi/2 (every term 1
                // for c = 0).  One rounding of a factor would otherwise repeat in every
                // direction with the same c; beyond pi/2 (more than a quarter turn between
                // nodes) the node loop below sums the terms.
                const double x = 0.5 * in[j].c * invN;
                if (fabs(x) <= 1.5707963267948966) {
                    if (x == 0.0) {
                        sr[j] = (double)Nk;
                        si[j] = 0.0;
                    } else {
                        double sh, ch;
                        sincos(0.5 * in[j].c, &sh, &ch);
                        const double m = sh / sin(x);
                        sr[j] = m * ch;
                        si[j] = m * sh;
                    }
                    continue;
                }
                const double c = in[j].c * kInv2Pi;
                const double A = c * invN, B = 0.5 * c * invN;
                double ar = 0.0, ai = 0.0;
                if constexpr (FP32) {
                    // The few nodes per direction do not average the hardware sin/cos error
                    // away, so the factor uses the correctly reduced single-precision sincospi.
                    for (int t = 0; t < Nk; ++t) {
                        const double a = fma((double)t, A, B);
                        const float fr = (float)(a - rint(a));
                        float sn, co;
                        sincospif(2.0f * fr, &sn, &co);
                        ar += (double)co;
                        ai += (double)sn;
                    }
                } else {
                    for (int t = 0; t < Nk; ++t) {
                        const double a = fma((double)t, A, B);
                        const double fr = a - rint(a);
                        double sn, co;
                        sincospi(2.0 * fr, &sn, &co);
                        ar += co;
                        ai += sn;
                    }
                }
                sr[j] = ar;
                si[j] = ai;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
        re[j] = sr[j] * invN;
        im[j] = si[j] * invN;
    }
}

// (cr + i ci) 2^E times (mr + i mi), renormalised to a largest part in [1/2, 1).
template <bool COMPLEX>
__device__ __forceinline__ void mul_renorm(double& cr, double& ci, int& E, double mr, double mi) {
    double nr, ni = 0.0;
    if constexpr (COMPLEX) {
        nr = fma(cr, mr, -ci * mi);
        ni = fma(cr, mi, ci * mr);
    } else {
        nr = cr * mr;
    }
    const double big = COMPLEX ? fmax(fabs(nr), fabs(ni)) : fabs(nr);
    if (big > 0.0 && big < INFINITY) {
        const int e = __builtin_amdgcn_frexp_exp(big);
        nr = ldexp(nr, -e);
        if constexpr (COMPLEX) ni = ldexp(ni, -e);
        E += e;
    }
    cr = nr;
    ci = ni;
}

template <int FAM, bool FP32>
__global__ __launch_bounds__(kMdiBlock) void mdi_lr_kernel(const MdiArgs a) {
    constexpr bool kComplex = FAM == kOscillatory;
    const int L = 1 << a.lanes_log2;
    const int gid = blockIdx.x * kMdiBlock + threadIdx.x;
    const int set = gid >> a.lanes_log2, li = gid & (L - 1);
    const bool active = set < a.nsets;

    // This lane's directions k = li, li + L, ... in increasing order, two at a time,
    // each pair's inputs loaded while the previous pair is summed.  Where every lane of
    // the wave has the same node count (every N_k equal, the usual case) the node loops
    // take it from a scalar register and 1/N_k is computed once per count; otherwise
    // each direction is summed on its own with its lane's count.  An N_k outside
    // [1, 2^20] (the caller's contract) gives NaN.
    double cr = 1.0, ci = 0.0;
    int E = 0;
    if (active && li < a.d) {
        const double* p = a.params + (size_t)set * a.P;
        DirIn n1 = load_dir<FAM>(p, a.d, a.N, li);
        DirIn n2 = li + L < a.d ? load_dir<FAM>(p, a.d, a.N, li + L) : n1;
        int n_inv = 0;  // the count whose reciprocal invN holds (0: none yet)
        double invN = 0.0;
        for (int k = li; k < a.d; k += 2 * L) {
            const bool two = k + L < a.d;
            const DirIn in[2] = {n1, n2};
            if (k + 2 * L < a.d) n1 = load_dir<FAM>(p, a.d, a.N, k + 2 * L);
            if (k + 3 * L < a.d) n2 = load_dir<FAM>(p, a.d, a.N, k + 3 * L);
            double re[2] = {1.0, 1.0}, im[2] = {0.0, 0.0};
            const int n0 = __builtin_amdgcn_readfirstlane(in[0].Nk);
            const bool bad0 = in[0].Nk < 1 || in[0].Nk > kMaxNodesPerDim;
            const bool bad1 = two && (in[1].Nk < 1 || in[1].Nk > kMaxNodesPerDim);
            if (__builtin_amdgcn_ballot_w64(in[0].Nk != n0 || (two && in[1].Nk != n0)) == 0 &&
                n0 >= 1 && n0 <= kMaxNodesPerDim) {
                if (n0 != n_inv) {
                    invN = 1.0 / (double)n0;
                    n_inv = n0;
                }
                if (two) {
                    direction_sums<FAM, FP32, 2>(in, n0, invN, re, im);
                } else {
                    const DirIn in1[1] = {in[0]};
                    double re1[1], im1[1];
                    direction_sums<FAM, FP32, 1>(in1, n0, invN, re1, im1);
                    re[0] = re1[0];
                    im[0] = im1[0];
                }
            } else {
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    if (j == 1 && !two) break;
                    if (j == 0 ? bad0 : bad1) {
                        re[j] = im[j] = __builtin_nan("");
                        continue;
                    }
                    const DirIn inj[1] = {in[j]};
                    double rej[1], imj[1];
                    direction_sums<FAM, FP32, 1>(inj, in[j].Nk, 1.0 / (double)in[j].Nk, rej, imj);
                    re[j] = rej[0];
                    im[j] = imj[0];
                }
            }
            mul_renorm<kComplex>(cr, ci, E, re[0], im[0]);
            if (two) mul_renorm<kComplex>(cr, ci, E, re[1], im[1]);
        }
    }
    // Partial products of the set's L lanes, combined by a butterfly over lane
    // distances 1, 2, 4, ...: products commute exactly, so both partners of every
    // exchange compute the same bits and the order is fixed by the lane structure.
    for (int off = 1; off < L; off <<= 1) {
        const double pr = __shfl_xor(cr, off, kWave);
        const double pi = kComplex ? __shfl_xor(ci, off, kWave) : 0.0;
        const int pe = __shfl_xor(E, off, kWave);
        E += pe;
        mul_renorm<kComplex>(cr, ci, E, pr, pi);
    }
    if (active && li == 0) {
        if constexpr (kComplex) {
            // the coefficient e^{2 pi i u} of the symbolic function before the sweeps
            double su, cu;
            sincospi(2.0 * a.params[(size_t)set * a.P], &su, &cu);
            double r = cr, i = ci;
            mul_renorm<true>(r, i, E, cu, su);
            cr = r;
        }
        a.q_out[set] = ldexp(cr, E);
    }
}

// Lanes per set: enough (set, lane) pairs for about eight waves per SIMD of the
// whole GPU (the kernel's FP64 chains need that many to keep the SIMD issuing), at
// most one wave per set and at most one lane per direction.
static int mdi_lanes_log2(int d, int nsets) {
    const int64_t want = (int64_t)device_cu_count() * 4 * 8 * kWave;
    int lg = 0;
    while (lg < 6 && (int64_t)nsets << lg < want && (2 << lg) <= d) ++lg;
    return lg;
}

template <int FAM, bool FP32>
static hipError_t launch_mdi_t(const MdiLaunch& L, hipStream_t stream) {
    MdiArgs a;
    a.d = L.d;
    a.N = L.N;
    a.params = L.params;
    a.P = L.P;
    a.nsets = L.nsets;
    a.lanes_log2 = mdi_lanes_log2(L.d, L.nsets);
    a.q_out = L.q_out;
    const int64_t threads = (int64_t)L.nsets << a.lanes_log2;
    const unsigned grid = (unsigned)((threads + kMdiBlock - 1) / kMdiBlock);
    hipLaunchKernelGGL((mdi_lr_kernel<FAM, FP32>), dim3(grid), dim3(kMdiBlock), 0, stream, a);
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
