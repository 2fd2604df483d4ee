// Host-side launchers of the HIP kernels (internal to libqmc.so).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace qmc {

// Threads per workgroup of the plain-sum kernel: 16 waves, so that one
// workgroup per CU already hides latency and the grid has few workgroups to
// dispatch and to reduce.
constexpr int kSumBlock = 1024;
// Workgroups per set that the plain-sum launcher may use: at most
// max(1, kMaxSumBlocks / nsets), never more than kMaxSumBlocksPerSet.
constexpr int kMaxSumBlocks = 2048;
constexpr int kMaxSumBlocksPerSet = 512;
// Parameter sets of one plain-sum call (the ticket layout holds this many).
constexpr int kMaxSumSets = 4096;

struct PlainLaunch {
    int d;
    uint32_t n;
    const int64_t* z;
    const double* shift;  // may be null
    int family;
    const double* params;
    int P;  // parameters per set
    int nsets;
    // Set s reads params + s * param_stride and shift + s * shift_stride: (P, 0) for
    // parameter sets sharing one shift, (0, d) for shifts sharing one parameter set.
    int param_stride;
    int shift_stride;
    int z_stride;  // int64 between the generating vectors of two sets (0: shared z)
    bool fp32;
    double* q_out;
    void* ws;
    int points_per_thread;  // 0 = choose automatically (4, 8 or 16)
    int max_blocks;         // 0 = choose automatically
};

int sum_blocks_per_set(int nsets);
size_t plain_workspace_bytes(int nsets);
hipError_t launch_lattice_sum(const PlainLaunch& a, hipStream_t stream);

// Mean and standard error of the mean of q[0..R) into stats[0..1] (one wave).
hipError_t launch_shift_stats(const double* q, int R, double* stats, hipStream_t stream);

hipError_t launch_lattice_points(int d, uint32_t n, const int64_t* z, int64_t i0, int64_t count,
                                 int32_t* k_out, hipStream_t stream);

struct MdiLaunch {
    int d;
    const int32_t* N;
    int family;
    const double* params;
    int P;
    int nsets;
    bool fp32;
    double* q_out;
};
hipError_t launch_mdi_lr(const MdiLaunch& a, hipStream_t stream);

// Adjoint of the plain rule for nsets parameter sets sharing the lattice.
constexpr int kMaxAdjBlocks = 1024;
constexpr int kMaxAdjDims = 512;
constexpr int kAdjSetsMaxParams = 65;  // parameters per set served by the set-batched adjoint (d <= 64)

struct AdjLaunch {
    int d;
    uint32_t n;
    const int64_t* z;
    const double* shift;
    int family;
    const double* params;
    int P;
    int nsets;
    bool fp32;
    const double* gq;  // may be null
    double* q_out;
    double* grad_out;
    void* ws;
};

int adjoint_blocks_per_set(int nsets);
size_t adjoint_workspace_bytes(int P, int nsets);
hipError_t launch_adjoint(const AdjLaunch& a, hipStream_t stream);

// Bernoulli product sums behind the lattice-quality criteria (criteria.hip).
struct BernoulliLaunch {
    int d;
    uint32_t n;
    const int64_t* z;  // [nz][d]
    int nz;            // <= kMaxSumSets
    int alpha;         // 2 or 4
    const double* a;   // [d]
    double* s_out;     // [nz]
    void* ws;
};
hipError_t launch_bernoulli_sum(const BernoulliLaunch& L, hipStream_t stream);

// A lattice-quality criterion: P_alpha of eq. 2.4, or e^2 of eq. 2.12 with
// product weights gamma (device, d entries) and beta (alpha = 2).
constexpr int kCritPAlpha = 0;
constexpr int kCritWce2 = 1;
struct CriterionSpec {
    int kind;
    int alpha;
    const double* gamma;  // kCritWce2 only
    double beta;
};

// The criterion of nz generating vectors (rows of z).
struct CriterionLaunch {
    int d;
    uint32_t n;
    const int64_t* z;  // [nz][d]
    int nz;
    CriterionSpec crit;
    double* out;       // [nz]
    void* ws;
};
hipError_t launch_criterion(const CriterionLaunch& L, hipStream_t stream);

struct SearchLaunch {
    int d;
    uint32_t n;
    CriterionSpec crit;
    int64_t a0;
    int count;
    double* s_out;     // [count]
    double* best_out;  // [2]
    void* ws;
};
hipError_t launch_korobov_search(const SearchLaunch& L, hipStream_t stream);

struct CbcLaunch {
    int d;
    uint32_t n;
    CriterionSpec crit;
    int64_t* z_out;  // [d]
    double* s_out;   // [d]
    void* ws;
};
hipError_t launch_cbc(const CbcLaunch& L, hipStream_t stream);

// Workspace of the criteria entry points: the zero region, the weights, then the
// larger of a table of kMaxSumSets generating vectors and the CBC vectors.
size_t criteria_workspace_bytes(int d, int64_t n);

// MDI-LR for integrands of the coordinate sum (mdi_sum.hip).
struct MdiSumLaunch {
    int d, N, N_last;
    int gfamily;           // 0 power (b, c, p), 1 Gaussian (c, w)
    const double* params;  // [nsets][P]
    int P;
    int nsets;
    bool fp32;
    double* q_out;
    void* ws;
};
hipError_t launch_mdi_sum(const MdiSumLaunch& L, hipStream_t stream);
// The states after d - 1 directions and two buffers of the same size.
size_t mdi_sum_workspace_bytes(int d, int N);

// The improved rule's tensor grid on a Korobov lattice (implr.hip).
struct ImplrLaunch {
    int d;
    uint32_t n;
    uint32_t a;
    uint32_t zd;          // z_d = a^{d-1} < n
    uint32_t nd;          // ceil(n / z_d)
    uint64_t grid;        // z_d n_d
    bool bitmap;          // count with the bitmap only (no order check)
    int64_t* nstar_out;   // device
    void* ws;
};
struct ImplrPointsLaunch {
    int d;
    uint32_t n;
    uint32_t a;
    uint32_t zd;
    uint64_t j0, count;   // j0 + count <= n
    uint64_t ld;          // >= count: s_out[i * ld + (j - j0)]
    int32_t* s_out;       // device
};
hipError_t launch_implr(const ImplrLaunch& L, hipStream_t stream);
hipError_t launch_implr_points(const ImplrPointsLaunch& L, hipStream_t stream);
size_t implr_workspace_bytes(uint64_t grid);

int device_cu_count();

}  // namespace qmc
