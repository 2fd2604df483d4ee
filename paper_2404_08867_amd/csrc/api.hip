// C ABI of libqmc.so: argument validation, error reporting and dispatch to the
// kernel launchers.  Nothing here allocates device memory; see include/qmc.h.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>

#include <mutex>

#include "qmc.h"
#include "common.hpp"
#include "kernels.hpp"
#include "status.hpp"

namespace {
// Message of the last failing call on this thread; a fixed buffer, so that no call
// allocates host memory either, on any path.
thread_local char g_last_error[512];
}

namespace qmc {

qmc_status fail(qmc_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return s;
}

qmc_status ok() {
    g_last_error[0] = '\0';
    return QMC_OK;
}

qmc_status from_hip(hipError_t e, const char* where) {
    if (e == hipSuccess) return ok();
    return fail(QMC_ERR_DEVICE, "%s: HIP error %d (%s)", where, (int)e, hipGetErrorString(e));
}

// Debug mode: with QMC_VALIDATE=1 in the environment, the device arrays whose
// ranges are the caller's contract (z_j in [0, n), shift_j in [0, 1)) are read back
// on the call's stream -- synchronously, after the work already queued there -- and
// checked before anything is launched.  A stream that is being captured into a
// graph cannot be synchronised, so there the check is skipped.
bool validate_mode() {
    const char* v = getenv("QMC_VALIDATE");
    return v && v[0] == '1';
}

bool capturing(hipStream_t stream) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(stream, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

// Reads the `count` entries of device array `dev` back on `stream` in chunks of 4 KiB
// through a buffer on the stack (no allocation) and sets *bad to the index of the
// first entry x with !good(x) (count if there is none) and *bad_value to that entry.
template <class T, class Good>
qmc_status scan_back(const T* dev, size_t count, hipStream_t stream, const char* what, Good good,
                     size_t* bad, T* bad_value) {
    constexpr size_t kChunk = 4096 / sizeof(T);
    T h[kChunk];
    for (size_t i0 = 0; i0 < count; i0 += kChunk) {
        const size_t m = count - i0 < kChunk ? count - i0 : kChunk;
        hipError_t e = hipMemcpyAsync(h, dev + i0, m * sizeof(T), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return from_hip(e, what);
        for (size_t i = 0; i < m; ++i)
            if (!good(h[i])) {
                *bad = i0 + i;
                *bad_value = h[i];
                return QMC_OK;
            }
    }
    *bad = count;
    return QMC_OK;
}

// z: `count` int64 entries, each in [0, n).
qmc_status validate_z(const int64_t* z, size_t count, int64_t n, void* stream, const char* what) {
    if (!validate_mode() || !z || capturing((hipStream_t)stream)) return QMC_OK;
    size_t i = 0;
    int64_t x = 0;
    qmc_status s = scan_back(z, count, (hipStream_t)stream, what,
                             [n](int64_t v) { return v >= 0 && v < n; }, &i, &x);
    if (s != QMC_OK) return s;
    if (i < count)
        return fail(QMC_ERR_INVALID_ARG, "%s: z[%zu] = %lld outside [0, %lld) (QMC_VALIDATE)", what, i,
                    (long long)x, (long long)n);
    return QMC_OK;
}

// shift: `count` doubles, each in [0, 1).
qmc_status validate_shift(const double* sh, size_t count, void* stream, const char* what) {
    if (!validate_mode() || !sh || capturing((hipStream_t)stream)) return QMC_OK;
    size_t i = 0;
    double x = 0.0;
    qmc_status s = scan_back(sh, count, (hipStream_t)stream, what,
                             [](double v) { return v >= 0.0 && v < 1.0; }, &i, &x);
    if (s != QMC_OK) return s;
    if (i < count)
        return fail(QMC_ERR_INVALID_ARG, "%s: shift[%zu] = %g outside [0, 1) (QMC_VALIDATE)", what, i, x);
    return QMC_OK;
}

}  // namespace qmc

namespace {

using qmc::fail;
using qmc::from_hip;
using qmc::ok;
using qmc::validate_shift;
using qmc::validate_z;

constexpr int kMaxD = 1024;
constexpr int64_t kMaxN = (int64_t)1 << 31;  // exclusive
constexpr int kMaxSets = qmc::kMaxSumSets;  // plain sums: one grid row and 33 counters per set
constexpr int kMaxMdiSets = 1 << 24;     // MDI-LR: sets are spread over workgroups
constexpr int64_t kMaxNodes = (int64_t)1 << 20;
constexpr int64_t kMaxExport = (int64_t)1 << 26;
constexpr int64_t kMaxCbcN = (int64_t)1 << 26;   // CBC keeps n + n/2 doubles
constexpr int32_t kMaxSumNodes = 1 << 20;
constexpr int64_t kMaxSumStates = (int64_t)1 << 20;
constexpr int64_t kMaxImplrLd = (int64_t)1 << 40;  // elements between rows of qmc_implr_points

int param_count(int family, int d) {
    switch (family) {
        case QMC_EXP_SUM: return d;
        case QMC_PRODUCT_PEAK: return 2 * d;
        case QMC_GAUSSIAN: return 2 * d;
        case QMC_OSCILLATORY: return d + 1;
        case QMC_EXP_QUADRATIC: return 2 * d;
        default: return -1;
    }
}

qmc_status check_common(int32_t d, int32_t family, int32_t nsets, int32_t precision,
                        int32_t max_sets = kMaxSets) {
    if (d < 1 || d > kMaxD) return fail(QMC_ERR_INVALID_ARG, "d = %d outside [1, %d]", d, kMaxD);
    if (param_count(family, d) < 0) return fail(QMC_ERR_INVALID_ARG, "unknown family %d", family);
    if (nsets < 1 || nsets > max_sets)
        return fail(QMC_ERR_INVALID_ARG, "nsets = %d outside [1, %d]", nsets, max_sets);
    if (precision != QMC_FP64 && precision != QMC_FP32_COMPENSATED)
        return fail(QMC_ERR_INVALID_ARG, "unknown precision %d", precision);
    return QMC_OK;
}

qmc_status check_workspace(const void* ws, size_t ws_bytes, size_t need) {
    if (!ws) return fail(QMC_ERR_WORKSPACE, "workspace pointer is NULL");
    if (((uintptr_t)ws) % 256 != 0) return fail(QMC_ERR_WORKSPACE, "workspace not 256-byte aligned");
    if (ws_bytes < need)
        return fail(QMC_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, need);
    return QMC_OK;
}

int64_t gcd64(int64_t a, int64_t b) {
    while (b) {
        const int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

}  // namespace

// ---------------------------------------------------------------------------
// Scratch of qmc_lattice_sum_noalloc: the plain sum's counter and tagged-slot region
// (qmc::kZeroBytes = 4 MiB), one copy per device in the library's code object, held
// until the process ends.  Its name stands for a host-side shadow in host code; the
// device address comes from hipGetSymbolAddress, once per device, and only that
// address is ever passed on.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[qmc::kZeroBytes];

namespace {

constexpr size_t kNoallocScratchBytes = qmc::kZeroBytes;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_addr[kMaxDevices];  // device address of `scratch` per device, null until set up

__global__ __launch_bounds__(256) void scratch_clear_kernel(uint4* p, size_t count) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// This device's scratch address.  The first call on a device (with the device
// current) looks the address up and clears the array with a kernel on `stream`
// (the plain sum needs its counters and slots zero, and leaves them zero when it
// completes).
qmc_status scratch_address(hipStream_t stream, void** addr) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return from_hip(e, "qmc_lattice_sum_noalloc: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(QMC_ERR_UNSUPPORTED, "qmc_lattice_sum_noalloc: device %d beyond the %d supported", dev,
                    kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return from_hip(e, "qmc_lattice_sum_noalloc: hipGetSymbolAddress(scratch)");
        if (!p || ((uintptr_t)p) % 256 != 0)
            return fail(QMC_ERR_DEVICE, "qmc_lattice_sum_noalloc: scratch address %p unusable", p);
        hipLaunchKernelGGL(scratch_clear_kernel, dim3(256), dim3(256), 0, stream, (uint4*)p,
                           kNoallocScratchBytes / sizeof(uint4));
        e = hipGetLastError();
        if (e != hipSuccess) return from_hip(e, "qmc_lattice_sum_noalloc: clearing the scratch");
        g_scratch_addr[dev] = p;
    }
    *addr = g_scratch_addr[dev];
    return QMC_OK;
}

}  // namespace

extern "C" {

const char* qmc_version(void) { return "qmc-mi355x 0.1.0 (gfx950)"; }

const char* qmc_status_string(qmc_status s) {
    switch (s) {
        case QMC_OK: return "ok";
        case QMC_ERR_INVALID_ARG: return "invalid argument";
        case QMC_ERR_UNSUPPORTED: return "unsupported";
        case QMC_ERR_WORKSPACE: return "workspace too small or misaligned";
        case QMC_ERR_OUT_OF_MEMORY: return "out of memory";
        case QMC_ERR_DEVICE: return "device error";
    }
    return "unknown status";
}

const char* qmc_last_error(void) { return g_last_error; }

qmc_status qmc_korobov(int32_t d, int64_t n, int64_t a, int64_t* z_out) {
    if (d < 1 || d > kMaxD) return fail(QMC_ERR_INVALID_ARG, "d = %d outside [1, %d]", d, kMaxD);
    if (n < 1 || n >= kMaxN) return fail(QMC_ERR_INVALID_ARG, "n = %lld outside [1, 2^31)", (long long)n);
    if (a < 0) return fail(QMC_ERR_INVALID_ARG, "a = %lld is negative", (long long)a);
    if (!z_out) return fail(QMC_ERR_INVALID_ARG, "z_out is NULL");
    // z_j = a^j mod n by repeated modular multiplication; residues < 2^31 so
    // every product fits in 62 bits.
    const int64_t am = a % n;
    int64_t r = 1 % n;
    for (int32_t j = 0; j < d; ++j) {
        z_out[j] = r;
        r = (r * am) % n;
    }
    return ok();
}

qmc_status qmc_mdi_lr_dims(int32_t d, int64_t a, int32_t n_mode, int64_t n_explicit,
                           int32_t* N_out) {
    if (d < 1 || d > kMaxD) return fail(QMC_ERR_INVALID_ARG, "d = %d outside [1, %d]", d, kMaxD);
    if (!N_out) return fail(QMC_ERR_INVALID_ARG, "N_out is NULL");
    if (a < 1 || a > kMaxNodes) return fail(QMC_ERR_INVALID_ARG, "a = %lld outside [1, 2^20]", (long long)a);
    switch (n_mode) {
        case QMC_N_A_POW_D:
            // z = (1, a, ..., a^{d-1}) is not reduced (n = a^d > a^{d-1}), so eq. 3.5 gives
            // N_i = lcm(a^{i-1}, a^i) / a^{i-1} = a and N_d = ceil(a^d / a^{d-1}) = a.
            for (int32_t k = 0; k < d; ++k) N_out[k] = (int32_t)a;
            return ok();
        case QMC_N_ONE_PLUS_A_POW_D:
            // Same z; N_d = ceil((1 + a^d) / a^{d-1}) = a + 1.
            if (a + 1 > kMaxNodes) return fail(QMC_ERR_INVALID_ARG, "N_d = a + 1 exceeds 2^20");
            for (int32_t k = 0; k + 1 < d; ++k) N_out[k] = (int32_t)a;
            N_out[d - 1] = (int32_t)(a + 1);
            return ok();
        case QMC_N_EXPLICIT: {
            const int64_t n = n_explicit;
            if (n < 1 || n >= kMaxN) return fail(QMC_ERR_INVALID_ARG, "n = %lld outside [1, 2^31)", (long long)n);
            int64_t zi = 1 % n;
            for (int32_t k = 0; k < d; ++k) {
                const int64_t zn = (zi * (a % n)) % n;
                int64_t Nk;
                if (k + 1 < d) {
                    if (zi == 0 || zn == 0)
                        return fail(QMC_ERR_INVALID_ARG, "z has a zero entry at %d; eq. 3.5 is undefined", k);
                    const int64_t g = gcd64(zi, zn);
                    const int64_t mn = zi < zn ? zi : zn;
                    Nk = (zi / g) * zn / mn;  // lcm / min
                } else {
                    if (zi == 0) return fail(QMC_ERR_INVALID_ARG, "z_d = 0; eq. 3.5 is undefined");
                    Nk = (n + zi - 1) / zi;
                }
                if (Nk < 1 || Nk > kMaxNodes)
                    return fail(QMC_ERR_INVALID_ARG, "N_%d = %lld exceeds 2^20", k + 1, (long long)Nk);
                N_out[k] = (int32_t)Nk;
                zi = zn;
            }
            return ok();
        }
        default:
            return fail(QMC_ERR_INVALID_ARG, "unknown n_mode %d", n_mode);
    }
}

qmc_status qmc_param_count(int32_t family, int32_t d, int32_t* count) {
    if (!count) return fail(QMC_ERR_INVALID_ARG, "count is NULL");
    if (d < 1 || d > kMaxD) return fail(QMC_ERR_INVALID_ARG, "d = %d outside [1, %d]", d, kMaxD);
    const int p = param_count(family, d);
    if (p < 0) return fail(QMC_ERR_INVALID_ARG, "unknown family %d", family);
    *count = p;
    return ok();
}

qmc_status qmc_workspace_size(int32_t max_d, int64_t max_n, int32_t max_sets, size_t* bytes) {
    if (!bytes) return fail(QMC_ERR_INVALID_ARG, "bytes is NULL");
    if (max_d < 1 || max_d > kMaxD) return fail(QMC_ERR_INVALID_ARG, "max_d = %d outside [1, %d]", max_d, kMaxD);
    if (max_n < 1 || max_n >= kMaxN) return fail(QMC_ERR_INVALID_ARG, "max_n outside [1, 2^31)");
    if (max_sets < 1 || max_sets > kMaxSets) return fail(QMC_ERR_INVALID_ARG, "max_sets outside [1, %d]", kMaxSets);
    // The counter region is fixed; the scratch per set shrinks as nsets grows,
    // so the bound is the maximum over nsets <= max_sets.
    size_t need = 0;
    for (int s = 1; s <= max_sets; s = (s < 64 ? s + 1 : s * 2)) {
        const size_t b = qmc::plain_workspace_bytes(s);
        if (b > need) need = b;
    }
    const size_t b = qmc::plain_workspace_bytes(max_sets);
    if (b > need) need = b;
    // The adjoint keeps one vector of P + 1 doubles per workgroup and group; its
    // set-batched form (small d) one vector per group of 32 sets, evaluated at the
    // largest P it serves.
    const int pmax = 2 * (max_d < qmc::kMaxAdjDims ? max_d : qmc::kMaxAdjDims) + 1;
    const int pset = pmax < qmc::kAdjSetsMaxParams ? pmax : qmc::kAdjSetsMaxParams;
    for (int s = 1; s <= max_sets; s = (s < 64 ? s + 1 : s * 2)) {
        size_t a = qmc::adjoint_workspace_bytes(pmax, s);
        if (a > need) need = a;
        a = qmc::adjoint_workspace_bytes(pset, s);
        if (a > need) need = a;
    }
    size_t a = qmc::adjoint_workspace_bytes(pmax, max_sets);
    if (a > need) need = a;
    a = qmc::adjoint_workspace_bytes(pset, max_sets);
    if (a > need) need = a;
    *bytes = need;
    return ok();
}

qmc_status qmc_lattice_sum_adjoint(int32_t d, int64_t n, const int64_t* z, const double* shift,
                                   int32_t family, const double* params, int32_t nsets,
                                   int32_t precision, const double* gq, double* q_out,
                                   double* grad_out, void* ws, size_t ws_bytes, void* stream) {
    qmc_status s = check_common(d, family, nsets, precision);
    if (s != QMC_OK) return s;
    if (d > qmc::kMaxAdjDims)
        return fail(QMC_ERR_UNSUPPORTED, "the adjoint supports d <= %d (d = %d)", qmc::kMaxAdjDims, d);
    if (n < 1 || n >= kMaxN) return fail(QMC_ERR_INVALID_ARG, "n = %lld outside [1, 2^31)", (long long)n);
    if (!z || !params || !q_out || !grad_out)
        return fail(QMC_ERR_INVALID_ARG, "z, params, q_out and grad_out must be non-NULL");
    const int P = param_count(family, d);
    s = check_workspace(ws, ws_bytes, qmc::adjoint_workspace_bytes(P, nsets));
    if (s != QMC_OK) return s;
    if ((s = validate_z(z, (size_t)d, n, stream, "qmc_lattice_sum_adjoint")) != QMC_OK) return s;
    if ((s = validate_shift(shift, (size_t)d, stream, "qmc_lattice_sum_adjoint")) != QMC_OK) return s;
    qmc::AdjLaunch L{};
    L.d = d;
    L.n = (uint32_t)n;
    L.z = z;
    L.shift = shift;
    L.family = family;
    L.params = params;
    L.P = P;
    L.nsets = nsets;
    L.fp32 = precision == QMC_FP32_COMPENSATED;
    L.gq = gq;
    L.q_out = q_out;
    L.grad_out = grad_out;
    L.ws = ws;
    return from_hip(qmc::launch_adjoint(L, (hipStream_t)stream), "qmc_lattice_sum_adjoint");
}

qmc_status qmc_lattice_sum(int32_t d, int64_t n, const int64_t* z, const double* shift,
                           int32_t family, const double* params, int32_t nsets,
                           int32_t precision, double* q_out, void* ws, size_t ws_bytes,
                           void* stream) {
    return qmc_lattice_sum_ex(d, n, z, shift, family, params, nsets, precision, q_out, ws,
                              ws_bytes, stream, nullptr);
}

qmc_status qmc_lattice_sum_ex(int32_t d, int64_t n, const int64_t* z, const double* shift,
                              int32_t family, const double* params, int32_t nsets,
                              int32_t precision, double* q_out, void* ws, size_t ws_bytes,
                              void* stream, const qmc_launch_config* cfg) {
    qmc_status s = check_common(d, family, nsets, precision);
    if (s != QMC_OK) return s;
    if (n < 1 || n >= kMaxN) return fail(QMC_ERR_INVALID_ARG, "n = %lld outside [1, 2^31)", (long long)n);
    if (!z || !params || !q_out) return fail(QMC_ERR_INVALID_ARG, "z, params and q_out must be non-NULL");
    s = check_workspace(ws, ws_bytes, qmc::plain_workspace_bytes(nsets));
    if (s != QMC_OK) return s;
    if ((s = validate_z(z, (size_t)d, n, stream, "qmc_lattice_sum")) != QMC_OK) return s;
    if ((s = validate_shift(shift, (size_t)d, stream, "qmc_lattice_sum")) != QMC_OK) return s;
    qmc::PlainLaunch L{};
    L.d = d;
    L.n = (uint32_t)n;
    L.z = z;
    L.shift = shift;
    L.family = family;
    L.params = params;
    L.P = param_count(family, d);
    L.nsets = nsets;
    L.param_stride = L.P;
    L.shift_stride = 0;
    L.z_stride = 0;
    L.fp32 = precision == QMC_FP32_COMPENSATED;
    L.q_out = q_out;
    L.ws = ws;
    L.points_per_thread = 0;
    L.max_blocks = 0;
    if (cfg) {
        const int m = cfg->points_per_thread;
        if (m != 0 && m != 4 && m != 8 && m != 16)
            return fail(QMC_ERR_INVALID_ARG, "points_per_thread = %d is not 0, 4, 8 or 16", m);
        if (cfg->max_blocks < 0 || cfg->max_blocks > qmc::kMaxSumBlocksPerSet)
            return fail(QMC_ERR_INVALID_ARG, "max_blocks = %d outside [0, %d]", cfg->max_blocks,
                        qmc::kMaxSumBlocksPerSet);
        L.points_per_thread = m;
        L.max_blocks = cfg->max_blocks;
    }
    return from_hip(qmc::launch_lattice_sum(L, (hipStream_t)stream), "qmc_lattice_sum");
}

qmc_status qmc_lattice_sum_noalloc(int32_t d, int64_t n, const int64_t* z, const double* shift,
                                   int32_t family, const double* params, int32_t nsets,
                                   int32_t precision, double* q_out, void* stream) {
    qmc_status s = check_common(d, family, nsets, precision);
    if (s != QMC_OK) return s;
    if (n < 1 || n >= kMaxN) return fail(QMC_ERR_INVALID_ARG, "n = %lld outside [1, 2^31)", (long long)n);
    if (!z || !params || !q_out) return fail(QMC_ERR_INVALID_ARG, "z, params and q_out must be non-NULL");
    const size_t need = qmc::plain_workspace_bytes(nsets);
    if (need > kNoallocScratchBytes)
        return fail(QMC_ERR_WORKSPACE,
                    "qmc_lattice_sum_noalloc: nsets = %d needs %zu bytes of scratch, the static scratch holds %zu",
                    nsets, need, kNoallocScratchBytes);
    if ((s = validate_z(z, (size_t)d, n, stream, "qmc_lattice_sum_noalloc")) != QMC_OK) return s;
    if ((s = validate_shift(shift, (size_t)d, stream, "qmc_lattice_sum_noalloc")) != QMC_OK) return s;
    void* ws = nullptr;
    if ((s = scratch_address((hipStream_t)stream, &ws)) != QMC_OK) return s;
    qmc::PlainLaunch L{};
    L.d = d;
    L.n = (uint32_t)n;
    L.z = z;
    L.shift = shift;
    L.family = family;
    L.params = params;
    L.P = param_count(family, d);
    L.nsets = nsets;
    L.param_stride = L.P;
    L.shift_stride = 0;
    L.z_stride = 0;
    L.fp32 = precision == QMC_FP32_COMPENSATED;
    L.q_out = q_out;
    L.ws = ws;
    L.points_per_thread = 0;
    L.max_blocks = 0;
    return from_hip(qmc::launch_lattice_sum(L, (hipStream_t)stream), "qmc_lattice_sum_noalloc");
}

qmc_status qmc_lattice_sum_shifts(int32_t d, int64_t n, const int64_t* z, const double* shifts,
                                  int32_t nshifts, int32_t family, const double* params,
                                  int32_t precision, double* q_out, double* stats_out, void* ws,
                                  size_t ws_bytes, void* stream) {
    qmc_status s = check_common(d, family, nshifts, precision);
    if (s != QMC_OK) return s;
    if (n < 1 || n >= kMaxN) return fail(QMC_ERR_INVALID_ARG, "n = %lld outside [1, 2^31)", (long long)n);
    if (!z || !shifts || !params || !q_out)
        return fail(QMC_ERR_INVALID_ARG, "z, shifts, params and q_out must be non-NULL");
    s = check_workspace(ws, ws_bytes, qmc::plain_workspace_bytes(nshifts));
    if (s != QMC_OK) return s;
    if ((s = validate_z(z, (size_t)d, n, stream, "qmc_lattice_sum_shifts")) != QMC_OK) return s;
    if ((s = validate_shift(shifts, (size_t)nshifts * (size_t)d, stream, "qmc_lattice_sum_shifts")) != QMC_OK)
        return s;
    qmc::PlainLaunch L{};
    L.d = d;
    L.n = (uint32_t)n;
    L.z = z;
    L.shift = shifts;
    L.family = family;
    L.params = params;
    L.P = param_count(family, d);
    L.nsets = nshifts;
    L.param_stride = 0;
    L.shift_stride = d;
    L.z_stride = 0;
    L.fp32 = precision == QMC_FP32_COMPENSATED;
    L.q_out = q_out;
    L.ws = ws;
    hipError_t e = qmc::launch_lattice_sum(L, (hipStream_t)stream);
    if (e == hipSuccess && stats_out) e = qmc::launch_shift_stats(q_out, nshifts, stats_out, (hipStream_t)stream);
    return from_hip(e, "qmc_lattice_sum_shifts");
}

qmc_status qmc_criteria_workspace_size(int32_t d, int64_t n, size_t* bytes) {
    if (d < 1 || d > kMaxD) return fail(QMC_ERR_INVALID_ARG, "d = %d outside [1, %d]", d, kMaxD);
    if (n < 2 || n >= kMaxN) return fail(QMC_ERR_INVALID_ARG, "n = %lld outside [2, 2^31)", (long long)n);
    if (!bytes) return fail(QMC_ERR_INVALID_ARG, "bytes must be non-NULL");
    *bytes = qmc::criteria_workspace_bytes(d, n);
    return ok();
}

static qmc_status check_criteria(int32_t d, int64_t n, int32_t alpha, const double* a) {
    if (d < 1 || d > kMaxD) return fail(QMC_ERR_INVALID_ARG, "d = %d outside [1, %d]", d, kMaxD);
    if (n < 2 || n >= kMaxN) return fail(QMC_ERR_INVALID_ARG, "n = %lld outside [2, 2^31)", (long long)n);
    if (alpha != 2 && alpha != 4) return fail(QMC_ERR_INVALID_ARG, "alpha = %d is not 2 or 4", alpha);
    if (!a) return fail(QMC_ERR_INVALID_ARG, "a must be non-NULL");
    return QMC_OK;
}

// gamma_j >= 0 (device) is the caller's contract, read back under QMC_VALIDATE.
static qmc_status validate_gamma(const double* gamma, int32_t d, void* stream, const char* what) {
    if (!qmc::validate_mode() || qmc::capturing((hipStream_t)stream)) return QMC_OK;
    size_t j = 0;
    double x = 0.0;
    qmc_status s = qmc::scan_back(gamma, (size_t)d, (hipStream_t)stream, what,
                                  [](double v) { return v >= 0.0 && v < INFINITY; }, &j, &x);
    if (s != QMC_OK) return s;
    if (j < (size_t)d)
        return fail(QMC_ERR_INVALID_ARG, "%s: gamma[%zu] = %g is not a finite weight >= 0 (QMC_VALIDATE)",
                    what, j, x);
    return QMC_OK;
}

// A criterion descriptor: P_alpha (alpha 2 or 4) or e^2 (gamma non-NULL, beta >= 0).
static qmc_status check_criterion(int32_t d, int64_t n, const qmc_criterion* c, void* stream, const char* what,
                                  qmc::CriterionSpec* out) {
    if (d < 1 || d > kMaxD) return fail(QMC_ERR_INVALID_ARG, "d = %d outside [1, %d]", d, kMaxD);
    if (n < 2 || n >= kMaxN) return fail(QMC_ERR_INVALID_ARG, "n = %lld outside [2, 2^31)", (long long)n);
    if (!c) return fail(QMC_ERR_INVALID_ARG, "criterion must be non-NULL");
    if (c->kind == QMC_CRIT_P_ALPHA) {
        if (c->alpha != 2 && c->alpha != 4)
            return fail(QMC_ERR_INVALID_ARG, "alpha = %d is not 2 or 4", c->alpha);
        *out = qmc::CriterionSpec{qmc::kCritPAlpha, c->alpha, nullptr, 0.0};
        return QMC_OK;
    }
    if (c->kind == QMC_CRIT_WCE2) {
        if (!c->gamma) return fail(QMC_ERR_INVALID_ARG, "gamma must be non-NULL for QMC_CRIT_WCE2");
        if (!(c->beta >= 0.0 && c->beta < INFINITY))
            return fail(QMC_ERR_INVALID_ARG, "beta = %g is not finite and >= 0", c->beta);
        qmc_status s = validate_gamma(c->gamma, d, stream, what);
        if (s != QMC_OK) return s;
        *out = qmc::CriterionSpec{qmc::kCritWce2, 2, c->gamma, c->beta};
        return QMC_OK;
    }
    return fail(QMC_ERR_INVALID_ARG, "unknown criterion kind %d", c->kind);
}

static qmc_status criterion_values(int32_t d, int64_t n, const int64_t* z, int32_t nz, const qmc_criterion* crit,
                                   double* out, void* ws, size_t ws_bytes, void* stream, const char* what) {
    qmc::CriterionSpec spec{};
    qmc_status s = check_criterion(d, n, crit, stream, what, &spec);
    if (s != QMC_OK) return s;
    if (nz < 1 || nz > kMaxSets) return fail(QMC_ERR_INVALID_ARG, "nz = %d outside [1, %d]", nz, kMaxSets);
    if (!z || !out) return fail(QMC_ERR_INVALID_ARG, "z and the output must be non-NULL");
    s = check_workspace(ws, ws_bytes, qmc::criteria_workspace_bytes(d, n));
    if (s != QMC_OK) return s;
    if ((s = validate_z(z, (size_t)nz * (size_t)d, n, stream, what)) != QMC_OK) return s;
    qmc::CriterionLaunch L{d, (uint32_t)n, z, nz, spec, out, ws};
    return from_hip(qmc::launch_criterion(L, (hipStream_t)stream), what);
}

qmc_status qmc_bernoulli_sum(int32_t d, int64_t n, const int64_t* z, int32_t nz, int32_t alpha,
                             const double* a, double* s_out, void* ws, size_t ws_bytes,
                             void* stream) {
    qmc_status s = check_criteria(d, n, alpha, a);
    if (s != QMC_OK) return s;
    if (nz < 1 || nz > kMaxSets) return fail(QMC_ERR_INVALID_ARG, "nz = %d outside [1, %d]", nz, kMaxSets);
    if (!z || !s_out) return fail(QMC_ERR_INVALID_ARG, "z and s_out must be non-NULL");
    s = check_workspace(ws, ws_bytes, qmc::plain_workspace_bytes(nz));
    if (s != QMC_OK) return s;
    if ((s = validate_z(z, (size_t)nz * (size_t)d, n, stream, "qmc_bernoulli_sum")) != QMC_OK) return s;
    qmc::BernoulliLaunch L{d, (uint32_t)n, z, nz, alpha, a, s_out, ws};
    return from_hip(qmc::launch_bernoulli_sum(L, (hipStream_t)stream), "qmc_bernoulli_sum");
}

qmc_status qmc_p_alpha(int32_t d, int64_t n, const int64_t* z, int32_t nz, int32_t alpha, double* p_out,
                       void* ws, size_t ws_bytes, void* stream) {
    const qmc_criterion c{QMC_CRIT_P_ALPHA, alpha, nullptr, 0.0};
    return criterion_values(d, n, z, nz, &c, p_out, ws, ws_bytes, stream, "qmc_p_alpha");
}

qmc_status qmc_shift_avg_wce2(int32_t d, int64_t n, const int64_t* z, int32_t nz, const double* gamma,
                              double beta, double* e2_out, void* ws, size_t ws_bytes, void* stream) {
    const qmc_criterion c{QMC_CRIT_WCE2, 2, gamma, beta};
    return criterion_values(d, n, z, nz, &c, e2_out, ws, ws_bytes, stream, "qmc_shift_avg_wce2");
}

qmc_status qmc_korobov_search(int32_t d, int64_t n, const qmc_criterion* crit, int64_t a0,
                              int32_t count, double* s_out, double* best_out, void* ws,
                              size_t ws_bytes, void* stream) {
    qmc::CriterionSpec spec{};
    qmc_status s = check_criterion(d, n, crit, stream, "qmc_korobov_search", &spec);
    if (s != QMC_OK) return s;
    if (a0 < 1 || count < 1 || a0 + (int64_t)count > n)
        return fail(QMC_ERR_INVALID_ARG, "candidates [%lld, %lld) outside [1, n)", (long long)a0,
                    (long long)(a0 + count));
    if (!s_out || !best_out) return fail(QMC_ERR_INVALID_ARG, "s_out and best_out must be non-NULL");
    s = check_workspace(ws, ws_bytes, qmc::criteria_workspace_bytes(d, n));
    if (s != QMC_OK) return s;
    qmc::SearchLaunch L{d, (uint32_t)n, spec, a0, count, s_out, best_out, ws};
    return from_hip(qmc::launch_korobov_search(L, (hipStream_t)stream), "qmc_korobov_search");
}

qmc_status qmc_cbc(int32_t d, int64_t n, const qmc_criterion* crit, int64_t* z_out,
                   double* s_out, void* ws, size_t ws_bytes, void* stream) {
    qmc::CriterionSpec spec{};
    qmc_status s = check_criterion(d, n, crit, stream, "qmc_cbc", &spec);
    if (s != QMC_OK) return s;
    if (n > kMaxCbcN) return fail(QMC_ERR_INVALID_ARG, "n = %lld above the CBC limit 2^26", (long long)n);
    if (!z_out || !s_out) return fail(QMC_ERR_INVALID_ARG, "z_out and s_out must be non-NULL");
    s = check_workspace(ws, ws_bytes, qmc::criteria_workspace_bytes(d, n));
    if (s != QMC_OK) return s;
    qmc::CbcLaunch L{d, (uint32_t)n, spec, z_out, s_out, ws};
    return from_hip(qmc::launch_cbc(L, (hipStream_t)stream), "qmc_cbc");
}

static qmc_status check_mdi_sum(int32_t d, int32_t N, int32_t N_last, int32_t gfamily) {
    if (d < 1 || d > kMaxD) return fail(QMC_ERR_INVALID_ARG, "d = %d outside [1, %d]", d, kMaxD);
    if (N < 1 || N > kMaxSumNodes) return fail(QMC_ERR_INVALID_ARG, "N = %d outside [1, %d]", N, kMaxSumNodes);
    if (N_last < 1 || N_last > kMaxSumNodes)
        return fail(QMC_ERR_INVALID_ARG, "N_last = %d outside [1, %d]", N_last, kMaxSumNodes);
    if ((int64_t)d * (N - 1) + 1 > kMaxSumStates)
        return fail(QMC_ERR_INVALID_ARG, "d (N - 1) + 1 states above 2^20");
    if (gfamily != QMC_SUM_POWER && gfamily != QMC_SUM_GAUSS)
        return fail(QMC_ERR_INVALID_ARG, "unknown sum family %d", gfamily);
    return QMC_OK;
}

qmc_status qmc_mdi_lr_sum_workspace_size(int32_t d, int32_t N, size_t* bytes) {
    qmc_status s = check_mdi_sum(d, N, 1, QMC_SUM_POWER);
    if (s != QMC_OK) return s;
    if (!bytes) return fail(QMC_ERR_INVALID_ARG, "bytes must be non-NULL");
    *bytes = qmc::mdi_sum_workspace_bytes(d, N);
    return ok();
}

qmc_status qmc_mdi_lr_sum(int32_t d, int32_t N, int32_t N_last, int32_t gfamily, const double* params,
                          int32_t nsets, int32_t precision, double* q_out, void* ws, size_t ws_bytes,
                          void* stream) {
    qmc_status s = check_mdi_sum(d, N, N_last, gfamily);
    if (s != QMC_OK) return s;
    if (nsets < 1 || nsets > kMaxMdiSets)
        return fail(QMC_ERR_INVALID_ARG, "nsets = %d outside [1, %d]", nsets, kMaxMdiSets);
    if (precision != QMC_FP64 && precision != QMC_FP32_COMPENSATED)
        return fail(QMC_ERR_INVALID_ARG, "unknown precision %d", precision);
    if (!params || !q_out) return fail(QMC_ERR_INVALID_ARG, "params and q_out must be non-NULL");
    s = check_workspace(ws, ws_bytes, qmc::mdi_sum_workspace_bytes(d, N));
    if (s != QMC_OK) return s;
    qmc::MdiSumLaunch L{d, N, N_last, gfamily, params, gfamily == QMC_SUM_POWER ? 3 : 2, nsets,
                        precision == QMC_FP32_COMPENSATED, q_out, ws};
    return from_hip(qmc::launch_mdi_sum(L, (hipStream_t)stream), "qmc_mdi_lr_sum");
}

// Korobov lattice with a^{d-1} < n: per-direction counts (eq. 3.5) and grid size.
static qmc_status implr_shape(int32_t d, int64_t n, int64_t a, int64_t* counts, uint64_t* grid,
                              int64_t* zd_out = nullptr) {
    if (d < 1 || d > 64) return fail(QMC_ERR_INVALID_ARG, "d = %d outside [1, 64]", d);
    if (n < 2 || n >= kMaxN) return fail(QMC_ERR_INVALID_ARG, "n = %lld outside [2, 2^31)", (long long)n);
    if (a < 1 || a >= n) return fail(QMC_ERR_INVALID_ARG, "a = %lld outside [1, n)", (long long)a);
    int64_t zd = 1;
    for (int i = 0; i + 1 < d; ++i) {
        if (zd > (n - 1) / a) return fail(QMC_ERR_INVALID_ARG, "a^(d-1) must be below n");
        zd *= a;
    }
    for (int i = 0; i + 1 < d; ++i)
        if (counts) counts[i] = a;
    const int64_t nd = (n + zd - 1) / zd;
    if (counts) counts[d - 1] = nd;
    *grid = (uint64_t)zd * (uint64_t)nd;
    if (zd_out) *zd_out = zd;
    return QMC_OK;
}

qmc_status qmc_implr_workspace_size(int32_t d, int64_t n, int64_t a, size_t* bytes) {
    uint64_t grid = 0;
    qmc_status s = implr_shape(d, n, a, nullptr, &grid);
    if (s != QMC_OK) return s;
    if (!bytes) return fail(QMC_ERR_INVALID_ARG, "bytes must be non-NULL");
    *bytes = qmc::implr_workspace_bytes(grid);
    return ok();
}

qmc_status qmc_implr_grid(int32_t d, int64_t n, int64_t a, int32_t method, int64_t* counts_host_out,
                          int64_t* nstar_out, void* ws, size_t ws_bytes, void* stream) {
    uint64_t grid = 0;
    int64_t zd = 0;
    qmc_status s = implr_shape(d, n, a, nullptr, &grid, &zd);
    if (s != QMC_OK) return s;
    if (method != QMC_IMPLR_AUTO && method != QMC_IMPLR_BITMAP)
        return fail(QMC_ERR_INVALID_ARG, "method = %d is not a qmc_implr_method", method);
    if (!nstar_out) return fail(QMC_ERR_INVALID_ARG, "nstar_out must be non-NULL");
    s = check_workspace(ws, ws_bytes, qmc::implr_workspace_bytes(grid));
    if (s != QMC_OK) return s;
    if (counts_host_out) implr_shape(d, n, a, counts_host_out, &grid);
    qmc::ImplrLaunch L{d, (uint32_t)n, (uint32_t)a, (uint32_t)zd, (uint32_t)((n + zd - 1) / zd), grid,
                       method == QMC_IMPLR_BITMAP, nstar_out, ws};
    return from_hip(qmc::launch_implr(L, (hipStream_t)stream), "qmc_implr_grid");
}

qmc_status qmc_implr_points(int32_t d, int64_t n, int64_t a, int64_t j0, int64_t count, int32_t* s_out,
                            int64_t ld, void* stream) {
    uint64_t grid = 0;
    int64_t zd = 0;
    qmc_status s = implr_shape(d, n, a, nullptr, &grid, &zd);
    if (s != QMC_OK) return s;
    if (j0 < 0 || count < 0 || j0 > n - count)
        return fail(QMC_ERR_INVALID_ARG, "points [%lld, %lld + %lld) outside [0, n)", (long long)j0,
                    (long long)j0, (long long)count);
    if (count > 0 && !s_out) return fail(QMC_ERR_INVALID_ARG, "s_out must be non-NULL");
    if (ld < count) return fail(QMC_ERR_INVALID_ARG, "ld = %lld below count = %lld", (long long)ld, (long long)count);
    // (d - 1) ld + count elements must be addressable; no device buffer comes near 2^40
    if (ld > kMaxImplrLd) return fail(QMC_ERR_INVALID_ARG, "ld = %lld above 2^40", (long long)ld);
    if ((uintptr_t)s_out % 4 != 0) return fail(QMC_ERR_INVALID_ARG, "s_out must be 4-byte aligned");
    qmc::ImplrPointsLaunch L{d, (uint32_t)n, (uint32_t)a, (uint32_t)zd, (uint64_t)j0, (uint64_t)count, (uint64_t)ld,
                             s_out};
    return from_hip(qmc::launch_implr_points(L, (hipStream_t)stream), "qmc_implr_points");
}

qmc_status qmc_lattice_points(int32_t d, int64_t n, const int64_t* z, int64_t i0, int64_t count,
                              int32_t* k_out, void* stream) {
    if (d < 1 || d > kMaxD) return fail(QMC_ERR_INVALID_ARG, "d = %d outside [1, %d]", d, kMaxD);
    if (n < 1 || n >= kMaxN) return fail(QMC_ERR_INVALID_ARG, "n = %lld outside [1, 2^31)", (long long)n);
    if (i0 < 0 || i0 >= kMaxN) return fail(QMC_ERR_INVALID_ARG, "i0 outside [0, 2^31)");
    if (count < 0 || count > kMaxExport) return fail(QMC_ERR_INVALID_ARG, "count outside [0, 2^26]");
    if (!z || (!k_out && count > 0)) return fail(QMC_ERR_INVALID_ARG, "z and k_out must be non-NULL");
    qmc_status s = validate_z(z, (size_t)d, n, stream, "qmc_lattice_points");
    if (s != QMC_OK) return s;
    return from_hip(qmc::launch_lattice_points(d, (uint32_t)n, z, i0, count, k_out, (hipStream_t)stream),
                    "qmc_lattice_points");
}

qmc_status qmc_mdi_lr(int32_t d, const int32_t* N, int32_t family, const double* params,
                      int32_t nsets, int32_t precision, double* q_out, void* ws, size_t ws_bytes,
                      void* stream) {
    (void)ws;
    (void)ws_bytes;  // the sweep needs no scratch space
    qmc_status s = check_common(d, family, nsets, precision, kMaxMdiSets);
    if (s != QMC_OK) return s;
    if (!N || !params || !q_out) return fail(QMC_ERR_INVALID_ARG, "N, params and q_out must be non-NULL");
    if (qmc::validate_mode() && !qmc::capturing((hipStream_t)stream)) {
        size_t k = 0;
        int32_t x = 0;
        s = qmc::scan_back(N, (size_t)d, (hipStream_t)stream, "qmc_mdi_lr",
                           [](int32_t v) { return v >= 1 && v <= kMaxNodes; }, &k, &x);
        if (s != QMC_OK) return s;
        if (k < (size_t)d)
            return fail(QMC_ERR_INVALID_ARG, "qmc_mdi_lr: N[%zu] = %d outside [1, 2^20] (QMC_VALIDATE)", k, x);
    }
    qmc::MdiLaunch L{};
    L.d = d;
    L.N = N;
    L.family = family;
    L.params = params;
    L.P = param_count(family, d);
    L.nsets = nsets;
    L.fp32 = precision == QMC_FP32_COMPENSATED;
    L.q_out = q_out;
    return from_hip(qmc::launch_mdi_lr(L, (hipStream_t)stream), "qmc_mdi_lr");
}

}  // extern "C"
