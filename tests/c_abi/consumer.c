/* A plain C consumer of libqmc.so: the HIP runtime API for device memory and a
 * stream, the C ABI of include/qmc.h for the computation, no Python and no torch.
 * It evaluates fixed problems and prints one "name value" line per result for the
 * GPU test that compares them with the FP64 oracle:
 *   - the Korobov vector z(a) for d = 4, n = 1009, a = 76 (qmc_korobov);
 *   - the plain rule (eq. 1.2, eq. 2.1) for the exponential of c . x on that lattice,
 *     c = (0.3, 0.6, 0.9, 1.2), in QMC_FP64 and QMC_FP32_COMPENSATED;
 *   - MDI-LR (Algorithm 2) for the Gaussian family, d = 3, N = (5, 6, 7),
 *     c = (0.5, 0.8, 1.1), w = (0.2, 0.5, 0.7), in QMC_FP64.
 * Exit status 0 on success, 2 on a HIP error, 3 on a library error. */
#include <stdio.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#include "qmc.h"

#define CHECK_HIP(x)                                                              \
    do {                                                                          \
        hipError_t e_ = (x);                                                      \
        if (e_ != hipSuccess) {                                                   \
            fprintf(stderr, "%s: HIP error %d\n", #x, (int)e_);                   \
            return 2;                                                             \
        }                                                                         \
    } while (0)
#define CHECK_QMC(x)                                                              \
    do {                                                                          \
        qmc_status s_ = (x);                                                      \
        if (s_ != QMC_OK) {                                                       \
            fprintf(stderr, "%s: %s (%s)\n", #x, qmc_status_string(s_), qmc_last_error()); \
            return 3;                                                             \
        }                                                                         \
    } while (0)

int main(void) {
    enum { D = 4, MD = 3 };
    const int64_t n = 1009, a = 76;
    int64_t z[D];
    CHECK_QMC(qmc_korobov(D, n, a, z));
    printf("korobov");
    for (int j = 0; j < D; ++j) printf(" %lld", (long long)z[j]);
    printf("\n");

    const double c[D] = {0.3, 0.6, 0.9, 1.2};
    size_t ws_bytes = 0;
    CHECK_QMC(qmc_workspace_size(D, n, 1, &ws_bytes));
    hipStream_t stream;
    CHECK_HIP(hipStreamCreate(&stream));
    int64_t* dz = NULL;
    double *dc = NULL, *dq = NULL;
    void* ws = NULL;
    CHECK_HIP(hipMalloc((void**)&dz, sizeof z));
    CHECK_HIP(hipMalloc((void**)&dc, sizeof c));
    CHECK_HIP(hipMalloc((void**)&dq, sizeof(double)));
    CHECK_HIP(hipMalloc(&ws, ws_bytes));
    CHECK_HIP(hipMemset(ws, 0, ws_bytes));  /* the zero region starts zero */
    CHECK_HIP(hipMemcpy(dz, z, sizeof z, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(dc, c, sizeof c, hipMemcpyHostToDevice));
    const int32_t precs[2] = {QMC_FP64, QMC_FP32_COMPENSATED};
    const char* names[2] = {"lattice_sum_fp64", "lattice_sum_fp32c"};
    for (int p = 0; p < 2; ++p) {
        double q = 0.0;
        CHECK_QMC(qmc_lattice_sum(D, n, dz, NULL, QMC_EXP_SUM, dc, 1, precs[p], dq, ws, ws_bytes,
                                  (void*)stream));
        CHECK_HIP(hipMemcpyAsync(&q, dq, sizeof q, hipMemcpyDeviceToHost, stream));
        CHECK_HIP(hipStreamSynchronize(stream));
        printf("%s %.17g\n", names[p], q);
    }

    const int32_t N[MD] = {5, 6, 7};
    const double gp[2 * MD] = {0.5, 0.8, 1.1, 0.2, 0.5, 0.7};  /* c[d], then w[d] */
    int32_t* dN = NULL;
    double* dgp = NULL;
    CHECK_HIP(hipMalloc((void**)&dN, sizeof N));
    CHECK_HIP(hipMalloc((void**)&dgp, sizeof gp));
    CHECK_HIP(hipMemcpy(dN, N, sizeof N, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(dgp, gp, sizeof gp, hipMemcpyHostToDevice));
    double qm = 0.0;
    CHECK_QMC(qmc_mdi_lr(MD, dN, QMC_GAUSSIAN, dgp, 1, QMC_FP64, dq, NULL, 0, (void*)stream));
    CHECK_HIP(hipMemcpyAsync(&qm, dq, sizeof qm, hipMemcpyDeviceToHost, stream));
    CHECK_HIP(hipStreamSynchronize(stream));
    printf("mdi_lr_fp64 %.17g\n", qm);

    CHECK_HIP(hipFree(dz));
    CHECK_HIP(hipFree(dc));
    CHECK_HIP(hipFree(dq));
    CHECK_HIP(hipFree(ws));
    CHECK_HIP(hipFree(dN));
    CHECK_HIP(hipFree(dgp));
    CHECK_HIP(hipStreamDestroy(stream));
    return 0;
}
