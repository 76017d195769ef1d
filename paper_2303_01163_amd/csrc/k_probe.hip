// Ceilings of the machine measured on the device itself (the roofline's denominators next to the
// datasheet figures): the FP64 MFMA rate of back-to-back v_mfma_f64_16x16x4f64 on every SIMD, and
// the HBM rate of a streaming copy.  Calibration only; the solver does not call them.
#include <functional>

#include "device_common.hpp"
#include "kernels.hpp"

namespace asdsm {

// Every wave runs `iters` rounds of eight independent MFMA chains (enough to keep the matrix pipe
// busy); the accumulators are summed into out so that nothing is optimised away.
__global__ __launch_bounds__(256) void k_probe_mfma_f64(double *out, int iters, double seed) {
    const int lane = threadIdx.x & 63;
    const double a = seed + 1e-3 * lane, b = seed - 1e-3 * lane;
    double4_t c[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) c[q] = double4_t{0.0, 0.0, 0.0, 0.0};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int q = 0; q < 8; ++q) c[q] = __builtin_amdgcn_mfma_f64_16x16x4f64((q & 1) ? a : b, (q & 2) ? a : b, c[q], 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) s += c[q][q & 3];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Streaming copy: four 16-byte loads in flight per thread, then their stores; non-temporal
// accesses (the data are touched once).
typedef double dbl2_t __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(256) void k_probe_copy(const dbl2_t *__restrict__ src, dbl2_t *__restrict__ dst,
                                                    long long n2) {
    const long long step = (long long)gridDim.x * 256;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n2; i += 4 * step) {
        dbl2_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i + u * step < n2) v[u] = __builtin_nontemporal_load(src + i + u * step);
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i + u * step < n2) __builtin_nontemporal_store(v[u], dst + i + u * step);
    }
}

constexpr int kProbeBlocks = 256 * 8;  // 8 blocks of 4 waves per CU: every SIMD can switch waves
size_t probe_mfma_scratch_bytes() { return (size_t)kProbeBlocks * 256 * sizeof(double); }

static int time_launches(hipStream_t st, int reps, float *ms, const std::function<void()> &launch) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = ASDSM_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = ASDSM_E_DEVICE;
    if (rc == ASDSM_OK) {
        launch();  // warm-up
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < reps; ++r) launch();
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(ms, e0, e1) != hipSuccess)
            rc = ASDSM_E_DEVICE;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return rc;
}

int probe_mfma_f64(double *scratch, int iters, hipStream_t st, double *tflops) {
    float ms = 0.f;
    const int rc = time_launches(st, 1, &ms, [&] {
        hipLaunchKernelGGL(k_probe_mfma_f64, dim3(kProbeBlocks), dim3(256), 0, st, scratch, iters, 1.0);
    });
    if (rc != ASDSM_OK) return rc;
    // 16 x 16 x 4 multiply-adds per MFMA, eight per round, issued by each wave of 64 lanes
    const double flops = 2.0 * 16 * 16 * 4 * 8.0 * iters * ((double)kProbeBlocks * 256 / 64);
    *tflops = flops / (ms * 1e-3) / 1e12;
    return ASDSM_OK;
}

int probe_copy(const double *src, double *dst, size_t bytes, int reps, hipStream_t st, double *tbps) {
    const long long n2 = (long long)(bytes / 16);
    float ms = 0.f;
    const int rc = time_launches(st, reps, &ms, [&] {
        hipLaunchKernelGGL(k_probe_copy, dim3(256 * 8), dim3(256), 0, st, (const dbl2_t *)src, (dbl2_t *)dst, n2);
    });
    if (rc != ASDSM_OK) return rc;
    *tbps = 2.0 * (double)(n2 * 16) * reps / (ms * 1e-3) / 1e12;  // read + write
    return ASDSM_OK;
}

}  // namespace asdsm
