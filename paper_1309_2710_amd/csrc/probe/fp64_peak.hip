// FP64 vector FMA throughput probe for the roofline's peak: every lane runs
// CHAINS independent FMA chains of `iters` steps (a <- a * b + c), so the
// dependent latency of one chain is covered by the others and by the other
// waves of the SIMD.  Built into its own library (librkc_probe.so), used by
// bench.py --peak; it is not part of the integrator's ABI.
#include <hip/hip_runtime.h>

namespace {

constexpr int CHAINS = 16;

__global__ __launch_bounds__(256) void fma_chains(double *out, int iters, double b, double c) {
    double a[CHAINS];
#pragma unroll
    for (int k = 0; k < CHAINS; ++k) a[k] = (double)(threadIdx.x + k) * 1e-3;
#pragma unroll 8
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < CHAINS; ++k) a[k] = __builtin_fma(a[k], b, c);
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < CHAINS; ++k) s += a[k];
    if (s == 12345.678) out[blockIdx.x] = s;   // keeps the chains live; never true in practice
}

}  // namespace

// Runs `blocks` workgroups of 256 lanes, `iters` steps of CHAINS FMAs per
// lane, after one untimed launch; returns 0 and the FP64 flops per second
// (2 per FMA) of the timed launch, or a negative value on a HIP error.
extern "C" int rkc_probe_fp64_fma(int blocks, int iters, double *flops_per_s, float *ms) {
    double *out = nullptr;
    if (hipMalloc(&out, sizeof(double) * (size_t)blocks) != hipSuccess) return -2;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipFree(out);
        return -3;
    }
    int rc = 0;
    const double b = 0.999999999, c = 1e-9;
    hipLaunchKernelGGL(fma_chains, dim3(blocks), dim3(256), 0, 0, out, iters, b, c);
    if (hipEventRecord(e0, 0) != hipSuccess) rc = -3;
    hipLaunchKernelGGL(fma_chains, dim3(blocks), dim3(256), 0, 0, out, iters, b, c);
    if (hipGetLastError() != hipSuccess || hipEventRecord(e1, 0) != hipSuccess ||
        hipEventSynchronize(e1) != hipSuccess)
        rc = -3;
    float t = 0.0f;
    if (rc == 0 && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = -3;
    if (rc == 0) {
        *ms = t;
        *flops_per_s = 2.0 * CHAINS * (double)iters * 256.0 * (double)blocks / (t * 1e-3);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    return rc;
}
