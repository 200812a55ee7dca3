// Measurement probe (part of the device translation unit perm_device.hip):
// the FP64 fused-multiply-add rate the chip sustains on independent chains,
// the measured counterpart of the spec-sheet FP64 vector peak.
namespace permgpu {

constexpr int kProbeBlock = 256;
constexpr int kProbeChains = 8;

// Every lane runs kProbeChains independent chains x <- x * m + c; the sum is
// written only under a condition that never holds for these inputs, which
// keeps the chains live without a store per lane.
__global__ __launch_bounds__(kProbeBlock) void k_probe_fma(double *out, int iters, double m, double c) {
    double x[kProbeChains];
#pragma unroll
    for (int j = 0; j < kProbeChains; j++) x[j] = 1e-3 * (double)(threadIdx.x + j);
    for (int i = 0; i < iters; i++) {
#pragma unroll
        for (int j = 0; j < kProbeChains; j++) x[j] = __builtin_fma(x[j], m, c);
    }
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kProbeChains; j++) s += x[j];
    if (s == -1.0) out[blockIdx.x] = s;
}

hipError_t launch_probe_fma(double *out, int blocks, int iters, hipStream_t s) {
    hipLaunchKernelGGL(k_probe_fma, dim3(blocks), dim3(kProbeBlock), 0, s, out, iters, 0.999999, 1e-7);
    return hipGetLastError();
}

double probe_fma_flops(int blocks, int iters) {
    return 2.0 * kProbeChains * (double)iters * (double)blocks * kProbeBlock;
}

}  // namespace permgpu
