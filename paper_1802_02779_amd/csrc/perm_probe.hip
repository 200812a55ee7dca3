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

// ------------------------------------------------------------ integer
// The integer sweep's arithmetic per term: a 64 x 64 -> 128-bit product
// added to a 128-bit sum (residue layers), folded mod p = 2^61 - c once per
// stored value; or a plain 64-bit addition (0/1 rows, plain layers).  Every
// lane runs kProbeChains independent sums; mode 0 folds each after 16
// products (about the terms of one stored value at n = 30), mode 1 adds.
namespace permgpu {

__device__ __forceinline__ uint64_t probe_fold61(unsigned __int128 x, uint64_t p) {
    const uint64_t M = (1ull << 61) - 1;
    const uint64_t c = (1ull << 61) - p;
    const unsigned __int128 y = (unsigned __int128)((uint64_t)x & M) + (unsigned __int128)c * (x >> 61);
    uint64_t z = ((uint64_t)y & M) + c * (uint64_t)(y >> 61);
    if (z >= p) z -= p;
    if (z >= p) z -= p;
    return z;
}

__global__ __launch_bounds__(kProbeBlock) void k_probe_int(uint64_t *out, int iters, int mode, uint64_t p,
                                                           uint64_t m) {
    uint64_t x[kProbeChains];
#pragma unroll
    for (int j = 0; j < kProbeChains; j++) x[j] = (uint64_t)(threadIdx.x * 7919u + j * 104729u) + p / 3;
    if (mode == 0) {
        for (int i = 0; i < iters; i++) {
#pragma unroll
            for (int j = 0; j < kProbeChains; j++) {
                unsigned __int128 acc = 0;
                uint64_t v = x[j];
#pragma unroll
                for (int t = 0; t < 16; t++) {
                    acc += (unsigned __int128)m * v;
                    v = (uint64_t)acc ^ (uint64_t)t;  // the next operand depends on the sum
                }
                x[j] = probe_fold61(acc, p);
            }
        }
    } else {
        for (int i = 0; i < iters; i++) {
#pragma unroll
            for (int t = 0; t < 16; t++) {
#pragma unroll
                for (int j = 0; j < kProbeChains; j++) x[j] += x[(j + 1) % kProbeChains];
            }
        }
    }
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < kProbeChains; j++) s ^= x[j];
    if (s == 0x123456789abcdefull) out[blockIdx.x] = s;
}

hipError_t launch_probe_int(uint64_t *out, int blocks, int iters, int mode, hipStream_t s) {
    const uint64_t p = (1ull << 61) - 1;
    hipLaunchKernelGGL(k_probe_int, dim3(blocks), dim3(kProbeBlock), 0, s, out, iters, mode, p,
                       (uint64_t)0x1d2c3b4a59687f01ull % p);
    return hipGetLastError();
}

// Terms (products with their 128-bit additions, or 64-bit additions) of one launch.
double probe_int_terms(int blocks, int iters) { return 16.0 * kProbeChains * (double)iters * (double)blocks * kProbeBlock; }

}  // namespace permgpu
