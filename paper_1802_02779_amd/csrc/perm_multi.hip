// Repeated columns: the stored-minor sweep over count vectors (part of the
// device translation unit perm_device.hip).
//
// Column j of the n x m input stands for mult[j] identical columns.  Every
// column subset with c_j copies of column j has the same minor, so layer k
// stores one value per count vector c (|c| = k, 0 <= c_j <= mult[j]):
//     G(c) = sum over j ascending with c_j > 0 of a[k-1][j] * G(c - e_j),
// the section-4 development along the last row with the repeating terms
// merged.  One launch per layer; a workgroup computes 256 consecutive ranks.
// Predecessors of an output in tile h (see perm_multi.h):
//   * low column i: the tile h of layer k-1, at the rank lowpred gives --
//     a gather inside one contiguous window;
//   * high column j: the tile h - e_j of layer k-1 at the same offset -- a
//     coalesced read of an aligned window.
// The chain visits the low columns, then the high windows, both ascending,
// so the terms come in ascending column order as the definition states.
#include "perm_multi.h"

namespace permgpu {

__global__ void k_multi_pack_c128(const double2 *__restrict__ a, int64_t lda, int n, int m,
                                  double2 *__restrict__ packed, double2 *__restrict__ layer1) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * m) return;
    const int i = e / m, j = e - i * m;
    const double2 v = a[(int64_t)i * lda + j];
    packed[e] = v;
    if (i == 0) layer1[j] = v;  // G(e_j) = a[0][j]; e_j has rank j in layer 1
}

hipError_t launch_multi_pack_c128(const void *a_dev, int64_t lda, int n, int m, void *packed, void *layer1,
                                  hipStream_t s) {
    const int tot = n * m;
    hipLaunchKernelGGL(k_multi_pack_c128, dim3((tot + 255) / 256), dim3(256), 0, s, (const double2 *)a_dev, lda, n,
                       m, (double2 *)packed, (double2 *)layer1);
    return hipGetLastError();
}

// Tile of this workgroup's outputs: the tiles overlapping the chunk go to
// LDS (at most kMultiBlock + 1 of them, plus the next one for the window
// end); each lane finds its own by binary search.
__device__ __forceinline__ uint32_t multi_stage_tiles(const MultiLayerArgs &g, uint4 *s_tile) {
    const uint32_t c = blockIdx.x;
    const uint32_t t0 = g.chunk_tile[c];
    const uint32_t nt = g.chunk_tile[c + 1] - t0 + 1;
    for (uint32_t i = threadIdx.x; i <= nt; i += kMultiBlock) s_tile[i] = g.tiles[t0 + i];
    return nt;
}

__device__ __forceinline__ uint32_t multi_find_tile(const uint4 *s_tile, uint32_t nt, uint32_t out) {
    uint32_t lo = 0, hi = nt - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (s_tile[mid].x <= out) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kMultiBlock) void k_multi_layer_c128(const double2 *__restrict__ prev,
                                                                 double2 *__restrict__ next,
                                                                 const double2 *__restrict__ row,
                                                                 const MultiLayerArgs g) {
    __shared__ uint4 s_tile[kMultiBlock + 2];
    __shared__ double2 s_row[kMultiMMax];
    const uint32_t nt = multi_stage_tiles(g, s_tile);
    for (int j = threadIdx.x; j < g.m; j += kMultiBlock) s_row[j] = row[j];
    __syncthreads();
    const uint32_t out = blockIdx.x * kMultiBlock + threadIdx.x;
    if (out >= g.size) return;
    const uint32_t ti = multi_find_tile(s_tile, nt, out);
    const uint4 T = s_tile[ti];
    const uint32_t wend = s_tile[ti + 1].w;
    const uint32_t r = out - T.x;
    double re = 0.0, im = 0.0;
    if (T.y > 0) {
        const uint32_t v = g.lowlist[g.lowoff[T.y] + r];
        const uint32_t *pred = g.lowpred + (size_t)v * g.L;
        for (int i = 0; i < g.L; i++) {
            const uint32_t q = pred[i];
            if (q != 0xffffffffu) cfma(re, im, s_row[i], prev[T.z + q]);
        }
    }
    for (uint32_t w = T.w; w < wend; w++) {
        const uint2 W = g.wins[w];
        cfma(re, im, s_row[W.y], prev[W.x + r]);
    }
    next[out] = make_double2(re, im);
}

hipError_t launch_multi_layer_c128(const void *prev, void *next, const void *row, const MultiLayerArgs &g,
                                   hipStream_t s) {
    hipLaunchKernelGGL(k_multi_layer_c128, dim3(g.nchunks), dim3(kMultiBlock), 0, s, (const double2 *)prev,
                       (double2 *)next, (const double2 *)row, g);
    return hipGetLastError();
}

// per = G(mult) * scale, scale = prod_j mult[j]! formed in double on the host.
__global__ void k_multi_readout_c128(const double2 *__restrict__ last, double scale, double2 *__restrict__ out) {
    if (threadIdx.x == 0) *out = make_double2(last[0].x * scale, last[0].y * scale);
}

hipError_t launch_multi_readout_c128(const void *last, double scale, void *out, hipStream_t s) {
    hipLaunchKernelGGL(k_multi_readout_c128, dim3(1), dim3(64), 0, s, (const double2 *)last, scale, (double2 *)out);
    return hipGetLastError();
}

// ------------------------------------------------------------- mod p
__global__ void k_multi_init_modp(const uint64_t *__restrict__ red, int n, int m, int rp,
                                  uint64_t *__restrict__ layer1, size_t plane) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rp * m) return;
    const int r = e / m, j = e - r * m;
    layer1[(size_t)r * plane + j] = red[(size_t)r * n * m + j];
}

hipError_t launch_multi_init_modp(const uint64_t *red, int n, int m, int rp, uint64_t *layer1, size_t plane,
                                  hipStream_t s) {
    hipLaunchKernelGGL(k_multi_init_modp, dim3((rp * m + 255) / 256), dim3(256), 0, s, red, n, m, rp, layer1,
                       plane);
    return hipGetLastError();
}

// Residues of a[k-1][*] for RP primes; each output sums at most m <= 64
// products below 2^122 exactly in 128 bits, then one fold.
template <int RP>
__global__ __launch_bounds__(kMultiBlock) void k_multi_layer_modp(const uint64_t *__restrict__ prev,
                                                                 uint64_t *__restrict__ next, size_t plane,
                                                                 const uint64_t *__restrict__ red, int n, int k,
                                                                 const uint64_t *__restrict__ primes,
                                                                 const MultiLayerArgs g) {
    __shared__ uint4 s_tile[kMultiBlock + 2];
    __shared__ uint64_t s_row[RP][kMultiMMax];
    const uint32_t nt = multi_stage_tiles(g, s_tile);
    for (int e = threadIdx.x; e < RP * g.m; e += kMultiBlock) {
        const int r = e / g.m, j = e - r * g.m;
        s_row[r][j] = red[(size_t)r * n * g.m + (size_t)(k - 1) * g.m + j];
    }
    __syncthreads();
    const uint32_t out = blockIdx.x * kMultiBlock + threadIdx.x;
    if (out >= g.size) return;
    const uint32_t ti = multi_find_tile(s_tile, nt, out);
    const uint4 T = s_tile[ti];
    const uint32_t wend = s_tile[ti + 1].w;
    const uint32_t rr = out - T.x;
    u128 acc[RP];
#pragma unroll
    for (int r = 0; r < RP; r++) acc[r] = 0;
    if (T.y > 0) {
        const uint32_t v = g.lowlist[g.lowoff[T.y] + rr];
        const uint32_t *pred = g.lowpred + (size_t)v * g.L;
        for (int i = 0; i < g.L; i++) {
            const uint32_t q = pred[i];
            if (q == 0xffffffffu) continue;
#pragma unroll
            for (int r = 0; r < RP; r++) acc[r] += (u128)s_row[r][i] * prev[(size_t)r * plane + T.z + q];
        }
    }
    for (uint32_t w = T.w; w < wend; w++) {
        const uint2 W = g.wins[w];
#pragma unroll
        for (int r = 0; r < RP; r++) acc[r] += (u128)s_row[r][W.y] * prev[(size_t)r * plane + W.x + rr];
    }
#pragma unroll
    for (int r = 0; r < RP; r++) next[(size_t)r * plane + out] = fold61(acc[r], primes[r]);
}

hipError_t launch_multi_layer_modp(const uint64_t *prev, uint64_t *next, size_t plane, const uint64_t *red, int n,
                                   int k, const uint64_t *primes, int rp, const MultiLayerArgs &g, hipStream_t s) {
    switch (rp) {
    case 1:
        hipLaunchKernelGGL(k_multi_layer_modp<1>, dim3(g.nchunks), dim3(kMultiBlock), 0, s, prev, next, plane, red,
                           n, k, primes, g);
        break;
    case 2:
        hipLaunchKernelGGL(k_multi_layer_modp<2>, dim3(g.nchunks), dim3(kMultiBlock), 0, s, prev, next, plane, red,
                           n, k, primes, g);
        break;
    case 3:
        hipLaunchKernelGGL(k_multi_layer_modp<3>, dim3(g.nchunks), dim3(kMultiBlock), 0, s, prev, next, plane, red,
                           n, k, primes, g);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace permgpu
