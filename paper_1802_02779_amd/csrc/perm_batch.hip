// Batched small-n Store-zechin permanents: one persistent launch.
//
// Each matrix (n <= 12) keeps its whole table of stored sub-permanents
// F(S) = per(rows 1..|S|, cols S) in LDS, indexed by the bitmask of S, and is
// evaluated layer by layer |S| = 2..n with the same per-entry arithmetic as
// the layer sweep (so batched and single results are bitwise equal):
//   F(S) = sum_{j in S, ascending} a[|S|-1][j] * F(S \ {j}).
// Work list: matrices sorted by cost (largest n first), cut into chunks of
// equal n; a chunk holds 256 / 2^group matrices, each served by 2^group
// threads.  Workgroups pull chunk indices from one atomic counter until the
// list is exhausted (every wave reaches the exit test).
#include "perm_internal.h"

namespace permgpu {

extern __constant__ BinomTable c_binom;
extern __device__ uint32_t g_highlist[1u << kHighBits];

constexpr int kBatchBlock = 256;
constexpr size_t kBatchLdsCap = 80 * 1024;  // two workgroups per CU

__device__ __forceinline__ uint32_t bbinom(int i, int j) { return c_binom.v[i][j]; }

__device__ __forceinline__ uint32_t highlist_block(int m) {
    uint32_t s = 0;
    for (int u = 0; u < m; u++) s += bbinom(kHighBits, u);
    return s;
}

__device__ __forceinline__ void bcfma(double &re, double &im, const double2 a, const double2 p) {
    re = __builtin_fma(a.x, p.x, re);
    re = __builtin_fma(-a.y, p.y, re);
    im = __builtin_fma(a.x, p.y, im);
    im = __builtin_fma(a.y, p.x, im);
}

size_t batch_lds_bytes(int nmax, int elem_bytes) {
    if (nmax < 0) nmax = 0;
    const size_t per = ((size_t)1 << nmax) + (size_t)nmax * nmax;
    size_t need = per * elem_bytes;
    if (need < kBatchLdsCap) need = kBatchLdsCap < 4 * need ? kBatchLdsCap : 4 * need;
    return need + 64;
}

int batch_blocks_per_cu(int nmax, int elem_bytes) {
    const size_t b = batch_lds_bytes(nmax, elem_bytes);
    int k = (int)((160 * 1024) / b);
    return k < 1 ? 1 : (k > 8 ? 8 : k);
}

__global__ void k_batch_reset(uint32_t *counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

hipError_t launch_batch_reset(uint32_t *counter, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, s, counter);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBatchBlock) void k_batch_c128(
    const double2 *__restrict__ mats, const int64_t *__restrict__ offsets,
    const uint32_t *__restrict__ order, const BatchChunk *__restrict__ chunks, uint32_t nchunks,
    uint32_t *counter, double2 *__restrict__ results) {
    extern __shared__ double2 bsm[];
    __shared__ uint32_t s_chunk;
    for (;;) {
        if (threadIdx.x == 0) s_chunk = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t c = s_chunk;
        __syncthreads();
        if (c >= nchunks) break;
        const BatchChunk ch = chunks[c];
        const int n = ch.n, lg = ch.group, G = 1 << lg;
        const int gi = threadIdx.x >> lg, lane = threadIdx.x & (G - 1);
        const int per = (1 << n) + n * n;
        double2 *tab = bsm + (size_t)gi * per;
        double2 *mat = tab + (1 << n);
        const bool active = gi < (int)ch.count;
        uint32_t mi = 0;
        if (active) {
            mi = order[ch.first + gi];
            const double2 *src = mats + offsets[mi];
            for (int i = lane; i < n * n; i += G) mat[i] = src[i];
        }
        __syncthreads();
        if (active)
            for (int j = lane; j < n; j += G) tab[1u << j] = mat[j];
        __syncthreads();
        for (int k = 2; k <= n; k++) {
            if (active) {
                const uint32_t cnt = bbinom(n, k);
                const uint32_t *ml = g_highlist + highlist_block(k);
                const double2 *arow = mat + (k - 1) * n;
                for (uint32_t i = lane; i < cnt; i += G) {
                    const uint32_t S = ml[i];
                    double re = 0.0, im = 0.0;
                    uint32_t b = S;
                    while (b) {
                        const int j = __ffs(b) - 1;
                        b &= b - 1;
                        bcfma(re, im, arow[j], tab[S ^ (1u << j)]);
                    }
                    tab[S] = make_double2(re, im);
                }
            }
            __syncthreads();
        }
        if (active && lane == 0)
            results[mi] = n == 0 ? make_double2(1.0, 0.0) : tab[(1u << n) - 1];
        __syncthreads();
    }
}

hipError_t launch_batch_c128(const void *mats, const int64_t *offsets, const uint32_t *order,
                             const BatchChunk *chunks, uint32_t nchunks, uint32_t *counter,
                             void *results, int nmax, int grid, hipStream_t s) {
    const size_t lds = batch_lds_bytes(nmax, 16);
    hipLaunchKernelGGL(k_batch_c128, dim3(grid), dim3(kBatchBlock), lds, s, (const double2 *)mats,
                       offsets, order, chunks, nchunks, counter, (double2 *)results);
    return hipGetLastError();
}

// ------------------------------------------------------------ integer
typedef unsigned __int128 u128b;

__device__ __forceinline__ uint64_t bfold61(u128b x, uint64_t p) {
    const uint64_t M = (1ull << 61) - 1;
    const uint64_t c = (1ull << 61) - p;
    const u128b y = (u128b)((uint64_t)x & M) + (u128b)c * (x >> 61);
    uint64_t z = ((uint64_t)y & M) + c * (uint64_t)(y >> 61);
    if (z >= p) z -= p;
    if (z >= p) z -= p;
    return z;
}

__global__ __launch_bounds__(kBatchBlock) void k_batch_modp(
    const int64_t *__restrict__ mats, const int64_t *__restrict__ offsets,
    const uint32_t *__restrict__ order, const BatchChunk *__restrict__ chunks, uint32_t nchunks,
    uint32_t *counter, const uint64_t *__restrict__ primes, int nprimes, uint64_t *__restrict__ res,
    uint32_t count) {
    extern __shared__ uint64_t bsu[];
    __shared__ uint32_t s_chunk;
    for (;;) {
        if (threadIdx.x == 0) s_chunk = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t c = s_chunk;
        __syncthreads();
        if (c >= nchunks) break;
        const BatchChunk ch = chunks[c];
        const int n = ch.n, lg = ch.group, G = 1 << lg;
        const int gi = threadIdx.x >> lg, lane = threadIdx.x & (G - 1);
        const int per = (1 << n) + n * n;
        uint64_t *tab = bsu + (size_t)gi * per;
        uint64_t *mat = tab + (1 << n);
        const bool active = gi < (int)ch.count;
        const uint32_t mi = active ? order[ch.first + gi] : 0u;
        const int64_t *src = mats + (active ? offsets[mi] : 0);
        for (int r = 0; r < nprimes; r++) {
            const uint64_t p = primes[r];
            if (active) {
                for (int i = lane; i < n * n; i += G) {
                    const int64_t v = src[i];
                    const uint64_t mag = v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v;
                    uint64_t m = mag % p;
                    if (v < 0 && m != 0) m = p - m;
                    mat[i] = m;
                }
            }
            __syncthreads();
            if (active)
                for (int j = lane; j < n; j += G) tab[1u << j] = mat[j];
            __syncthreads();
            for (int k = 2; k <= n; k++) {
                if (active) {
                    const uint32_t cnt = bbinom(n, k);
                    const uint32_t *ml = g_highlist + highlist_block(k);
                    const uint64_t *arow = mat + (k - 1) * n;
                    for (uint32_t i = lane; i < cnt; i += G) {
                        const uint32_t S = ml[i];
                        u128b acc = 0;
                        uint32_t b = S;
                        while (b) {
                            const int j = __ffs(b) - 1;
                            b &= b - 1;
                            acc += (u128b)arow[j] * tab[S ^ (1u << j)];
                        }
                        tab[S] = bfold61(acc, p);
                    }
                }
                __syncthreads();
            }
            if (active && lane == 0)
                res[(size_t)r * count + mi] = n == 0 ? 1u : tab[(1u << n) - 1];
            __syncthreads();
        }
    }
}

hipError_t launch_batch_modp(const int64_t *mats, const int64_t *offsets, const uint32_t *order,
                             const BatchChunk *chunks, uint32_t nchunks, uint32_t *counter,
                             const uint64_t *primes, int nprimes, uint64_t *res, uint32_t count,
                             int nmax, int grid, hipStream_t s) {
    const size_t lds = batch_lds_bytes(nmax, 8);
    hipLaunchKernelGGL(k_batch_modp, dim3(grid), dim3(kBatchBlock), lds, s, mats, offsets, order,
                       chunks, nchunks, counter, primes, nprimes, res, count);
    return hipGetLastError();
}

}  // namespace permgpu
