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
// Masks below 2^12 in batch order (see batch_mask_list), filled once per device.
__device__ uint16_t g_batch_masks[1u << kBatchNMax];

constexpr int kBatchBlock = 256;   // integer batched kernel
constexpr int kBatchBlockC = kBatchBlockComplex;  // complex batched kernel
// Matrix area per workgroup: four order-10 matrices (4 * (2^10 + 100) * 16 B);
// with the 8 KB mask list two workgroups still share a CU's 160 KB.
constexpr size_t kBatchLdsCap = 4 * ((1 << 10) + 100) * 16;

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

// LDS of one workgroup: the masks below 2^nmax sorted by (popcount, value)
// as u16 (copied once per workgroup), then the matrix area: B/G matrices of
// (2^n table entries + n*n matrix entries) each.
__host__ __device__ size_t batch_mask_bytes(int) { return ((size_t)2 << kBatchNMax) + 16; }

// The complex kernel always takes the whole cap: its 512-thread workgroups
// at 128 VGPRs are limited to two per CU by registers anyway, and a larger
// area lets a chunk hold more small matrices.  The integer kernel (256
// threads) keeps its area near its need so that more workgroups fit a CU.
size_t batch_area_bytes(int nmax, int elem_bytes) {
    if (nmax < 0) nmax = 0;
    const size_t per = ((size_t)1 << nmax) + (size_t)nmax * nmax;
    size_t need = per * elem_bytes;
    if (need < kBatchLdsCap) need = (elem_bytes == 16 || kBatchLdsCap < 4 * need) ? kBatchLdsCap : 4 * need;
    return need;
}

size_t batch_lds_bytes(int nmax, int elem_bytes) {
    return batch_mask_bytes(nmax) + batch_area_bytes(nmax, elem_bytes) + 64;
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

__device__ __forceinline__ uint32_t mask_block(int nmax, int k) {
    uint32_t s = 0;
    for (int u = 0; u < k; u++) s += bbinom(nmax, u);
    return s;
}

// The mask list (built on the host, see batch_mask_list) is copied into LDS
// once per workgroup.
__device__ __forceinline__ void load_masks(uint16_t *s_masks) {
    for (uint32_t i = threadIdx.x; i < (1u << kBatchNMax); i += blockDim.x) s_masks[i] = g_batch_masks[i];
}

// F(S) of an order-N matrix lives at table position (2^N - 1) - S (the
// complement of S): the predecessor F(S \ {j}) of any j in S is then at
// position + 2^j, a constant offset that folds into the LDS instruction.
template <int N>
__device__ __forceinline__ uint32_t cpos(uint32_t S) { return ((1u << N) - 1u) - S; }

constexpr int cbinom(int n, int k) {
    if (k < 0 || k > n) return 0;
    int r = 1;
    for (int i = 1; i <= k; i++) r = r * (n - k + i) / i;
    return r;
}

// F({x, y}) for x < y: the stored value of layer 2, formed from the matrix
// (row 0 entries are the stored values of layer 1) with its chain, j = x then
// j = y.
__device__ __forceinline__ double2 pair_value(const double2 *mat, int N, uint32_t x, uint32_t y) {
    double re = 0.0, im = 0.0;
    bcfma(re, im, mat[N + x], mat[y]);
    bcfma(re, im, mat[N + y], mat[x]);
    return make_double2(re, im);
}

// One chunk of matrices of order N.  Layer by layer, each lane computes whole
// stored values F(S) with the fixed chain over the columns of S in ascending
// order (k is a compile-time constant in each unrolled layer).  Layers 1 and
// 2 are not stored: layer 3 forms its predecessors from the matrix with the
// same chains (pair_value).  Layer N - 1 has N values, all in the first N
// lanes of one wave, so the last value is formed after a wave-level fence
// instead of a workgroup barrier; groups of at most 64 lanes (one wave) use
// such fences between all their layers.
// mi is the result index of this thread's matrix (read with the prefetch).
template <int N>
__device__ __forceinline__ void batch_chunk_c128(const BatchChunk ch, int nmax, const uint16_t *s_masks, double2 *area,
                                                 uint32_t mi, double2 *__restrict__ results) {
    static_assert(N >= 3, "orders below 3 take batch_chunk_tiny_c128");
    const int lg = ch.group, G = 1 << lg;
    const int gi = threadIdx.x >> lg, lane = threadIdx.x & (G - 1);
    constexpr int PER = (1 << N) + N * N;
    double2 *tab = area + (size_t)gi * PER;
    const double2 *mat = tab + (1 << N);
    const bool active = gi < (int)ch.count;
#pragma unroll
    for (int k = 3; k <= N; k++) {
        // the last layer (one value) in lane 0 of the wave that holds layer N - 1
        const bool last = k == N;
        if (last && N > 3) __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        if (active && (!last || lane == 0)) {
            const uint16_t *ml = s_masks + mask_block(kBatchNMax, k);
            // row k-1 of A, read per term at the lane's own column
            const double2 *rowk = mat + (k - 1) * N;
            const int cnt = cbinom(N, k);
            uint32_t Sn = lane < cnt ? ml[lane] : 0u;
            for (int i = lane; i < cnt; i += G) {
                const uint32_t S = Sn;
                if (i + G < cnt) Sn = ml[i + G];
                const double2 *t0 = tab + cpos<N>(S);
                // the k columns of S, lowest first (every lane of the layer has
                // exactly k): each term's predecessor and coefficient are read
                // into distinct registers before the chain starts, so a round
                // waits for LDS once and issues no masked-off work
                double2 p[N], c[N];
                uint32_t Sr = S;
#pragma unroll
                for (int u = 0; u < N; u++) {
                    if (u < k) {
                        const uint32_t j = (uint32_t)__builtin_ctz(Sr);
                        Sr &= Sr - 1u;
                        if (k == 3) {
                            const uint32_t rest = S ^ (1u << j);
                            const uint32_t x = (uint32_t)__builtin_ctz(rest);
                            p[u] = pair_value(mat, N, x, (uint32_t)__builtin_ctz(rest ^ (1u << x)));
                        } else {
                            p[u] = t0[1u << j];
                        }
                        c[u] = rowk[j];
                    }
                }
                double re = 0.0, im = 0.0;
#pragma unroll
                for (int u = 0; u < N; u++)
                    if (u < k) bcfma(re, im, c[u], p[u]);
                if (last) results[mi] = make_double2(re, im);
                else tab[cpos<N>(S)] = make_double2(re, im);
            }
        }
        if (k < N - 1) {
            // a group of at most 64 lanes lies in one wave: its layers need
            // only that wave's LDS traffic ordered (the branch is uniform)
            if (G <= 64) __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            else __syncthreads();
        }
    }
    __syncthreads();
}

// Orders 0..2 (rare): trivial values, written directly.
__device__ __forceinline__ void batch_chunk_tiny_c128(const BatchChunk ch, const double2 *__restrict__ mats,
                                      const int64_t *__restrict__ offsets, const uint32_t *__restrict__ order,
                                      double2 *__restrict__ results) {
    for (uint32_t g = threadIdx.x; g < ch.count; g += blockDim.x) {
        const uint32_t mi = order ? order[ch.first + g] : ch.first + g;
        const double2 *a = mats + (offsets ? offsets[ch.first + g] : 0);
        double2 r;
        if (ch.n == 0) {
            r = make_double2(1.0, 0.0);
        } else if (ch.n == 1) {
            r = a[0];
        } else {  // F({0,1}) = a[1][0] * a[0][1] + a[1][1] * a[0][0], chain over j = 0, 1
            double re = 0.0, im = 0.0;
            bcfma(re, im, a[2], a[1]);
            bcfma(re, im, a[3], a[0]);
            r = make_double2(re, im);
        }
        results[mi] = r;
    }
    __syncthreads();
}

// Entries of a chunk's matrices staged through registers: thread i holds
// flat entry i (the planner keeps (B / G) * n * n <= B for the workgroup size
// B), so the whole next chunk is in flight in four registers, together with
// the result index of the thread's matrix.
struct ChunkPrefetch {
    double2 v;
    uint32_t mi;
    int64_t off;  // element offset of the matrix holding flat entry threadIdx.x
};

// offsets[] is in work-list order (entry ch.first + g is the chunk's g-th
// matrix).  Two phases: the offset and result index of the thread's matrix
// first, then (once the offset has arrived) the matrix entry itself.
__device__ __forceinline__ void prefetch_index(ChunkPrefetch &R, const BatchChunk ch,
                                               const int64_t *__restrict__ offsets,
                                               const uint32_t *__restrict__ order) {
    const uint32_t nn = (uint32_t)ch.n * ch.n, tot = nn * ch.count, f = threadIdx.x;
    R.off = 0;
    if (f < tot && offsets) R.off = offsets[ch.first + f / nn];
    const uint32_t gi = threadIdx.x >> ch.group;
    R.mi = gi < ch.count ? (order ? order[ch.first + gi] : ch.first + gi) : 0u;
}

__device__ __forceinline__ void prefetch_entry(ChunkPrefetch &R, const BatchChunk ch,
                                               const double2 *__restrict__ mats) {
    const uint32_t nn = (uint32_t)ch.n * ch.n, tot = nn * ch.count, f = threadIdx.x;
    if (f < tot) R.v = mats[R.off + (f - (f / nn) * nn)];
}

__device__ __forceinline__ void prefetch_chunk(ChunkPrefetch &R, const BatchChunk ch,
                                               const double2 *__restrict__ mats,
                                               const int64_t *__restrict__ offsets,
                                               const uint32_t *__restrict__ order) {
    prefetch_index(R, ch, offsets, order);
    prefetch_entry(R, ch, mats);
}

__device__ __forceinline__ void stage_chunk(const ChunkPrefetch &R, const BatchChunk ch, double2 *area) {
    const uint32_t nn = (uint32_t)ch.n * ch.n, tot = nn * ch.count, f = threadIdx.x;
    if (f < tot) {
        const uint32_t g = f / nn, e = f - g * nn;
        area[(size_t)g * ((1u << ch.n) + nn) + (1u << ch.n) + e] = R.v;
    }
}

// Chunk descriptors travel as two raw words: loaded with a vector load (its
// latency is tracked apart from LDS traffic) and made wave-uniform only
// where they are used.
__device__ __forceinline__ uint2 chunk_raw(const BatchChunk *chunks, uint32_t c) {
    return *reinterpret_cast<const uint2 *>(chunks + c);
}

__device__ __forceinline__ BatchChunk chunk_from(uint2 w) {
    BatchChunk c;
    c.first = __builtin_amdgcn_readfirstlane(w.x);
    const uint32_t y = __builtin_amdgcn_readfirstlane(w.y);
    c.count = (uint16_t)(y & 0xffffu);
    c.n = (uint8_t)((y >> 16) & 0xffu);
    c.group = (uint8_t)(y >> 24);
    return c;
}

// Chunks are claimed from the counter in groups of kClaimGroup consecutive
// chunks (group q covers chunks q*K .. q*K+K-1): fewer trips to the shared
// counter, while the group size stays small next to the list so that faster
// workgroups still take more of the work.  The list is sorted by cost, so
// the last groups hold the cheapest chunks.
constexpr uint32_t kClaimGroup = 4;

// Index sequence of one workgroup: the chunks of its current group, then of
// the next claimed group.  Two claimed groups are kept ahead of the current
// one; taking one out of that queue issues a claim for its replacement, whose
// value arrives at the end of the same loop iteration.
struct ChunkSeq {
    uint32_t q, j;    // group and position of the last index handed out
    uint32_t f0, f1;  // the two claimed groups that follow
    uint32_t K, nch;
    // next index (>= nch once the list is exhausted); sets pop when it moved
    // into a new group
    __device__ __forceinline__ uint32_t next(bool &pop) {
        if (j + 1 < K && q * K + j + 1 < nch) {
            j++;
            pop = false;
        } else {
            q = f0;
            f0 = f1;
            j = 0;
            pop = true;
        }
        return q * K + j;
    }
};

// With single.count == 1 the launch solves that one chunk (matrix 0 at
// offset 0, no work list, no counter); otherwise it runs the persistent loop.
// The loop is pipelined so that no round trip to memory sits between two
// chunks: while chunk i is computed, the matrices of chunk i+1 are in flight
// to registers, the descriptor of chunk i+2 is being read and, when chunk i+2
// opened a new group, the claim of a further group is in flight.  A claimed
// index at or beyond nchunks means the list is exhausted; since the counter
// only grows, a workgroup that stops holds no unprocessed chunk.
// At most 128 VGPRs: two 512-thread workgroups must share a CU.
__global__ __launch_bounds__(kBatchBlockC) __attribute__((amdgpu_waves_per_eu(4))) void k_batch_c128(
    const double2 *__restrict__ mats, const int64_t *__restrict__ offsets,
    const uint32_t *__restrict__ order, const BatchChunk *chunks, uint32_t nchunks,
    uint32_t *counter, double2 *__restrict__ results, int nmax, const BatchChunk single) {
    extern __shared__ double2 bsm[];
    __shared__ uint32_t s_claim;
    uint16_t *s_masks = (uint16_t *)bsm;
    double2 *area = bsm + batch_mask_bytes(nmax) / sizeof(double2);
    load_masks(s_masks);
    const bool one = single.count != 0;
    const uint32_t nch = one ? 1u : nchunks;
    if (threadIdx.x == 0 && !one) s_claim = atomicAdd(counter, 3u);  // groups q, q + 1, q + 2
    __syncthreads();
    const uint32_t q0 = one ? 0u : __builtin_amdgcn_readfirstlane(s_claim);
    ChunkSeq seq{q0, 0u, q0 + 1, q0 + 2, one ? 1u : kClaimGroup, nch};
    const uint32_t c0 = q0 * seq.K;
    if (c0 >= nch) return;  // uniform: every thread read the same index
    bool pop1, pop2;
    const uint32_t c1 = seq.next(pop1);
    uint32_t c2 = seq.next(pop2);
    const uint32_t pops = (pop1 ? 1u : 0u) + (pop2 ? 1u : 0u);
    __syncthreads();  // everyone has read s_claim
    if (pops && !one) {  // refill the queue of claimed groups (start-up only)
        if (threadIdx.x == 0) s_claim = atomicAdd(counter, pops);
        __syncthreads();
        const uint32_t base = __builtin_amdgcn_readfirstlane(s_claim);
        if (pops == 2) {
            seq.f0 = base;
            seq.f1 = base + 1;
        } else {
            seq.f1 = base;
        }
        __syncthreads();  // everyone has read s_claim
    }
    BatchChunk ch = one ? single : chunk_from(chunk_raw(chunks, c0));
    bool have1 = c1 < nch;
    BatchChunk ch1 = ch;
    if (have1) ch1 = chunk_from(chunk_raw(chunks, c1));
    ChunkPrefetch R;
    prefetch_chunk(R, ch, mats, offsets, order);
    for (;;) {
        // staging waits for the registers filled by the previous prefetch;
        // everything issued after it stays in flight during the compute
        if (ch.n >= 3) stage_chunk(R, ch, area);
        const uint32_t mi = R.mi;
        // nothing newer than the previous prefetch is in flight here; settling
        // it on every path (orders <= 2 skip the staging) keeps the compiler
        // from waiting for the loads below when it refills R
        __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0)
        // next chunk: its offsets and result indices, then the descriptor of
        // the one after it (index clamped to the list, so the load needs no
        // branch of its own; the single-matrix launch has no list), then its
        // matrix entries, then a claim if a group was taken from the queue;
        // all stay in flight during the compute
        if (have1) prefetch_index(R, ch1, offsets, order);
        const bool have2 = c2 < nch;
        uint2 d2 = make_uint2(0u, 0u);
        if (!one) d2 = chunk_raw(chunks, have2 ? c2 : 0u);  // decoded after the compute
        if (have1) prefetch_entry(R, ch1, mats);
        bool pop;
        const uint32_t c3 = seq.next(pop);
        // atomicInc (not atomicAdd) keeps the compiler from turning this
        // single-lane claim into a wave-wide pattern that waits for it here
        uint32_t claimed = 0;
        if (pop && !one && threadIdx.x == 0) claimed = atomicInc(counter, 0xffffffffu);  // used after the compute
        __syncthreads();  // the staged matrices are visible to every thread
        switch (ch.n) {
        case 12: batch_chunk_c128<12>(ch, nmax, s_masks, area, mi, results); break;
        case 11: batch_chunk_c128<11>(ch, nmax, s_masks, area, mi, results); break;
        case 10: batch_chunk_c128<10>(ch, nmax, s_masks, area, mi, results); break;
        case 9: batch_chunk_c128<9>(ch, nmax, s_masks, area, mi, results); break;
        case 8: batch_chunk_c128<8>(ch, nmax, s_masks, area, mi, results); break;
        case 7: batch_chunk_c128<7>(ch, nmax, s_masks, area, mi, results); break;
        case 6: batch_chunk_c128<6>(ch, nmax, s_masks, area, mi, results); break;
        case 5: batch_chunk_c128<5>(ch, nmax, s_masks, area, mi, results); break;
        case 4: batch_chunk_c128<4>(ch, nmax, s_masks, area, mi, results); break;
        case 3: batch_chunk_c128<3>(ch, nmax, s_masks, area, mi, results); break;
        default: batch_chunk_tiny_c128(ch, mats, offsets, order, results); break;
        }
        if (pop && !one) {  // uniform
            // every chunk body ends with a barrier, so all reads of the
            // previous s_claim are done before it is overwritten here
            if (threadIdx.x == 0) s_claim = claimed;
            __syncthreads();
            seq.f1 = __builtin_amdgcn_readfirstlane(s_claim);
        }
        if (!have1) break;  // uniform
        ch = ch1;
        if (have2) ch1 = chunk_from(d2);
        have1 = have2;
        c2 = c3;
    }
}

hipError_t launch_batch_c128(const void *mats, const int64_t *offsets, const uint32_t *order,
                             const BatchChunk *chunks, uint32_t nchunks, uint32_t *counter,
                             void *results, int nmax, int grid, hipStream_t s) {
    const size_t lds = batch_lds_bytes(nmax, 16);
    const BatchChunk none{0, 0, 0, 0};
    hipLaunchKernelGGL(k_batch_c128, dim3(grid), dim3(kBatchBlockC), lds, s, (const double2 *)mats,
                       offsets, order, chunks, nchunks, counter, (double2 *)results, nmax, none);
    return hipGetLastError();
}

hipError_t launch_single_c128(const void *mat, int n, void *result, hipStream_t s) {
    const size_t lds = batch_lds_bytes(n, 16);
    int lg = 0;
    while ((1 << lg) < kBatchBlockC) lg++;
    const BatchChunk one{0, 1, (uint8_t)n, (uint8_t)lg};
    hipLaunchKernelGGL(k_batch_c128, dim3(1), dim3(kBatchBlockC), lds, s, (const double2 *)mat, nullptr,
                       nullptr, nullptr, 0u, nullptr, (double2 *)result, n, one);
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
    uint32_t count, const BatchChunk single) {
    extern __shared__ uint64_t bsu_all[];
    __shared__ uint32_t s_chunk;
    uint64_t *bsu = bsu_all;
    const bool one = single.count != 0;
    for (uint32_t iter = 0;; iter++) {
        if (threadIdx.x == 0) s_chunk = one ? iter : atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t c = s_chunk;
        __syncthreads();
        if (one ? c >= 1u : c >= nchunks) break;
        const BatchChunk ch = one ? single : chunks[c];
        const int n = ch.n, lg = ch.group, G = 1 << lg;
        const int gi = threadIdx.x >> lg, lane = threadIdx.x & (G - 1);
        const int per = (1 << n) + n * n;
        uint64_t *tab = bsu + (size_t)gi * per;
        uint64_t *mat = tab + (1 << n);
        const bool active = gi < (int)ch.count;
        const uint32_t mi = active ? (order ? order[ch.first + gi] : ch.first + gi) : 0u;
        const int64_t *src = mats + (active && offsets ? offsets[mi] : 0);
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
    const BatchChunk none{0, 0, 0, 0};
    hipLaunchKernelGGL(k_batch_modp, dim3(grid), dim3(kBatchBlock), lds, s, mats, offsets, order,
                       chunks, nchunks, counter, primes, nprimes, res, count, none);
    return hipGetLastError();
}

hipError_t launch_single_modp(const int64_t *mat, int n, const uint64_t *primes, int nprimes, uint64_t *res,
                              hipStream_t s) {
    const size_t lds = batch_lds_bytes(n, 8);
    int lg = 0;
    while ((1 << lg) < kBatchBlock) lg++;
    const BatchChunk one{0, 1, (uint8_t)n, (uint8_t)lg};
    hipLaunchKernelGGL(k_batch_modp, dim3(1), dim3(kBatchBlock), lds, s, mat, nullptr, nullptr, nullptr, 0u,
                       nullptr, primes, nprimes, res, 1u, one);
    return hipGetLastError();
}

hipError_t upload_batch_masks(const uint16_t *host, hipStream_t s) {
    return hipMemcpyToSymbolAsync(HIP_SYMBOL(g_batch_masks), host, sizeof(uint16_t) << kBatchNMax, 0,
                                  hipMemcpyHostToDevice, s);
}

}  // namespace permgpu
