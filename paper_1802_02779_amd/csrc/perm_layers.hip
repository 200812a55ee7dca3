// Layer sweep of the Store-zechin permanent on gfx950.
//
// Section 4 of the paper develops per(A) along the last row and stores every
// sub-permanent once.  Here the stored values F(S) = per(rows 1..|S|, cols S)
// are evaluated layer by layer (|S| = 1, 2, ..., n); layer k needs only layer
// k-1:  F(S) = sum_{j in S, ascending} a[k-1][j] * F(S \ {j})  (0-based row).
// Tiling, ranks and tables are described in perm_internal.h.
//
// Complex arithmetic: one fixed FMA chain per output over j ascending
//   re = fma(a.re, p.re, re); re = fma(-a.im, p.im, re);
//   im = fma(a.re, p.im, im); im = fma(a.im, p.re, im);
// Integer arithmetic: residues mod p = 2^61 - c; the sum of the k products
// is kept exact in 128 bits and folded once per output.
#include "perm_internal.h"

namespace permgpu {

__constant__ BinomTable c_binom = make_binom();
__device__ uint32_t g_lowtab[kLowtabEntries];
__device__ uint32_t g_highlist[1u << kHighBits];

__device__ __forceinline__ uint32_t dbinom(int i, int j) { return c_binom.v[i][j]; }

// ------------------------------------------------------------------ tables
__global__ void k_build_lowtab(int t) {
    uint32_t L = blockIdx.x * blockDim.x + threadIdx.x;
    if (L >= (1u << t) || L == 0) return;
    const int kp = __popc(L);
    // columns of L ascending and the colex rank of L
    int cols[kTMax];
    uint32_t rank = 0;
    {
        uint32_t b = L;
        for (int i = 0; i < kp; i++) {
            int c = __ffs(b) - 1;
            b &= b - 1;
            cols[i] = c;
            rank += dbinom(c, i + 1);
        }
    }
    uint32_t off = 0;  // lowtab_t_base(t) + lowtab_kp_off(t, kp)
    for (int u = 1; u < t; u++) off += (uint32_t)u << (u - 1);
    for (int u = 1; u < kp; u++) off += (uint32_t)u * dbinom(t, u);
    const uint32_t ck = dbinom(t, kp);
    for (int p = 0; p < kp; p++) {
        // rank of L without its p-th column: columns above p move down one place
        uint32_t r = 0;
        for (int i = 0; i < kp; i++) {
            if (i < p) r += dbinom(cols[i], i + 1);
            else if (i > p) r += dbinom(cols[i], i);
        }
        g_lowtab[off + (uint32_t)p * ck + rank] = r | ((uint32_t)cols[p] << 16);
    }
}

__global__ void k_build_highlist() {
    uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= (1u << kHighBits)) return;
    const int pop = __popc(m);
    uint32_t off = 0;
    for (int u = 0; u < pop; u++) off += dbinom(kHighBits, u);
    uint32_t rank = 0, b = m;
    for (int i = 1; b; i++) {
        int c = __ffs(b) - 1;
        b &= b - 1;
        rank += dbinom(c, i);
    }
    g_highlist[off + rank] = m;
}

static bool g_tables_ready[64];

hipError_t ensure_tables(int device, hipStream_t s) {
    if (device < 0 || device >= 64) return hipErrorInvalidDevice;
    if (g_tables_ready[device]) return hipSuccess;
    for (int t = 1; t <= kTMax; t++) {
        uint32_t threads = 1u << t;
        hipLaunchKernelGGL(k_build_lowtab, dim3((threads + 255) / 256), dim3(256), 0, s, t);
    }
    hipLaunchKernelGGL(k_build_highlist, dim3((1u << kHighBits) / 256), dim3(256), 0, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    static uint16_t masks[1u << kBatchNMax];
    static bool masks_built = false;
    if (!masks_built) {
        batch_mask_list(kBatchNMax, masks);
        masks_built = true;
    }
    e = upload_batch_masks(masks, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e == hipSuccess) g_tables_ready[device] = true;
    return e;
}

// -------------------------------------------------------------- planning
uint32_t plan_layer(int n, int k, int t, int chunk, int nt_store, uint32_t thin_below, LayerArgs *a) {
    const int nh = n - t;
    a->n = n;
    a->k = k;
    a->t = t;
    a->chunk = chunk;
    a->nt_store = nt_store;
    a->binary_row = 0;
    a->ngroups = 0;
    a->thin_groups = 0;
    a->lds_window = 0;
    uint32_t tiles = 0, thin_out = 0;
    const int kp_lo = k - nh > 0 ? k - nh : 0;
    const int kp_hi = k < t ? k : t;
    for (int kp = kp_lo; kp <= kp_hi; kp++) {
        const int m = k - kp;
        const uint32_t ck = binom_host(t, kp);
        if (ck < thin_below) {
            const int g = a->thin_groups++;
            a->t_kp[g] = kp;
            a->t_ck[g] = ck;
            a->t_out_start[g] = thin_out;
            a->t_low_off[g] = lowtab_t_base(t) + lowtab_kp_off(t, kp);
            a->t_high_off[g] = highlist_off(m);
            thin_out += binom_host(nh, m) * ck;
            continue;
        }
        const int g = a->ngroups++;
        a->kp[g] = kp;
        a->start[g] = tiles;
        a->ck[g] = ck;
        a->low_off[g] = lowtab_t_base(t) + lowtab_kp_off(t, kp);
        a->high_off[g] = highlist_off(m);
        tiles += binom_host(nh, m);
        if (kp >= 1 && binom_host(t, kp - 1) > a->lds_window) a->lds_window = binom_host(t, kp - 1);
    }
    a->start[a->ngroups] = tiles;
    a->t_out_start[a->thin_groups] = thin_out;
    a->big_blocks = tiles;
    return tiles + (thin_out + 255) / 256;
}

size_t layer_lds_bytes_c128(const LayerArgs &a) {
    const size_t tiled = (size_t)(a.lds_window + a.t + 32) * 16 + 32 * 4;
    const size_t thin = 33 * 33 * 4 + 32 * 16;
    return tiled > thin ? tiled : thin;
}

size_t layer_lds_bytes_modp(const LayerArgs &a, int rp) {
    const size_t tiled = (size_t)rp * (a.lds_window + a.t + 32) * 8 + 32 * 4;
    const size_t thin = (33 * 33 + 1) * 4 + (size_t)rp * 32 * 8;
    return tiled > thin ? tiled : thin;
}

// XCD-aware order.  Workgroup b is dispatched to XCD b % 8 as that XCD's
// (b / 8)-th workgroup.  With chunk C > 0, each XCD takes runs of C
// consecutive tiles (tiles that share high windows then meet in one L2)
// while the eight XCDs stay on neighbouring runs (the chip-wide working set
// stays small).  Tiles past the last full round of 8*C keep their order.
// A bijection on [0, G).
__device__ __forceinline__ uint32_t xcd_chunk_remap(uint32_t b, uint32_t G, uint32_t C) {
    const uint32_t round = 8u * C;
    if (C == 0 || b >= (G / round) * round) return b;
    const uint32_t x = b & 7u, s = b >> 3;
    return ((s / C) * 8u + x) * C + (s % C);
}

struct TileInfo {
    int g, kp, m;
    uint32_t T, ck, base_out, base_low;
};

__device__ __forceinline__ TileInfo decode_tile(const LayerArgs &A) {
    TileInfo ti;
    const uint32_t tile = xcd_chunk_remap(blockIdx.x, A.big_blocks, (uint32_t)A.chunk);
    int g = 0;
    while (g + 1 < A.ngroups && A.start[g + 1] <= tile) g++;
    ti.g = g;
    ti.kp = A.kp[g];
    ti.m = A.k - ti.kp;
    ti.ck = A.ck[g];
    ti.T = g_highlist[A.high_off[g] + (tile - A.start[g])];
    uint32_t bo = 0, bl = 0, b = ti.T;
    for (int i = 1; b; i++) {
        const int h = __ffs(b) - 1 + A.t;
        b &= b - 1;
        bo += dbinom(h, ti.kp + i);
        bl += dbinom(h, ti.kp - 1 + i);
    }
    ti.base_out = bo;
    ti.base_low = bl;
    return ti;
}

// Base rank (in layer k-1) of the high window that removes the q-th high
// column (q = 0..m-1), and that column.
__device__ __forceinline__ uint32_t high_window_base(uint32_t T, int t, int kp, int q, int *col) {
    uint32_t base = 0, b = T;
    for (int i = 0; b; i++) {
        const int h = __ffs(b) - 1 + t;
        b &= b - 1;
        if (i < q) base += dbinom(h, kp + i + 1);
        else if (i > q) base += dbinom(h, kp + i);
        else *col = h;
    }
    return base;
}

// ---------------------------------------------------------- complex128
__device__ __forceinline__ void cfma(double &re, double &im, const double2 a, const double2 p) {
    re = __builtin_fma(a.x, p.x, re);
    re = __builtin_fma(-a.y, p.y, re);
    im = __builtin_fma(a.x, p.y, im);
    im = __builtin_fma(a.y, p.x, im);
}

__global__ void k_pack_c128(const double2 *__restrict__ a, int64_t lda, int n,
                            double2 *__restrict__ packed, double2 *__restrict__ layer1) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * n) return;
    const int r = i / n, c = i - r * n;
    const double2 v = a[(int64_t)r * lda + c];
    packed[i] = v;
    if (r == 0) layer1[c] = v;  // F({c}) = a[0][c]; rank of {c} is c
}

hipError_t launch_pack_c128(const void *a_dev, int64_t lda, int n, void *packed, void *layer1,
                            hipStream_t s) {
    const int tot = n * n;
    hipLaunchKernelGGL(k_pack_c128, dim3((tot + 255) / 256), dim3(256), 0, s,
                       (const double2 *)a_dev, lda, n, (double2 *)packed, (double2 *)layer1);
    return hipGetLastError();
}

constexpr int kLayerBlock = 256;

// Per-thread path for groups whose tiles are too small to fill a workgroup:
// each thread computes one whole output.  Low predecessors come through the
// rank table from the tile's window (small, cached), high predecessors from
// the aligned windows (neighbouring threads read neighbouring entries).
__device__ void layer_c128_thin(const double2 *__restrict__ prev, double2 *__restrict__ next,
                                const double2 *__restrict__ A, const LayerArgs &args, double2 *smem) {
    uint32_t *s_bin = (uint32_t *)smem;               // C(i, j) at [i * 33 + j]
    double2 *s_arow = (double2 *)(s_bin + 33 * 33);   // row k-1 of A
    const int tid = threadIdx.x;
    for (int i = tid; i < 33 * 33; i += kLayerBlock) s_bin[i] = c_binom.v[i / 33][i % 33];
    if (tid < args.n) s_arow[tid] = A[(size_t)(args.k - 1) * args.n + tid];
    __syncthreads();
    const uint32_t gid = (blockIdx.x - args.big_blocks) * kLayerBlock + tid;
    if (gid >= args.t_out_start[args.thin_groups]) return;
    int g = 0;
    while (g + 1 < args.thin_groups && args.t_out_start[g + 1] <= gid) g++;
    const int kp = args.t_kp[g], t = args.t;
    const uint32_t ck = args.t_ck[g], local = gid - args.t_out_start[g];
    const uint32_t tile = local / ck, r = local - tile * ck;
    const uint32_t T = g_highlist[args.t_high_off[g] + tile];
    // ranks: output base, low-window base, and the base of the first high window
    uint32_t base_out = 0, base_low = 0, base_h = 0;
    {
        uint32_t b = T;
        for (int i = 1; b; i++) {
            const int h = __ffs(b) - 1 + t;
            b &= b - 1;
            base_out += s_bin[h * 33 + kp + i];
            base_low += s_bin[h * 33 + kp + i - 1];
            if (i >= 2) base_h += s_bin[h * 33 + kp + i - 1];
        }
    }
    double re = 0.0, im = 0.0;
    const uint32_t *lt = g_lowtab + args.t_low_off[g];
    for (int p = 0; p < kp; p++) {
        const uint32_t e = lt[(uint32_t)p * ck + r];
        cfma(re, im, s_arow[e >> 16], prev[base_low + (e & 0xffffu)]);
    }
    // high columns ascending; the window that removes the q-th one starts at
    // base_q, with base_{q+1} = base_q + C(h_q, k'+q) - C(h_{q+1}, k'+q)
    uint32_t b = T;
    int q = 1, hprev = 0;
    while (b) {
        const int h = __ffs(b) - 1 + t;
        b &= b - 1;
        if (q > 1) base_h = base_h + s_bin[hprev * 33 + kp + q - 1] - s_bin[h * 33 + kp + q - 1];
        cfma(re, im, s_arow[h], prev[base_h + r]);
        hprev = h;
        q++;
    }
    double2 *out = next + base_out + r;
    if (args.nt_store) {
        __builtin_nontemporal_store(re, &out->x);
        __builtin_nontemporal_store(im, &out->y);
    } else {
        *out = make_double2(re, im);
    }
}

__global__ __launch_bounds__(kLayerBlock) void k_layer_c128(const double2 *__restrict__ prev,
                                                            double2 *__restrict__ next,
                                                            const double2 *__restrict__ A,
                                                            const LayerArgs args) {
    extern __shared__ double2 smem[];
    if (blockIdx.x >= args.big_blocks) {
        layer_c128_thin(prev, next, A, args, smem);
        return;
    }
    const int tid = threadIdx.x;
    const TileInfo ti = decode_tile(args);
    const int t = args.t;
    const double2 *arow = A + (size_t)(args.k - 1) * args.n;

    double2 *s_win = smem;
    double2 *s_arow = smem + args.lds_window;
    double2 *s_ha = s_arow + t;
    uint32_t *s_hb = (uint32_t *)(s_ha + 32);

    if (tid < ti.m) {
        int col = 0;
        s_hb[tid] = high_window_base(ti.T, t, ti.kp, tid, &col);
        s_ha[tid] = arow[col];
    }
    if (tid < t) s_arow[tid] = arow[tid];
    if (ti.kp >= 1) {
        const uint32_t w = dbinom(t, ti.kp - 1);
        const double2 *src = prev + ti.base_low;
        for (uint32_t i = tid; i < w; i += kLayerBlock) s_win[i] = src[i];
    }
    __syncthreads();

    const uint32_t ck = ti.ck;
    const uint32_t *lt = g_lowtab + args.low_off[ti.g];
    double2 *out = next + ti.base_out;
    for (uint32_t r = tid; r < ck; r += kLayerBlock) {
        double re = 0.0, im = 0.0;
        // low columns, ascending (all below t)
        int p = 0;
        for (; p + 4 <= ti.kp; p += 4) {
            uint32_t e[4];
#pragma unroll
            for (int u = 0; u < 4; u++) e[u] = lt[(uint32_t)(p + u) * ck + r];
#pragma unroll
            for (int u = 0; u < 4; u++) cfma(re, im, s_arow[e[u] >> 16], s_win[e[u] & 0xffffu]);
        }
        for (; p < ti.kp; p++) {
            const uint32_t e = lt[(uint32_t)p * ck + r];
            cfma(re, im, s_arow[e >> 16], s_win[e & 0xffffu]);
        }
        // high columns, ascending (all >= t); windows aligned with the tile
        int q = 0;
        for (; q + 4 <= ti.m; q += 4) {
            double2 w[4];
#pragma unroll
            for (int u = 0; u < 4; u++) w[u] = prev[s_hb[q + u] + r];
#pragma unroll
            for (int u = 0; u < 4; u++) cfma(re, im, s_ha[q + u], w[u]);
        }
        for (; q < ti.m; q++) cfma(re, im, s_ha[q], prev[s_hb[q] + r]);
        if (args.nt_store) {
            __builtin_nontemporal_store(re, &out[r].x);
            __builtin_nontemporal_store(im, &out[r].y);
        } else {
            out[r] = make_double2(re, im);
        }
    }
}

hipError_t launch_layer_c128(const void *prev, void *next, const void *packed,
                             const LayerArgs &a, uint32_t grid, hipStream_t s) {
    const size_t lds = layer_lds_bytes_c128(a);
    hipLaunchKernelGGL(k_layer_c128, dim3(grid), dim3(kLayerBlock), lds, s, (const double2 *)prev,
                       (double2 *)next, (const double2 *)packed, a);
    return hipGetLastError();
}

__global__ void k_readout_c128(const double2 *last, double2 *result) {
    if (threadIdx.x == 0) *result = last[0];
}

hipError_t launch_readout_c128(const void *last, void *result, hipStream_t s) {
    hipLaunchKernelGGL(k_readout_c128, dim3(1), dim3(64), 0, s, (const double2 *)last,
                       (double2 *)result);
    return hipGetLastError();
}

// ------------------------------------------------------------- mod p
typedef unsigned __int128 u128;

// x mod p for p = 2^61 - c (c small): 2^61 = c (mod p), folded twice.
__device__ __forceinline__ uint64_t fold61(u128 x, uint64_t p) {
    const uint64_t M = (1ull << 61) - 1;
    const uint64_t c = (1ull << 61) - p;
    const u128 y = (u128)((uint64_t)x & M) + (u128)c * (x >> 61);
    uint64_t z = ((uint64_t)y & M) + c * (uint64_t)(y >> 61);
    if (z >= p) z -= p;
    if (z >= p) z -= p;
    return z;
}

__global__ void k_reduce_modp(const int64_t *__restrict__ a, int n, const uint64_t *__restrict__ primes,
                              int rp, uint64_t *__restrict__ red, uint64_t *__restrict__ layer1,
                              size_t plane) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * n) return;
    const int64_t v = a[i];
    for (int r = 0; r < rp; r++) {
        const uint64_t p = primes[r];
        const uint64_t mag = v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v;
        uint64_t m = mag % p;
        if (v < 0 && m != 0) m = p - m;
        red[(size_t)r * n * n + i] = m;
        if (i < n) layer1[(size_t)r * plane + i] = m;
    }
}

hipError_t launch_reduce_modp(const int64_t *a_dev, int n, const uint64_t *primes, int rp,
                              uint64_t *red, uint64_t *layer1, size_t plane, hipStream_t s) {
    const int tot = n * n;
    hipLaunchKernelGGL(k_reduce_modp, dim3((tot + 255) / 256), dim3(256), 0, s, a_dev, n, primes, rp,
                       red, layer1, plane);
    return hipGetLastError();
}

// Per-thread path of the integer sweep (see layer_c128_thin).
template <int RP, bool BIN>
__device__ void layer_modp_thin(const uint64_t *__restrict__ prev, uint64_t *__restrict__ next, size_t plane,
                                const uint64_t *__restrict__ red, const uint64_t *__restrict__ primes,
                                const LayerArgs &args, uint64_t *smem) {
    uint32_t *s_bin = (uint32_t *)smem;                 // C(i, j) at [i * 33 + j]
    uint64_t *s_arow = (uint64_t *)(s_bin + 33 * 33 + 1);  // RP x 32 residues of row k-1 (8-byte aligned)
    const int tid = threadIdx.x, n = args.n;
    for (int i = tid; i < 33 * 33; i += kLayerBlock) s_bin[i] = c_binom.v[i / 33][i % 33];
    if (tid < n) {
#pragma unroll
        for (int r = 0; r < RP; r++) s_arow[r * 32 + tid] = red[(size_t)r * n * n + (size_t)(args.k - 1) * n + tid];
    }
    __syncthreads();
    const uint32_t gid = (blockIdx.x - args.big_blocks) * kLayerBlock + tid;
    if (gid >= args.t_out_start[args.thin_groups]) return;
    int g = 0;
    while (g + 1 < args.thin_groups && args.t_out_start[g + 1] <= gid) g++;
    const int kp = args.t_kp[g], t = args.t;
    const uint32_t ck = args.t_ck[g], local = gid - args.t_out_start[g];
    const uint32_t tile = local / ck, rr = local - tile * ck;
    const uint32_t T = g_highlist[args.t_high_off[g] + tile];
    uint32_t base_out = 0, base_low = 0, base_h = 0;
    {
        uint32_t b = T;
        for (int i = 1; b; i++) {
            const int h = __ffs(b) - 1 + t;
            b &= b - 1;
            base_out += s_bin[h * 33 + kp + i];
            base_low += s_bin[h * 33 + kp + i - 1];
            if (i >= 2) base_h += s_bin[h * 33 + kp + i - 1];
        }
    }
    u128 acc[RP];
#pragma unroll
    for (int r = 0; r < RP; r++) acc[r] = 0;
    const uint32_t *lt = g_lowtab + args.t_low_off[g];
    for (int p = 0; p < kp; p++) {
        const uint32_t e = lt[(uint32_t)p * ck + rr];
        const uint32_t idx = base_low + (e & 0xffffu), col = e >> 16;
        if (BIN) {
            if (s_arow[col] != 0) {
#pragma unroll
                for (int r = 0; r < RP; r++) acc[r] += prev[(size_t)r * plane + idx];
            }
        } else {
#pragma unroll
            for (int r = 0; r < RP; r++) {
                const uint64_t a = s_arow[r * 32 + col];
                if (a != 0) acc[r] += (u128)a * prev[(size_t)r * plane + idx];
            }
        }
    }
    uint32_t b = T;
    int q = 1, hprev = 0;
    while (b) {
        const int h = __ffs(b) - 1 + t;
        b &= b - 1;
        if (q > 1) base_h = base_h + s_bin[hprev * 33 + kp + q - 1] - s_bin[h * 33 + kp + q - 1];
        const uint32_t idx = base_h + rr;
        if (BIN) {
            if (s_arow[h] != 0) {
#pragma unroll
                for (int r = 0; r < RP; r++) acc[r] += prev[(size_t)r * plane + idx];
            }
        } else {
#pragma unroll
            for (int r = 0; r < RP; r++) {
                const uint64_t a = s_arow[r * 32 + h];
                if (a != 0) acc[r] += (u128)a * prev[(size_t)r * plane + idx];
            }
        }
        hprev = h;
        q++;
    }
#pragma unroll
    for (int r = 0; r < RP; r++) next[(size_t)r * plane + base_out + rr] = fold61(acc[r], primes[r]);
}

// BIN: every entry of this layer's row of A is 0 or 1 (then equal in every
// residue), so a term is either skipped or a plain addition.
template <int RP, bool BIN>
__global__ __launch_bounds__(kLayerBlock) void k_layer_modp(const uint64_t *__restrict__ prev,
                                                            uint64_t *__restrict__ next, size_t plane,
                                                            const uint64_t *__restrict__ red,
                                                            const uint64_t *__restrict__ primes,
                                                            const LayerArgs args) {
    extern __shared__ uint64_t smem_u[];
    if (blockIdx.x >= args.big_blocks) {
        layer_modp_thin<RP, BIN>(prev, next, plane, red, primes, args, smem_u);
        return;
    }
    const int tid = threadIdx.x;
    const TileInfo ti = decode_tile(args);
    const int t = args.t, n = args.n;
    const uint32_t W = args.lds_window;

    uint64_t *s_win = smem_u;                       // RP x W
    uint64_t *s_arow = smem_u + (size_t)RP * W;     // RP x t
    uint64_t *s_ha = s_arow + RP * t;               // RP x 32
    uint32_t *s_hb = (uint32_t *)(s_ha + RP * 32);  // 32

    if (tid < ti.m) {
        int col = 0;
        s_hb[tid] = high_window_base(ti.T, t, ti.kp, tid, &col);
#pragma unroll
        for (int r = 0; r < RP; r++) s_ha[r * 32 + tid] = red[(size_t)r * n * n + (size_t)(args.k - 1) * n + col];
    }
    if (tid < t) {
#pragma unroll
        for (int r = 0; r < RP; r++) s_arow[r * t + tid] = red[(size_t)r * n * n + (size_t)(args.k - 1) * n + tid];
    }
    if (ti.kp >= 1) {
        const uint32_t w = dbinom(t, ti.kp - 1);
        for (uint32_t i = tid; i < w; i += kLayerBlock) {
#pragma unroll
            for (int r = 0; r < RP; r++) s_win[r * W + i] = prev[(size_t)r * plane + ti.base_low + i];
        }
    }
    __syncthreads();

    uint64_t pr[RP];
#pragma unroll
    for (int r = 0; r < RP; r++) pr[r] = primes[r];
    const uint32_t ck = ti.ck;
    const uint32_t *lt = g_lowtab + args.low_off[ti.g];
    for (uint32_t rr = tid; rr < ck; rr += kLayerBlock) {
        u128 acc[RP];
#pragma unroll
        for (int r = 0; r < RP; r++) acc[r] = 0;
        for (int p = 0; p < ti.kp; p++) {
            const uint32_t e = lt[(uint32_t)p * ck + rr];
            const uint32_t idx = e & 0xffffu, col = e >> 16;
            if (BIN) {
                if (s_arow[col] != 0) {
#pragma unroll
                    for (int r = 0; r < RP; r++) acc[r] += s_win[r * W + idx];
                }
            } else {
#pragma unroll
                for (int r = 0; r < RP; r++) {
                    const uint64_t a = s_arow[r * t + col];
                    if (a != 0) acc[r] += (u128)a * s_win[r * W + idx];
                }
            }
        }
        for (int q = 0; q < ti.m; q++) {
            const uint32_t base = s_hb[q] + rr;
            if (BIN) {
                if (s_ha[q] != 0) {
#pragma unroll
                    for (int r = 0; r < RP; r++) acc[r] += prev[(size_t)r * plane + base];
                }
            } else {
#pragma unroll
                for (int r = 0; r < RP; r++) {
                    const uint64_t a = s_ha[r * 32 + q];
                    if (a != 0) acc[r] += (u128)a * prev[(size_t)r * plane + base];
                }
            }
        }
#pragma unroll
        for (int r = 0; r < RP; r++) next[(size_t)r * plane + ti.base_out + rr] = fold61(acc[r], pr[r]);
    }
}

template <bool BIN>
static void launch_modp_t(const uint64_t *prev, uint64_t *next, size_t plane, const uint64_t *red,
                          const uint64_t *primes, int rp, const LayerArgs &a, uint32_t grid, size_t lds,
                          hipStream_t s) {
    switch (rp) {
    case 1:
        hipLaunchKernelGGL((k_layer_modp<1, BIN>), dim3(grid), dim3(kLayerBlock), lds, s, prev, next, plane,
                           red, primes, a);
        break;
    case 2:
        hipLaunchKernelGGL((k_layer_modp<2, BIN>), dim3(grid), dim3(kLayerBlock), lds, s, prev, next, plane,
                           red, primes, a);
        break;
    default:
        hipLaunchKernelGGL((k_layer_modp<3, BIN>), dim3(grid), dim3(kLayerBlock), lds, s, prev, next, plane,
                           red, primes, a);
        break;
    }
}

hipError_t launch_layer_modp(const uint64_t *prev, uint64_t *next, size_t plane, const uint64_t *red,
                             const uint64_t *primes, int rp, const LayerArgs &a, uint32_t grid,
                             hipStream_t s) {
    if (rp < 1 || rp > kRPMax) return hipErrorInvalidValue;
    const size_t lds = layer_lds_bytes_modp(a, rp);
    if (a.binary_row) launch_modp_t<true>(prev, next, plane, red, primes, rp, a, grid, lds, s);
    else launch_modp_t<false>(prev, next, plane, red, primes, rp, a, grid, lds, s);
    return hipGetLastError();
}

__global__ void k_readout_modp(const uint64_t *last, size_t plane, int rp, uint64_t *out) {
    const int r = threadIdx.x;
    if (r < rp) out[r] = last[(size_t)r * plane];
}

hipError_t launch_readout_modp(const uint64_t *last, size_t plane, int rp, uint64_t *out,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_readout_modp, dim3(1), dim3(64), 0, s, last, plane, rp, out);
    return hipGetLastError();
}

}  // namespace permgpu
