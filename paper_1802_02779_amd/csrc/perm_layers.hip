// Layer sweep of the Store-zechin permanent on gfx950: rank tables, layer
// planning and tile decoding shared by the complex128 and mod-p layer kernels.
//
// Section 4 of the paper develops per(A) along the last row and stores every
// sub-permanent once.  Here the stored values F(S) = per(rows 1..|S|, cols S)
// are evaluated layer by layer (|S| = 1, 2, ..., n); layer k needs only layer
// k-1:  F(S) = sum_{j in S, ascending} a[k-1][j] * F(S \ {j})  (0-based row).
// Tiling, ranks and tables are described in perm_internal.h.
#include "perm_internal.h"

namespace permgpu {

__constant__ BinomTable c_binom = make_binom();
__device__ uint32_t g_lowmask[kLowmaskEntries];
__device__ uint32_t g_highlist[1u << kHighBits];

__device__ __forceinline__ uint32_t dbinom(int i, int j) { return c_binom.v[i][j]; }

// ------------------------------------------------------------------ tables
// lowmask entries of the k'-subsets L of [0, t), one thread per L != 0.
__global__ void k_build_lowmask(int t) {
    const uint32_t L = blockIdx.x * blockDim.x + threadIdx.x;
    if (L >= (1u << t) || L == 0) return;
    const int kp = __popc(L);
    uint32_t rank = 0, tb = 0;  // sum_i C(l_i, i + 1) (colex rank), sum_i C(l_i, i)
    uint32_t b = L;
    for (int i = 0; b; i++) {
        const int c = __ffs(b) - 1;
        b &= b - 1;
        rank += dbinom(c, i + 1);
        tb += dbinom(c, i);
    }
    g_lowmask[lowmask_t_base(t) + lowmask_kp_off(t, kp) + rank] = L | (tb << 16);
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
        hipLaunchKernelGGL(k_build_lowmask, dim3((threads + 255) / 256), dim3(256), 0, s, t);
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
uint32_t plan_layer(int n, int k, int t, int chunk, int nt_store, uint32_t thin_below, LayerArgs *a, bool pad8) {
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
    a->zorder = nullptr;
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
            a->t_lmask_off[g] = lowmask_t_base(t) + lowmask_kp_off(t, kp);
            a->t_high_off[g] = highlist_off(m);
            thin_out += binom_host(nh, m) * ck;
            continue;
        }
        const int g = a->ngroups++;
        a->kp[g] = kp;
        a->start[g] = tiles;
        a->ck[g] = ck;
        a->lmask_off[g] = lowmask_t_base(t) + lowmask_kp_off(t, kp);
        a->high_off[g] = highlist_off(m);
        tiles += pad8 ? (binom_host(nh, m) + 7u) & ~7u : binom_host(nh, m);
        if (kp >= 1 && binom_host(t, kp - 1) > a->lds_window) a->lds_window = binom_host(t, kp - 1);
    }
    a->start[a->ngroups] = tiles;
    a->t_out_start[a->thin_groups] = thin_out;
    a->big_blocks = tiles;
    return tiles + (thin_out + 255) / 256;
}

size_t layer_lds_bytes_c128(const LayerArgs &a) {
    const size_t tiled = (size_t)(a.lds_window + a.t + 32) * 16 + 32 * 4 + (size_t)kTMax * kLowBinDim * 4;
    const size_t thin = (size_t)kBinomWords * 4 + kRowSlots * 16;
    return tiled > thin ? tiled : thin;
}

size_t layer_lds_bytes_modp(const LayerArgs &a, int rp) {
    const size_t tiled = (size_t)rp * (a.lds_window + a.t + 32) * 8 + 32 * 4 + (size_t)kTMax * kLowBinDim * 4;
    const size_t thin = (size_t)kBinomWords * 4 + (size_t)rp * kRowSlots * 8;
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
    bool empty;  // padding slot of the cache-aware order: the workgroup has no tile
};

// The workgroup's tile (group, k', m, high part T; the same in every lane).
// Its ranks come from tile_bases_wave.
__device__ __forceinline__ TileInfo decode_tile(const LayerArgs &A) {
    TileInfo ti;
    const uint32_t tile = A.zorder ? blockIdx.x : xcd_chunk_remap(blockIdx.x, A.big_blocks, (uint32_t)A.chunk);
    int g = 0;
    while (g + 1 < A.ngroups && A.start[g + 1] <= tile) g++;
    ti.g = g;
    ti.kp = A.kp[g];
    ti.m = A.k - ti.kp;
    ti.ck = A.ck[g];
    const uint32_t T =
        A.zorder ? A.zorder[A.zoff[g] + (tile - A.start[g])] : g_highlist[A.high_off[g] + (tile - A.start[g])];
    ti.T = __builtin_amdgcn_readfirstlane(T);
    ti.empty = ti.T == kNoTile;
    if (ti.empty) ti.T = 0;
    ti.base_out = ti.base_low = 0;
    return ti;
}

// Inclusive prefix sum over lanes 0..31 of a wave with DPP lane moves (no
// LDS round trips): four shifts inside each row of 16 lanes, then lane 15
// added to the next row.  Lanes 32..63 hold the scan of their own half.
static_assert(kHighBits < 32, "tile_bases_wave keeps the high columns in lanes 0..31");
__device__ __forceinline__ uint32_t scan32_dpp(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    return v;
}

// A tile's ranks from its high columns h_0 < ... < h_{m-1} (all >= t), with
// A_i = C(h_i, k' + i + 1) and B_i = C(h_i, k' + i):
//   first output rank            sum_i A_i,
//   low window (layer k-1)       sum_i B_i,
//   window without h_q           sum_{i<q} A_i + sum_{i>q} B_i.
// One lane per high column and two prefix sums over lanes 0..31, so the
// wave gets them in one round of table reads instead of a loop over the
// columns.  Every lane
// of the calling wave must call it; lane q < m receives its window base and
// h_q, every lane the tile's two bases.
__device__ __forceinline__ void tile_bases_wave(const LayerArgs &A, TileInfo &ti, uint32_t &hb, int &col) {
    const int lane = threadIdx.x & 63;
    uint32_t b = ti.T;
    for (int j = 0; j < lane && b; j++) b &= b - 1;  // lane-th set bit of T lowest
    const bool act = lane < ti.m;
    const int h = act ? __ffs(b) - 1 + A.t : 0;
    const uint32_t a = act ? dbinom(h, ti.kp + lane + 1) : 0u;
    const uint32_t c = act ? dbinom(h, ti.kp + lane) : 0u;
    // m <= kHighBits < 32: lane 31 holds the totals
    const uint32_t ia = scan32_dpp(a), ic = scan32_dpp(c);
    const uint32_t tot_c = __builtin_amdgcn_readlane(ic, 31);
    ti.base_out = __builtin_amdgcn_readlane(ia, 31);
    ti.base_low = tot_c;
    hb = (ia - a) + (tot_c - ic);
    col = h;
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

// Threads per workgroup of both layer kernels.
constexpr int kLayerBlock = 256;

// The whole binomial table into LDS (C(i, j) at [i * kBinomDim + j]) by a
// workgroup of kLayerBlock threads: every thread's loads are issued before
// its LDS writes, so the copy costs one memory latency.
__device__ __forceinline__ void stage_binomials(uint32_t *s_bin, int tid) {
    constexpr int kPer = (kBinomDim * kBinomDim + kLayerBlock - 1) / kLayerBlock;
    uint32_t v[kPer];
#pragma unroll
    for (int u = 0; u < kPer; u++) {
        const int i = tid + u * kLayerBlock;
        if (i < kBinomDim * kBinomDim) v[u] = c_binom.v[i / kBinomDim][i % kBinomDim];
    }
#pragma unroll
    for (int u = 0; u < kPer; u++) {
        const int i = tid + u * kLayerBlock;
        if (i < kBinomDim * kBinomDim) s_bin[i] = v[u];
    }
}

}  // namespace permgpu
