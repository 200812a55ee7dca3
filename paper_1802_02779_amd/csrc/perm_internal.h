// Internal declarations of libpermgpu shared by its HIP and host sources.
//
// Stored sub-permanents (section 4 of the paper): F(S) = per(rows 1..|S|,
// columns S).  Layer k holds F(S) for every k-subset S of the n columns,
// ranked in colexicographic order:
//     rank(S) = sum_{i=1..k} C(s_i, i),   s_1 < ... < s_k   (0-based columns),
// which is also increasing bitmask order.  The layer sweep computes layer k
// from layer k-1 tile by tile.  A tile fixes the "high" part T = S & [t, n)
// (|T| = m) and runs over every "low" part L = S & [0, t) with |L| = k' = k-m:
//   * the tile's outputs have contiguous ranks  base(T, k') + rank_t(L),
//     rank_t(L) in [0, C(t, k'));
//   * removing a low column l in L leads to layer k-1 entries with the same T
//     and |L| = k'-1: one contiguous window of C(t, k'-1) entries, staged in
//     LDS; the entry of L \ {l_p} is found from L and running binomial sums
//     (table "lowmask" below);
//   * removing a high column h in T leads to a window of C(t, k') entries
//     aligned 1:1 with the tile's outputs (same rank_t(L)): read straight from
//     HBM, coalesced.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace permgpu {

constexpr int kNMax = 34;
constexpr int kTMax = 15;        // largest low window (columns) of a tile
constexpr int kHighBits = 22;    // largest high part (columns) of a tile (n - t at n = 34, t = 12)
constexpr int kBatchNMax = 12;   // largest order of the on-chip batched kernel
constexpr int kRPMax = 3;        // primes that share one integer sweep
constexpr int kMaxGroups = 32;   // k' groups in one layer launch
constexpr int kBatchBlockComplex = 512;  // threads of a complex batched workgroup
constexpr int kBatchBlockInt = 256;      // threads of an integer batched workgroup

// Cache-aware tile order (perm_order.cpp): built for high parts of at most
// this many columns; an empty slot of a padded group holds kNoTile.
constexpr int kOrderNhMax = 18;
constexpr uint32_t kNoTile = 0xffffffffu;

constexpr int kBinomDim = kNMax + 1;  // C(i, j) for 0 <= i, j <= kNMax (all below 2^32)

struct BinomTable {
    uint32_t v[kBinomDim][kBinomDim];
};

constexpr BinomTable make_binom() {
    BinomTable b{};
    for (int i = 0; i <= kNMax; i++) {
        b.v[i][0] = 1;
        for (int j = 1; j <= i; j++)
            b.v[i][j] = b.v[i - 1][j - 1] + (j <= i - 1 ? b.v[i - 1][j] : 0u);
    }
    return b;
}

inline constexpr BinomTable kBinom = make_binom();

// LDS copies of the binomial table (per-thread paths): words rounded up to a
// 16-byte multiple so that what follows is aligned; slots for one row of A.
constexpr int kBinomWords = (kBinomDim * kBinomDim + 3) & ~3;
constexpr int kRowSlots = 36;  // >= kNMax
static_assert(kRowSlots >= kNMax, "row slots");

constexpr uint32_t binom_host(int i, int j) {
    return (i < 0 || j < 0 || i > kNMax || j > kNMax) ? 0u : kBinom.v[i][j];
}

// lowmask layout: for each t in 1..kTMax, for each k' in 0..t, entry
// [rank_t(L)] = L | (sum_i C(l_i, i)) << 16 for the k'-subsets L of [0, t)
// (l_0 < l_1 < ...): the low part of output rank_t(L) of a tile, and the sum
// that gives the ranks of its predecessors with one table read per output:
//   rank_t(L \ {l_p}) = sum_{i<p} C(l_i, i+1) + sum_{i>p} C(l_i, i).
constexpr uint32_t lowmask_t_base(int t) { return (2u << (t - 1)) - 2u; }  // sum_{s < t} 2^s
constexpr uint32_t lowmask_kp_off(int t, int kp) {  // sum_{k'' < k'} C(t, k'')
    uint32_t s = 0;
    for (int u = 0; u < kp; u++) s += binom_host(t, u);
    return s;
}
constexpr uint32_t kLowmaskEntries = lowmask_t_base(kTMax + 1);
// LDS binomials of the tiled path: C(c, i) at [c * kLowBinDim + i], c < t, i <= kTMax.
constexpr int kLowBinDim = kTMax + 1;

// highlist: every mask below 2^kHighBits, sorted by (popcount, value).
// Masks of popcount m below 2^nh are the first C(nh, m) entries of block m.
constexpr uint32_t highlist_off(int m) {
    uint32_t s = 0;
    for (int u = 0; u < m; u++) s += binom_host(kHighBits, u);
    return s;
}

struct LayerArgs {
    int n, k, t;
    int ngroups;
    int chunk;                // XCD chunking of the tile order (0 = hardware order)
    int nt_store;             // non-temporal stores of the outputs
    int binary_row;           // integer path: this layer's row of A is all 0/1
    uint32_t lds_window;      // entries reserved for the largest low window
    int32_t kp[kMaxGroups];   // k' of group g
    uint32_t start[kMaxGroups + 1];  // first tile of group g (prefix sums)
    uint32_t ck[kMaxGroups];         // C(t, k'): outputs per tile
    uint32_t lmask_off[kMaxGroups];  // lowmask offset of (t, k')
    uint32_t high_off[kMaxGroups];   // highlist offset of popcount m = k - k'
    // Groups whose tiles have fewer than `thin_below` outputs are not tiled:
    // workgroups past big_blocks give one output to each thread instead.
    uint32_t big_blocks;
    int thin_groups;
    int32_t t_kp[kMaxGroups];
    uint32_t t_ck[kMaxGroups];
    uint32_t t_out_start[kMaxGroups + 1];  // prefix sums of the thin groups' outputs
    uint32_t t_lmask_off[kMaxGroups];
    uint32_t t_high_off[kMaxGroups];
    // Cache-aware tile order (null: colex order with XCD chunking).  Tile
    // b - start[g] of group g is zorder[zoff[g] + b - start[g]]: its high
    // part, or kNoTile for a padding slot.  Group starts are multiples of 8.
    const uint32_t *zorder;
    uint32_t zoff[kMaxGroups];
};

// Fills LayerArgs for layer k of order n with low window t; groups with
// fewer than thin_below outputs per tile go to the per-thread path.  With
// pad8 every tiled group takes a multiple of 8 workgroups (for zorder).
// Returns the grid size (tiled workgroups + per-thread workgroups).
uint32_t plan_layer(int n, int k, int t, int chunk, int nt_store, uint32_t thin_below, LayerArgs *a,
                    bool pad8 = false);

// Dynamic LDS bytes of a layer launch.
size_t layer_lds_bytes_c128(const LayerArgs &a);
size_t layer_lds_bytes_modp(const LayerArgs &a, int rp);

// ---- launchers (perm_layers.hip); all return hipError_t of the launch ----
hipError_t ensure_tables(int device, hipStream_t s);
hipError_t launch_pack_c128(const void *a_dev, int64_t lda, int n, void *packed, void *layer1,
                            hipStream_t s);
hipError_t launch_layer_c128(const void *prev, void *next, const void *packed,
                             const LayerArgs &a, uint32_t grid, hipStream_t s);
hipError_t launch_readout_c128(const void *last, void *result, hipStream_t s);

// Integer path: `rp` primes share the sweep; tables are rp planes of `plane`
// entries each.  `red` holds rp reduced copies of the matrix (rp * n * n).
// A prime of 0 means plain 64-bit two's-complement arithmetic (entries as
// they are, outputs truncated to 64 bits), for layers bounded below 2^63.
hipError_t launch_reduce_modp(const int64_t *a_dev, int n, const uint64_t *primes, int rp,
                              uint64_t *red, uint64_t *layer1, size_t plane, hipStream_t s);
hipError_t launch_layer_modp(const uint64_t *prev, uint64_t *next, size_t plane,
                             const uint64_t *red, const uint64_t *primes, int rp,
                             const LayerArgs &a, uint32_t grid, hipStream_t s);
hipError_t launch_readout_modp(const uint64_t *last, size_t plane, int rp, uint64_t *out,
                               hipStream_t s);
// count plain 64-bit values of one layer (src) to rp residue planes (dst).
hipError_t launch_int64_to_modp(const uint64_t *src, uint64_t *dst, size_t plane, size_t count,
                                const uint64_t *primes, int rp, hipStream_t s);

// ---- allocation-free solve (perm_noalloc.hip) ----
// Device address and size of the file-scope scratch array on the current
// device (looked up once per device).
hipError_t noalloc_scratch(void **ptr, size_t *bytes);

// ---- batched on-chip kernel (perm_batch.hip) ----
struct BatchChunk {
    uint32_t first;   // index into the sorted order
    uint16_t count;   // matrices in this chunk (same n)
    uint8_t n;
    uint8_t group;    // log2 of threads per matrix (a workgroup holds block / 2^group matrices)
};

hipError_t launch_batch_reset(uint32_t *counter, hipStream_t s);
hipError_t launch_batch_c128(const void *mats, const int64_t *offsets, const uint32_t *order,
                             const BatchChunk *chunks, uint32_t nchunks, uint32_t *counter,
                             void *results, int nmax, int grid, hipStream_t s);
// One matrix of order n (packed row-major at mat, device) through the batched
// kernel in a single workgroup; writes per(A) to *result (device).
hipError_t launch_single_c128(const void *mat, int n, void *result, hipStream_t s);
// Same for residues: res[r] = per(A) mod primes[r], r < nprimes.
hipError_t launch_single_modp(const int64_t *mat, int n, const uint64_t *primes, int nprimes, uint64_t *res,
                              hipStream_t s);
hipError_t upload_batch_masks(const uint16_t *host, hipStream_t s);

// ---- Ryser's formula, Gray-code walk (perm_ryser.hip) ----
// AT (n x n, column j contiguous) from a device matrix with leading dim lda.
hipError_t launch_ryser_transpose_c128(const void *a_dev, int64_t lda, int n, void *at, hipStream_t s);
// 2^(n-m) threads of 2^m codes each in `blocks` workgroups of 256 (the
// last may be partial); partial[blocks] sums, then *out = per(A) (device).
hipError_t launch_ryser_c128(const void *at, int n, int m, void *partial, uint32_t blocks, void *out,
                             hipStream_t s);
// Residues: atr[r*n*n + j*n + i] = a[i][j] mod primes[r] (device), for
// r < nprimes; res[r] = per(A) mod primes[r] (device); partial holds
// nprimes * blocks values.
hipError_t launch_ryser_modp(const uint64_t *atr, const uint64_t *primes, int nprimes, int n, int m,
                             uint64_t *partial, uint32_t blocks, uint64_t *res, hipStream_t s);
hipError_t launch_batch_modp(const int64_t *mats, const int64_t *offsets, const uint32_t *order,
                             const BatchChunk *chunks, uint32_t nchunks, uint32_t *counter,
                             const uint64_t *primes, int nprimes, uint64_t *res, uint32_t count,
                             int nmax, int grid, hipStream_t s);
size_t batch_lds_bytes(int nmax, int elem_bytes);
// Masks below 2^nmax grouped by popcount; inside a popcount the masks with
// highest bit h come after all lower ones (so the masks of popcount k below
// 2^n are the first C(n,k) entries for every n <= nmax), and each run of one
// highest bit is interleaved by the mask's low three bits so that eight
// neighbouring lanes read eight different LDS bank groups.
void batch_mask_list(int nmax, uint16_t *out);
size_t batch_area_bytes(int nmax, int elem_bytes);
int batch_blocks_per_cu(int nmax, int elem_bytes);

}  // namespace permgpu
