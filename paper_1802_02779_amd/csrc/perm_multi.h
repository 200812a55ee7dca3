// Internal interface of the repeated-column sweep (count-vector tables):
// the plan layout the host builds and the device launches that read it.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace permgpu {

constexpr int kMultiBlock = 256;     // threads per tile workgroup
constexpr int kMultiMMax = 64;       // distinct columns
constexpr int kMultiWinMax = 3072;   // largest low window staged in LDS (entries)
constexpr int kMultiThin = 128;      // tiles with at most this many outputs take one wave each
// Residue sweeps stage a workgroup tile's low window (RP planes) in LDS up to
// this size; larger windows (above 2389 entries with three planes, which only
// plans of billions of count vectors reach) are read from cache instead.
constexpr size_t kMultiModpLdsMax = 56 * 1024;

// Layer k of the sweep over count vectors c with |c| = k, in colex order
// (last column most significant).  Columns 0..L-1 are "low", L..m-1 "high".
// The vectors sharing a high part h form one contiguous tile; their low
// parts (sum kp = k - |h|) run in colex order, WL[kp] of them.  The rank of
// a vector is sum_j G_j(P_j, c_j) with P_j = c_0 + ... + c_j and
// G_j(P, c) = sum_{v < c} W_j(P - v), W_j(s) = vectors over columns < j
// with sum s; for a tile's first vector only the high terms are nonzero.
//   G        [j - L][P][c] for high columns j, P in 0..n, c in 0..tmax;
//   hlist    high parts as mixed-radix indices (column L least significant),
//            sorted by |h| then index; those with |h| = q start at qoff[q];
//   hstride, hradix  per high column: stride of its digit and mult + 1;
//   lp16     per low sum kp, at kpoff[kp] (16-bit units): L x WL[kp] ranks,
//            [i][r] = rank of (low part r) - e_i among the low parts of sum
//            kp - 1, or 0xffff when that low part has no copy of column i;
//   WL       low parts per sum.
// Tile b of layer k is hlist[tile0 + b].  Tiles [0, thin_lo) and
// [thin_hi, ntiles) are thin (few outputs): thin_wg workgroups take four of
// them each, one per wave; the tiles between take a workgroup each.
struct MultiLayerArgs {
    const uint32_t *G;
    const uint32_t *hlist;
    const uint32_t *hstride;
    const uint32_t *hradix;
    const uint16_t *lp16;
    const uint32_t *kpoff;
    const uint32_t *WL;
    uint32_t tile0;
    uint32_t ntiles;
    uint32_t thin_lo, thin_hi, thin_wg;
    int n, m, L, SL, k, tmax1;
};

hipError_t launch_multi_pack_c128(const void *a_dev, int64_t lda, int n, int m, void *packed, void *layer1,
                                  hipStream_t s);
hipError_t launch_multi_layer_c128(const void *prev, void *next, const void *row, const MultiLayerArgs &g,
                                   uint32_t max_window, hipStream_t s);
hipError_t launch_multi_readout_c128(const void *last, double scale, void *out, hipStream_t s);
// red: residues [prime][n][m]; layer1 planes get row 0.  A prime of 0 means
// plain 64-bit arithmetic (red holds the entries themselves).
hipError_t launch_multi_init_modp(const uint64_t *red, int n, int m, int rp, uint64_t *layer1, size_t plane,
                                  hipStream_t s);
// A layer of plain 64-bit values to rp residue planes (perm_layer_modp.hip).
hipError_t launch_int64_to_modp(const uint64_t *src, uint64_t *dst, size_t plane, size_t count,
                                const uint64_t *primes, int rp, hipStream_t s);
hipError_t launch_multi_layer_modp(const uint64_t *prev, uint64_t *next, size_t plane, const uint64_t *red,
                                   const uint64_t *primes, int rp, const MultiLayerArgs &g, uint32_t max_window,
                                   hipStream_t s);

// FP64 FMA probe (perm_probe.hip): `blocks` workgroups of independent
// chains, `iters` steps each; probe_fma_flops gives the flops of one launch.
hipError_t launch_probe_fma(double *out, int blocks, int iters, hipStream_t s);
double probe_fma_flops(int blocks, int iters);
// Integer probe (perm_probe.hip): mode 0 = 128-bit sums of 64 x 64-bit
// products folded mod 2^61 - 1 every 16 terms, mode 1 = 64-bit additions;
// probe_int_terms gives the terms of one launch.
hipError_t launch_probe_int(uint64_t *out, int blocks, int iters, int mode, hipStream_t s);
double probe_int_terms(int blocks, int iters);

}  // namespace permgpu
