// Internal interface of the repeated-column sweep (count-vector tables):
// the plan layout the host builds and the device launches that read it.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace permgpu {

constexpr int kMultiBlock = 256;  // outputs per workgroup (one rank chunk)
constexpr int kMultiMMax = 64;    // distinct columns

// One layer k of the sweep over count vectors c with |c| = k.  The layer is
// laid out in colex order (last column most significant).  Columns 0..L-1
// are "low", L..m-1 "high"; all vectors sharing the high part h form one
// contiguous tile whose low parts (sum kp = k - |h|) run in colex order.
//   tiles[i] = {base_out, kp, low_base, win_off} for the layer's tiles in rank
//              order, then one sentinel {size, 0, 0, total windows}; low_base
//              is the first rank of tile h in layer k-1 (used when kp > 0);
//   wins[w]  = {base_in, col}: the tile h - e_col of layer k-1, aligned 1:1
//              with tile h (same low part, same offset), ascending col;
//   chunk_tile[c] = the tile holding output c * kMultiBlock, and at
//              [nchunks] the tile holding the last output;
//   lowlist  = low parts (mixed-radix index v = sum_i c_i * prod_{i'<i}
//              (mult[i'] + 1)) grouped by sum, colex within a sum, sum kp
//              starting at lowoff[kp];
//   lowpred[v * L + i] = rank of v - e_i among the low parts of its sum, or
//              0xffffffff when c_i = 0.
struct MultiLayerArgs {
    const uint4 *tiles;
    const uint2 *wins;
    const uint32_t *chunk_tile;
    const uint32_t *lowlist;
    const uint32_t *lowoff;
    const uint32_t *lowpred;
    uint32_t size;
    uint32_t nchunks;
    int L;
    int m;
};

hipError_t launch_multi_pack_c128(const void *a_dev, int64_t lda, int n, int m, void *packed, void *layer1,
                                  hipStream_t s);
hipError_t launch_multi_layer_c128(const void *prev, void *next, const void *row, const MultiLayerArgs &g,
                                   hipStream_t s);
hipError_t launch_multi_readout_c128(const void *last, double scale, void *out, hipStream_t s);
// red: residues [prime][n][m]; layer1 planes get row 0.
hipError_t launch_multi_init_modp(const uint64_t *red, int n, int m, int rp, uint64_t *layer1, size_t plane,
                                  hipStream_t s);
hipError_t launch_multi_layer_modp(const uint64_t *prev, uint64_t *next, size_t plane, const uint64_t *red, int n,
                                   int k, const uint64_t *primes, int rp, const MultiLayerArgs &g, hipStream_t s);

}  // namespace permgpu
