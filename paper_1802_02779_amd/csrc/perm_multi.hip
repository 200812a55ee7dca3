// Repeated columns: the stored-minor sweep over count vectors (part of the
// device translation unit perm_device.hip).
//
// Column j of the n x m input stands for mult[j] identical columns.  Every
// column subset with c_j copies of column j has the same minor, so layer k
// stores one value per count vector c (|c| = k, 0 <= c_j <= mult[j]):
//     G(c) = sum over j ascending with c_j > 0 of a[k-1][j] * G(c - e_j),
// the section-4 development along the last row with the repeating terms
// merged.  One launch per layer, one workgroup per tile (high part h):
//   * the tile's first rank, the first rank of tile h in layer k-1 (its low
//     predecessors) and of each tile h - e_j (high predecessors) come from
//     the closed-form colex rank, one lane per high column;
//   * low predecessors: the window of tile h in layer k-1 is staged in LDS
//     once; the 16-bit rank table gives each output's offsets, read
//     coalesced (lanes are consecutive outputs);
//   * high predecessors: tile h - e_j of layer k-1 at the same offset --
//     coalesced reads of an aligned window.
// The chain visits the low columns, then the high columns, both ascending,
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

// Per-tile scratch in LDS.
struct MultiTileLds {
    uint32_t wbase[kMultiMMax];  // first rank of tile h - e_col in layer k-1, compacted
    uint32_t wcol[kMultiMMax];   // its column
    uint32_t base_out, kp, low_base, nh;
};

// Workgroup -> tile: runs of kMultiXcdRun consecutive tiles on one XCD
// (workgroups are dealt to the 8 XCDs in turn), so tiles that read the same
// predecessor windows share that XCD's L2; 0 keeps the identity.  b is the
// workgroup's index among the `ntiles` workgroups of its kind.
constexpr uint32_t kMultiXcdRun = 64;

__device__ __forceinline__ uint32_t multi_tile_index(uint32_t b, uint32_t ntiles) {
    if (kMultiXcdRun == 0) return b;
    const uint32_t span = 8u * kMultiXcdRun;
    if (b >= (ntiles / span) * span) return b;
    const uint32_t r = b % span;
    return (b - r) + (r % 8u) * kMultiXcdRun + r / 8u;
}

// Inclusive prefix sum over the 64 lanes of a wave: the 32-lane scan, then
// lane 31's total added to the upper half.
__device__ __forceinline__ uint32_t scan64_dpp(uint32_t v) {
    v = scan32_dpp(v);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

// Decodes tile `tile` of layer k and its predecessor tiles into t, in one
// wave (lane = 0..63, all lanes present) with one lane per high column j
// (prefix sums by DPP lane moves):
//   P_j  = kp + h_L + ... + h_j,
//   base = sum_j G_j(P_j, h_j)                       (this tile, layer k),
//   low  = sum_j G_j(P_j - 1, h_j)                   (tile h, layer k-1, low sum kp-1),
//   win_j = sum_{i<j} G_i(P_i, h_i) + G_j(P_j - 1, h_j - 1)
//         + sum_{i>j} G_i(P_i - 1, h_i)               (tile h - e_j, layer k-1).
// The caller makes t visible to the readers with a barrier.
__device__ __forceinline__ void decode_tile(const MultiLayerArgs &g, uint32_t tile, MultiTileLds &t, int lane) {
    const int mh = g.m - g.L;
    const bool act = lane < mh;
    const uint32_t x = g.hlist[g.tile0 + tile];
    const uint32_t h = act ? (x / g.hstride[lane]) % g.hradix[lane] : 0u;
    const uint32_t ph = scan64_dpp(h);
    const int kp = g.k - (int)__builtin_amdgcn_readlane(ph, 63);
    const int P = kp + (int)ph;
    const uint32_t *Gj = g.G + (size_t)(act ? lane : 0) * (g.n + 1) * g.tmax1;
    const uint32_t a = act ? Gj[(size_t)P * g.tmax1 + h] : 0u;
    const uint32_t b = (act && P >= 1) ? Gj[(size_t)(P - 1) * g.tmax1 + h] : 0u;
    const uint32_t c = (act && h > 0) ? Gj[(size_t)(P - 1) * g.tmax1 + h - 1] : 0u;
    const uint32_t pa = scan64_dpp(a), pb = scan64_dpp(b);
    const uint32_t tot_a = __builtin_amdgcn_readlane(pa, 63), tot_b = __builtin_amdgcn_readlane(pb, 63);
    const uint64_t has = __ballot(act && h > 0);
    if (act && h > 0) {
        const int slot = __popcll(has & ((1ull << lane) - 1));
        t.wbase[slot] = (pa - a) + c + (tot_b - pb);
        t.wcol[slot] = (uint32_t)(g.L + lane);
    }
    if (lane == 0) {
        t.base_out = tot_a;
        t.kp = (uint32_t)kp;
        t.low_base = tot_b;
        t.nh = (uint32_t)__popcll(has);
    }
}

// The high terms of output r, in column order after the low ones, four
// windows' loads in flight.
__device__ __forceinline__ void multi_high_c128(double &re, double &im, const double2 *__restrict__ prev,
                                                const double2 *s_row, const MultiTileLds &t, uint32_t r) {
    const uint32_t nh = t.nh;
    uint32_t w = 0;
    for (; w + 4 <= nh; w += 4) {
        double2 p[4];
#pragma unroll
        for (int u = 0; u < 4; u++) p[u] = prev[t.wbase[w + u] + r];
#pragma unroll
        for (int u = 0; u < 4; u++) cfma(re, im, s_row[t.wcol[w + u]], p[u]);
    }
    for (; w < nh; w++) cfma(re, im, s_row[t.wcol[w]], prev[t.wbase[w] + r]);
}

// Workgroups [0, thin_wg) take four thin tiles each, one per wave, their low
// predecessors gathered straight from the previous layer (a thin tile's
// window is a few cache lines); the others take one tile each with its low
// window staged in LDS.  Both keep the canonical chain: low columns first,
// then high columns, in column order.
__global__ __launch_bounds__(kMultiBlock) void k_multi_layer_c128(const double2 *__restrict__ prev,
                                                                 double2 *__restrict__ next,
                                                                 const double2 *__restrict__ row,
                                                                 const MultiLayerArgs g) {
    extern __shared__ double2 s_win[];
    __shared__ double2 s_row[kMultiMMax];
    __shared__ MultiTileLds tl[kMultiBlock / 64];
    const int tid = threadIdx.x;
    for (int j = tid; j < g.m; j += kMultiBlock) s_row[j] = row[j];
    const uint32_t b = blockIdx.x;
    if (b < g.thin_wg) {
        const int wv = tid >> 6, lane = tid & 63;
        const uint32_t i = b * (kMultiBlock / 64) + (uint32_t)wv;
        const bool valid = i < g.thin_lo + (g.ntiles - g.thin_hi);
        if (valid) decode_tile(g, i < g.thin_lo ? i : g.thin_hi + (i - g.thin_lo), tl[wv], lane);
        __syncthreads();
        if (!valid) return;
        const MultiTileLds &t = tl[wv];
        const uint32_t kp = t.kp, nout = g.WL[kp];
        const uint16_t *lp = g.lp16 + g.kpoff[kp];
        const double2 *low = prev + t.low_base;
        for (uint32_t r = lane; r < nout; r += 64) {
            double re = 0.0, im = 0.0;
            if (kp >= 1) {
                // four columns' index and value loads in flight at a time
                int c = 0;
                for (; c + 4 <= g.L; c += 4) {
                    uint32_t q[4];
                    double2 v[4];
#pragma unroll
                    for (int u = 0; u < 4; u++) q[u] = lp[(size_t)(c + u) * nout + r];
#pragma unroll
                    for (int u = 0; u < 4; u++)
                        if (q[u] != 0xffffu) v[u] = low[q[u]];
#pragma unroll
                    for (int u = 0; u < 4; u++)
                        if (q[u] != 0xffffu) cfma(re, im, s_row[c + u], v[u]);
                }
                for (; c < g.L; c++) {
                    const uint32_t q = lp[(size_t)c * nout + r];
                    if (q != 0xffffu) cfma(re, im, s_row[c], low[q]);
                }
            }
            multi_high_c128(re, im, prev, s_row, t, r);
            next[t.base_out + r] = make_double2(re, im);
        }
        return;
    }
    MultiTileLds &t = tl[0];
    if (tid < 64) decode_tile(g, g.thin_lo + multi_tile_index(b - g.thin_wg, g.thin_hi - g.thin_lo), t, tid);
    __syncthreads();
    const uint32_t kp = t.kp, base_out = t.base_out;
    if (kp >= 1) {
        // two of a thread's loads in flight before their stores
        const uint32_t nwin = g.WL[kp - 1];
        const double2 *src = prev + t.low_base;
        for (uint32_t e = tid; e < nwin; e += 2 * kMultiBlock) {
            const bool b1 = e + kMultiBlock < nwin;
            const double2 v0 = src[e];
            double2 v1;
            if (b1) v1 = src[e + kMultiBlock];
            s_win[e] = v0;
            if (b1) s_win[e + kMultiBlock] = v1;
        }
    }
    __syncthreads();
    const uint32_t nout = g.WL[kp];
    const uint16_t *lp = g.lp16 + g.kpoff[kp];
    for (uint32_t r = tid; r < nout; r += kMultiBlock) {
        double re = 0.0, im = 0.0;
        if (kp >= 1) {
            // eight columns' index loads in flight at a time
            int i = 0;
            for (; i + 8 <= g.L; i += 8) {
                uint32_t q[8];
#pragma unroll
                for (int u = 0; u < 8; u++) q[u] = lp[(size_t)(i + u) * nout + r];
#pragma unroll
                for (int u = 0; u < 8; u++)
                    if (q[u] != 0xffffu) cfma(re, im, s_row[i + u], s_win[q[u]]);
            }
            for (; i < g.L; i++) {
                const uint32_t q = lp[(size_t)i * nout + r];
                if (q != 0xffffu) cfma(re, im, s_row[i], s_win[q]);
            }
        }
        multi_high_c128(re, im, prev, s_row, t, r);
        next[base_out + r] = make_double2(re, im);
    }
}

hipError_t launch_multi_layer_c128(const void *prev, void *next, const void *row, const MultiLayerArgs &g,
                                   uint32_t max_window, hipStream_t s) {
    if (max_window > (uint32_t)kMultiWinMax || g.thin_lo > g.thin_hi || g.thin_hi > g.ntiles ||
        (uint64_t)g.thin_wg * (kMultiBlock / 64) < (uint64_t)g.thin_lo + (g.ntiles - g.thin_hi))
        return hipErrorInvalidValue;
    const uint32_t grid = g.thin_wg + (g.thin_hi - g.thin_lo);
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(k_multi_layer_c128, dim3(grid), dim3(kMultiBlock), (size_t)max_window * 16, s,
                       (const double2 *)prev, (double2 *)next, (const double2 *)row, g);
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
// products below 2^122 exactly in 128 bits, then one fold (the prime 0:
// plain 64-bit arithmetic, see out_modp).  High predecessors are read from
// HBM / cache; low ones from the tile's window staged in LDS (STAGED: RP
// planes of nwin values in s_win) or, for thin tiles, gathered from the
// previous layer.
template <int RP, bool STAGED>
__device__ __forceinline__ void multi_output_modp(const uint64_t *__restrict__ prev, uint64_t *__restrict__ next,
                                                  size_t plane, const uint64_t (*s_row)[kMultiMMax],
                                                  const uint64_t *__restrict__ primes, const MultiLayerArgs &g,
                                                  const MultiTileLds &t, const uint16_t *lp, uint32_t nout,
                                                  uint32_t rr, const uint64_t *s_win, uint32_t nwin) {
    u128 acc[RP];
#pragma unroll
    for (int r = 0; r < RP; r++) acc[r] = 0;
    if (t.kp >= 1) {
        // four columns' index loads in flight at a time
        int i = 0;
        for (; i + 4 <= g.L; i += 4) {
            uint32_t q[4];
#pragma unroll
            for (int u = 0; u < 4; u++) q[u] = lp[(size_t)(i + u) * nout + rr];
#pragma unroll
            for (int u = 0; u < 4; u++)
                if (q[u] != 0xffffu) {
#pragma unroll
                    for (int r = 0; r < RP; r++)
                        acc[r] += (u128)s_row[r][i + u] *
                                  (STAGED ? s_win[r * nwin + q[u]] : prev[(size_t)r * plane + t.low_base + q[u]]);
                }
        }
        for (; i < g.L; i++) {
            const uint32_t q = lp[(size_t)i * nout + rr];
            if (q == 0xffffu) continue;
#pragma unroll
            for (int r = 0; r < RP; r++)
                acc[r] += (u128)s_row[r][i] * (STAGED ? s_win[r * nwin + q] : prev[(size_t)r * plane + t.low_base + q]);
        }
    }
    for (uint32_t w = 0; w < t.nh; w++) {
        const uint32_t col = t.wcol[w], b = t.wbase[w];
#pragma unroll
        for (int r = 0; r < RP; r++) acc[r] += (u128)s_row[r][col] * prev[(size_t)r * plane + b + rr];
    }
#pragma unroll
    for (int r = 0; r < RP; r++) next[(size_t)r * plane + t.base_out + rr] = out_modp(acc[r], primes[r]);
}

// The same split into thin tiles (one per wave) and workgroup tiles as the
// complex sweep.  STAGE: workgroup tiles stage their low window in LDS (RP
// planes of the largest window fit the launch's LDS).
template <int RP, bool STAGE>
__global__ __launch_bounds__(kMultiBlock) void k_multi_layer_modp(const uint64_t *__restrict__ prev,
                                                                 uint64_t *__restrict__ next, size_t plane,
                                                                 const uint64_t *__restrict__ red,
                                                                 const uint64_t *__restrict__ primes,
                                                                 const MultiLayerArgs g) {
    extern __shared__ uint64_t s_winu[];  // RP x the largest low window
    __shared__ uint64_t s_row[RP][kMultiMMax];
    __shared__ MultiTileLds tl[kMultiBlock / 64];
    const int tid = threadIdx.x;
    for (int e = tid; e < RP * g.m; e += kMultiBlock) {
        const int r = e / g.m, j = e - r * g.m;
        s_row[r][j] = red[(size_t)r * g.n * g.m + (size_t)(g.k - 1) * g.m + j];
    }
    const uint32_t b = blockIdx.x;
    if (b < g.thin_wg) {
        const int wv = tid >> 6, lane = tid & 63;
        const uint32_t i = b * (kMultiBlock / 64) + (uint32_t)wv;
        const bool valid = i < g.thin_lo + (g.ntiles - g.thin_hi);
        if (valid) decode_tile(g, i < g.thin_lo ? i : g.thin_hi + (i - g.thin_lo), tl[wv], lane);
        __syncthreads();
        if (!valid) return;
        const MultiTileLds &t = tl[wv];
        const uint32_t nout = g.WL[t.kp];
        const uint16_t *lp = g.lp16 + g.kpoff[t.kp];
        for (uint32_t rr = lane; rr < nout; rr += 64)
            multi_output_modp<RP, false>(prev, next, plane, s_row, primes, g, t, lp, nout, rr, nullptr, 0);
        return;
    }
    if (tid < 64) decode_tile(g, g.thin_lo + multi_tile_index(b - g.thin_wg, g.thin_hi - g.thin_lo), tl[0], tid);
    __syncthreads();
    const MultiTileLds &t = tl[0];
    const uint32_t nout = g.WL[t.kp];
    const uint16_t *lp = g.lp16 + g.kpoff[t.kp];
    if (!STAGE) {
        for (uint32_t rr = tid; rr < nout; rr += kMultiBlock)
            multi_output_modp<RP, false>(prev, next, plane, s_row, primes, g, t, lp, nout, rr, nullptr, 0);
        return;
    }
    // the low window of every plane in LDS, two of a thread's loads in flight
    // before their stores
    const uint32_t nwin = t.kp >= 1 ? g.WL[t.kp - 1] : 0u;
    for (uint32_t e = tid; e < RP * nwin; e += 2 * kMultiBlock) {
        const uint32_t e1 = e + kMultiBlock;
        const uint32_t r0 = e / nwin, r1 = e1 / nwin;
        const uint64_t v0 = prev[(size_t)r0 * plane + t.low_base + (e - r0 * nwin)];
        uint64_t v1 = 0;
        if (e1 < RP * nwin) v1 = prev[(size_t)r1 * plane + t.low_base + (e1 - r1 * nwin)];
        s_winu[e] = v0;
        if (e1 < RP * nwin) s_winu[e1] = v1;
    }
    __syncthreads();
    for (uint32_t rr = tid; rr < nout; rr += kMultiBlock)
        multi_output_modp<RP, true>(prev, next, plane, s_row, primes, g, t, lp, nout, rr, s_winu, nwin);
}

template <int RP>
static void launch_multi_modp_t(const uint64_t *prev, uint64_t *next, size_t plane, const uint64_t *red,
                                const uint64_t *primes, const MultiLayerArgs &g, uint32_t grid, uint32_t max_window,
                                hipStream_t s) {
    const size_t lds = (size_t)max_window * 8 * RP;
    if (lds <= kMultiModpLdsMax)
        hipLaunchKernelGGL((k_multi_layer_modp<RP, true>), dim3(grid), dim3(kMultiBlock), lds, s, prev, next, plane,
                           red, primes, g);
    else
        hipLaunchKernelGGL((k_multi_layer_modp<RP, false>), dim3(grid), dim3(kMultiBlock), 0, s, prev, next, plane,
                           red, primes, g);
}

hipError_t launch_multi_layer_modp(const uint64_t *prev, uint64_t *next, size_t plane, const uint64_t *red,
                                   const uint64_t *primes, int rp, const MultiLayerArgs &g, uint32_t max_window,
                                   hipStream_t s) {
    if (max_window > (uint32_t)kMultiWinMax || g.thin_lo > g.thin_hi || g.thin_hi > g.ntiles ||
        (uint64_t)g.thin_wg * (kMultiBlock / 64) < (uint64_t)g.thin_lo + (g.ntiles - g.thin_hi))
        return hipErrorInvalidValue;
    const uint32_t grid = g.thin_wg + (g.thin_hi - g.thin_lo);
    if (grid == 0) return hipSuccess;
    switch (rp) {
    case 1: launch_multi_modp_t<1>(prev, next, plane, red, primes, g, grid, max_window, s); break;
    case 2: launch_multi_modp_t<2>(prev, next, plane, red, primes, g, grid, max_window, s); break;
    case 3: launch_multi_modp_t<3>(prev, next, plane, red, primes, g, grid, max_window, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace permgpu
