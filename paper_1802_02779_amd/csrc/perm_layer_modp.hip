// Integer layer sweep of the Store-zechin permanent on gfx950 (part of the
// device translation unit perm_device.hip; tables, planning and tile decoding
// come from perm_layers.hip).
//
// Residues mod p = 2^61 - c: the sum of the k products of one stored value is
// kept exact in 128 bits and folded once per output.  The value p = 0 selects
// plain 64-bit two's-complement arithmetic instead (entries taken as they are,
// each output truncated to 64 bits): exact for the layers whose stored values
// and partial sums the host has bounded below 2^63.
namespace permgpu {

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

// One output: folded mod p, or (p = 0) the low 64 bits of the exact sum.
__device__ __forceinline__ uint64_t out_modp(u128 x, uint64_t p) { return p == 0 ? (uint64_t)x : fold61(x, p); }

__global__ void k_reduce_modp(const int64_t *__restrict__ a, int n, const uint64_t *__restrict__ primes,
                              int rp, uint64_t *__restrict__ red, uint64_t *__restrict__ layer1,
                              size_t plane) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * n) return;
    const int64_t v = a[i];
    for (int r = 0; r < rp; r++) {
        const uint64_t p = primes[r];
        const uint64_t mag = v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v;
        uint64_t m = (uint64_t)v;
        if (p != 0) {
            m = mag % p;
            if (v < 0 && m != 0) m = p - m;
        }
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
    uint32_t *s_bin = (uint32_t *)smem;                 // C(i, j) at [i * kBinomDim + j]
    uint64_t *s_arow = (uint64_t *)(s_bin + kBinomWords);  // RP x kRowSlots residues of row k-1
    const int tid = threadIdx.x, n = args.n;
    stage_binomials(s_bin, tid);
    if (tid < n) {
#pragma unroll
        for (int r = 0; r < RP; r++) s_arow[r * kRowSlots + tid] = red[(size_t)r * n * n + (size_t)(args.k - 1) * n + tid];
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
            base_out += s_bin[h * kBinomDim + kp + i];
            base_low += s_bin[h * kBinomDim + kp + i - 1];
            if (i >= 2) base_h += s_bin[h * kBinomDim + kp + i - 1];
        }
    }
    u128 acc[RP];
#pragma unroll
    for (int r = 0; r < RP; r++) acc[r] = 0;
    // low columns: the output's low part L and sum_i C(l_i, i) from one
    // table entry, predecessor ranks from running sums
    const uint32_t e = kp > 0 ? g_lowmask[args.t_lmask_off[g] + rr] : 0u;
    uint32_t bl = e & 0xffffu;
    const uint32_t totb = e >> 16;
    uint32_t pa = 0, pb = 0;
    for (int p = 0; bl; p++) {
        const int col = __ffs(bl) - 1;
        bl &= bl - 1;
        const uint32_t cb = s_bin[col * kBinomDim + p];
        const uint32_t idx = base_low + pa + totb - pb - cb;
        pa += s_bin[col * kBinomDim + p + 1];
        pb += cb;
        if (BIN) {
            if (s_arow[col] != 0) {
#pragma unroll
                for (int r = 0; r < RP; r++) acc[r] += prev[(size_t)r * plane + idx];
            }
        } else {
#pragma unroll
            for (int r = 0; r < RP; r++) {
                const uint64_t a = s_arow[r * kRowSlots + col];
                if (a != 0) acc[r] += (u128)a * prev[(size_t)r * plane + idx];
            }
        }
    }
    uint32_t b = T;
    int q = 1, hprev = 0;
    while (b) {
        const int h = __ffs(b) - 1 + t;
        b &= b - 1;
        if (q > 1) base_h = base_h + s_bin[hprev * kBinomDim + kp + q - 1] - s_bin[h * kBinomDim + kp + q - 1];
        const uint32_t idx = base_h + rr;
        if (BIN) {
            if (s_arow[h] != 0) {
#pragma unroll
                for (int r = 0; r < RP; r++) acc[r] += prev[(size_t)r * plane + idx];
            }
        } else {
#pragma unroll
            for (int r = 0; r < RP; r++) {
                const uint64_t a = s_arow[r * kRowSlots + h];
                if (a != 0) acc[r] += (u128)a * prev[(size_t)r * plane + idx];
            }
        }
        hprev = h;
        q++;
    }
#pragma unroll
    for (int r = 0; r < RP; r++) next[(size_t)r * plane + base_out + rr] = out_modp(acc[r], primes[r]);
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
    TileInfo ti = decode_tile(args);
    if (ti.empty) return;  // uniform: the whole workgroup has no tile
    uint32_t hbw;
    int hcolw;
    tile_bases_wave(args, ti, hbw, hcolw);  // every wave: the tile's bases; wave 0: the window bases
    const int t = args.t, n = args.n;
    const uint32_t W = args.lds_window;

    uint64_t *s_win = smem_u;                       // RP x W
    uint64_t *s_arow = smem_u + (size_t)RP * W;     // RP x t
    uint64_t *s_ha = s_arow + RP * t;               // RP x 32
    uint32_t *s_hb = (uint32_t *)(s_ha + RP * 32);  // 32
    uint32_t *s_bn = s_hb + 32;                     // C(c, i) at [c * kLowBinDim + i], c < t
    __shared__ uint32_t s_mact;

    for (int i = tid; i < t * kLowBinDim; i += kLayerBlock) s_bn[i] = dbinom(i / kLowBinDim, i % kLowBinDim);

    // high windows whose coefficient is nonzero for some prime, compacted
    // (a zero residue contributes nothing, so dropping it is exact)
    if (tid < 32) {
        const bool in = tid < ti.m;
        const int col = in ? hcolw : 0;
        const uint32_t hb = in ? hbw : 0u;
        uint64_t a[RP];
        bool nz = false;
#pragma unroll
        for (int r = 0; r < RP; r++) {
            a[r] = in ? red[(size_t)r * n * n + (size_t)(args.k - 1) * n + col] : 0u;
            nz |= a[r] != 0;
        }
        const uint64_t act = __ballot(in && nz);  // lanes 0..31 of wave 0
        if (in && nz) {
            const int slot = __popcll(act & ((1ull << tid) - 1));
            s_hb[slot] = hb;
#pragma unroll
            for (int r = 0; r < RP; r++) s_ha[r * 32 + slot] = a[r];
        }
        if (tid == 0) s_mact = (uint32_t)__popcll(act);
    }
    if (tid < t) {
#pragma unroll
        for (int r = 0; r < RP; r++) s_arow[r * t + tid] = red[(size_t)r * n * n + (size_t)(args.k - 1) * n + tid];
    }
    if (ti.kp >= 1) {
        // the low window, up to four entries per plane and thread in flight
        // before their stores
        const uint32_t w = dbinom(t, ti.kp - 1);
        for (uint32_t i0 = tid; i0 < w; i0 += 4 * kLayerBlock) {
            uint64_t v[4][RP];
#pragma unroll
            for (int u = 0; u < 4; u++)
                if (i0 + u * kLayerBlock < w) {
#pragma unroll
                    for (int r = 0; r < RP; r++) v[u][r] = prev[(size_t)r * plane + ti.base_low + i0 + u * kLayerBlock];
                }
#pragma unroll
            for (int u = 0; u < 4; u++)
                if (i0 + u * kLayerBlock < w) {
#pragma unroll
                    for (int r = 0; r < RP; r++) s_win[r * W + i0 + u * kLayerBlock] = v[u][r];
                }
        }
    }
    __syncthreads();

    uint64_t pr[RP];
#pragma unroll
    for (int r = 0; r < RP; r++) pr[r] = primes[r];
    const uint32_t ck = ti.ck;
    const uint32_t *lm = g_lowmask + args.lmask_off[ti.g];
    const int mact = (int)s_mact;
    for (uint32_t rr = tid; rr < ck; rr += kLayerBlock) {
        u128 acc[RP];
#pragma unroll
        for (int r = 0; r < RP; r++) acc[r] = 0;
        // Integer sums are exact in any order, so on the add-only path with
        // one plane (the plain 64-bit layers of a 0/1 row, most of a 0/1
        // solve) the loads of the first eight active high windows (HBM) are
        // issued before the low terms (one table entry, then LDS) and arrive
        // while those run (n = 30 0/1: 12.39 -> 12.12 ms).  With products or
        // more planes the registers this takes cost more than the overlap
        // gains (26x26 entries 0..9: 3.27 -> 3.47 ms), so there the windows
        // are read after the low terms.
        constexpr int kPre = (RP == 1 && BIN) ? 8 : 0;
        uint64_t hw[kPre > 0 ? kPre : 1][RP];
#pragma unroll
        for (int u = 0; u < kPre; u++)
            if (u < mact) {
#pragma unroll
                for (int r = 0; r < RP; r++) hw[u][r] = prev[(size_t)r * plane + s_hb[u] + rr];
            }
        // low columns: output rr's low part L and sum_i C(l_i, i) come from
        // one table entry; the window rank of L without its p-th column is
        // sum_{i<p} C(l_i, i+1) + sum_{i>p} C(l_i, i) (running sums over the
        // columns of L, binomials from LDS)
        {
            const uint32_t e = ti.kp > 0 ? lm[rr] : 0u;
            uint32_t b = e & 0xffffu;
            const uint32_t totb = e >> 16;
            uint32_t pa = 0, pb = 0;  // sum_{i<p} C(l_i, i+1), sum_{i<p} C(l_i, i)
            for (int p = 0; b; p++) {
                const int col = __ffs(b) - 1;
                b &= b - 1;
                const uint32_t cb = s_bn[col * kLowBinDim + p], ca = s_bn[col * kLowBinDim + p + 1];
                const uint32_t idx = pa + totb - pb - cb;
                pa += ca;
                pb += cb;
                if (BIN) {
                    if (s_arow[col] != 0) {
#pragma unroll
                        for (int r = 0; r < RP; r++) acc[r] += s_win[r * W + idx];
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < RP; r++) acc[r] += (u128)s_arow[r * t + col] * s_win[r * W + idx];
                }
            }
        }
        // the prefetched high windows, then the rest four at a time
#pragma unroll
        for (int u = 0; u < kPre; u++)
            if (u < mact) {
#pragma unroll
                for (int r = 0; r < RP; r++)
                    acc[r] += BIN ? (u128)hw[u][r] : (u128)s_ha[r * 32 + u] * hw[u][r];
            }
        int q = kPre;
        for (; q + 4 <= mact; q += 4) {
            uint64_t w[4][RP];
#pragma unroll
            for (int u = 0; u < 4; u++)
#pragma unroll
                for (int r = 0; r < RP; r++) w[u][r] = prev[(size_t)r * plane + s_hb[q + u] + rr];
#pragma unroll
            for (int u = 0; u < 4; u++)
#pragma unroll
                for (int r = 0; r < RP; r++)
                    acc[r] += BIN ? (u128)w[u][r] : (u128)s_ha[r * 32 + q + u] * w[u][r];
        }
        for (; q < mact; q++) {
#pragma unroll
            for (int r = 0; r < RP; r++) {
                const uint64_t v = prev[(size_t)r * plane + s_hb[q] + rr];
                acc[r] += BIN ? (u128)v : (u128)s_ha[r * 32 + q] * v;
            }
        }
#pragma unroll
        for (int r = 0; r < RP; r++) next[(size_t)r * plane + ti.base_out + rr] = out_modp(acc[r], pr[r]);
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

// A layer of plain 64-bit values (two's complement) to residues mod rp primes:
// dst plane r, entry i = src[i] mod primes[r] in [0, p).
__global__ void k_int64_to_modp(const uint64_t *__restrict__ src, uint64_t *__restrict__ dst, size_t plane,
                                size_t count, const uint64_t *__restrict__ primes, int rp) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int64_t v = (int64_t)src[i];
    const uint64_t mag = v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v;
    for (int r = 0; r < rp; r++) {
        const uint64_t p = primes[r];
        uint64_t m = fold61((u128)mag, p);
        if (v < 0 && m != 0) m = p - m;
        dst[(size_t)r * plane + i] = m;
    }
}

hipError_t launch_int64_to_modp(const uint64_t *src, uint64_t *dst, size_t plane, size_t count,
                                const uint64_t *primes, int rp, hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_int64_to_modp, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, src, dst, plane,
                       count, primes, rp);
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
