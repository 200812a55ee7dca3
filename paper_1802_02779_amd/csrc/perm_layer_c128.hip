// Complex128 layer sweep of the Store-zechin permanent on gfx950 (part of
// the device translation unit perm_device.hip; tables, planning and tile
// decoding come from perm_layers.hip).
//
// Layer k from layer k-1:  F(S) = sum_{j in S, ascending} a[k-1][j] * F(S \ {j})
// with one fixed FMA chain per output
//   re = fma(a.re, p.re, re); re = fma(-a.im, p.im, re);
//   im = fma(a.re, p.im, im); im = fma(a.im, p.re, im);
namespace permgpu {

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

// Terms whose loads one thread of the per-thread path has in flight together.
constexpr int kThinGroup = 4;

// Per-thread path for groups whose tiles are too small to fill a workgroup:
// each thread computes one whole output.  Low predecessors are read from the
// tile's window at ranks computed from the output's low part (small, cached),
// high predecessors from the aligned windows (neighbouring threads read
// neighbouring entries).
__device__ void layer_c128_thin(const double2 *__restrict__ prev, double2 *__restrict__ next,
                                const double2 *__restrict__ A, const LayerArgs &args, double2 *smem) {
    uint32_t *s_bin = (uint32_t *)smem;                  // C(i, j) at [i * kBinomDim + j]
    double2 *s_arow = (double2 *)(s_bin + kBinomWords);  // row k-1 of A
    const int tid = threadIdx.x;
    stage_binomials(s_bin, tid);
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
            base_out += s_bin[h * kBinomDim + kp + i];
            base_low += s_bin[h * kBinomDim + kp + i - 1];
            if (i >= 2) base_h += s_bin[h * kBinomDim + kp + i - 1];
        }
    }
    // terms in groups of kThinGroup: the group's loads are issued before
    // its FMAs (one memory latency per group, not per term); the FMA order
    // is the chain's
    // low columns: one table entry gives the output's low part L and
    // sum_i C(l_i, i); the rank of L without its p-th column is
    // sum_{i<p} C(l_i, i+1) + sum_{i>p} C(l_i, i)
    double re = 0.0, im = 0.0;
    {
        const uint32_t e = kp > 0 ? g_lowmask[args.t_lmask_off[g] + r] : 0u;
        uint32_t bl = e & 0xffffu;
        const uint32_t totb = e >> 16;
        uint32_t pa = 0, pb = 0;
        for (int p = 0; p < kp; p += kThinGroup) {
            int col[kThinGroup];
            double2 w[kThinGroup];
#pragma unroll
            for (int u = 0; u < kThinGroup; u++)
                if (p + u < kp) {
                    col[u] = __ffs(bl) - 1;
                    bl &= bl - 1;
                    const uint32_t cb = s_bin[col[u] * kBinomDim + p + u];
                    w[u] = prev[base_low + pa + totb - pb - cb];
                    pa += s_bin[col[u] * kBinomDim + p + u + 1];
                    pb += cb;
                }
#pragma unroll
            for (int u = 0; u < kThinGroup; u++)
                if (p + u < kp) cfma(re, im, s_arow[col[u]], w[u]);
        }
    }
    // high columns ascending; the window that removes the q-th one starts at
    // base_q, with base_{q+1} = base_q + C(h_q, k'+q) - C(h_{q+1}, k'+q)
    uint32_t b = T;
    int q = 1, hprev = 0;
    while (b) {
        int hh[kThinGroup];
        uint32_t bb[kThinGroup];
        int cnt = 0;
#pragma unroll
        for (int u = 0; u < kThinGroup; u++) {
            if (b) {
                const int h = __ffs(b) - 1 + t;
                b &= b - 1;
                if (q > 1)
                    base_h = base_h + s_bin[hprev * kBinomDim + kp + q - 1] - s_bin[h * kBinomDim + kp + q - 1];
                hh[u] = h;
                bb[u] = base_h;
                hprev = h;
                q++;
                cnt++;
            }
        }
        double2 w[kThinGroup];
#pragma unroll
        for (int u = 0; u < kThinGroup; u++)
            if (u < cnt) w[u] = prev[bb[u] + r];
#pragma unroll
        for (int u = 0; u < kThinGroup; u++)
            if (u < cnt) cfma(re, im, s_arow[hh[u]], w[u]);
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
    TileInfo ti = decode_tile(args);
    if (ti.empty) return;  // uniform: the whole workgroup has no tile
    const int t = args.t;
    const double2 *arow = A + (size_t)(args.k - 1) * args.n;
    uint32_t hb;
    int hcol;
    tile_bases_wave(args, ti, hb, hcol);  // every wave: the tile's bases; wave 0: the window bases

    double2 *s_win = smem;
    double2 *s_arow = smem + args.lds_window;
    double2 *s_ha = s_arow + t;
    uint32_t *s_hb = (uint32_t *)(s_ha + 32);
    uint32_t *s_bn = s_hb + 32;  // C(c, i) at [c * kLowBinDim + i], c < t

    for (int i = tid; i < t * kLowBinDim; i += kLayerBlock) s_bn[i] = dbinom(i / kLowBinDim, i % kLowBinDim);
    if (tid < ti.m) {  // wave 0 (m <= 22)
        s_hb[tid] = hb;
        s_ha[tid] = arow[hcol];
    }
    if (tid < t) s_arow[tid] = arow[tid];
    if (ti.kp >= 1) {
        const uint32_t w = dbinom(t, ti.kp - 1);
        const double2 *src = prev + ti.base_low;
        // two of a thread's loads in flight before their stores (one round
        // trip less for windows above 256 entries; four in flight was slower)
        for (uint32_t i0 = tid; i0 < w; i0 += 2 * kLayerBlock) {
            double2 v0, v1;
            const bool b1 = i0 + kLayerBlock < w;
            v0 = src[i0];
            if (b1) v1 = src[i0 + kLayerBlock];
            s_win[i0] = v0;
            if (b1) s_win[i0 + kLayerBlock] = v1;
        }
    }
    __syncthreads();

    const uint32_t ck = ti.ck;
    const uint32_t *lm = g_lowmask + args.lmask_off[ti.g];
    double2 *out = next + ti.base_out;
    for (uint32_t r = tid; r < ck; r += kLayerBlock) {
        double re = 0.0, im = 0.0;
        // low columns, ascending (all below t).  Output r's low part L is the
        // r-th k'-subset of [0, t) in colex order; one table entry gives L and
        // sum_i C(l_i, i), and the window rank of L without its p-th column,
        // sum_{i<p} C(l_i, i+1) + sum_{i>p} C(l_i, i), follows from running
        // sums with binomials read from LDS.
        {
            const uint32_t e = ti.kp > 0 ? lm[r] : 0u;
            uint32_t b = e & 0xffffu;
            const uint32_t totb = e >> 16;
            uint32_t pa = 0, pb = 0;  // sum_{i<p} C(l_i, i+1), sum_{i<p} C(l_i, i)
            for (int p = 0; b; p++) {
                const int col = __ffs(b) - 1;
                b &= b - 1;
                const uint32_t cb = s_bn[col * kLowBinDim + p];
                cfma(re, im, s_arow[col], s_win[pa + totb - pb - cb]);
                pa += s_bn[col * kLowBinDim + p + 1];
                pb += cb;
            }
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

}  // namespace permgpu
