// Complex128 block sweep of the Store-zechin permanent on gfx950 (part of
// the device translation unit perm_device.hip; rank tables come from
// perm_layers.hip).
//
// The stored values F(S) and the chain of each one are those of the layer
// sweep; only the grouping differs.  A block holds F(T u L) for one high
// part T of the columns [t, n) and every low part L of [0, t): 2^t values of
// all popcounts, ordered by |L| ("low level" k') and colex rank of L inside a
// level.  For a block of high level m = |T| the predecessor that removes a
// low column has the same T and sits one low level below in the same block
// (kept in LDS), and the one that removes a high column h is at the same
// position of block T \ {h}, of high level m - 1 (read from HBM, consecutive
// lanes reading consecutive entries).  One launch per high level m; inside a
// block the low levels run in order with one workgroup barrier each.  No
// value is ever staged back from HBM as a low window: a value is written once
// and read again only as a high predecessor.
namespace permgpu {

__global__ __launch_bounds__(kBlockThreads) void k_block_c128(const double2 *__restrict__ prev,
                                                              double2 *__restrict__ cur,
                                                              const double2 *__restrict__ A,
                                                              const BlockArgs args) {
    extern __shared__ double2 smem[];
    const int tid = threadIdx.x, t = args.t, m = args.m, n = args.n;
    const uint32_t W = args.lds_level;
    double2 *s_lv0 = smem;                    // low levels of even k'
    double2 *s_lv1 = smem + W;                // low levels of odd k'
    double2 *s_row = smem + 2 * W;            // row k-1 of A, double-buffered by k'
    uint32_t *s_hb = (uint32_t *)(s_row + 2 * kRowSlots);  // block of T \ {h_q} in level m-1
    uint32_t *s_hc = s_hb + 32;                            // column h_q

    const uint32_t b = xcd_chunk_remap(blockIdx.x, args.nblocks, args.chunk);
    const uint32_t T = g_highlist[args.high_off + b];  // high part, as positions 0..n-t-1
    if (tid < m) {
        // colex rank of T without its tid-th element, among the (m-1)-subsets
        uint32_t rank = 0, bb = T;
        int col = 0;
        for (int i = 0; bb; i++) {
            const int h = __ffs(bb) - 1;
            bb &= bb - 1;
            if (i < tid) rank += dbinom(h, i + 1);
            else if (i > tid) rank += dbinom(h, i);
            else col = h;
        }
        s_hb[tid] = rank;
        s_hc[tid] = (uint32_t)(col + t);
    }
    const size_t BS = (size_t)1 << t;
    double2 *out = cur + (size_t)b * BS;
    for (int kp = 0; kp <= t; kp++) {
        const int k = m + kp;
        double2 *row = s_row + (kp & 1) * kRowSlots;
        if (k >= 1 && tid < n) row[tid] = A[(size_t)(k - 1) * n + tid];
        __syncthreads();  // row, s_hb/s_hc and the previous low level are in LDS
        const uint32_t ck = dbinom(t, kp), base = args.loff[kp];
        double2 *lv_out = (kp & 1) ? s_lv1 : s_lv0;
        const double2 *lv_in = (kp & 1) ? s_lv0 : s_lv1;
        const uint32_t *lt = g_lowtab + args.low_off[kp];
        for (uint32_t r = tid; r < ck; r += kBlockThreads) {
            double2 v;
            if (k <= 1) {
                // F(empty) = 1 is never read; F({j}) = a[0][j] is a copy, as in
                // the layer sweep (the colex rank of {l} is l)
                v = k == 0 ? make_double2(1.0, 0.0) : (kp == 1 ? row[r] : row[s_hc[0]]);
            } else {
                double re = 0.0, im = 0.0;
                // low columns, ascending (all below t): this block, level k'-1
                int p = 0;
                for (; p + 4 <= kp; p += 4) {
                    uint32_t e[4];
#pragma unroll
                    for (int u = 0; u < 4; u++) e[u] = lt[(uint32_t)(p + u) * ck + r];
#pragma unroll
                    for (int u = 0; u < 4; u++) cfma(re, im, row[e[u] >> 16], lv_in[e[u] & 0xffffu]);
                }
                for (; p < kp; p++) {
                    const uint32_t e = lt[(uint32_t)p * ck + r];
                    cfma(re, im, row[e >> 16], lv_in[e & 0xffffu]);
                }
                // high columns, ascending (all >= t): same position of the
                // blocks of level m-1, four loads in flight at a time
                const double2 *src = prev + base + r;
                int q = 0;
                for (; q + 4 <= m; q += 4) {
                    double2 w[4];
#pragma unroll
                    for (int u = 0; u < 4; u++) w[u] = src[(size_t)s_hb[q + u] * BS];
#pragma unroll
                    for (int u = 0; u < 4; u++) cfma(re, im, row[s_hc[q + u]], w[u]);
                }
                for (; q < m; q++) cfma(re, im, row[s_hc[q]], src[(size_t)s_hb[q] * BS]);
                v = make_double2(re, im);
            }
            out[base + r] = v;
            if (kp < t) lv_out[r] = v;
        }
    }
}

uint32_t plan_block(int n, int t, int m, int chunk, BlockArgs *a) {
    a->n = n;
    a->t = t;
    a->m = m;
    a->nblocks = binom_host(n - t, m);
    a->high_off = highlist_off(m);
    a->chunk = (uint32_t)(chunk > 0 ? chunk : 0);
    a->lds_level = binom_host(t, t / 2);
    uint32_t s = 0;
    for (int kp = 0; kp <= t; kp++) {
        a->loff[kp] = s;
        a->low_off[kp] = lowtab_t_base(t) + lowtab_kp_off(t, kp);
        s += binom_host(t, kp);
    }
    a->loff[t + 1] = s;
    return a->nblocks;
}

size_t block_lds_bytes_c128(const BlockArgs &a) {
    return ((size_t)2 * a.lds_level + 2 * kRowSlots) * 16 + 64 * 4;
}

hipError_t launch_block_c128(const void *prev, void *cur, const void *packed, const BlockArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_block_c128, dim3(a.nblocks), dim3(kBlockThreads), block_lds_bytes_c128(a), s,
                       (const double2 *)prev, (double2 *)cur, (const double2 *)packed, a);
    return hipGetLastError();
}

// The permanent is F(all columns): block 0 of the last level, last position.
__global__ void k_block_readout_c128(const double2 *last, size_t pos, double2 *result) {
    if (threadIdx.x == 0) *result = last[pos];
}

hipError_t launch_block_readout_c128(const void *last, int t, void *result, hipStream_t s) {
    hipLaunchKernelGGL(k_block_readout_c128, dim3(1), dim3(64), 0, s, (const double2 *)last,
                       ((size_t)1 << t) - 1, (double2 *)result);
    return hipGetLastError();
}

}  // namespace permgpu
