// Ryser's formula (eq. 4 of the paper) on gfx950: the comparison method of
// the paper's section 3 and Table 4, as an alternative path behind the same
// C ABI (part of the device translation unit perm_device.hip).
//
//   per(A) = (-1)^n * sum over column subsets S of (-1)^|S| * prod_i r_i(S),
//   r_i(S) = sum_{j in S} a[i][j].
//
// Subsets are visited in binary-reflected Gray-code order: x = 0 .. 2^n - 1
// (64-bit codes),
// S(x) = x ^ (x >> 1), so consecutive subsets differ in column ctz(x) and
// the row sums change by one column.  Thread g owns the 2^m consecutive
// codes x = g*2^m + t (t < 2^m); for t > 0 the changed column is ctz(t) for
// every thread, so the column is wave-uniform and comes through scalar loads
// of the transposed matrix.  Each thread starts from row sums computed
// directly for its first subset, so rounding drift spans at most 2^m updates.
// No table is stored: the path is FP64-bound, not memory-bound.
//
// The per-thread sums are reduced in a fixed order (workgroup tree, then one
// workgroup over the partial sums), so the result does not depend on
// scheduling.  Integer matrices use the same walk on residues mod p.
namespace permgpu {

constexpr int kRyserBlock = 256;

// AT[j*n + i] = A[i*lda + j] (column j contiguous); complex.
__global__ void k_ryser_transpose_c128(const double2 *__restrict__ a, int64_t lda, int n,
                                       double2 *__restrict__ at) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n * n) return;
    const int i = k / n, j = k - i * n;
    at[(size_t)j * n + i] = a[(int64_t)i * lda + j];
}

hipError_t launch_ryser_transpose_c128(const void *a_dev, int64_t lda, int n, void *at, hipStream_t s) {
    const int tot = n * n;
    hipLaunchKernelGGL(k_ryser_transpose_c128, dim3((tot + 255) / 256), dim3(256), 0, s, (const double2 *)a_dev,
                       lda, n, (double2 *)at);
    return hipGetLastError();
}

// Fixed-order tree sum of one value per thread of the workgroup; thread 0
// returns the total.
__device__ __forceinline__ double2 ryser_block_sum(double2 v, double2 *s) {
    s[threadIdx.x] = v;
    __syncthreads();
    for (int w = kRyserBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double2 o = s[threadIdx.x + w];
            s[threadIdx.x] = make_double2(s[threadIdx.x].x + o.x, s[threadIdx.x].y + o.y);
        }
        __syncthreads();
    }
    return s[0];
}

__device__ __forceinline__ void ryser_cmul(double &ar, double &ai, double br, double bi) {
    const double nr = __builtin_fma(-ai, bi, ar * br);
    const double ni = __builtin_fma(ai, br, ar * bi);
    ar = nr;
    ai = ni;
}

// prod_i (rr[i] + i*ri[i]) as four interleaved partial products (rows
// i = c mod 4 in ascending order), combined as (P0*P1)*(P2*P3): short
// dependency chains with few temporaries.
template <int N>
__device__ __forceinline__ void ryser_product(const double *rr, const double *ri, double &pr, double &pi) {
    constexpr int L = N < 4 ? N : 4;
    double cr[L], ci[L];
#pragma unroll
    for (int c = 0; c < L; c++) {
        cr[c] = rr[c];
        ci[c] = ri[c];
    }
#pragma unroll
    for (int i = L; i < N; i++) ryser_cmul(cr[i % L], ci[i % L], rr[i], ri[i]);
    if constexpr (L == 4) {
        ryser_cmul(cr[0], ci[0], cr[1], ci[1]);
        ryser_cmul(cr[2], ci[2], cr[3], ci[3]);
        ryser_cmul(cr[0], ci[0], cr[2], ci[2]);
    } else {
#pragma unroll
        for (int c = 1; c < L; c++) ryser_cmul(cr[0], ci[0], cr[c], ci[c]);
    }
    pr = cr[0];
    pi = ci[0];
}

// One thread per 2^m consecutive Gray codes; threads g >= nthreads add 0.
template <int N>
__global__ __launch_bounds__(kRyserBlock) void k_ryser_c128(const double2 *__restrict__ at, int m,
                                                           uint32_t nthreads, double2 *__restrict__ partial) {
    __shared__ double2 red[kRyserBlock];
    const uint32_t g = blockIdx.x * kRyserBlock + threadIdx.x;
    double accr = 0.0, acci = 0.0;
    if (g < nthreads) {
        const uint64_t x0 = (uint64_t)g << m;
        uint64_t S = x0 ^ (x0 >> 1);
        double rr[N], ri[N];
#pragma unroll
        for (int i = 0; i < N; i++) rr[i] = ri[i] = 0.0;
        // row sums of the first subset, columns in ascending order
        for (int j = 0; j < N; j++) {
            if ((S >> j) & 1u) {
                const double2 *col = at + (size_t)j * N;
#pragma unroll
                for (int i = 0; i < N; i++) {
                    rr[i] += col[i].x;
                    ri[i] += col[i].y;
                }
            }
        }
        double sg = (__builtin_popcountll(S) & 1) ? -1.0 : 1.0;
        double pr, pi;
        ryser_product<N>(rr, ri, pr, pi);
        accr = sg * pr;
        acci = sg * pi;
        // inside the range only columns below m (at most 13) change: 32 bits suffice
        uint32_t Slo = (uint32_t)S;
        const uint32_t steps = 1u << m;
        for (uint32_t t = 1; t < steps; t++) {
            // next code: column j = ctz(t) enters or leaves S
            const int j = __builtin_ctz(t);
            Slo ^= 1u << j;
            const double s = ((Slo >> j) & 1u) ? 1.0 : -1.0;
            const double2 *col = at + (size_t)j * N;
#pragma unroll
            for (int i = 0; i < N; i++) {
                rr[i] = __builtin_fma(s, col[i].x, rr[i]);
                ri[i] = __builtin_fma(s, col[i].y, ri[i]);
            }
            sg = -sg;
            ryser_product<N>(rr, ri, pr, pi);
            accr = __builtin_fma(sg, pr, accr);
            acci = __builtin_fma(sg, pi, acci);
        }
    }
    const double2 tot = ryser_block_sum(make_double2(accr, acci), red);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// Sum of the per-workgroup partial sums in a fixed order, times (-1)^n.
// 0 - x and x + 0 leave every nonzero value unchanged and give +0 for a zero
// sum, so an exactly zero permanent comes out as +0 whatever the parity.
__global__ __launch_bounds__(kRyserBlock) void k_ryser_final_c128(const double2 *__restrict__ partial, uint32_t np,
                                                                 int n, double2 *__restrict__ out) {
    __shared__ double2 red[kRyserBlock];
    double sr = 0.0, si = 0.0;
    for (uint32_t k = threadIdx.x; k < np; k += kRyserBlock) {
        sr += partial[k].x;
        si += partial[k].y;
    }
    const double2 tot = ryser_block_sum(make_double2(sr, si), red);
    if (threadIdx.x == 0)
        *out = (n & 1) ? make_double2(0.0 - tot.x, 0.0 - tot.y) : make_double2(tot.x + 0.0, tot.y + 0.0);
}

template <int N>
static hipError_t launch_ryser_n(const double2 *at, int m, uint32_t nthreads, uint32_t blocks, double2 *partial,
                                 hipStream_t s) {
    hipLaunchKernelGGL(k_ryser_c128<N>, dim3(blocks), dim3(kRyserBlock), 0, s, at, m, nthreads, partial);
    return hipGetLastError();
}

hipError_t launch_ryser_c128(const void *at, int n, int m, void *partial, uint32_t blocks, void *out,
                             hipStream_t s) {
    const uint32_t nthreads = 1u << (n - m);
    const double2 *A = (const double2 *)at;
    double2 *P = (double2 *)partial;
    hipError_t e = hipErrorInvalidValue;
    switch (n) {
#define PERM_RYSER_CASE(K) \
    case K: e = launch_ryser_n<K>(A, m, nthreads, blocks, P, s); break;
        PERM_RYSER_CASE(1) PERM_RYSER_CASE(2) PERM_RYSER_CASE(3) PERM_RYSER_CASE(4) PERM_RYSER_CASE(5)
        PERM_RYSER_CASE(6) PERM_RYSER_CASE(7) PERM_RYSER_CASE(8) PERM_RYSER_CASE(9) PERM_RYSER_CASE(10)
        PERM_RYSER_CASE(11) PERM_RYSER_CASE(12) PERM_RYSER_CASE(13) PERM_RYSER_CASE(14) PERM_RYSER_CASE(15)
        PERM_RYSER_CASE(16) PERM_RYSER_CASE(17) PERM_RYSER_CASE(18) PERM_RYSER_CASE(19) PERM_RYSER_CASE(20)
        PERM_RYSER_CASE(21) PERM_RYSER_CASE(22) PERM_RYSER_CASE(23) PERM_RYSER_CASE(24) PERM_RYSER_CASE(25)
        PERM_RYSER_CASE(26) PERM_RYSER_CASE(27) PERM_RYSER_CASE(28) PERM_RYSER_CASE(29) PERM_RYSER_CASE(30)
        PERM_RYSER_CASE(31) PERM_RYSER_CASE(32) PERM_RYSER_CASE(33) PERM_RYSER_CASE(34)
#undef PERM_RYSER_CASE
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ryser_final_c128, dim3(1), dim3(kRyserBlock), 0, s, (const double2 *)P, blocks, n,
                       (double2 *)out);
    return hipGetLastError();
}

// ------------------------------------------------------------- mod p
// The same walk on residues mod p = 2^61 - c (one prime per grid row):
// row sums in [0, p), products folded with fold61, signed terms added mod p.

__device__ __forceinline__ uint64_t ryser_addmod(uint64_t x, uint64_t y, uint64_t p) {
    const uint64_t z = x + y;  // < 2^62
    return z >= p ? z - p : z;
}

__device__ __forceinline__ uint64_t ryser_mulmod(uint64_t x, uint64_t y, uint64_t p) {
    return fold61((u128)x * y, p);
}

template <int N>
__device__ __forceinline__ uint64_t ryser_product_modp(const uint64_t *r, uint64_t p) {
    constexpr int L = N < 4 ? N : 4;
    uint64_t c[L];
#pragma unroll
    for (int k = 0; k < L; k++) c[k] = r[k];
#pragma unroll
    for (int i = L; i < N; i++) c[i % L] = ryser_mulmod(c[i % L], r[i], p);
#pragma unroll
    for (int k = 1; k < L; k++) c[0] = ryser_mulmod(c[0], c[k], p);
    return c[0];
}

__device__ __forceinline__ uint64_t ryser_block_sum_modp(uint64_t v, uint64_t p, uint64_t *s) {
    s[threadIdx.x] = v;
    __syncthreads();
    for (int w = kRyserBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] = ryser_addmod(s[threadIdx.x], s[threadIdx.x + w], p);
        __syncthreads();
    }
    return s[0];
}

// atr: prime r's transposed residues at atr[r*n*n + j*n + i]; partial[r*gridDim.x + block]
template <int N>
__global__ __launch_bounds__(kRyserBlock) void k_ryser_modp(const uint64_t *__restrict__ atr,
                                                           const uint64_t *__restrict__ primes, int m,
                                                           uint32_t nthreads, uint64_t *__restrict__ partial) {
    __shared__ uint64_t red[kRyserBlock];
    const uint64_t p = primes[blockIdx.y];
    const uint64_t *at = atr + (size_t)blockIdx.y * N * N;
    const uint32_t g = blockIdx.x * kRyserBlock + threadIdx.x;
    uint64_t acc = 0;
    if (g < nthreads) {
        const uint64_t x0 = (uint64_t)g << m;
        uint64_t S = x0 ^ (x0 >> 1);
        uint64_t r[N];
#pragma unroll
        for (int i = 0; i < N; i++) r[i] = 0;
        for (int j = 0; j < N; j++) {
            if ((S >> j) & 1u) {
                const uint64_t *col = at + (size_t)j * N;
#pragma unroll
                for (int i = 0; i < N; i++) r[i] = ryser_addmod(r[i], col[i], p);
            }
        }
        bool neg = __builtin_popcountll(S) & 1;
        uint64_t pr = ryser_product_modp<N>(r, p);
        acc = neg ? (pr ? p - pr : 0) : pr;
        uint32_t Slo = (uint32_t)S;  // only columns below m change
        const uint32_t steps = 1u << m;
        for (uint32_t t = 1; t < steps; t++) {
            const int j = __builtin_ctz(t);
            Slo ^= 1u << j;
            const bool add = (Slo >> j) & 1u;
            const uint64_t *col = at + (size_t)j * N;
#pragma unroll
            for (int i = 0; i < N; i++) {
                const uint64_t a = col[i];
                r[i] = ryser_addmod(r[i], add ? a : (a ? p - a : 0), p);
            }
            neg = !neg;
            pr = ryser_product_modp<N>(r, p);
            acc = ryser_addmod(acc, neg ? (pr ? p - pr : 0) : pr, p);
        }
    }
    const uint64_t tot = ryser_block_sum_modp(acc, p, red);
    if (threadIdx.x == 0) partial[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = tot;
}

// res[r] = (-1)^n * (sum of prime r's partial sums) mod p_r, fixed order
__global__ __launch_bounds__(kRyserBlock) void k_ryser_final_modp(const uint64_t *__restrict__ partial, uint32_t np,
                                                                 const uint64_t *__restrict__ primes, int n,
                                                                 uint64_t *__restrict__ res) {
    __shared__ uint64_t red[kRyserBlock];
    const uint64_t p = primes[blockIdx.x];
    const uint64_t *pp = partial + (size_t)blockIdx.x * np;
    uint64_t s = 0;
    for (uint32_t k = threadIdx.x; k < np; k += kRyserBlock) s = ryser_addmod(s, pp[k], p);
    const uint64_t tot = ryser_block_sum_modp(s, p, red);
    if (threadIdx.x == 0) res[blockIdx.x] = (n & 1) ? (tot ? p - tot : 0) : tot;
}

template <int N>
static hipError_t launch_ryser_modp_n(const uint64_t *atr, const uint64_t *primes, int nprimes, int m,
                                      uint32_t nthreads, uint32_t blocks, uint64_t *partial, hipStream_t s) {
    hipLaunchKernelGGL(k_ryser_modp<N>, dim3(blocks, nprimes), dim3(kRyserBlock), 0, s, atr, primes, m, nthreads,
                       partial);
    return hipGetLastError();
}

hipError_t launch_ryser_modp(const uint64_t *atr, const uint64_t *primes, int nprimes, int n, int m,
                             uint64_t *partial, uint32_t blocks, uint64_t *res, hipStream_t s) {
    const uint32_t nthreads = 1u << (n - m);
    hipError_t e = hipErrorInvalidValue;
    switch (n) {
#define PERM_RYSER_CASE(K) \
    case K: e = launch_ryser_modp_n<K>(atr, primes, nprimes, m, nthreads, blocks, partial, s); break;
        PERM_RYSER_CASE(1) PERM_RYSER_CASE(2) PERM_RYSER_CASE(3) PERM_RYSER_CASE(4) PERM_RYSER_CASE(5)
        PERM_RYSER_CASE(6) PERM_RYSER_CASE(7) PERM_RYSER_CASE(8) PERM_RYSER_CASE(9) PERM_RYSER_CASE(10)
        PERM_RYSER_CASE(11) PERM_RYSER_CASE(12) PERM_RYSER_CASE(13) PERM_RYSER_CASE(14) PERM_RYSER_CASE(15)
        PERM_RYSER_CASE(16) PERM_RYSER_CASE(17) PERM_RYSER_CASE(18) PERM_RYSER_CASE(19) PERM_RYSER_CASE(20)
        PERM_RYSER_CASE(21) PERM_RYSER_CASE(22) PERM_RYSER_CASE(23) PERM_RYSER_CASE(24) PERM_RYSER_CASE(25)
        PERM_RYSER_CASE(26) PERM_RYSER_CASE(27) PERM_RYSER_CASE(28) PERM_RYSER_CASE(29) PERM_RYSER_CASE(30)
        PERM_RYSER_CASE(31) PERM_RYSER_CASE(32) PERM_RYSER_CASE(33) PERM_RYSER_CASE(34)
#undef PERM_RYSER_CASE
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ryser_final_modp, dim3(nprimes), dim3(kRyserBlock), 0, s, (const uint64_t *)partial, blocks,
                       primes, n, res);
    return hipGetLastError();
}

}  // namespace permgpu
