/*
 * CPU oracle for the permanent -- TEST INFRASTRUCTURE ONLY.
 *
 * Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline leg may
 * load this library.  It shares no code, header, table or constant with the
 * HIP library under paper_1802_02779_amd/: it is written from the paper.
 *
 * What it computes (Su & Zheng, section 4 "Store-zechin"): the permanent of
 * an n x n matrix developed along the last row, recursively, with every
 * sub-permanent stored once and reused.  A stored sub-permanent is
 *
 *     F(S) = per(rows 0..|S|-1 of A, columns S),   S a subset of {0..n-1},
 *
 * i.e. the paper's A_{u;v} with u = the last n-|S| rows and v = the
 * complement of S (notation of section 4).  Development of the last of its
 * rows (property 4 of section 3.1) gives
 *
 *     F(S) = sum over j in S, ascending, of a[|S|-1][j] * F(S \ {j}),
 *     F({j}) = a[0][j],  F(empty) = 1.
 *
 * The tables are indexed by the bitmask of S (2^n entries).  Two evaluation
 * orders of the same stored values are offered:
 *   memo   -- the paper's order: recurse from F({0..n-1}) along the last
 *             row, evaluate each F(S) the first time it is needed, store it;
 *             single-threaded;
 *   layers -- every F(S) with |S| = k before any with |S| = k+1 (k = 2..n);
 *             OpenMP over the masks of one popcount.
 * Each F(S) has exactly one arithmetic definition (below), so both orders
 * produce bitwise-identical tables.
 *
 * Arithmetic of one stored value:
 *   complex128: acc = 0 + 0i; for j ascending in S, with a = a[k-1][j] and
 *     p = F(S\{j}):  acc.re = fma( a.re, p.re, acc.re);
 *                    acc.re = fma(-a.im, p.im, acc.re);
 *                    acc.im = fma( a.re, p.im, acc.im);
 *                    acc.im = fma( a.im, p.re, acc.im);
 *     (round to nearest even, no reassociation; the paper works in exact
 *     arithmetic and fixes no order, so this one is chosen and documented).
 *   mod p (p < 2^61): acc = sum of a*p as an exact unsigned 128-bit integer
 *     (at most 30 terms below 2^122 each, so no overflow), then acc % p.
 *   |A| (per of entrywise moduli, for the complex tolerance): the complex
 *     chain's real part with a = |a_ij| (hypot) and non-negative values.
 *
 * Ryser's formula (eq. 4 of the paper, section 3) is the comparison method:
 *   per(A) = (-1)^n sum_{S} (-1)^|S| prod_i r_i(S),  r_i(S) = sum_{j in S} a_ij.
 * Its exact value is pinned in the Python oracle; here oracle_ryser_bound
 * gives a rigorous bound on the rounding error of an fp64 evaluation of it
 * (see that function).
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC.
 * Returns 0 on success, -1 on bad arguments, -2 when memory runs out.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_N_MAX 30

typedef unsigned __int128 u128;

static int popcount32(uint32_t x) { return __builtin_popcount(x); }

/* ---------------------------------------------------------------- complex */

typedef struct {
    int n;
    const double *a; /* row-major, interleaved (re, im), n*n entries */
    double *tab;     /* 2^n entries of (re, im) */
    uint8_t *done;   /* 2^n bits */
} c128_state;

static void c128_value(const double *a, int n, const double *tab, uint32_t S,
                       double *out_re, double *out_im)
{
    int k = popcount32(S);
    const double *row = a + 2 * (size_t)(k - 1) * (size_t)n;
    double re = 0.0, im = 0.0;
    for (int j = 0; j < n; j++) {
        if (!((S >> j) & 1u))
            continue;
        uint32_t P = S & ~(1u << j);
        double ar = row[2 * j], ai = row[2 * j + 1];
        double pr = tab[2 * (size_t)P], pi = tab[2 * (size_t)P + 1];
        re = fma(ar, pr, re);
        re = fma(-ai, pi, re);
        im = fma(ar, pi, im);
        im = fma(ai, pr, im);
    }
    *out_re = re;
    *out_im = im;
}

static void c128_memo_visit(c128_state *st, uint32_t S)
{
    /* The paper's order: develop along the last row; evaluate each needed
     * minor (recursively) the first time, then reuse the stored value. */
    if (st->done[S >> 3] & (1u << (S & 7)))
        return;
    for (int j = 0; j < st->n; j++) {
        if ((S >> j) & 1u) {
            uint32_t P = S & ~(1u << j);
            c128_memo_visit(st, P);
        }
    }
    c128_value(st->a, st->n, st->tab, S, &st->tab[2 * (size_t)S], &st->tab[2 * (size_t)S + 1]);
    st->done[S >> 3] |= (uint8_t)(1u << (S & 7));
}

static int c128_setup(int n, const double *a, double **tab, uint8_t **done)
{
    size_t N = (size_t)1 << n;
    *tab = (double *)malloc(2 * N * sizeof(double));
    *done = (uint8_t *)calloc((N + 7) / 8, 1);
    if (!*tab || !*done) {
        free(*tab);
        free(*done);
        return -2;
    }
    for (int j = 0; j < n; j++) {
        uint32_t S = 1u << j;
        (*tab)[2 * (size_t)S] = a[2 * j];
        (*tab)[2 * (size_t)S + 1] = a[2 * j + 1];
        (*done)[S >> 3] |= (uint8_t)(1u << (S & 7));
    }
    return 0;
}

/* mode: 0 = memo (paper's order, one thread), 1 = layers (OpenMP) */
int oracle_per_c128(int n, const double *a, int mode, int nthreads, double *out)
{
    if (n < 0 || n > ORACLE_N_MAX || !out || (n > 0 && !a))
        return -1;
    if (n == 0) {
        out[0] = 1.0;
        out[1] = 0.0;
        return 0;
    }
    if (n == 1) {
        out[0] = a[0];
        out[1] = a[1];
        return 0;
    }
    double *tab;
    uint8_t *done;
    int rc = c128_setup(n, a, &tab, &done);
    if (rc)
        return rc;
    uint32_t full = (uint32_t)(((uint64_t)1 << n) - 1);
    if (mode == 0) {
        c128_state st = {n, a, tab, done};
        c128_memo_visit(&st, full);
    } else {
        int64_t N = (int64_t)1 << n;
#ifdef _OPENMP
        if (nthreads > 0)
            omp_set_num_threads(nthreads);
#endif
        for (int k = 2; k <= n; k++) {
#pragma omp parallel for schedule(static, 4096)
            for (int64_t S = 0; S < N; S++) {
                if (popcount32((uint32_t)S) != k)
                    continue;
                c128_value(a, n, tab, (uint32_t)S, &tab[2 * S], &tab[2 * S + 1]);
            }
        }
    }
    out[0] = tab[2 * (size_t)full];
    out[1] = tab[2 * (size_t)full + 1];
    free(tab);
    free(done);
    return 0;
}

/* ------------------------------------------------------------------ |A| */

int oracle_per_abs(int n, const double *a, int nthreads, double *out)
{
    if (n < 0 || n > ORACLE_N_MAX || !out || (n > 0 && !a))
        return -1;
    if (n == 0) {
        *out = 1.0;
        return 0;
    }
    size_t N = (size_t)1 << n;
    double *mod = (double *)malloc((size_t)n * n * sizeof(double));
    double *tab = (double *)malloc(N * sizeof(double));
    if (!mod || !tab) {
        free(mod);
        free(tab);
        return -2;
    }
    for (size_t i = 0; i < (size_t)n * n; i++)
        mod[i] = hypot(a[2 * i], a[2 * i + 1]);
    for (int j = 0; j < n; j++)
        tab[(size_t)1 << j] = mod[j];
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#endif
    for (int k = 2; k <= n; k++) {
        const double *row = mod + (size_t)(k - 1) * n;
#pragma omp parallel for schedule(static, 4096)
        for (int64_t S = 0; S < (int64_t)N; S++) {
            if (popcount32((uint32_t)S) != k)
                continue;
            double acc = 0.0;
            for (int j = 0; j < n; j++)
                if ((S >> j) & 1)
                    acc = fma(row[j], tab[S & ~((int64_t)1 << j)], acc);
            tab[S] = acc;
        }
    }
    *out = tab[N - 1];
    free(mod);
    free(tab);
    return 0;
}

/* ----------------------------------------------------------------- mod p */

typedef struct {
    int n;
    const uint64_t *a; /* residues in [0, p), row-major */
    uint64_t p;
    uint64_t *tab;
    uint8_t *done;
} modp_state;

static uint64_t modp_value(const uint64_t *a, int n, uint64_t p, const uint64_t *tab, uint32_t S)
{
    int k = popcount32(S);
    const uint64_t *row = a + (size_t)(k - 1) * n;
    u128 acc = 0;
    for (int j = 0; j < n; j++)
        if ((S >> j) & 1u)
            acc += (u128)row[j] * tab[S & ~(1u << j)];
    return (uint64_t)(acc % p);
}

static void modp_memo_visit(modp_state *st, uint32_t S)
{
    if (st->done[S >> 3] & (1u << (S & 7)))
        return;
    for (int j = 0; j < st->n; j++)
        if ((S >> j) & 1u)
            modp_memo_visit(st, S & ~(1u << j));
    st->tab[S] = modp_value(st->a, st->n, st->p, st->tab, S);
    st->done[S >> 3] |= (uint8_t)(1u << (S & 7));
}

/* a: residues in [0, p); p must be below 2^61 so 30 products fit 128 bits. */
int oracle_per_modp(int n, const uint64_t *a, uint64_t p, int mode, int nthreads, uint64_t *out)
{
    if (n < 0 || n > ORACLE_N_MAX || !out || (n > 0 && !a) || p < 2 || p >= ((uint64_t)1 << 61))
        return -1;
    for (size_t i = 0; i < (size_t)n * n; i++)
        if (a[i] >= p)
            return -1;
    if (n == 0) {
        *out = 1 % p;
        return 0;
    }
    if (n == 1) {
        *out = a[0];
        return 0;
    }
    size_t N = (size_t)1 << n;
    uint64_t *tab = (uint64_t *)malloc(N * sizeof(uint64_t));
    uint8_t *done = (uint8_t *)calloc((N + 7) / 8, 1);
    if (!tab || !done) {
        free(tab);
        free(done);
        return -2;
    }
    for (int j = 0; j < n; j++) {
        uint32_t S = 1u << j;
        tab[S] = a[j];
        done[S >> 3] |= (uint8_t)(1u << (S & 7));
    }
    uint32_t full = (uint32_t)(N - 1);
    if (mode == 0) {
        modp_state st = {n, a, p, tab, done};
        modp_memo_visit(&st, full);
    } else {
#ifdef _OPENMP
        if (nthreads > 0)
            omp_set_num_threads(nthreads);
#endif
        for (int k = 2; k <= n; k++) {
#pragma omp parallel for schedule(static, 4096)
            for (int64_t S = 0; S < (int64_t)N; S++) {
                if (popcount32((uint32_t)S) != k)
                    continue;
                tab[S] = modp_value(a, n, p, tab, (uint32_t)S);
            }
        }
    }
    *out = tab[full];
    free(tab);
    free(done);
    return 0;
}

/* Number of OpenMP threads a parallel region would use (for reporting). */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------ Ryser bound */
/*
 * Upper bound E on |computed - per(A)| for an fp64 complex evaluation of
 * eq. (4) (unit roundoff u = 2^-53) that
 *   (a) splits the 2^n subsets into ranges of at most 2^mm consecutive
 *       subsets of a one-column-change order, forms the row sums of each
 *       range's first subset directly (at most n additions) and then changes
 *       them by one column per subset with one rounding each;
 *   (b) multiplies the n row sums with complex products whose components
 *       are each rounded twice (a product, then a fused multiply-add), in
 *       any order;
 *   (c) adds the 2^n signed products with every product passing through at
 *       most `depth` additions.
 * Error model, with B_i = sum_j |a_ij| and r_i(S) the exact row sums:
 *   each component of a computed row sum is off by at most
 *   (gamma_n + 2^mm u) B_i, so |computed r_i - r_i| <= eps_i
 *   = sqrt(2) (gamma_n + 2^mm u) B_i  (gamma_k = k u / (1 - k u));
 *   one complex product has relative error at most eta = 2 sqrt(2) u
 *   (each component: two roundings of terms bounded by |a| |b|, whose sum is
 *   at most |a||b| by Cauchy-Schwarz), so a computed product is within
 *   ((1+eta)^(n-1) - 1) prod(|r_i| + eps_i) of the product of the computed
 *   row sums;
 *   summation adds at most sqrt(2) gamma_depth times the sum of the moduli.
 * Hence, with T(S) = (1+eta)^(n-1) prod_i (|r_i(S)| + eps_i),
 *   E = sum_S [T(S) - prod_i |r_i(S)|] + sqrt(2) gamma_depth sum_S T(S).
 * The row sums here are themselves computed in fp64 (directly, at most n
 * additions), so eps_i is enlarged by sqrt(2) gamma_n B_i to cover them, and
 * the result is multiplied by 1.01 for the rounding of this computation.
 */
static double gamma_k(double k) { const double u = ldexp(1.0, -53); return k * u / (1.0 - k * u); }

int oracle_ryser_bound(int n, const double *a, int mm, int depth, int nthreads, double *out)
{
    if (n < 1 || n > 24 || !a || !out || mm < 0 || mm > 40 || depth < 0) return -1;
    const double u = ldexp(1.0, -53);
    double eps[ORACLE_N_MAX];
    for (int i = 0; i < n; i++) {
        double b = 0.0;
        for (int j = 0; j < n; j++) b += hypot(a[2 * (i * n + j)], a[2 * (i * n + j) + 1]);
        b *= 1.0 + gamma_k(n + 1);  /* the sum above is itself rounded */
        eps[i] = sqrt(2.0) * (2.0 * gamma_k(n) + ldexp(1.0, mm) * u) * b;
    }
    const double grow = pow(1.0 + 2.0 * sqrt(2.0) * u, n - 1);
    const uint32_t full = (uint32_t)1 << n;
    double excess = 0.0, total = 0.0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(static, 4096) reduction(+ : excess, total)
    for (uint32_t S = 0; S < full; S++) {
        double t = grow, p = 1.0;
        for (int i = 0; i < n; i++) {
            double rr = 0.0, ri = 0.0;
            for (int j = 0; j < n; j++)
                if ((S >> j) & 1u) {
                    rr += a[2 * (i * n + j)];
                    ri += a[2 * (i * n + j) + 1];
                }
            const double m = hypot(rr, ri);
            t *= m + eps[i];
            p *= m;
        }
        excess += t - p;
        total += t;
    }
    *out = 1.01 * (excess + sqrt(2.0) * gamma_k(depth) * total);
    return 0;
}

/* ------------------------------------------------------ repeated columns */
/*
 * Permanent of the n x n matrix whose columns are column j of the n x m
 * matrix a repeated mult[j] >= 1 times (sum of mult = n): the output
 * amplitudes of bunched bosons.  Copies of one column are identical, so
 * every column subset with the same number c_j of copies of each column has
 * the same stored minor (section 4's stored sub-permanents, one per count
 * vector c instead of one per subset):
 *
 *     G(c) = sum over j ascending with c_j > 0 of a[|c|-1][j] * G(c - e_j),
 *     G(e_j) = a[0][j],  G(0) = 1,
 *
 * where G(c) counts each assignment of rows 0..|c|-1 to distinct columns
 * with c_j rows on column j once; an assignment stands for prod_j c_j!
 * bijections onto the copies, so per = G(mult) * prod_j mult[j]!.
 * With every mult[j] = 1 the table and the chain are exactly the subset
 * tables above (same terms in the same order).
 *
 * Table: one entry per count vector, mixed-radix index
 * idx(c) = sum_j c_j * stride_j, stride_0 = 1, stride_{j+1} = stride_j *
 * (mult[j] + 1).  Evaluation layer by layer (|c| = 2..n), OpenMP within a
 * layer.  Complex arithmetic: the chain of oracle_per_c128; the result is
 * G(mult) times f, f = 1.0 multiplied in double by 2, ..., mult[j] for
 * j = 0, 1, ... in turn (each factor exact while below 2^53), as two real
 * products.  The mod p variant returns G(mult) mod p (unscaled).
 */
#define ORACLE_MULTI_N_MAX 64
#define ORACLE_MULTI_STATES ((int64_t)1 << 29)

static int multi_layout(int n, int m, const int32_t *mult, int64_t *stride, int64_t *states)
{
    if (n < 0 || n > ORACLE_MULTI_N_MAX || m < 0 || m > n || (m > 0 && !mult))
        return -1;
    int64_t s = 1, tot = 0;
    for (int j = 0; j < m; j++) {
        if (mult[j] < 1)
            return -1;
        tot += mult[j];
        stride[j] = s;
        s *= (int64_t)mult[j] + 1;
        if (s > ORACLE_MULTI_STATES)
            return -2;
    }
    stride[m] = s;
    if (tot != n)
        return -1;
    *states = s;
    return 0;
}

/* digit sum of every index (the layer it belongs to) */
static uint8_t *multi_layers(int m, const int32_t *mult, int64_t D)
{
    uint8_t *ks = (uint8_t *)malloc((size_t)D);
    int32_t dig[ORACLE_MULTI_N_MAX] = {0};
    if (!ks)
        return NULL;
    int sum = 0;
    for (int64_t i = 0; i < D; i++) {
        ks[i] = (uint8_t)sum;
        for (int j = 0; j < m; j++) { /* odometer step */
            if (dig[j] < mult[j]) {
                dig[j]++;
                sum++;
                break;
            }
            sum -= dig[j];
            dig[j] = 0;
        }
    }
    return ks;
}

int oracle_multi_c128(int n, int m, const int32_t *mult, const double *a, int nthreads, double *out)
{
    int64_t stride[ORACLE_MULTI_N_MAX + 1], D;
    int rc = multi_layout(n, m, mult, stride, &D);
    if (rc || !out || (n > 0 && !a))
        return rc ? rc : -1;
    if (n == 0) {
        out[0] = 1.0;
        out[1] = 0.0;
        return 0;
    }
    double *tab = (double *)malloc(2 * (size_t)D * sizeof(double));
    uint8_t *ks = multi_layers(m, mult, D);
    if (!tab || !ks) {
        free(tab);
        free(ks);
        return -2;
    }
    for (int j = 0; j < m; j++) {
        tab[2 * stride[j]] = a[2 * j];
        tab[2 * stride[j] + 1] = a[2 * j + 1];
    }
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#endif
    for (int k = 2; k <= n; k++) {
        const double *row = a + 2 * (size_t)(k - 1) * (size_t)m;
#pragma omp parallel for schedule(static, 4096)
        for (int64_t idx = 0; idx < D; idx++) {
            if (ks[idx] != k)
                continue;
            double re = 0.0, im = 0.0;
            for (int j = 0; j < m; j++) {
                if ((idx / stride[j]) % ((int64_t)mult[j] + 1) == 0)
                    continue;
                const int64_t P = idx - stride[j];
                const double ar = row[2 * j], ai = row[2 * j + 1];
                const double pr = tab[2 * P], pi = tab[2 * P + 1];
                re = fma(ar, pr, re);
                re = fma(-ai, pi, re);
                im = fma(ar, pi, im);
                im = fma(ai, pr, im);
            }
            tab[2 * idx] = re;
            tab[2 * idx + 1] = im;
        }
    }
    double f = 1.0;
    for (int j = 0; j < m; j++)
        for (int v = 2; v <= mult[j]; v++)
            f *= (double)v;
    out[0] = tab[2 * (D - 1)] * f;
    out[1] = tab[2 * (D - 1) + 1] * f;
    free(tab);
    free(ks);
    return 0;
}

/* r: n x m residues in [0, p), p < 2^61 (at most 64 products below 2^122
 * each, so the 128-bit sum cannot overflow); out = G(mult) mod p. */
int oracle_multi_modp(int n, int m, const int32_t *mult, const uint64_t *r, uint64_t p, int nthreads,
                      uint64_t *out)
{
    int64_t stride[ORACLE_MULTI_N_MAX + 1], D;
    int rc = multi_layout(n, m, mult, stride, &D);
    if (rc || !out || (n > 0 && !r) || p < 2 || p >= ((uint64_t)1 << 61))
        return rc ? rc : -1;
    for (size_t i = 0; i < (size_t)n * m; i++)
        if (r[i] >= p)
            return -1;
    if (n == 0) {
        *out = 1 % p;
        return 0;
    }
    uint64_t *tab = (uint64_t *)malloc((size_t)D * sizeof(uint64_t));
    uint8_t *ks = multi_layers(m, mult, D);
    if (!tab || !ks) {
        free(tab);
        free(ks);
        return -2;
    }
    for (int j = 0; j < m; j++)
        tab[stride[j]] = r[j];
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#endif
    for (int k = 2; k <= n; k++) {
        const uint64_t *row = r + (size_t)(k - 1) * (size_t)m;
#pragma omp parallel for schedule(static, 4096)
        for (int64_t idx = 0; idx < D; idx++) {
            if (ks[idx] != k)
                continue;
            u128 acc = 0;
            for (int j = 0; j < m; j++)
                if ((idx / stride[j]) % ((int64_t)mult[j] + 1) != 0)
                    acc += (u128)row[j] * tab[idx - stride[j]];
            tab[idx] = (uint64_t)(acc % p);
        }
    }
    *out = tab[D - 1];
    free(tab);
    free(ks);
    return 0;
}

/* ------------------------------------------------- eq. (4) mod p, O(n) memory */
/*
 * Ryser's formula (eq. 4 of the paper, section 3.3) in exact modular
 * arithmetic, for orders beyond the reach of the 2^n tables above:
 *
 *     per(A) = (-1)^n  sum over column subsets S of (-1)^|S| prod_i r_i(S),
 *     r_i(S) = sum_{j in S} a_ij.
 *
 * Everything is reduced mod a prime p = 2^61 - c (1 <= c < 2^16), so the
 * result is exact mod p; Garner on several primes gives the integer.  The
 * subsets are visited in binary-reflected Gray-code order (the g-th subset is
 * g XOR (g >> 1); going from g-1 to g flips exactly the column ctz(g)), so
 * each step changes every row sum by one entry.  The 2^n codes are cut into
 * blocks; a block forms the row sums of its first subset directly.  Memory is
 * O(n) per thread.  This is an independent method from the stored minors
 * above: it shares no step with them.
 *
 * Multiplication mod p = 2^61 - c (the classical pseudo-Mersenne
 * reduction): z = x*y < 2^122 is written z = hi*2^61 + lo, and
 * 2^61 = c (mod p), so z = lo + c*hi (mod p); twice, then subtract p while
 * the value is >= p.
 */
#define ORACLE_RYSER_N_MAX 40

static uint64_t mulmod_pm61(uint64_t x, uint64_t y, uint64_t p, uint64_t c)
{
    const uint64_t m61 = ((uint64_t)1 << 61) - 1;
    u128 z = (u128)x * y;                       /* < 2^122 */
    u128 w = (z >> 61) * c + (uint64_t)(z & m61); /* < 2^61 * 2^16 + 2^61 */
    uint64_t v = (uint64_t)(w & m61) + (uint64_t)(w >> 61) * c; /* < 2^61 + 2^33 */
    while (v >= p)
        v -= p;
    return v;
}

static uint64_t addmod(uint64_t x, uint64_t y, uint64_t p) { uint64_t s = x + y; return s >= p ? s - p : s; }
static uint64_t submod(uint64_t x, uint64_t y, uint64_t p) { return x >= y ? x - y : x + p - y; }

/* x * y mod p, exposed so a test can check the reduction against exact
 * integer arithmetic. */
uint64_t oracle_mulmod_pm61(uint64_t x, uint64_t y, uint64_t p)
{
    return mulmod_pm61(x, y, p, ((uint64_t)1 << 61) - p);
}

/* a: n x n residues in [0, p), row-major; p = 2^61 - c with 1 <= c < 2^16. */
int oracle_ryser_modp(int n, const uint64_t *a, uint64_t p, int nthreads, uint64_t *out)
{
    const uint64_t two61 = (uint64_t)1 << 61;
    if (n < 0 || n > ORACLE_RYSER_N_MAX || !out || (n > 0 && !a) || p >= two61 || two61 - p >= (1u << 16))
        return -1;
    for (size_t i = 0; i < (size_t)n * n; i++)
        if (a[i] >= p)
            return -1;
    if (n == 0) {
        *out = 1;
        return 0;
    }
    const uint64_t c = two61 - p;
    const int bb = n < 16 ? n : 16;          /* codes per block: 2^bb */
    const int64_t blocks = (int64_t)1 << (n - bb);
    uint64_t pos = 0, neg = 0;               /* sums of terms with sign + and - */
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        uint64_t r[ORACLE_RYSER_N_MAX];
        uint64_t my_pos = 0, my_neg = 0;
#pragma omp for schedule(dynamic, 1)
        for (int64_t blk = 0; blk < blocks; blk++) {
            const uint64_t g0 = (uint64_t)blk << bb;
            uint64_t S = g0 ^ (g0 >> 1);
            for (int i = 0; i < n; i++) {
                uint64_t s = 0;
                for (int j = 0; j < n; j++)
                    if ((S >> j) & 1u)
                        s = addmod(s, a[(size_t)i * n + j], p);
                r[i] = s;
            }
            for (uint64_t g = g0; g < g0 + ((uint64_t)1 << bb); g++) {
                if (g != g0) {
                    const int col = __builtin_ctzll(g);
                    S ^= (uint64_t)1 << col;
                    if ((S >> col) & 1u)
                        for (int i = 0; i < n; i++) r[i] = addmod(r[i], a[(size_t)i * n + col], p);
                    else
                        for (int i = 0; i < n; i++) r[i] = submod(r[i], a[(size_t)i * n + col], p);
                }
                /* prod_i r_i: two interleaved chains (even and odd rows) */
                uint64_t e = 1, o = 1;
                int i = 0;
                for (; i + 1 < n; i += 2) {
                    e = mulmod_pm61(e, r[i], p, c);
                    o = mulmod_pm61(o, r[i + 1], p, c);
                }
                if (i < n)
                    e = mulmod_pm61(e, r[i], p, c);
                const uint64_t term = mulmod_pm61(e, o, p, c);
                /* sign (-1)^(n - |S|) */
                if (((n - __builtin_popcountll(S)) & 1) == 0)
                    my_pos = addmod(my_pos, term, p);
                else
                    my_neg = addmod(my_neg, term, p);
            }
        }
#pragma omp critical
        {
            pos = addmod(pos, my_pos, p);
            neg = addmod(neg, my_neg, p);
        }
    }
    *out = submod(pos, neg, p);
    return 0;
}

/* -------------------------------------------- Gaussian integers mod p (exact) */
/*
 * The stored sub-permanents of section 4 for a matrix of Gaussian integers
 * g_ij = x_ij + i y_ij, reduced mod a prime p < 2^61: every value is a pair
 * (re, im) of residues, and a product follows (x + iy)(u + iv) =
 * (xu - yv) + i(xv + yu).  Sums are exact 128-bit integers (at most 40
 * products below 2^122 per part) reduced once per stored value.  With
 * A = 2^-b G (a dyadic complex matrix), per(A) = 2^-nb per(G) exactly, so
 * Garner over enough primes gives the exact permanent of A and hence the
 * true rounding error of any fp64 evaluation.  Layers mode, OpenMP.
 */
#define ORACLE_GAUSS_N_MAX 26

int oracle_per_gauss_modp(int n, const uint64_t *re, const uint64_t *im, uint64_t p, int nthreads,
                          uint64_t *out)
{
    if (n < 0 || n > ORACLE_GAUSS_N_MAX || !out || (n > 0 && (!re || !im)) || p < 2 ||
        p >= ((uint64_t)1 << 61))
        return -1;
    for (size_t i = 0; i < (size_t)n * n; i++)
        if (re[i] >= p || im[i] >= p)
            return -1;
    if (n == 0) {
        out[0] = 1 % p;
        out[1] = 0;
        return 0;
    }
    size_t N = (size_t)1 << n;
    uint64_t *tab = (uint64_t *)malloc(2 * N * sizeof(uint64_t));
    if (!tab)
        return -2;
    for (int j = 0; j < n; j++) {
        tab[2 * ((size_t)1 << j)] = re[j];
        tab[2 * ((size_t)1 << j) + 1] = im[j];
    }
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#endif
    for (int k = 2; k <= n; k++) {
        const uint64_t *xr = re + (size_t)(k - 1) * n, *yr = im + (size_t)(k - 1) * n;
#pragma omp parallel for schedule(static, 4096)
        for (int64_t S = 0; S < (int64_t)N; S++) {
            if (popcount32((uint32_t)S) != k)
                continue;
            /* re = sum x*u - sum y*v, im = sum x*v + sum y*u */
            u128 xu = 0, yv = 0, xv = 0, yu = 0;
            for (int j = 0; j < n; j++) {
                if (!((S >> j) & 1))
                    continue;
                const size_t P = (size_t)(S & ~((int64_t)1 << j));
                const uint64_t u = tab[2 * P], v = tab[2 * P + 1];
                xu += (u128)xr[j] * u;
                yv += (u128)yr[j] * v;
                xv += (u128)xr[j] * v;
                yu += (u128)yr[j] * u;
            }
            const uint64_t a1 = (uint64_t)(xu % p), a2 = (uint64_t)(yv % p);
            tab[2 * S] = a1 >= a2 ? a1 - a2 : a1 + p - a2;
            tab[2 * S + 1] = (uint64_t)((xv % p + yu % p) % p);
        }
    }
    out[0] = tab[2 * (N - 1)];
    out[1] = tab[2 * (N - 1) + 1];
    free(tab);
    return 0;
}

/* ------------------------------------------------ many small complex matrices */
/*
 * oracle_per_c128 (memo mode, the paper's order) for each of `count`
 * matrices packed row-major back to back: matrix i has order ns[i] <= 20
 * and starts at complex element offsets[i] of mats; out[2i], out[2i+1] get
 * its permanent.  OpenMP over the matrices (each one single-threaded).
 */
int oracle_per_c128_many(int64_t count, const int32_t *ns, const int64_t *offsets, const double *mats,
                         int nthreads, double *out)
{
    if (count < 0 || (count > 0 && (!ns || !offsets || !mats || !out)))
        return -1;
    for (int64_t i = 0; i < count; i++)
        if (ns[i] < 0 || ns[i] > 20 || offsets[i] < 0)
            return -1;
    int bad = 0;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 256) reduction(| : bad)
    for (int64_t i = 0; i < count; i++) {
        if (oracle_per_c128(ns[i], mats + 2 * offsets[i], 0, 1, out + 2 * i) != 0)
            bad = 1;
    }
    return bad ? -2 : 0;
}
