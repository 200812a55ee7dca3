// C ABI of libpermgpu (include/perm.h): validation, planning, workspace
// carving, the integer path's primes / bound / Chinese remaindering, the
// batch work list and graph cache, tuning and profiling.
//
// Paper: Su & Zheng, section 3.1 eq. (1) (the permanent), section 4
// (Store-zechin: development along the last row with stored minors).
#include "perm_host.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>

namespace permgpu {

typedef unsigned __int128 u128h;

// ------------------------------------------------------------------ errors
static thread_local std::string t_err;

int set_error(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return code;
}

int hip_error(hipError_t e, const char *what) {
    return set_error(PERM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCALL(expr, what)                              \
    do {                                                 \
        hipError_t _e = (expr);                          \
        if (_e != hipSuccess) return hip_error(_e, what); \
    } while (0)

double now_seconds() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ----------------------------------------------------------------- device
static std::mutex g_dev_mu;

int prepare_device(hipStream_t s, int *device) {
    int dev = 0;
    HIPCALL(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_dev_mu);
    HIPCALL(ensure_tables(dev, s), "building rank tables");
    if (device) *device = dev;
    return PERM_OK;
}

static int cu_count() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return 256;
    return cus;
}

// ------------------------------------------------------------------ primes
// Deterministic Miller-Rabin for 64-bit odd x with the first 12 prime bases.
static uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128h)a * b % m); }

static uint64_t powmod64(uint64_t a, uint64_t e, uint64_t m) {
    uint64_t r = 1 % m;
    a %= m;
    while (e) {
        if (e & 1) r = mulmod64(r, a, m);
        a = mulmod64(a, a, m);
        e >>= 1;
    }
    return r;
}

static bool is_prime64(uint64_t x) {
    static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (x < 2) return false;
    for (uint64_t b : bases)
        if (x % b == 0) return x == b;
    uint64_t d = x - 1;
    int s = 0;
    while (!(d & 1)) {
        d >>= 1;
        s++;
    }
    for (uint64_t a : bases) {
        uint64_t y = powmod64(a, d, x);
        if (y == 1 || y == x - 1) continue;
        bool comp = true;
        for (int i = 1; i < s; i++) {
            y = mulmod64(y, y, x);
            if (y == x - 1) {
                comp = false;
                break;
            }
        }
        if (comp) return false;
    }
    return true;
}

const std::vector<uint64_t> &primes61() {
    static std::vector<uint64_t> ps;
    static std::once_flag once;
    std::call_once(once, [] {
        for (uint64_t x = ((uint64_t)1 << 61) - 1; (int)ps.size() < PERM_MAX_PRIMES; x -= 2)
            if (is_prime64(x)) ps.push_back(x);
    });
    return ps;
}

// Smallest R with prod_{r<R} p_r > 2 * |per(A)| bound, where the bound is
// min(prod_i sum_j |a_ij|, n! max|a_ij|^n), evaluated in log2 with margin.
static int primes_needed(int n, const int64_t *a, int64_t lda) {
    double bits_rows = 0.0, bits_fact = 0.0;
    uint64_t mx = 0;
    bool zero_row = false;
    for (int i = 0; i < n; i++) {
        u128h s = 0;
        for (int j = 0; j < n; j++) {
            const int64_t v = a[(int64_t)i * lda + j];
            const uint64_t m = v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v;
            s += m;
            mx = std::max(mx, m);
        }
        if (s == 0) zero_row = true;
        else bits_rows += std::log2((double)s);
    }
    if (zero_row || mx == 0) return 1;
    for (int i = 2; i <= n; i++) bits_fact += std::log2((double)i);
    bits_fact += n * std::log2((double)mx);
    const double need = std::min(bits_rows, bits_fact) * (1.0 + 1e-12) + 2.0;  // > 2B, margin
    const auto &ps = primes61();
    double have = 0.0;
    int r = 0;
    while (have <= need && r < PERM_MAX_PRIMES) have += std::log2((double)ps[r++]);
    return r;
}

// Layers 1..K whose stored values provably lie in [-(2^63 - 1), 2^63 - 1]
// (returns K, 0 <= K <= n): expanding along row k - 1, |F(S)| for |S| = k is
// at most min(R_{k-1}, k M_{k-1}) times the bound of layer k - 1, with
// R_i = sum_j |a_ij| and M_i = max_j |a_ij| (the terms of S have at most k
// columns).  Those layers can run in plain 64-bit arithmetic: sums taken
// mod 2^64 recover a value in that range exactly.
static int plain_int64_layers(int n, const int64_t *a) {
    const u128h lim = ((u128h)1 << 63) - 1;
    u128h B = 1;
    int K = 0;
    for (int k = 1; k <= n; k++) {
        u128h R = 0, M = 0;
        for (int j = 0; j < n; j++) {
            const int64_t v = a[(size_t)(k - 1) * n + j];
            const u128h m = v < 0 ? (u128h)((uint64_t)0 - (uint64_t)v) : (u128h)v;
            R += m;
            if (m > M) M = m;
        }
        const u128h kM = (u128h)k * M, f = R < kM ? R : kM;
        if (f != 0 && B > lim / f) break;
        B *= f;
        K = k;
    }
    return K;
}

// ------------------------------------------------- Chinese remaindering
// Mixed-radix (Garner) digits d_i with v = sum d_i prod_{j<i} p_j.
static void garner_digits(const uint64_t *res, const uint64_t *p, int R, std::vector<uint64_t> &d) {
    d.assign(R, 0);
    for (int i = 0; i < R; i++) {
        // v_{<i} mod p_i by Horner from the top digit
        uint64_t acc = 0;
        for (int j = i - 1; j >= 0; j--) acc = (mulmod64(acc, p[j] % p[i], p[i]) + d[j] % p[i]) % p[i];
        uint64_t scale = 1;
        for (int j = 0; j < i; j++) scale = mulmod64(scale, p[j] % p[i], p[i]);
        const uint64_t inv = powmod64(scale, p[i] - 2, p[i]);
        const uint64_t diff = (res[i] + p[i] - acc) % p[i];
        d[i] = mulmod64(diff, inv, p[i]);
    }
}

typedef std::vector<uint64_t> Big;  // little-endian limbs

static void big_mul_add(Big &x, uint64_t m, uint64_t add) {
    u128h carry = add;
    for (auto &l : x) {
        const u128h t = (u128h)l * m + carry;
        l = (uint64_t)t;
        carry = t >> 64;
    }
    if (carry) x.push_back((uint64_t)carry);
}

static void big_trim(Big &x) {
    while (!x.empty() && x.back() == 0) x.pop_back();
}

static int big_cmp(const Big &a, const Big &b) {
    if (a.size() != b.size()) return a.size() < b.size() ? -1 : 1;
    for (size_t i = a.size(); i-- > 0;)
        if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    return 0;
}

static Big big_sub(const Big &a, const Big &b) {  // a >= b
    Big r(a.size());
    uint64_t borrow = 0;
    for (size_t i = 0; i < a.size(); i++) {
        const uint64_t bi = i < b.size() ? b[i] : 0;
        const u128h t = (u128h)a[i] - bi - borrow;
        r[i] = (uint64_t)t;
        borrow = (uint64_t)(t >> 64) ? 1 : 0;
    }
    big_trim(r);
    return r;
}

// Recombine residues of R primes, lift to (-P/2, P/2], check the redundant
// prime p[R] against res[R], multiply by the factors in *scale if given.
// Returns PERM_OK, PERM_EDEVICE (redundant prime) or PERM_ERANGE (limbs).
int crt_to_int(const uint64_t *res, const uint64_t *p, int R, perm_int_t *out,
               const std::vector<uint64_t> *scale) {
    std::vector<uint64_t> d;
    garner_digits(res, p, R, d);
    Big v{0}, P{1};
    // Horner: v = d_{R-1}; v = v * p_{i} + d_i for i = R-2..0
    v.assign(1, d[R - 1]);
    for (int i = R - 2; i >= 0; i--) big_mul_add(v, p[i], d[i]);
    for (int i = 0; i < R; i++) big_mul_add(P, p[i], 0);
    big_trim(v);
    big_trim(P);
    // lift: negative when 2v > P
    Big twice = v;
    big_mul_add(twice, 2, 0);
    big_trim(twice);
    int sign = 1;
    Big mag = v;
    if (big_cmp(twice, P) > 0) {
        mag = big_sub(P, v);
        sign = -1;
    }
    big_trim(mag);
    if (mag.empty()) sign = 0;
    // redundant check: v mod q (minus P mod q when lifted)
    const uint64_t q = p[R];
    uint64_t vq = d[R - 1] % q;
    for (int i = R - 2; i >= 0; i--) vq = (mulmod64(vq, p[i] % q, q) + d[i] % q) % q;
    if (sign < 0) {
        uint64_t Pq = 1;
        for (int i = 0; i < R; i++) Pq = mulmod64(Pq, p[i] % q, q);
        vq = (vq + q - Pq) % q;
    }
    if (vq != res[R])
        return set_error(PERM_EDEVICE, "redundant prime %llu disagrees with the recombined value",
                         (unsigned long long)q);
    if (scale && !mag.empty()) {
        for (uint64_t f : *scale) big_mul_add(mag, f, 0);
        big_trim(mag);
    }
    if (mag.size() > PERM_INT_LIMBS)
        return set_error(scale ? PERM_ERANGE : PERM_EDEVICE, "result needs %zu limbs (> %d)", mag.size(),
                         PERM_INT_LIMBS);
    std::memset(out, 0, sizeof *out);
    out->sign = sign;
    out->nlimbs = (uint32_t)mag.size();
    for (size_t i = 0; i < mag.size(); i++) out->limb[i] = mag[i];
    return PERM_OK;
}

static void int_from_i64(int64_t v, perm_int_t *out) {
    std::memset(out, 0, sizeof *out);
    if (v == 0) return;
    out->sign = v < 0 ? -1 : 1;
    out->nlimbs = 1;
    out->limb[0] = v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v;
}

// ----------------------------------------------------------------- tuning
static std::mutex g_tune_mu;
static perm_tuning_t g_tune;  // zero = defaults
static bool g_tune_init = false;

static void tune_init_locked() {
    if (g_tune_init) return;
    std::memset(&g_tune, 0, sizeof g_tune);
    for (int n = 0; n <= PERM_N_MAX; n++) g_tune.layer_xcd_remap[n] = -1;
    g_tune_init = true;
}

static int default_layer_t(int n) {
    int t = n - 12;
    if (t < 6) t = 6;
    if (t > 12) t = 12;
    if (t > n) t = n;
    return t;
}

static int valid_layer_t(int n, int t) {
    if (n < 2) return n;
    if (t < 1) t = 1;
    if (t > kTMax) t = kTMax;
    if (t > n) t = n;
    if (n - t > kHighBits) t = n - kHighBits;
    return t;
}

int tuned_layer_t(int n) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_init_locked();
    const int t = g_tune.layer_t[n] ? g_tune.layer_t[n] : default_layer_t(n);
    return valid_layer_t(n, t);
}

int tuned_layer_remap(int n) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_init_locked();
    const int r = g_tune.layer_xcd_remap[n];
    return r >= 0 ? r : (n >= 20 ? 64 : 0);
}

// Tiles with fewer outputs than this go to the per-thread path.
uint32_t tuned_layer_thin(int n) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_init_locked();
    const int v = g_tune.layer_thin[n];
    return v < 0 ? 0u : (v == 0 ? 128u : (uint32_t)v);
}

int tuned_layer_flags(int n) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_init_locked();
    return g_tune.layer_flags[n];
}

// Low columns of the integer sweep's plain 64-bit layers: layer_t, or one
// more with bit 1 of layer_flags (8-byte values fill a window of t + 1
// columns with about the bytes of a complex window of t).
static int tuned_plain_layer_t(int n) {
    const int t = tuned_layer_t(n);
    return (tuned_layer_flags(n) & 2) ? valid_layer_t(n, t + 1) : t;
}

// Threads per matrix in the batched kernel: a power of two in [16, block]
// with block/G matrices fitting the workgroup's LDS and, for the complex
// kernel, its register staging of one matrix entry per thread (the integer
// kernel reads its matrices directly; it keeps at most 4 entries per thread).
int tuned_batch_group(int n, size_t lds_bytes, int elem_bytes, int block) {
    int g;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_init_locked();
        g = g_tune.batch_group[n];
    }
    if (g == 0) {
        // as few threads per matrix as the LDS area and the register staging
        // allow (the loops below raise it): chunks carry as many matrices as
        // possible, and each chunk costs a claim and a prefetch round trip
        static const int defaults[PERM_BATCH_N_MAX + 1] = {16, 16, 16, 16, 16, 16, 16, 16, 16, 16, 16, 16, 16};
        g = defaults[n];
    }
    if (g > block) g = block;
    const size_t per = (((size_t)1 << n) + (size_t)n * n) * elem_bytes;
    while (g < block && (size_t)(block / g) * per > lds_bytes) g *= 2;
    const int stage = elem_bytes == 16 ? 1 : 4;
    while (g < block && (block / g) * n * n > stage * block) g *= 2;
    return g;
}

// ----------------------------------------------------------------- profile
static std::mutex g_prof_mu;
static std::atomic<bool> g_prof_on{false};
struct ProfEv {
    int kind;
    hipEvent_t a, b;
};
static std::vector<ProfEv> g_prof_events;
static std::vector<hipEvent_t> g_prof_pool;
static int64_t g_prof_plain_layers = 0;

bool profiling_on() { return g_prof_on.load(std::memory_order_relaxed); }

hipEvent_t profile_event() {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void profile_record(int kind, hipEvent_t a, hipEvent_t b) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_events.push_back({kind, a, b});
}

void profile_count_plain(int layers) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_plain_layers += layers;
}

// ------------------------------------------------------- complex solve
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static size_t max_layer(int n) {
    uint32_t m = 0;
    for (int k = 0; k <= n; k++) m = std::max(m, binom_host(n, k));
    return m;
}

size_t c128_workspace_bytes(int n) {
    if (n < 2) return 256;
    return align256((size_t)n * n * 16) + 256 + 2 * align256(max_layer(n) * 16);
}

int solve_c128_device(int n, const void *a_dev, int64_t lda, void *result_dev, void *ws,
                      size_t ws_bytes, hipStream_t s, bool allow_profile, bool allow_order) {
    if (n == 0) {
        static const perm_c128_t one = {1.0, 0.0};
        HIPCALL(hipMemcpyAsync(result_dev, &one, sizeof one, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
        return PERM_OK;
    }
    if (n == 1) {
        HIPCALL(hipMemcpyAsync(result_dev, a_dev, 16, hipMemcpyDeviceToDevice, s), "hipMemcpyAsync");
        return PERM_OK;
    }
    const size_t need = c128_workspace_bytes(n);
    if (!ws || ws_bytes < need)
        return set_error(PERM_ENOMEM, "workspace of %zu bytes < %zu needed for n=%d", ws_bytes, need, n);
    int rc = prepare_device(s, nullptr);
    if (rc) return rc;
    char *base = (char *)ws;
    void *packed = base;
    if (n <= kBatchNMax) {
        // one launch of the on-chip kernel: the whole table stays in LDS
        const void *mat = a_dev;
        if (lda != n) {
            HIPCALL(launch_pack_c128(a_dev, lda, n, packed, base + align256((size_t)n * n * 16) + 256, s),
                    "pack kernel");
            mat = packed;
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        const bool prof = allow_profile && profiling_on();
        if (prof) {
            e0 = profile_event();
            e1 = profile_event();
            if (e0) (void)hipEventRecord(e0, s);
        }
        HIPCALL(launch_single_c128(mat, n, result_dev, s), "small-n kernel");
        if (prof && e0 && e1) {
            (void)hipEventRecord(e1, s);
            profile_record(2, e0, e1);
        }
        return PERM_OK;
    }
    const size_t lay = align256(max_layer(n) * 16);
    char *buf0 = base + align256((size_t)n * n * 16) + 256;
    char *buf1 = buf0 + lay;
    HIPCALL(launch_pack_c128(a_dev, lda, n, packed, buf0, s), "pack kernel");
    const int t = tuned_layer_t(n);
    const int chunk = tuned_layer_remap(n);
    const int nt = tuned_layer_flags(n) & 1;
    const uint32_t thin = tuned_layer_thin(n);
    const bool order = allow_order && (tuned_layer_flags(n) & 4) && n - t <= kOrderNhMax;
    const bool prof = allow_profile && profiling_on();
    char *prev = buf0, *next = buf1;
    for (int k = 2; k <= n; k++) {
        LayerArgs args;
        const uint32_t grid = plan_layer(n, k, t, chunk, nt, thin, &args, order);
        if (order) {
            const int orc = apply_tile_order(n, k, t, thin, chunk, 16, s, &args);
            if (orc) return orc;
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (prof) {
            e0 = profile_event();
            e1 = profile_event();
            if (e0) (void)hipEventRecord(e0, s);
        }
        HIPCALL(launch_layer_c128(prev, next, packed, args, grid, s), "layer kernel");
        if (prof && e0 && e1) {
            (void)hipEventRecord(e1, s);
            profile_record(0, e0, e1);
        }
        std::swap(prev, next);
    }
    HIPCALL(launch_readout_c128(prev, result_dev, s), "readout kernel");
    return PERM_OK;
}

// --------------------------------------------------------- integer solve
// Workspace: matrix (n*n int64) | primes (40) | residues out (40) |
//            reduced matrices (kRPMax * n*n) | 2 * rp * maxC layer planes.
static size_t int_fixed_bytes(int n) {
    return align256((size_t)n * n * 8) + 2 * align256(PERM_MAX_PRIMES * 8) +
           align256((size_t)kRPMax * n * n * 8);
}

static size_t int_workspace_bytes(int n, int rp) {
    if (n < 2) return 256;
    return int_fixed_bytes(n) + 2 * align256((size_t)rp * max_layer(n) * 8);
}

static int solve_int(int n, const int64_t *a, int64_t lda, perm_int_t *out, void *ws, size_t ws_bytes,
                     hipStream_t s) {
    if (n == 0) {
        int_from_i64(1, out);
        return PERM_OK;
    }
    if (n == 1) {
        int_from_i64(a[0], out);
        return PERM_OK;
    }
    if (!ws || ws_bytes < int_workspace_bytes(n, 1))
        return set_error(PERM_ENOMEM, "workspace of %zu bytes < %zu needed for n=%d", ws_bytes,
                         int_workspace_bytes(n, 1), n);
    int rp = kRPMax;
    while (rp > 1 && int_workspace_bytes(n, rp) > ws_bytes) rp--;
    int rc = prepare_device(s, nullptr);
    if (rc) return rc;

    const int R = primes_needed(n, a, lda);
    const int Rt = R + 1;  // one redundant prime
    if (Rt > PERM_MAX_PRIMES) return set_error(PERM_ERANGE, "needs %d primes (> %d)", Rt, PERM_MAX_PRIMES);
    const auto &ps = primes61();

    std::vector<int64_t> packed((size_t)n * n);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) packed[(size_t)i * n + j] = a[(int64_t)i * lda + j];

    char *base = (char *)ws;
    int64_t *d_a = (int64_t *)base;
    uint64_t *d_primes = (uint64_t *)(base + align256((size_t)n * n * 8));
    uint64_t *d_res = (uint64_t *)((char *)d_primes + align256(PERM_MAX_PRIMES * 8));
    uint64_t *d_red = (uint64_t *)((char *)d_res + align256(PERM_MAX_PRIMES * 8));
    char *lay0 = base + int_fixed_bytes(n);
    const size_t plane = max_layer(n);
    uint64_t *buf0 = (uint64_t *)lay0;
    uint64_t *buf1 = (uint64_t *)(lay0 + align256((size_t)rp * plane * 8));

    // the primes, then a 0 that selects plain 64-bit arithmetic
    std::vector<uint64_t> up(ps.begin(), ps.begin() + Rt);
    up.push_back(0);
    const uint64_t *d_plain = Rt < PERM_MAX_PRIMES ? d_primes + Rt : nullptr;
    HIPCALL(hipMemcpyAsync(d_a, packed.data(), packed.size() * 8, hipMemcpyHostToDevice, s), "upload matrix");
    HIPCALL(hipMemcpyAsync(d_primes, up.data(), std::min<size_t>(up.size(), PERM_MAX_PRIMES) * 8,
                           hipMemcpyHostToDevice, s),
            "upload primes");
    if (n <= kBatchNMax) {
        // one launch of the on-chip kernel for every prime
        HIPCALL(launch_single_modp(d_a, n, d_primes, Rt, d_res, s), "small-n kernel");
        std::vector<uint64_t> res(Rt);
        HIPCALL(hipMemcpyAsync(res.data(), d_res, Rt * 8, hipMemcpyDeviceToHost, s), "download residues");
        HIPCALL(hipStreamSynchronize(s), "hipStreamSynchronize");
        return crt_to_int(res.data(), ps.data(), R, out);
    }
    const int t = tuned_layer_t(n);
    const int chunk = tuned_layer_remap(n);
    const bool prof = profiling_on();
    std::vector<int> binary(n, 1);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            const int64_t v = packed[(size_t)i * n + j];
            if (v != 0 && v != 1) binary[i] = 0;
        }
    // layers 2..K in plain 64-bit arithmetic (one plane), then residues
    const int K = d_plain ? plain_int64_layers(n, packed.data()) : 0;
    const int t_plain = tuned_plain_layer_t(n);
    const uint32_t thin = tuned_layer_thin(n);
    const bool order_on = tuned_layer_flags(n) & 4;
    auto layer = [&](uint64_t *prev, uint64_t *next, int k, const uint64_t *primes, int cnt, int tk) -> int {
        LayerArgs args;
        const bool order = order_on && n - tk <= kOrderNhMax;
        const uint32_t grid = plan_layer(n, k, tk, chunk, 0, thin, &args, order);
        if (order) {
            const int orc = apply_tile_order(n, k, tk, thin, chunk, 8 * cnt, s, &args);
            if (orc) return orc;
        }
        args.binary_row = binary[k - 1];
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (prof) {
            e0 = profile_event();
            e1 = profile_event();
            if (e0) (void)hipEventRecord(e0, s);
        }
        HIPCALL(launch_layer_modp(prev, next, plane, d_red, primes, cnt, args, grid, s), "modp layer kernel");
        if (prof && e0 && e1) {
            (void)hipEventRecord(e1, s);
            profile_record(1, e0, e1);
        }
        return PERM_OK;
    };
    // With more primes than one sweep carries, the plain layer K is kept for
    // the later groups in the tail of buf1's last plane, when the residue
    // layers (at most max_{k >= K} C(n, k) entries of a plane) and the
    // conversion leave that tail untouched; the plain layers then run once.
    uint64_t *keep = nullptr;
    if (K >= 2 && Rt > rp && rp >= 2) {
        size_t after = 0;
        for (int k = K; k <= n; k++) after = std::max<size_t>(after, binom_host(n, k));
        if (after + n + binom_host(n, K) <= plane)
            keep = buf1 + (size_t)(rp - 1) * plane + (plane - binom_host(n, K));
    }
    for (int s0 = 0; s0 < Rt; s0 += rp) {
        const int cnt = std::min(rp, Rt - s0);
        uint64_t *prev = buf0, *next = buf1;
        int k0 = 2;
        if (K >= 2 && keep && s0 > 0) {
            HIPCALL(launch_int64_to_modp(keep, prev, plane, binom_host(n, K), d_primes + s0, cnt, s),
                    "int64 to residues kernel");
            HIPCALL(launch_reduce_modp(d_a, n, d_primes + s0, cnt, d_red, next, plane, s), "reduce kernel");
            k0 = K + 1;
        } else if (K >= 2) {
            HIPCALL(launch_reduce_modp(d_a, n, d_plain, 1, d_red, prev, plane, s), "reduce kernel");
            for (int k = 2; k <= K; k++) {
                if ((rc = layer(prev, next, k, d_plain, 1, t_plain)) != PERM_OK) return rc;
                std::swap(prev, next);
            }
            if (prof) profile_count_plain(K - 1);
            if (keep)
                HIPCALL(hipMemcpyAsync(keep, prev, (size_t)binom_host(n, K) * 8, hipMemcpyDeviceToDevice, s),
                        "keep plain layer");
            HIPCALL(launch_int64_to_modp(prev, next, plane, binom_host(n, K), d_primes + s0, cnt, s),
                    "int64 to residues kernel");
            std::swap(prev, next);
            // the free buffer takes the reduced first row, which is not used
            HIPCALL(launch_reduce_modp(d_a, n, d_primes + s0, cnt, d_red, next, plane, s), "reduce kernel");
            k0 = K + 1;
        } else {
            HIPCALL(launch_reduce_modp(d_a, n, d_primes + s0, cnt, d_red, prev, plane, s), "reduce kernel");
        }
        for (int k = k0; k <= n; k++) {
            if ((rc = layer(prev, next, k, d_primes + s0, cnt, t)) != PERM_OK) return rc;
            std::swap(prev, next);
        }
        HIPCALL(launch_readout_modp(prev, plane, cnt, d_res + s0, s), "readout kernel");
    }
    std::vector<uint64_t> res(Rt);
    HIPCALL(hipMemcpyAsync(res.data(), d_res, Rt * 8, hipMemcpyDeviceToHost, s), "download residues");
    HIPCALL(hipStreamSynchronize(s), "hipStreamSynchronize");
    return crt_to_int(res.data(), ps.data(), R, out);
}

// -------------------------------------------------------------- batch
void batch_mask_list(int nmax, uint16_t *out) {
    size_t pos = 0;
    for (int k = 0; k <= nmax; k++) {
        if (k == 0) {
            out[pos++] = 0;
            continue;
        }
        for (int h = k - 1; h < nmax; h++) {
            // masks of popcount k with highest bit h, in increasing order, bucketed by low bits
            std::vector<uint16_t> bucket[8];
            for (uint32_t m = 1u << h; m < (2u << h); m++)
                if (__builtin_popcount(m) == k) bucket[m & 7].push_back((uint16_t)m);
            size_t idx[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (bool more = true; more;) {
                more = false;
                for (int b = 0; b < 8; b++)
                    if (idx[b] < bucket[b].size()) {
                        out[pos++] = bucket[b][idx[b]++];
                        more = true;
                    }
            }
        }
    }
}

struct BatchPlan {
    std::vector<uint32_t> order;
    std::vector<BatchChunk> chunks;
    int nmax = 0;
};

static void build_batch_plan(int count, const int32_t *ns, size_t lds, int elem, int block, BatchPlan &bp) {
    bp.order.resize(count);
    std::iota(bp.order.begin(), bp.order.end(), 0u);
    // largest cost first (cost grows with n); stable keeps input order inside an n
    std::stable_sort(bp.order.begin(), bp.order.end(), [&](uint32_t x, uint32_t y) { return ns[x] > ns[y]; });
    bp.chunks.clear();
    bp.nmax = 0;
    for (int i = 0; i < count; i++) bp.nmax = std::max(bp.nmax, (int)ns[i]);
    int i = 0;
    while (i < count) {
        const int n = ns[bp.order[i]];
        const int G = tuned_batch_group(n, lds, elem, block);
        const int per = block / G;
        int j = i;
        while (j < count && ns[bp.order[j]] == n && j - i < per) j++;
        BatchChunk c;
        c.first = (uint32_t)i;
        c.count = (uint16_t)(j - i);
        c.n = (uint8_t)n;
        int lg = 0;
        while ((1 << lg) < G) lg++;
        c.group = (uint8_t)lg;
        bp.chunks.push_back(c);
        i = j;
    }
}

struct BatchLayout {
    size_t counter, order, offsets, chunks, primes, res, mats, total;
};

static BatchLayout batch_layout(perm_dtype_t dt, int count, const int32_t *ns) {
    BatchLayout L{};
    size_t off = 0;
    L.counter = off;
    off += 256;
    L.order = off;
    off += align256((size_t)count * 4);
    L.offsets = off;
    off += align256((size_t)count * 8);
    L.chunks = off;
    off += align256((size_t)count * sizeof(BatchChunk));
    if (dt == PERM_INT64) {
        size_t elems = 0;
        for (int i = 0; i < count; i++) elems += (size_t)ns[i] * ns[i];
        L.primes = off;
        off += align256(PERM_MAX_PRIMES * 8);
        L.res = off;
        off += align256((size_t)PERM_MAX_PRIMES * count * 8);
        L.mats = off;
        off += align256(elems * 8);
    }
    L.total = off;
    return L;
}

struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    const void *mats = nullptr;
    void *results = nullptr;
    int count = -1;
};
static std::mutex g_graph_mu;
static std::map<void *, GraphEntry> g_graphs;  // keyed by workspace

// Orders in 0..PERM_BATCH_N_MAX, offsets >= 0, a matrix pointer when any
// order is positive.
static int validate_batch(int count, const int32_t *ns, const int64_t *offsets, const void *mats) {
    bool any_entries = false;
    for (int i = 0; i < count; i++) {
        if (ns[i] < 0) return set_error(PERM_EINVAL, "ns[%d] = %d < 0", i, ns[i]);
        if (ns[i] > PERM_BATCH_N_MAX)
            return set_error(PERM_ERANGE, "ns[%d] = %d > %d (use perm_solve)", i, ns[i], PERM_BATCH_N_MAX);
        if (offsets[i] < 0) return set_error(PERM_EINVAL, "offsets[%d] < 0", i);
        any_entries |= ns[i] > 0;
    }
    if (!mats && any_entries) return set_error(PERM_EINVAL, "null matrix pointer");
    return PERM_OK;
}

static int batch_c128(int count, const int32_t *ns, const int64_t *offsets, const void *mats, void *results,
                      void *ws, size_t ws_bytes, hipStream_t s, uint32_t flags) {
    const bool use_graph = (flags & PERM_BATCH_GRAPH) != 0;
    const bool reuse = (flags & PERM_BATCH_REUSE) != 0;
    std::unique_lock<std::mutex> glk(g_graph_mu);
    GraphEntry *ge = nullptr;
    if (use_graph) {
        auto it = g_graphs.find(ws);
        if (it != g_graphs.end() && it->second.mats == mats && it->second.results == results &&
            it->second.count == count && reuse)
            ge = &it->second;
    }
    if (!ge) {
        const int vrc = validate_batch(count, ns, offsets, mats);
        if (vrc) return vrc;
    }
    const BatchLayout L = batch_layout(PERM_COMPLEX128, count, ns);
    if (ws_bytes < L.total)
        return set_error(PERM_ENOMEM, "batch workspace of %zu bytes < %zu needed", ws_bytes, L.total);
    int rc = prepare_device(s, nullptr);
    if (rc) return rc;
    char *base = (char *)ws;
    uint32_t *d_counter = (uint32_t *)(base + L.counter);
    if (!ge) {
        int nmax = 0;
        for (int i = 0; i < count; i++) nmax = std::max(nmax, (int)ns[i]);
        const size_t lds = batch_area_bytes(nmax, 16);
        BatchPlan bp;
        build_batch_plan(count, ns, lds, 16, kBatchBlockComplex, bp);
        const uint32_t nchunks = (uint32_t)bp.chunks.size();
        HIPCALL(hipMemcpyAsync(base + L.order, bp.order.data(), (size_t)count * 4, hipMemcpyHostToDevice, s),
                "upload order");
        // the kernel reads offsets in work-list order (one dependent load fewer)
        std::vector<int64_t> soff(count);
        for (int i = 0; i < count; i++) soff[i] = offsets[bp.order[i]];
        HIPCALL(hipMemcpyAsync(base + L.offsets, soff.data(), (size_t)count * 8, hipMemcpyHostToDevice, s),
                "upload offsets");
        HIPCALL(hipMemcpyAsync(base + L.chunks, bp.chunks.data(), nchunks * sizeof(BatchChunk),
                               hipMemcpyHostToDevice, s),
                "upload chunks");
        const int grid = std::max(1, std::min<int>((int)nchunks, cu_count() * batch_blocks_per_cu(nmax, 16)));
        auto enqueue = [&](hipStream_t q) -> hipError_t {
            hipError_t e = launch_batch_reset(d_counter, q);
            if (e != hipSuccess) return e;
            return launch_batch_c128(mats, (const int64_t *)(base + L.offsets), (const uint32_t *)(base + L.order),
                                     (const BatchChunk *)(base + L.chunks), nchunks, d_counter, results, nmax,
                                     grid, q);
        };
        if (!use_graph) {
            glk.unlock();
            hipEvent_t e0 = nullptr, e1 = nullptr;
            const bool prof = profiling_on();
            if (prof) {
                e0 = profile_event();
                e1 = profile_event();
                if (e0) (void)hipEventRecord(e0, s);
            }
            HIPCALL(enqueue(s), "batch kernel");
            if (prof && e0 && e1) {
                (void)hipEventRecord(e1, s);
                profile_record(2, e0, e1);
            }
            if (flags & PERM_BATCH_SYNC) HIPCALL(hipStreamSynchronize(s), "hipStreamSynchronize");
            return PERM_OK;
        }
        // capture on a private stream, replay on the caller's
        auto &slot = g_graphs[ws];
        if (slot.exec) {
            (void)hipGraphExecDestroy(slot.exec);
            slot.exec = nullptr;
        }
        if (slot.graph) {
            (void)hipGraphDestroy(slot.graph);
            slot.graph = nullptr;
        }
        hipStream_t cap;
        HIPCALL(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "hipStreamCreate");
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t le = enqueue(cap);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(cap, &g);
            if (le != hipSuccess) e = le;
            if (e == hipSuccess) {
                slot.graph = g;
                e = hipGraphInstantiate(&slot.exec, g, nullptr, nullptr, 0);
            }
        }
        (void)hipStreamDestroy(cap);
        if (e != hipSuccess) {
            g_graphs.erase(ws);
            return hip_error(e, "batch graph capture");
        }
        slot.mats = mats;
        slot.results = results;
        slot.count = count;
        ge = &slot;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool prof = profiling_on();
    if (prof) {
        e0 = profile_event();
        e1 = profile_event();
        if (e0) (void)hipEventRecord(e0, s);
    }
    hipError_t e = hipGraphLaunch(ge->exec, s);
    glk.unlock();
    if (e != hipSuccess) return hip_error(e, "hipGraphLaunch");
    if (prof && e0 && e1) {
        (void)hipEventRecord(e1, s);
        profile_record(2, e0, e1);
    }
    if (flags & PERM_BATCH_SYNC) HIPCALL(hipStreamSynchronize(s), "hipStreamSynchronize");
    return PERM_OK;
}

static int batch_int(int count, const int32_t *ns, const int64_t *offsets, const int64_t *mats,
                     perm_int_t *results, void *ws, size_t ws_bytes, hipStream_t s) {
    const BatchLayout L = batch_layout(PERM_INT64, count, ns);
    if (ws_bytes < L.total)
        return set_error(PERM_ENOMEM, "batch workspace of %zu bytes < %zu needed", ws_bytes, L.total);
    int rc = prepare_device(s, nullptr);
    if (rc) return rc;
    // pack host matrices, count primes per matrix
    std::vector<int64_t> dev_off(count);
    std::vector<int> R(count);
    size_t elems = 0;
    int Rmax = 1;
    for (int i = 0; i < count; i++) {
        dev_off[i] = (int64_t)elems;
        elems += (size_t)ns[i] * ns[i];
        R[i] = ns[i] >= 2 ? primes_needed(ns[i], mats + offsets[i], ns[i]) : 1;
        Rmax = std::max(Rmax, R[i] + 1);
    }
    if (Rmax > PERM_MAX_PRIMES) return set_error(PERM_ERANGE, "needs %d primes", Rmax);
    std::vector<int64_t> packed(elems);
    for (int i = 0; i < count; i++)
        std::memcpy(&packed[dev_off[i]], mats + offsets[i], (size_t)ns[i] * ns[i] * 8);
    int nmax = 0;
    for (int i = 0; i < count; i++) nmax = std::max(nmax, (int)ns[i]);
    const size_t lds = batch_lds_bytes(nmax, 8) - 64;
    BatchPlan bp;
    build_batch_plan(count, ns, lds, 8, kBatchBlockInt, bp);
    const uint32_t nchunks = (uint32_t)bp.chunks.size();
    char *base = (char *)ws;
    const auto &ps = primes61();
    HIPCALL(hipMemcpyAsync(base + L.order, bp.order.data(), (size_t)count * 4, hipMemcpyHostToDevice, s), "upload");
    HIPCALL(hipMemcpyAsync(base + L.offsets, dev_off.data(), (size_t)count * 8, hipMemcpyHostToDevice, s), "upload");
    HIPCALL(hipMemcpyAsync(base + L.chunks, bp.chunks.data(), nchunks * sizeof(BatchChunk), hipMemcpyHostToDevice, s),
            "upload");
    HIPCALL(hipMemcpyAsync(base + L.primes, ps.data(), Rmax * 8, hipMemcpyHostToDevice, s), "upload");
    if (elems) HIPCALL(hipMemcpyAsync(base + L.mats, packed.data(), elems * 8, hipMemcpyHostToDevice, s), "upload");
    HIPCALL(launch_batch_reset((uint32_t *)(base + L.counter), s), "reset");
    const int grid = std::max(1, std::min<int>((int)nchunks, cu_count() * batch_blocks_per_cu(nmax, 8)));
    HIPCALL(launch_batch_modp((const int64_t *)(base + L.mats), (const int64_t *)(base + L.offsets),
                              (const uint32_t *)(base + L.order), (const BatchChunk *)(base + L.chunks), nchunks,
                              (uint32_t *)(base + L.counter), (const uint64_t *)(base + L.primes), Rmax,
                              (uint64_t *)(base + L.res), (uint32_t)count, nmax, grid, s),
            "batch modp kernel");
    std::vector<uint64_t> res((size_t)Rmax * count);
    HIPCALL(hipMemcpyAsync(res.data(), base + L.res, res.size() * 8, hipMemcpyDeviceToHost, s), "download");
    HIPCALL(hipStreamSynchronize(s), "hipStreamSynchronize");
    std::vector<uint64_t> r1(Rmax);
    for (int i = 0; i < count; i++) {
        if (ns[i] == 0) {
            int_from_i64(1, &results[i]);
            continue;
        }
        if (ns[i] == 1) {
            int_from_i64(mats[offsets[i]], &results[i]);
            continue;
        }
        for (int r = 0; r <= R[i]; r++) r1[r] = res[(size_t)r * count + i];
        int rc2 = crt_to_int(r1.data(), ps.data(), R[i], &results[i]);
        if (rc2) return rc2;
    }
    return PERM_OK;
}

// -------------------------------------------------------------- ryser
// Threads of the Gray-code walk: 2^hb of them, each over 2^(n-hb) codes.
// 2^21 threads keep the last wave of workgroups small next to the whole
// (three workgroups of 256 per CU fit the register budget at n = 28..30);
// 2^7 codes per thread keep the direct start (n*n additions) near 5 % of a
// thread's work; small orders use one code per thread.
static int ryser_high_bits(int n) {
    int hb = n - 7;
    const int lo = std::min(n, 12);
    if (hb < lo) hb = lo;
    if (hb > 21) hb = 21;
    return hb;
}

static uint32_t ryser_blocks(int n) { return (uint32_t)(((1u << ryser_high_bits(n)) + 255u) / 256u); }

// [matrix slot n*n][transposed n*n][partial sums][result], 256-byte aligned
struct RyserLayout {
    size_t mat, at, partial, result, total;
};

static RyserLayout ryser_layout(int n) {
    RyserLayout L{};
    const size_t nn = (size_t)n * n * 16;
    L.mat = 0;
    L.at = align256(nn);
    L.partial = L.at + align256(nn);
    L.result = L.partial + align256((size_t)ryser_blocks(n) * 16);
    L.total = L.result + 256;
    return L;
}

size_t ryser_c128_workspace_bytes(int n) { return n < 1 ? 256 : ryser_layout(n).total; }

// Integer layout: [residues, transposed, one n*n plane per prime][primes]
// [partial sums per prime][residues of the result], room for PERM_MAX_PRIMES.
struct RyserIntLayout {
    size_t atr, primes, partial, res, total;
};

static RyserIntLayout ryser_int_layout(int n) {
    RyserIntLayout L{};
    L.atr = 0;
    L.primes = align256((size_t)PERM_MAX_PRIMES * n * n * 8);
    L.partial = L.primes + align256(PERM_MAX_PRIMES * 8);
    L.res = L.partial + align256((size_t)PERM_MAX_PRIMES * ryser_blocks(n) * 8);
    L.total = L.res + align256(PERM_MAX_PRIMES * 8);
    return L;
}

size_t ryser_int_workspace_bytes(int n) { return n < 2 ? 256 : ryser_int_layout(n).total; }

// Exact integer permanent by eq. (4): residues mod the primes the bound asks
// for plus one redundant, Chinese remaindering on the host (as solve_int).
static int ryser_int(int n, const int64_t *a, int64_t lda, perm_int_t *out, void *ws, size_t ws_bytes,
                     hipStream_t s) {
    if (n == 0) {
        int_from_i64(1, out);
        return PERM_OK;
    }
    if (n == 1) {
        int_from_i64(a[0], out);
        return PERM_OK;
    }
    const size_t need = ryser_int_workspace_bytes(n);
    if (!ws || ws_bytes < need)
        return set_error(PERM_ENOMEM, "workspace of %zu bytes < %zu needed for n=%d", ws_bytes, need, n);
    int rc = prepare_device(s, nullptr);
    if (rc) return rc;
    const int R = primes_needed(n, a, lda);
    const int Rt = R + 1;  // one redundant prime
    if (Rt > PERM_MAX_PRIMES) return set_error(PERM_ERANGE, "needs %d primes (> %d)", Rt, PERM_MAX_PRIMES);
    const auto &ps = primes61();
    std::vector<uint64_t> atr((size_t)Rt * n * n);
    for (int r = 0; r < Rt; r++) {
        const uint64_t p = ps[r];
        for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++) {
                const int64_t v = a[(int64_t)i * lda + j];
                const uint64_t mag = v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v;
                uint64_t m = mag % p;
                if (v < 0 && m != 0) m = p - m;
                atr[(size_t)r * n * n + (size_t)j * n + i] = m;
            }
    }
    const RyserIntLayout L = ryser_int_layout(n);
    char *base = (char *)ws;
    uint64_t *d_atr = (uint64_t *)(base + L.atr), *d_primes = (uint64_t *)(base + L.primes);
    uint64_t *d_part = (uint64_t *)(base + L.partial), *d_res = (uint64_t *)(base + L.res);
    HIPCALL(hipMemcpyAsync(d_atr, atr.data(), atr.size() * 8, hipMemcpyHostToDevice, s), "upload residues");
    HIPCALL(hipMemcpyAsync(d_primes, ps.data(), Rt * 8, hipMemcpyHostToDevice, s), "upload primes");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool prof = profiling_on();
    if (prof) {
        e0 = profile_event();
        e1 = profile_event();
        if (e0) (void)hipEventRecord(e0, s);
    }
    const int hb = ryser_high_bits(n);
    HIPCALL(launch_ryser_modp(d_atr, d_primes, Rt, n, n - hb, d_part, ryser_blocks(n), d_res, s),
            "ryser modp kernel");
    if (prof && e0 && e1) {
        (void)hipEventRecord(e1, s);
        profile_record(3, e0, e1);
    }
    std::vector<uint64_t> res(Rt);
    HIPCALL(hipMemcpyAsync(res.data(), d_res, Rt * 8, hipMemcpyDeviceToHost, s), "download residues");
    HIPCALL(hipStreamSynchronize(s), "hipStreamSynchronize");
    return crt_to_int(res.data(), ps.data(), R, out);
}

// a_dev (device, lda) -> *result_dev (device), stream-ordered
static int ryser_c128_device(int n, const void *a_dev, int64_t lda, void *result_dev, void *ws, size_t ws_bytes,
                             hipStream_t s) {
    const size_t need = ryser_c128_workspace_bytes(n);
    if (!ws || ws_bytes < need)
        return set_error(PERM_ENOMEM, "workspace of %zu bytes < %zu needed for n=%d", ws_bytes, need, n);
    if (n == 0) {
        static const perm_c128_t one = {1.0, 0.0};
        HIPCALL(hipMemcpyAsync(result_dev, &one, 16, hipMemcpyHostToDevice, s), "write result");
        return PERM_OK;
    }
    int rc = prepare_device(s, nullptr);
    if (rc) return rc;
    const RyserLayout L = ryser_layout(n);
    char *base = (char *)ws;
    const int hb = ryser_high_bits(n);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool prof = profiling_on();
    if (prof) {
        e0 = profile_event();
        e1 = profile_event();
        if (e0) (void)hipEventRecord(e0, s);
    }
    HIPCALL(launch_ryser_transpose_c128(a_dev, lda, n, base + L.at, s), "ryser transpose");
    HIPCALL(launch_ryser_c128(base + L.at, n, n - hb, base + L.partial, ryser_blocks(n), result_dev, s),
            "ryser kernel");
    if (prof && e0 && e1) {
        (void)hipEventRecord(e1, s);
        profile_record(3, e0, e1);
    }
    return PERM_OK;
}

}  // namespace permgpu

// ======================================================================
//                                C ABI
// ======================================================================
using namespace permgpu;

extern "C" {

const char *perm_last_error(void) { return t_err.c_str(); }

int perm_version(void) { return 10000; }

int perm_prime(int i, uint64_t *p) {
    if (!p || i < 0 || i >= PERM_MAX_PRIMES) return set_error(PERM_EINVAL, "prime index %d out of range", i);
    *p = primes61()[i];
    return PERM_OK;
}

size_t perm_workspace_bytes(perm_dtype_t dt, int n) {
    if (n < 0 || n > PERM_N_MAX) return 0;
    if (dt == PERM_COMPLEX128) return c128_workspace_bytes(n);
    if (dt == PERM_INT64) return int_workspace_bytes(n, kRPMax);
    return 0;
}

int perm_solve(perm_dtype_t dt, int n, const void *a, int64_t lda, void *result, void *workspace,
               size_t ws_bytes, void *stream) {
    try {
        t_err.clear();
        if (dt != PERM_COMPLEX128 && dt != PERM_INT64) return set_error(PERM_EINVAL, "bad dtype %d", (int)dt);
        if (n < 0) return set_error(PERM_EINVAL, "n = %d < 0", n);
        if (n > PERM_N_MAX) return set_error(PERM_ERANGE, "n = %d > %d", n, PERM_N_MAX);
        if (!result || (n > 0 && !a)) return set_error(PERM_EINVAL, "null pointer");
        if (n > 0 && lda < n) return set_error(PERM_EINVAL, "lda = %lld < n = %d", (long long)lda, n);
        hipStream_t s = (hipStream_t)stream;
        if (dt == PERM_INT64) return solve_int(n, (const int64_t *)a, lda, (perm_int_t *)result, workspace, ws_bytes, s);
        perm_c128_t *out = (perm_c128_t *)result;
        if (n == 0) {
            out->re = 1.0;
            out->im = 0.0;
            return PERM_OK;
        }
        if (n == 1) {
            *out = *(const perm_c128_t *)a;
            return PERM_OK;
        }
        const size_t need = c128_workspace_bytes(n);
        if (!workspace || ws_bytes < need)
            return set_error(PERM_ENOMEM, "workspace of %zu bytes < %zu needed for n=%d", ws_bytes, need, n);
        // host matrix -> the workspace's matrix slot (packed, lda = n); the
        // pack kernel then reads and rewrites it in place; result -> slot
        std::vector<perm_c128_t> packed((size_t)n * n);
        const perm_c128_t *src = (const perm_c128_t *)a;
        for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++) packed[(size_t)i * n + j] = src[(int64_t)i * lda + j];
        char *base = (char *)workspace;
        void *d_res = base + ((size_t)n * n * 16 + 255) / 256 * 256;
        HIPCALL(hipMemcpyAsync(base, packed.data(), packed.size() * 16, hipMemcpyHostToDevice, s), "upload matrix");
        int rc = solve_c128_device(n, base, n, d_res, workspace, ws_bytes, s);
        if (rc) return rc;
        HIPCALL(hipMemcpyAsync(out, d_res, 16, hipMemcpyDeviceToHost, s), "download result");
        HIPCALL(hipStreamSynchronize(s), "hipStreamSynchronize");
        return PERM_OK;
    } catch (const std::exception &e) {
        return set_error(PERM_EDEVICE, "internal error: %s", e.what());
    } catch (...) {
        return set_error(PERM_EDEVICE, "internal error");
    }
}

int perm_solve_async(int n, const perm_c128_t *a_dev, int64_t lda, perm_c128_t *result_dev, void *workspace,
                     size_t ws_bytes, void *stream) {
    try {
        t_err.clear();
        if (n < 0) return set_error(PERM_EINVAL, "n = %d < 0", n);
        if (n > PERM_N_MAX) return set_error(PERM_ERANGE, "n = %d > %d", n, PERM_N_MAX);
        if (!result_dev || (n > 0 && !a_dev)) return set_error(PERM_EINVAL, "null pointer");
        if (n > 0 && lda < n) return set_error(PERM_EINVAL, "lda = %lld < n = %d", (long long)lda, n);
        return solve_c128_device(n, a_dev, lda, result_dev, workspace, ws_bytes, (hipStream_t)stream);
    } catch (...) {
        return set_error(PERM_EDEVICE, "internal error");
    }
}

int perm_solve_async_noalloc(int n, const perm_c128_t *a_dev, int64_t lda, perm_c128_t *result_dev,
                             void *stream) {
    try {
        t_err.clear();
        if (n < 0) return set_error(PERM_EINVAL, "n = %d < 0", n);
        if (n > PERM_NOALLOC_N_MAX)
            return set_error(PERM_ERANGE, "n = %d > %d: the allocation-free solve keeps its tables in a fixed "
                             "%zu-byte device array", n, PERM_NOALLOC_N_MAX, (size_t)PERM_NOALLOC_SCRATCH_BYTES);
        if (!result_dev || (n > 0 && !a_dev)) return set_error(PERM_EINVAL, "null pointer");
        if (n > 0 && lda < n) return set_error(PERM_EINVAL, "lda = %lld < n = %d", (long long)lda, n);
        void *ws = nullptr;
        size_t ws_bytes = 0;
        HIPCALL(noalloc_scratch(&ws, &ws_bytes), "hipGetSymbolAddress(scratch)");
        if (c128_workspace_bytes(n) > ws_bytes)
            return set_error(PERM_EDEVICE, "internal error: order %d needs %zu scratch bytes, the array holds %zu", n,
                             c128_workspace_bytes(n), ws_bytes);
        // profiling events are not created here: hipEventCreate allocates
        return solve_c128_device(n, a_dev, lda, result_dev, ws, ws_bytes, (hipStream_t)stream, false, false);
    } catch (...) {
        return set_error(PERM_EDEVICE, "internal error");
    }
}

size_t perm_ryser_workspace_bytes(perm_dtype_t dt, int n) {
    if (n < 0 || n > PERM_N_MAX) return 0;
    if (dt == PERM_COMPLEX128) return ryser_c128_workspace_bytes(n);
    if (dt == PERM_INT64) return ryser_int_workspace_bytes(n);
    return 0;
}

int perm_ryser(perm_dtype_t dt, int n, const void *a, int64_t lda, void *result, void *workspace,
               size_t ws_bytes, void *stream) {
    try {
        t_err.clear();
        if (dt != PERM_COMPLEX128 && dt != PERM_INT64) return set_error(PERM_EINVAL, "bad dtype %d", (int)dt);
        if (n < 0) return set_error(PERM_EINVAL, "n = %d < 0", n);
        if (n > PERM_N_MAX) return set_error(PERM_ERANGE, "n = %d > %d", n, PERM_N_MAX);
        if (!result || (n > 0 && !a)) return set_error(PERM_EINVAL, "null pointer");
        if (n > 0 && lda < n) return set_error(PERM_EINVAL, "lda = %lld < n = %d", (long long)lda, n);
        if (dt == PERM_INT64)
            return ryser_int(n, (const int64_t *)a, lda, (perm_int_t *)result, workspace, ws_bytes,
                             (hipStream_t)stream);
        perm_c128_t *out = (perm_c128_t *)result;
        if (n == 0) {
            out->re = 1.0;
            out->im = 0.0;
            return PERM_OK;
        }
        const size_t need = ryser_c128_workspace_bytes(n);
        if (!workspace || ws_bytes < need)
            return set_error(PERM_ENOMEM, "workspace of %zu bytes < %zu needed for n=%d", ws_bytes, need, n);
        hipStream_t s = (hipStream_t)stream;
        const RyserLayout L = ryser_layout(n);
        std::vector<perm_c128_t> packed((size_t)n * n);
        const perm_c128_t *src = (const perm_c128_t *)a;
        for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++) packed[(size_t)i * n + j] = src[(int64_t)i * lda + j];
        char *base = (char *)workspace;
        HIPCALL(hipMemcpyAsync(base + L.mat, packed.data(), packed.size() * 16, hipMemcpyHostToDevice, s),
                "upload matrix");
        int rc = ryser_c128_device(n, base + L.mat, n, base + L.result, workspace, ws_bytes, s);
        if (rc) return rc;
        HIPCALL(hipMemcpyAsync(out, base + L.result, 16, hipMemcpyDeviceToHost, s), "download result");
        HIPCALL(hipStreamSynchronize(s), "hipStreamSynchronize");
        return PERM_OK;
    } catch (const std::exception &e) {
        return set_error(PERM_EDEVICE, "internal error: %s", e.what());
    } catch (...) {
        return set_error(PERM_EDEVICE, "internal error");
    }
}

int perm_ryser_async(int n, const perm_c128_t *a_dev, int64_t lda, perm_c128_t *result_dev, void *workspace,
                     size_t ws_bytes, void *stream) {
    try {
        t_err.clear();
        if (n < 0) return set_error(PERM_EINVAL, "n = %d < 0", n);
        if (n > PERM_N_MAX) return set_error(PERM_ERANGE, "n = %d > %d", n, PERM_N_MAX);
        if (!result_dev || (n > 0 && !a_dev)) return set_error(PERM_EINVAL, "null pointer");
        if (n > 0 && lda < n) return set_error(PERM_EINVAL, "lda = %lld < n = %d", (long long)lda, n);
        return ryser_c128_device(n, a_dev, lda, result_dev, workspace, ws_bytes, (hipStream_t)stream);
    } catch (...) {
        return set_error(PERM_EDEVICE, "internal error");
    }
}

size_t perm_batch_workspace_bytes(perm_dtype_t dt, int count, const int32_t *ns) {
    if (count < 0 || (count > 0 && !ns)) return 0;
    if (dt != PERM_COMPLEX128 && dt != PERM_INT64) return 0;
    return batch_layout(dt, count, ns).total;
}

int perm_solve_batch(perm_dtype_t dt, int count, const int32_t *ns, const int64_t *offsets, const void *mats,
                     void *results, void *workspace, size_t ws_bytes, void *stream, uint32_t flags) {
    try {
        t_err.clear();
        if (dt != PERM_COMPLEX128 && dt != PERM_INT64) return set_error(PERM_EINVAL, "bad dtype %d", (int)dt);
        if (count < 0) return set_error(PERM_EINVAL, "count < 0");
        if (flags & ~(PERM_BATCH_SYNC | PERM_BATCH_GRAPH | PERM_BATCH_REUSE))
            return set_error(PERM_EINVAL, "unknown flags 0x%x", flags);
        if (count == 0) return PERM_OK;
        if (!ns || !offsets || !results || !workspace) return set_error(PERM_EINVAL, "null pointer");
        hipStream_t s = (hipStream_t)stream;
        if (dt == PERM_INT64) {
            const int rc = validate_batch(count, ns, offsets, mats);
            if (rc) return rc;
            return batch_int(count, ns, offsets, (const int64_t *)mats, (perm_int_t *)results, workspace, ws_bytes, s);
        }
        // the complex path validates whenever it builds a work list (a replayed
        // graph was validated when it was captured)
        return batch_c128(count, ns, offsets, mats, results, workspace, ws_bytes, s, flags);
    } catch (const std::exception &e) {
        return set_error(PERM_EDEVICE, "internal error: %s", e.what());
    } catch (...) {
        return set_error(PERM_EDEVICE, "internal error");
    }
}

// ------------------------------------------------------------ tuning ABI
int perm_tuning_get(perm_tuning_t *out) {
    if (!out) return set_error(PERM_EINVAL, "null pointer");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_init_locked();
    *out = g_tune;
    return PERM_OK;
}

int perm_tuning_set(const perm_tuning_t *in) {
    if (!in) return set_error(PERM_EINVAL, "null pointer");
    for (int n = 0; n <= PERM_N_MAX; n++) {
        const int t = in->layer_t[n];
        if (t != 0 && (t < 1 || t > kTMax || t > n || n - t > kHighBits))
            return set_error(PERM_EINVAL, "layer_t[%d] = %d impossible", n, t);
        if (in->layer_xcd_remap[n] < -1 || in->layer_xcd_remap[n] > 4096)
            return set_error(PERM_EINVAL, "layer_xcd_remap[%d] = %d", n, in->layer_xcd_remap[n]);
        if (in->layer_flags[n] & ~7)
            return set_error(PERM_EINVAL, "layer_flags[%d] = %d", n, in->layer_flags[n]);
        if (in->layer_thin[n] < -1 || in->layer_thin[n] > 65536)
            return set_error(PERM_EINVAL, "layer_thin[%d] = %d", n, in->layer_thin[n]);
    }
    for (int n = 0; n <= PERM_BATCH_N_MAX; n++) {
        const int g = in->batch_group[n];
        if (g != 0 && (g < 16 || g > kBatchBlockComplex || (g & (g - 1))))
            return set_error(PERM_EINVAL, "batch_group[%d] = %d (power of two in 16..%d)", n, g,
                             kBatchBlockComplex);
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune = *in;
    g_tune_init = true;
    return PERM_OK;
}

int perm_tuning_key(char *buf, size_t len) {
    if (!buf || len == 0) return set_error(PERM_EINVAL, "null buffer");
    int dev = 0, rt = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return set_error(PERM_EDEVICE, "no device");
    (void)hipRuntimeGetVersion(&rt);
    char arch[64];
    std::snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
    for (char *c = arch; *c; c++)
        if (*c == ':') {
            *c = 0;
            break;
        }
    std::snprintf(buf, len, "%s/cu%d/hip%d", arch, prop.multiProcessorCount, rt);
    return PERM_OK;
}

// Reads up to `count` integers of the array `name`; a shorter array (a file
// written when fewer orders existed) leaves the remaining entries unchanged.
static bool json_int_array(const std::string &s, const char *name, int *out, int count) {
    const std::string pat = std::string("\"") + name + "\"";
    size_t p = s.find(pat);
    if (p == std::string::npos) return false;
    p = s.find('[', p);
    if (p == std::string::npos) return false;
    const char *c = s.c_str() + p + 1;
    while (*c == ' ' || *c == '\n' || *c == '\t') c++;
    for (int i = 0; i < count && *c != ']'; i++) {
        char *end = nullptr;
        long v = std::strtol(c, &end, 10);
        if (end == c) return false;
        out[i] = (int)v;
        c = end;
        while (*c == ' ' || *c == ',' || *c == '\n' || *c == '\t') c++;
    }
    return *c == ']';
}

int perm_tuning_load(const char *path) {
    if (!path) return set_error(PERM_EINVAL, "null path");
    FILE *f = std::fopen(path, "rb");
    if (!f) return set_error(PERM_ENOTFOUND, "cannot open %s", path);
    std::string s;
    char buf[4096];
    size_t r;
    while ((r = std::fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, r);
    std::fclose(f);
    char key[256];
    int rc = perm_tuning_key(key, sizeof key);
    if (rc) return rc;
    const std::string want = std::string("\"key\": \"") + key + "\"";
    if (s.find(want) == std::string::npos) return set_error(PERM_ENOTFOUND, "tuning file is for another device");
    perm_tuning_t t;
    std::memset(&t, 0, sizeof t);
    for (int n = 0; n <= PERM_N_MAX; n++) t.layer_xcd_remap[n] = -1;
    // every array is optional (a file from an older library lacks the newer
    // ones: those keep their defaults); a present array must be complete
    struct {
        const char *name;
        int *v;
        int cnt;
    } arrays[] = {{"layer_t", t.layer_t, PERM_N_MAX + 1},
                  {"layer_xcd_remap", t.layer_xcd_remap, PERM_N_MAX + 1},
                  {"layer_flags", t.layer_flags, PERM_N_MAX + 1},
                  {"layer_thin", t.layer_thin, PERM_N_MAX + 1},
                  {"batch_group", t.batch_group, PERM_BATCH_N_MAX + 1}};
    for (auto &a : arrays) {
        const std::string pat = std::string("\"") + a.name + "\"";
        if (s.find(pat) == std::string::npos) continue;
        if (!json_int_array(s, a.name, a.v, a.cnt))
            return set_error(PERM_EINVAL, "malformed array %s in tuning file %s", a.name, path);
    }
    return perm_tuning_set(&t);
}

int perm_tuning_save(const char *path) {
    if (!path) return set_error(PERM_EINVAL, "null path");
    char key[256];
    int rc = perm_tuning_key(key, sizeof key);
    if (rc) return rc;
    perm_tuning_t t;
    perm_tuning_get(&t);
    FILE *f = std::fopen(path, "wb");
    if (!f) return set_error(PERM_EINVAL, "cannot write %s", path);
    std::fprintf(f, "{\n  \"key\": \"%s\",\n", key);
    auto arr = [&](const char *name, const int *v, int cnt, bool last) {
        std::fprintf(f, "  \"%s\": [", name);
        for (int i = 0; i < cnt; i++) std::fprintf(f, "%s%d", i ? ", " : "", v[i]);
        std::fprintf(f, "]%s\n", last ? "" : ",");
    };
    arr("layer_t", t.layer_t, PERM_N_MAX + 1, false);
    arr("layer_xcd_remap", t.layer_xcd_remap, PERM_N_MAX + 1, false);
    arr("layer_flags", t.layer_flags, PERM_N_MAX + 1, false);
    arr("layer_thin", t.layer_thin, PERM_N_MAX + 1, false);
    arr("batch_group", t.batch_group, PERM_BATCH_N_MAX + 1, true);
    std::fprintf(f, "}\n");
    std::fclose(f);
    return PERM_OK;
}

// ---------------------------------------------------------- profile ABI
int perm_profile_enable(int on) {
    g_prof_on.store(on != 0);
    return PERM_OK;
}

int perm_profile_read(perm_profile_t *out) {
    if (!out) return set_error(PERM_EINVAL, "null pointer");
    std::vector<ProfEv> evs;
    int64_t plain = 0;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        evs.swap(g_prof_events);
        plain = g_prof_plain_layers;
        g_prof_plain_layers = 0;
    }
    std::memset(out, 0, sizeof *out);
    out->int_plain_layers = plain;
    int rc = PERM_OK;
    for (auto &e : evs) {
        float ms = 0.f;
        hipError_t he = hipEventSynchronize(e.b);
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e.a, e.b);
        if (he != hipSuccess) rc = hip_error(he, "profile events");
        if (e.kind == 0) {
            out->layer_c128_ms += ms;
            out->layer_c128_launches++;
        } else if (e.kind == 1) {
            out->layer_modp_ms += ms;
            out->layer_modp_launches++;
        } else if (e.kind == 2) {
            out->batch_ms += ms;
            out->batch_launches++;
        } else if (e.kind == 3) {
            out->ryser_ms += ms;
            out->ryser_launches++;
        } else if (e.kind == 4) {
            out->multi_c128_ms += ms;
            out->multi_c128_launches++;
        } else {
            out->multi_modp_ms += ms;
            out->multi_modp_launches++;
        }
    }
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto &e : evs) {
        g_prof_pool.push_back(e.a);
        g_prof_pool.push_back(e.b);
    }
    return rc;
}

}  // extern "C"
