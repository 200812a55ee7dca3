// Host side of the repeated-column path (include/perm.h, "repeated
// columns"): plans of the count-vector layers, workspace carving, the
// complex and integer solves and their C ABI.
//
// Paper: Su & Zheng, section 4 (stored minors, development along the last
// row); section 2 (boson-sampling amplitudes are permanents of submatrices
// of the interferometer unitary -- a detector hit by t photons repeats its
// column t times).
#include "perm_host.h"
#include "perm_multi.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>

namespace permgpu {

#define MHIP(expr, what)                                  \
    do {                                                  \
        hipError_t _e = (expr);                           \
        if (_e != hipSuccess) return hip_error(_e, what); \
    } while (0)

namespace {

constexpr uint64_t kLowTarget = 1 << 14;     // low parts wanted per tile group
constexpr uint64_t kHighMax = 1ull << 20;    // high parts at most
constexpr uint64_t kPredMax = 1ull << 26;    // lowpred entries at most
constexpr uint64_t kPlanMax = 1ull << 30;    // plan bytes at most
constexpr uint64_t kSat = ~0ull;
constexpr uint32_t kNone = 0xffffffffu;

uint64_t sat_add(uint64_t a, uint64_t b) { return a > kSat - b ? kSat : a + b; }
uint64_t sat_mul(uint64_t a, uint64_t b) { return (b != 0 && a > kSat / b) ? kSat : a * b; }
size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

typedef unsigned __int128 u128m;

struct MultiPlan {
    int n = 0, m = 0, L = 0, SL = 0;
    std::vector<int32_t> mult;
    uint64_t states = 0, low_states = 0;
    std::vector<uint32_t> size;  // layer sizes, k = 0..n
    uint32_t max_layer = 0;
    std::vector<uint32_t> WL;    // low parts of sum s, s = 0..SL
    // device image in 32-bit words; every section starts on 256 bytes
    std::vector<uint32_t> blob;
    size_t low_list = 0, low_off = 0, low_pred = 0;
    std::vector<size_t> tiles, wins, chunks;  // word offsets of layer k (k >= 2)
    std::vector<uint32_t> ntiles, nchunks;
    uint64_t total_tiles = 0, total_wins = 0;
    // device copies of blob, per device index (guarded by g_plan_mu; freed
    // only when the plan leaves the cache, never at exit)
    mutable std::map<int, void *> dev;
};

// W[j][s]: count vectors over columns 0..j-1 with sum s (saturating).
std::vector<std::vector<uint64_t>> prefix_counts(int n, int m, const int32_t *t) {
    std::vector<std::vector<uint64_t>> W(m + 1, std::vector<uint64_t>(n + 1, 0));
    W[0][0] = 1;
    for (int j = 0; j < m; j++)
        for (int s = 0; s <= n; s++) {
            uint64_t acc = 0;
            for (int v = 0; v <= t[j] && v <= s; v++) acc = sat_add(acc, W[j][s - v]);
            W[j + 1][s] = acc;
        }
    return W;
}

size_t section(std::vector<uint32_t> &b) {
    b.resize((b.size() + 63) & ~(size_t)63, 0);
    return b.size();
}

int build_plan(int n, int m, const int32_t *t, MultiPlan &P) {
    P.n = n;
    P.m = m;
    P.mult.assign(t, t + m);
    const auto W = prefix_counts(n, m, t);
    P.size.assign(n + 1, 0);
    for (int k = 0; k <= n; k++) {
        if (W[m][k] >= (1ull << 32))
            return set_error(PERM_ERANGE, "layer %d holds %llu count vectors (2^32 or more)", k,
                             (unsigned long long)W[m][k]);
        P.size[k] = (uint32_t)W[m][k];
        P.max_layer = std::max(P.max_layer, P.size[k]);
    }
    std::vector<uint64_t> PL(m + 1, 1), PH(m + 1, 1);
    for (int j = 0; j < m; j++) PL[j + 1] = sat_mul(PL[j], (uint64_t)t[j] + 1);
    for (int j = m - 1; j >= 0; j--) PH[j] = sat_mul(PH[j + 1], (uint64_t)t[j] + 1);
    P.states = PL[m];
    int L = 1;
    while (L < m && PL[L] < kLowTarget) L++;
    while (L < m && PH[L] > kHighMax) L++;
    if (PL[L] == kSat || sat_mul(PL[L], (uint64_t)L) > kPredMax || PH[L] > kHighMax)
        return set_error(PERM_ERANGE, "repeated-column plan too large (%llu low parts, %llu high parts)",
                         (unsigned long long)PL[L], (unsigned long long)PH[L]);
    P.L = L;
    P.low_states = PL[L];
    P.SL = 0;
    for (int j = 0; j < L; j++) P.SL += t[j];
    P.WL.assign(P.SL + 1, 0);
    for (int s = 0; s <= P.SL; s++) P.WL[s] = (uint32_t)W[L][s];  // <= layer size < 2^32

    // low parts: colex order inside each sum is increasing mixed-radix index
    const uint32_t DL = (uint32_t)PL[L];
    std::vector<uint32_t> cnt(P.SL + 1, 0), rankL(DL), lowoff(P.SL + 2, 0), lowlist(DL),
        lowpred((size_t)DL * L, kNone);
    std::vector<uint8_t> sumL(DL);
    {
        std::vector<int> d(L, 0);
        int sum = 0;
        for (uint32_t v = 0; v < DL; v++) {
            sumL[v] = (uint8_t)sum;
            rankL[v] = cnt[sum]++;
            for (int i = 0; i < L; i++)
                if (d[i] > 0) lowpred[(size_t)v * L + i] = rankL[v - (uint32_t)PL[i]];
            for (int i = 0; i < L; i++) {  // odometer
                if (d[i] < t[i]) {
                    d[i]++;
                    sum++;
                    break;
                }
                sum -= d[i];
                d[i] = 0;
            }
        }
    }
    for (int s = 0; s <= P.SL; s++) lowoff[s + 1] = lowoff[s] + cnt[s];
    for (uint32_t v = 0; v < DL; v++) lowlist[lowoff[sumL[v]] + rankL[v]] = v;
    std::vector<uint32_t> &b = P.blob;
    P.low_list = section(b);
    b.insert(b.end(), lowlist.begin(), lowlist.end());
    P.low_off = section(b);
    b.insert(b.end(), lowoff.begin(), lowoff.end());
    P.low_pred = section(b);
    b.insert(b.end(), lowpred.begin(), lowpred.end());

    // high parts: tiles of layer k in increasing mixed-radix index of h with
    // column L least significant (= colex), each of WL[k - |h|] outputs
    const int mh = m - L;
    std::vector<uint64_t> SH(mh + 1, 1);
    for (int j = 0; j < mh; j++) SH[j + 1] = SH[j] * ((uint64_t)t[L + j] + 1);
    const uint64_t DH = SH[mh];
    std::vector<int64_t> prevb(DH, -1), curb(DH, -1);
    P.tiles.assign(n + 1, 0);
    P.wins.assign(n + 1, 0);
    P.chunks.assign(n + 1, 0);
    P.ntiles.assign(n + 1, 0);
    P.nchunks.assign(n + 1, 0);
    std::vector<uint32_t> tl, wl, cl;
    std::vector<int> d(mh, 0);
    for (int k = 1; k <= n; k++) {
        tl.clear();
        wl.clear();
        std::fill(d.begin(), d.end(), 0);
        int q = 0;
        uint64_t base = 0;
        for (uint64_t x = 0; x < DH; x++) {
            const int kp = k - q;
            if (kp < 0 || kp > P.SL) {
                curb[x] = -1;
            } else {
                curb[x] = (int64_t)base;
                if (k >= 2) {
                    int64_t lb = 0;
                    if (kp >= 1) {
                        lb = prevb[x];
                        if (lb < 0) return set_error(PERM_EDEVICE, "plan: missing low tile (layer %d)", k);
                    }
                    tl.push_back((uint32_t)base);
                    tl.push_back((uint32_t)kp);
                    tl.push_back((uint32_t)lb);
                    tl.push_back((uint32_t)(wl.size() / 2));
                    for (int j = 0; j < mh; j++) {
                        if (d[j] == 0) continue;
                        const int64_t pb = prevb[x - SH[j]];
                        if (pb < 0) return set_error(PERM_EDEVICE, "plan: missing high tile (layer %d)", k);
                        wl.push_back((uint32_t)pb);
                        wl.push_back((uint32_t)(L + j));
                    }
                }
                base += P.WL[kp];
            }
            for (int j = 0; j < mh; j++) {  // odometer
                if (d[j] < t[L + j]) {
                    d[j]++;
                    q++;
                    break;
                }
                q -= d[j];
                d[j] = 0;
            }
        }
        if (base != P.size[k]) return set_error(PERM_EDEVICE, "plan: layer %d size %llu != %u", k,
                                                (unsigned long long)base, P.size[k]);
        if (k >= 2) {
            const uint32_t nt = (uint32_t)(tl.size() / 4);
            tl.push_back(P.size[k]);
            tl.push_back(0);
            tl.push_back(0);
            tl.push_back((uint32_t)(wl.size() / 2));
            const uint32_t nch = (P.size[k] + kMultiBlock - 1) / kMultiBlock;
            cl.assign(nch + 1, 0);
            uint32_t ti = 0;
            for (uint32_t c = 0; c < nch; c++) {
                const uint64_t first = (uint64_t)c * kMultiBlock;
                while (ti + 1 < nt && tl[4 * (ti + 1)] <= first) ti++;
                cl[c] = ti;
            }
            cl[nch] = nt - 1;  // every tile is nonempty: the last one holds the last output
            P.tiles[k] = section(b);
            b.insert(b.end(), tl.begin(), tl.end());
            P.wins[k] = section(b);
            b.insert(b.end(), wl.begin(), wl.end());
            P.chunks[k] = section(b);
            b.insert(b.end(), cl.begin(), cl.end());
            P.ntiles[k] = nt;
            P.nchunks[k] = nch;
            P.total_tiles += nt;
            P.total_wins += wl.size() / 2;
            if ((uint64_t)b.size() * 4 > kPlanMax)
                return set_error(PERM_ERANGE, "repeated-column plan above %llu bytes", (unsigned long long)kPlanMax);
        }
        std::swap(prevb, curb);
    }
    section(b);
    return PERM_OK;
}

MultiLayerArgs layer_args(const MultiPlan &P, const char *d_blob, int k) {
    MultiLayerArgs g;
    g.tiles = (const uint4 *)(d_blob + P.tiles[k] * 4);
    g.wins = (const uint2 *)(d_blob + P.wins[k] * 4);
    g.chunk_tile = (const uint32_t *)(d_blob + P.chunks[k] * 4);
    g.lowlist = (const uint32_t *)(d_blob + P.low_list * 4);
    g.lowoff = (const uint32_t *)(d_blob + P.low_off * 4);
    g.lowpred = (const uint32_t *)(d_blob + P.low_pred * 4);
    g.size = P.size[k];
    g.nchunks = P.nchunks[k];
    g.L = P.L;
    g.m = P.m;
    return g;
}

// ---------------------------------------------------------- plan checker
// Independent of the builder: closed-form colex rank / unrank of count
// vectors, compared with what the tables give for each checked output.
struct Ranker {
    int n, m;
    const int32_t *t;
    std::vector<std::vector<uint64_t>> W;
    uint64_t rank(const std::vector<int> &c) const {
        uint64_t r = 0;
        int P = 0;
        for (int j = 0; j < m; j++) {
            P += c[j];
            for (int v = 0; v < c[j]; v++) r += W[j][P - v];
        }
        return r;
    }
    void unrank(int k, uint64_t r, std::vector<int> &c) const {
        int R = k;
        for (int j = m - 1; j >= 0; j--) {
            int v = 0;
            for (; v <= t[j] && v <= R; v++) {
                if (r < W[j][R - v]) break;
                r -= W[j][R - v];
            }
            c[j] = v;
            R -= v;
        }
    }
};

int check_plan(const MultiPlan &P, uint64_t *checked) {
    Ranker rk{P.n, P.m, P.mult.data(), prefix_counts(P.n, P.m, P.mult.data())};
    uint64_t all = 0;
    for (int k = 2; k <= P.n; k++) all += P.size[k];
    const bool full = all <= (1ull << 22);
    const uint32_t *B = P.blob.data();
    const uint32_t *lowlist = B + P.low_list, *lowoff = B + P.low_off, *lowpred = B + P.low_pred;
    std::vector<uint64_t> PL(P.L + 1, 1);
    for (int i = 0; i < P.L; i++) PL[i + 1] = PL[i] * ((uint64_t)P.mult[i] + 1);
    std::vector<int> c(P.m), e(P.m);
    uint64_t done = 0;
    for (int k = 2; k <= P.n; k++) {
        const uint32_t size = P.size[k], nt = P.ntiles[k], nch = P.nchunks[k];
        const uint32_t *T = B + P.tiles[k], *Wn = B + P.wins[k], *C = B + P.chunks[k];
        // tiles: contiguous, nonempty, sized WL[kp]; sentinel at the end
        for (uint32_t i = 0; i < nt; i++) {
            const uint32_t kp = T[4 * i + 1];
            if ((int)kp > P.SL || T[4 * i] + P.WL[kp] != T[4 * (i + 1)] || T[4 * i + 3] > T[4 * (i + 1) + 3])
                return set_error(PERM_EDEVICE, "plan check: layer %d tile %u malformed", k, i);
        }
        if (T[0] != 0 || T[4 * nt] != size) return set_error(PERM_EDEVICE, "plan check: layer %d tile bounds", k);
        // chunks: tile of the first output, at most kMultiBlock + 1 tiles each
        for (uint32_t ch = 0; ch <= nch; ch++) {
            const uint64_t o = ch < nch ? (uint64_t)ch * kMultiBlock : size - 1;
            const uint32_t ti = C[ch];
            if (ti >= nt || T[4 * ti] > o || T[4 * (ti + 1)] <= o)
                return set_error(PERM_EDEVICE, "plan check: layer %d chunk %u", k, ch);
            if (ch < nch && C[ch + 1] - C[ch] + 1 > (uint32_t)kMultiBlock + 1)
                return set_error(PERM_EDEVICE, "plan check: layer %d chunk %u spans too many tiles", k, ch);
        }
        const uint32_t step = (full || size <= 4096) ? 1 : std::max<uint32_t>(1, size / 4096);
        // every `step`-th output and the last one
        auto after = [&](uint64_t r) -> uint64_t {
            if (r == size - 1) return size;
            return r + step < size ? r + step : size - 1;
        };
        uint32_t ti = 0;
        for (uint64_t r = 0; r < size; r = after(r)) {
            while (T[4 * (ti + 1)] <= r) ti++;
            rk.unrank(k, r, c);
            const uint32_t base = T[4 * ti], kp = T[4 * ti + 1], lb = T[4 * ti + 2];
            const uint32_t w0 = T[4 * ti + 3], w1 = T[4 * (ti + 1) + 3];
            const uint32_t loc = (uint32_t)(r - base);
            int sl = 0;
            for (int i = 0; i < P.L; i++) sl += c[i];
            if ((uint32_t)sl != kp) return set_error(PERM_EDEVICE, "plan check: layer %d rank %llu low sum", k,
                                                     (unsigned long long)r);
            const uint32_t v = lowlist[lowoff[kp] + loc];
            uint64_t vv = 0;
            for (int i = 0; i < P.L; i++) vv += (uint64_t)c[i] * PL[i];
            if (v != vv) return set_error(PERM_EDEVICE, "plan check: layer %d rank %llu low part", k,
                                          (unsigned long long)r);
            uint32_t w = w0;
            for (int j = 0; j < P.m; j++) {
                if (c[j] == 0) {
                    if (j < P.L && lowpred[(size_t)v * P.L + j] != kNone)
                        return set_error(PERM_EDEVICE, "plan check: layer %d rank %llu spurious low %d", k,
                                         (unsigned long long)r, j);
                    continue;
                }
                e = c;
                e[j]--;
                const uint64_t want = rk.rank(e);
                uint64_t got;
                if (j < P.L) {
                    const uint32_t q = lowpred[(size_t)v * P.L + j];
                    if (q == kNone) return set_error(PERM_EDEVICE, "plan check: missing low %d", j);
                    got = (uint64_t)lb + q;
                } else {
                    if (w >= w1 || Wn[2 * w + 1] != (uint32_t)j)
                        return set_error(PERM_EDEVICE, "plan check: layer %d rank %llu window of column %d", k,
                                         (unsigned long long)r, j);
                    got = (uint64_t)Wn[2 * w] + loc;
                    w++;
                }
                if (got != want || want >= P.size[k - 1])
                    return set_error(PERM_EDEVICE, "plan check: layer %d rank %llu column %d: %llu != %llu", k,
                                     (unsigned long long)r, j, (unsigned long long)got, (unsigned long long)want);
            }
            if (w != w1) return set_error(PERM_EDEVICE, "plan check: layer %d rank %llu extra windows", k,
                                          (unsigned long long)r);
            done++;
        }
    }
    *checked = done;
    return PERM_OK;
}

// ------------------------------------------------------------ plan cache
// Host plans by multiplicity vector, each with its device copies; at most
// kPlanCache plans and kDevPlanBytes of device copies, least recently used
// dropped first.
std::mutex g_plan_mu;
std::map<std::vector<int32_t>, std::shared_ptr<const MultiPlan>> g_plans;
std::deque<std::vector<int32_t>> g_plan_order;
size_t g_dev_plan_bytes = 0;
constexpr size_t kPlanCache = 16;
constexpr size_t kDevPlanBytes = (size_t)2 << 30;

void drop_oldest_locked() {
    auto it = g_plans.find(g_plan_order.front());
    g_plan_order.pop_front();
    if (it == g_plans.end()) return;
    if (!it->second->dev.empty()) {
        // a queued launch may still read the tables
        (void)hipDeviceSynchronize();
        for (auto &d : it->second->dev) {
            (void)hipFree(d.second);
            g_dev_plan_bytes -= it->second->blob.size() * 4;
        }
        it->second->dev.clear();
    }
    g_plans.erase(it);
}

int get_plan(int n, int m, const int32_t *t, std::shared_ptr<const MultiPlan> &out) {
    std::vector<int32_t> key(t, t + m);
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        auto it = g_plans.find(key);
        if (it != g_plans.end()) {
            out = it->second;
            return PERM_OK;
        }
    }
    auto P = std::make_shared<MultiPlan>();
    const int rc = build_plan(n, m, t, *P);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) {  // built meanwhile by another thread
        out = it->second;
        return PERM_OK;
    }
    while (g_plans.size() >= kPlanCache) drop_oldest_locked();
    g_plans[key] = P;
    g_plan_order.push_back(key);
    out = P;
    return PERM_OK;
}

// Device copy of the plan's tables on the current device (uploaded once).
int device_plan(const MultiPlan &P, const char **out) {
    int dev = 0;
    MHIP(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto it = P.dev.find(dev);
    if (it != P.dev.end()) {
        *out = (const char *)it->second;
        return PERM_OK;
    }
    const size_t bytes = P.blob.size() * 4;
    while (g_dev_plan_bytes + bytes > kDevPlanBytes && g_plan_order.size() > 1 &&
           g_plans.find(g_plan_order.front())->second.get() != &P)
        drop_oldest_locked();
    void *ptr = nullptr;
    MHIP(hipMalloc(&ptr, bytes), "hipMalloc (repeated-column plan)");
    const hipError_t e = hipMemcpy(ptr, P.blob.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(ptr);
        return hip_error(e, "upload repeated-column plan");
    }
    P.dev[dev] = ptr;
    g_dev_plan_bytes += bytes;
    *out = (const char *)ptr;
    return PERM_OK;
}

// -------------------------------------------------------------- checks
// PERM_OK for a plan-path shape, 1 for the subset path (every count 1),
// negative on error.
int validate(int n, int m, const int32_t *t, const void *a, int64_t lda) {
    if (n < 0 || m < 0) return set_error(PERM_EINVAL, "negative size");
    if (n > PERM_MULTI_N_MAX) return set_error(PERM_ERANGE, "n=%d above %d", n, PERM_MULTI_N_MAX);
    if (m > n || (n > 0 && m == 0)) return set_error(PERM_EINVAL, "m=%d distinct columns for n=%d", m, n);
    if (m > 0 && !t) return set_error(PERM_EINVAL, "null multiplicities");
    int sum = 0;
    for (int j = 0; j < m; j++) {
        if (t[j] < 1) return set_error(PERM_EINVAL, "multiplicity %d of column %d below 1", t[j], j);
        sum += t[j];
    }
    if (sum != n) return set_error(PERM_EINVAL, "multiplicities sum to %d, not n=%d", sum, n);
    if (n > 0 && (!a || lda < m)) return set_error(PERM_EINVAL, "null matrix or lda < m");
    if (m == n) {
        if (n > PERM_N_MAX) return set_error(PERM_ERANGE, "no repeated column and n=%d above %d", n, PERM_N_MAX);
        return 1;
    }
    return PERM_OK;
}

double scale_c128(const MultiPlan &P) {
    double f = 1.0;
    for (int j = 0; j < P.m; j++)
        for (int v = 2; v <= P.mult[j]; v++) f *= (double)v;
    return f;
}

// ------------------------------------------------------------- complex
struct LayoutC {
    size_t packed, res, buf0, buf1, total;
};

LayoutC layout_c128(const MultiPlan &P) {
    LayoutC L;
    L.packed = 0;
    L.res = a256((size_t)P.n * P.m * 16);
    L.buf0 = L.res + 256;
    L.buf1 = L.buf0 + a256((size_t)P.max_layer * 16);
    L.total = L.buf1 + a256((size_t)P.max_layer * 16);
    return L;
}

int multi_c128_device(const MultiPlan &P, const void *a_dev, int64_t lda, void *result_dev, void *ws,
                      size_t ws_bytes, hipStream_t s) {
    const LayoutC Ly = layout_c128(P);
    if (!ws || ws_bytes < Ly.total)
        return set_error(PERM_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, Ly.total);
    const char *d_plan = nullptr;
    const int rc = device_plan(P, &d_plan);
    if (rc) return rc;
    char *base = (char *)ws;
    MHIP(launch_multi_pack_c128(a_dev, lda, P.n, P.m, base + Ly.packed, base + Ly.buf0, s), "pack kernel");
    char *prev = base + Ly.buf0, *next = base + Ly.buf1;
    const bool prof = profiling_on();
    for (int k = 2; k <= P.n; k++) {
        const MultiLayerArgs g = layer_args(P, d_plan, k);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (prof) {
            e0 = profile_event();
            e1 = profile_event();
            if (e0) (void)hipEventRecord(e0, s);
        }
        MHIP(launch_multi_layer_c128(prev, next, base + Ly.packed + (size_t)(k - 1) * P.m * 16, g, s),
             "repeated-column layer kernel");
        if (prof && e0 && e1) {
            (void)hipEventRecord(e1, s);
            profile_record(4, e0, e1);
        }
        std::swap(prev, next);
    }
    MHIP(launch_multi_readout_c128(prev, scale_c128(P), result_dev, s), "readout kernel");
    return PERM_OK;
}

// ------------------------------------------------------------- integer
// Primes for |G| <= |per| <= min(prod_i sum_j |a_ij| mult[j], n! max|a|^n).
int primes_needed_multi(const MultiPlan &P, const int64_t *a, int64_t lda) {
    double bits_rows = 0.0, bits_fact = 0.0;
    uint64_t mx = 0;
    for (int i = 0; i < P.n; i++) {
        u128m s = 0;
        for (int j = 0; j < P.m; j++) {
            const int64_t v = a[(int64_t)i * lda + j];
            const uint64_t mag = v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v;
            s += (u128m)mag * (uint64_t)P.mult[j];
            mx = std::max(mx, mag);
        }
        if (s == 0) return 1;
        bits_rows += std::log2((double)s);
    }
    if (mx == 0) return 1;
    for (int i = 2; i <= P.n; i++) bits_fact += std::log2((double)i);
    bits_fact += P.n * std::log2((double)mx);
    const double need = std::min(bits_rows, bits_fact) * (1.0 + 1e-12) + 2.0;
    const auto &ps = primes61();
    double have = 0.0;
    int r = 0;
    while (have <= need && r < PERM_MAX_PRIMES) have += std::log2((double)ps[r++]);
    return have > need ? r : PERM_MAX_PRIMES + 1;
}

struct LayoutI {
    size_t primes, res, red, bufs;
};

LayoutI layout_int(const MultiPlan &P) {
    LayoutI L;
    L.primes = 0;
    L.res = a256(PERM_MAX_PRIMES * 8);
    L.red = L.res + a256(PERM_MAX_PRIMES * 8);
    L.bufs = L.red + a256((size_t)PERM_MAX_PRIMES * P.n * P.m * 8);
    return L;
}

size_t int_bytes(const MultiPlan &P, int rp) { return layout_int(P).bufs + 2 * a256((size_t)rp * P.max_layer * 8); }

int multi_int(const MultiPlan &P, const int64_t *a, int64_t lda, perm_int_t *out, void *ws, size_t ws_bytes,
              hipStream_t s) {
    if (!ws || ws_bytes < int_bytes(P, 1))
        return set_error(PERM_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, int_bytes(P, 1));
    int rp = kRPMax;
    while (rp > 1 && int_bytes(P, rp) > ws_bytes) rp--;
    const int R = primes_needed_multi(P, a, lda);
    const int Rt = R + 1;
    if (Rt > PERM_MAX_PRIMES) return set_error(PERM_ERANGE, "needs more than %d primes", PERM_MAX_PRIMES - 1);
    const auto &ps = primes61();
    const size_t nm = (size_t)P.n * P.m;
    std::vector<uint64_t> red(Rt * nm);
    for (int r = 0; r < Rt; r++)
        for (int i = 0; i < P.n; i++)
            for (int j = 0; j < P.m; j++) {
                const int64_t v = a[(int64_t)i * lda + j];
                const uint64_t mag = v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v;
                uint64_t x = mag % ps[r];
                if (v < 0 && x != 0) x = ps[r] - x;
                red[r * nm + (size_t)i * P.m + j] = x;
            }
    const LayoutI Ly = layout_int(P);
    char *base = (char *)ws;
    uint64_t *d_primes = (uint64_t *)(base + Ly.primes), *d_res = (uint64_t *)(base + Ly.res);
    uint64_t *d_red = (uint64_t *)(base + Ly.red);
    const size_t plane = P.max_layer;
    uint64_t *buf0 = (uint64_t *)(base + Ly.bufs);
    uint64_t *buf1 = (uint64_t *)(base + Ly.bufs + a256((size_t)rp * plane * 8));
    MHIP(hipMemcpyAsync(d_primes, ps.data(), Rt * 8, hipMemcpyHostToDevice, s), "upload primes");
    MHIP(hipMemcpyAsync(d_red, red.data(), red.size() * 8, hipMemcpyHostToDevice, s), "upload residues");
    const char *d_plan = nullptr;
    const int rc = device_plan(P, &d_plan);
    if (rc) return rc;
    const bool prof = profiling_on();
    for (int s0 = 0; s0 < Rt; s0 += rp) {
        const int cnt = std::min(rp, Rt - s0);
        const uint64_t *gred = d_red + (size_t)s0 * nm;
        MHIP(launch_multi_init_modp(gred, P.n, P.m, cnt, buf0, plane, s), "init kernel");
        uint64_t *prev = buf0, *next = buf1;
        for (int k = 2; k <= P.n; k++) {
            const MultiLayerArgs g = layer_args(P, d_plan, k);
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (prof) {
                e0 = profile_event();
                e1 = profile_event();
                if (e0) (void)hipEventRecord(e0, s);
            }
            MHIP(launch_multi_layer_modp(prev, next, plane, gred, P.n, k, d_primes + s0, cnt, g, s),
                 "repeated-column modp layer kernel");
            if (prof && e0 && e1) {
                (void)hipEventRecord(e1, s);
                profile_record(5, e0, e1);
            }
            std::swap(prev, next);
        }
        MHIP(launch_readout_modp(prev, plane, cnt, d_res + s0, s), "readout kernel");
    }
    std::vector<uint64_t> res(Rt);
    MHIP(hipMemcpyAsync(res.data(), d_res, Rt * 8, hipMemcpyDeviceToHost, s), "download residues");
    MHIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    std::vector<uint64_t> scale;
    for (int j = 0; j < P.m; j++)
        for (int v = 2; v <= P.mult[j]; v++) scale.push_back((uint64_t)v);
    return crt_to_int(res.data(), ps.data(), R, out, &scale);
}

}  // namespace
}  // namespace permgpu

using namespace permgpu;

extern "C" {

size_t perm_multi_workspace_bytes(perm_dtype_t dt, int n, int m, const int32_t *mult) {
    if (dt != PERM_INT64 && dt != PERM_COMPLEX128) return 0;
    static const int64_t dummy = 0;
    const int v = validate(n, m, mult, &dummy, m);
    if (v < 0) return 0;
    if (v == 1) return perm_workspace_bytes(dt, n);
    std::shared_ptr<const MultiPlan> P;
    if (get_plan(n, m, mult, P)) return 0;
    return dt == PERM_COMPLEX128 ? layout_c128(*P).total : int_bytes(*P, kRPMax);
}

int perm_solve_multi(perm_dtype_t dt, int n, int m, const int32_t *mult, const void *a, int64_t lda, void *result,
                     void *workspace, size_t ws_bytes, void *stream) {
    if (dt != PERM_INT64 && dt != PERM_COMPLEX128) return set_error(PERM_EINVAL, "bad dtype");
    if (!result) return set_error(PERM_EINVAL, "null result");
    const int v = validate(n, m, mult, a, lda);
    if (v < 0) return v;
    if (v == 1) return perm_solve(dt, n, a, lda, result, workspace, ws_bytes, stream);
    std::shared_ptr<const MultiPlan> P;
    int rc = get_plan(n, m, mult, P);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (dt == PERM_INT64) return multi_int(*P, (const int64_t *)a, lda, (perm_int_t *)result, workspace, ws_bytes, s);
    const LayoutC Ly = layout_c128(*P);
    if (!workspace || ws_bytes < Ly.total)
        return set_error(PERM_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, Ly.total);
    char *base = (char *)workspace;
    MHIP(hipMemcpy2DAsync(base + Ly.packed, (size_t)m * 16, a, (size_t)lda * 16, (size_t)m * 16, n,
                          hipMemcpyHostToDevice, s),
         "upload matrix");
    rc = multi_c128_device(*P, base + Ly.packed, m, base + Ly.res, workspace, ws_bytes, s);
    if (rc) return rc;
    MHIP(hipMemcpyAsync(result, base + Ly.res, 16, hipMemcpyDeviceToHost, s), "download result");
    MHIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    return PERM_OK;
}

int perm_solve_multi_async(int n, int m, const int32_t *mult, const perm_c128_t *a_dev, int64_t lda,
                           perm_c128_t *result_dev, void *workspace, size_t ws_bytes, void *stream) {
    if (!result_dev) return set_error(PERM_EINVAL, "null result");
    const int v = validate(n, m, mult, a_dev, lda);
    if (v < 0) return v;
    if (v == 1) return perm_solve_async(n, a_dev, lda, result_dev, workspace, ws_bytes, stream);
    std::shared_ptr<const MultiPlan> P;
    const int rc = get_plan(n, m, mult, P);
    if (rc) return rc;
    return multi_c128_device(*P, a_dev, lda, result_dev, workspace, ws_bytes, (hipStream_t)stream);
}

int perm_multi_plan_info(int n, int m, const int32_t *mult, int check, perm_multi_plan_info_t *out) {
    if (!out) return set_error(PERM_EINVAL, "null pointer");
    std::memset(out, 0, sizeof *out);
    static const int64_t dummy = 0;
    const int v = validate(n, m, mult, &dummy, m);
    if (v < 0) return v;
    if (v == 1) {
        out->states = n < 64 ? (1ull << n) : 0;
        return PERM_OK;
    }
    MultiPlan P;
    int rc = build_plan(n, m, mult, P);
    if (rc) return rc;
    out->L = P.L;
    out->states = P.states;
    out->low_states = P.low_states;
    out->max_layer = P.max_layer;
    out->tiles = P.total_tiles;
    out->windows = P.total_wins;
    out->plan_bytes = P.blob.size() * 4;
    if (check) {
        uint64_t done = 0;
        rc = check_plan(P, &done);
        if (rc) return rc;
        out->checked = done;
    }
    return PERM_OK;
}

}  // extern "C"
