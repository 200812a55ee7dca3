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

constexpr uint32_t kLowWindow = 1024;        // largest low window wanted (entries)
constexpr uint64_t kHighMax = 1ull << 24;    // high parts at most (the list costs 4 B each)
constexpr uint64_t kPlanMax = 1ull << 30;    // plan bytes at most
constexpr uint64_t kSat = ~0ull;
constexpr uint32_t kNone = 0xffffffffu;

uint64_t sat_add(uint64_t a, uint64_t b) { return a > kSat - b ? kSat : a + b; }
uint64_t sat_mul(uint64_t a, uint64_t b) { return (b != 0 && a > kSat / b) ? kSat : a * b; }
size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

typedef unsigned __int128 u128m;

struct MultiPlan {
    int n = 0, m = 0, L = 0, SL = 0, SH = 0, tmax1 = 1;
    std::vector<int32_t> mult;
    uint64_t states = 0, low_states = 0, high_states = 0;
    std::vector<uint32_t> size;  // layer sizes, k = 0..n
    uint32_t max_layer = 0;
    std::vector<uint32_t> WL;    // low parts of sum s, s = 0..SL
    uint32_t max_window = 0;     // max WL
    std::vector<uint32_t> qoff;  // high parts with |h| = q start at qoff[q] in hlist
    // device image in 32-bit words; every section starts on 256 bytes
    std::vector<uint32_t> blob;
    size_t oG = 0, ohlist = 0, ohstride = 0, ohradix = 0, olp16 = 0, okpoff = 0, oWL = 0;
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

uint32_t max_of(const std::vector<uint64_t> &v, int upto) {
    uint64_t x = 0;
    for (int s = 0; s <= upto && s < (int)v.size(); s++) x = std::max(x, v[s]);
    return (uint32_t)std::min<uint64_t>(x, kNone);
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
    // the most low columns whose largest low window stays at kLowWindow
    // entries; more while the high parts exceed kHighMax (up to the LDS cap)
    int L = 1;
    while (L < m && max_of(W[L + 1], n) <= kLowWindow) L++;
    while (L < m && PH[L] > kHighMax && max_of(W[L + 1], n) <= (uint32_t)kMultiWinMax) L++;
    if (PH[L] > kHighMax || max_of(W[L], n) > (uint32_t)kMultiWinMax)
        return set_error(PERM_ERANGE, "repeated-column plan too large (%llu high parts)",
                         (unsigned long long)PH[L]);
    P.L = L;
    P.low_states = PL[L];
    P.high_states = PH[L];
    P.SL = 0;
    for (int j = 0; j < L; j++) P.SL += t[j];
    P.SH = n - P.SL;
    P.WL.assign(P.SL + 1, 0);
    for (int s = 0; s <= P.SL; s++) P.WL[s] = (uint32_t)W[L][s];
    P.max_window = max_of(W[L], n);
    const int mh = m - L;
    int tmax = 0;
    for (int j = L; j < m; j++) tmax = std::max(tmax, (int)t[j]);
    P.tmax1 = tmax + 1;

    std::vector<uint32_t> &b = P.blob;
    // G_j(P, c) = sum_{v < c} W_j(P - v) for the high columns
    P.oG = section(b);
    for (int j = L; j < m; j++)
        for (int p = 0; p <= n; p++)
            for (int c = 0; c <= tmax; c++) {
                uint64_t g = 0;
                for (int v = 0; v < c && v <= p; v++) g = sat_add(g, W[j][p - v]);
                b.push_back((uint32_t)std::min<uint64_t>(g, kNone));
            }
    // high parts sorted by |h| (counting sort), then index
    const uint32_t DH = (uint32_t)PH[L];
    std::vector<uint8_t> hs(DH);
    {
        std::vector<int> d(mh, 0);
        int q = 0, nz = 0;
        for (uint32_t x = 0; x < DH; x++) {
            hs[x] = (uint8_t)q;
            // tile h is in layers q..q+SL; one high window per nonzero digit
            const int k0 = std::max(2, q), k1 = std::min(n, q + P.SL);
            if (k1 >= k0) P.total_wins += (uint64_t)nz * (uint64_t)(k1 - k0 + 1);
            for (int j = 0; j < mh; j++) {
                if (d[j] < t[L + j]) {
                    if (d[j] == 0) nz++;
                    d[j]++;
                    q++;
                    break;
                }
                q -= d[j];
                nz--;
                d[j] = 0;
            }
        }
    }
    P.qoff.assign(P.SH + 2, 0);
    for (uint32_t x = 0; x < DH; x++) P.qoff[hs[x] + 1]++;
    for (int q = 0; q <= P.SH; q++) P.qoff[q + 1] += P.qoff[q];
    P.ohlist = section(b);
    b.resize(b.size() + DH);
    {
        std::vector<uint32_t> fill(P.qoff.begin(), P.qoff.end() - 1);
        for (uint32_t x = 0; x < DH; x++) b[P.ohlist + fill[hs[x]]++] = x;
    }
    P.ohstride = section(b);
    {
        uint32_t st = 1;
        for (int j = L; j < m; j++) {
            b.push_back(st);
            st *= (uint32_t)t[j] + 1;
        }
    }
    P.ohradix = section(b);
    for (int j = L; j < m; j++) b.push_back((uint32_t)t[j] + 1);

    // low parts: colex order inside each sum is increasing mixed-radix index
    const uint32_t DL = (uint32_t)PL[L];
    std::vector<uint32_t> cnt(P.SL + 1, 0), rankL(DL);
    std::vector<uint8_t> sumL(DL);
    std::vector<std::vector<uint32_t>> bysum(P.SL + 1);
    {
        std::vector<int> d(L, 0);
        int sum = 0;
        for (uint32_t v = 0; v < DL; v++) {
            sumL[v] = (uint8_t)sum;
            rankL[v] = cnt[sum]++;
            bysum[sum].push_back(v);
            for (int i = 0; i < L; i++) {
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
    std::vector<uint16_t> lp;
    std::vector<uint32_t> kpoff(P.SL + 2, 0);
    for (int kp = 0; kp <= P.SL; kp++) {
        kpoff[kp] = (uint32_t)lp.size();
        const auto &vs = bysum[kp];
        const size_t base = lp.size();
        lp.resize(base + (size_t)L * vs.size(), 0xffff);
        for (size_t r = 0; r < vs.size(); r++) {
            uint32_t v = vs[r];
            for (int i = 0; i < L; i++) {
                const uint32_t digit = (v / (uint32_t)PL[i]) % ((uint32_t)t[i] + 1);
                if (digit > 0) lp[base + (size_t)i * vs.size() + r] = (uint16_t)rankL[v - (uint32_t)PL[i]];
            }
        }
    }
    kpoff[P.SL + 1] = (uint32_t)lp.size();
    if (lp.size() & 1) lp.push_back(0xffff);
    P.olp16 = section(b);
    {
        const size_t w0 = b.size();
        b.resize(w0 + lp.size() / 2);
        std::memcpy(b.data() + w0, lp.data(), lp.size() * 2);
    }
    P.okpoff = section(b);
    b.insert(b.end(), kpoff.begin(), kpoff.end());
    P.oWL = section(b);
    b.insert(b.end(), P.WL.begin(), P.WL.end());
    section(b);
    for (int k = 2; k <= n; k++) {
        const int qlo = std::max(0, k - P.SL), qhi = std::min(k, P.SH);
        if (qlo <= qhi) P.total_tiles += P.qoff[qhi + 1] - P.qoff[qlo];
    }
    if ((uint64_t)b.size() * 4 > kPlanMax)
        return set_error(PERM_ERANGE, "repeated-column plan above %llu bytes", (unsigned long long)kPlanMax);
    return PERM_OK;
}

// Launch arguments of layer k.  The runs of |h| groups at either end of the
// layer whose tiles have at most kMultiThin outputs (WL[k - |h|]) are its
// thin tiles.
MultiLayerArgs layer_args(const MultiPlan &P, const char *d_blob, int k) {
    MultiLayerArgs g;
    const uint32_t *w = (const uint32_t *)d_blob;
    g.G = w + P.oG;
    g.hlist = w + P.ohlist;
    g.hstride = w + P.ohstride;
    g.hradix = w + P.ohradix;
    g.lp16 = (const uint16_t *)(w + P.olp16);
    g.kpoff = w + P.okpoff;
    g.WL = w + P.oWL;
    const int qlo = std::max(0, k - P.SL), qhi = std::min(k, P.SH);
    g.tile0 = P.qoff[qlo];
    g.ntiles = qlo <= qhi ? P.qoff[qhi + 1] - P.qoff[qlo] : 0;
    g.thin_lo = 0;
    g.thin_hi = g.ntiles;
    if (qlo <= qhi) {
        int a = qlo, b = qhi;
        while (a <= qhi && P.WL[k - a] <= (uint32_t)kMultiThin) a++;
        while (b >= a && P.WL[k - b] <= (uint32_t)kMultiThin) b--;
        g.thin_lo = P.qoff[a] - g.tile0;
        g.thin_hi = P.qoff[b + 1] - g.tile0;
    }
    g.thin_wg = (g.thin_lo + (g.ntiles - g.thin_hi) + kMultiBlock / 64 - 1) / (kMultiBlock / 64);
    g.n = P.n;
    g.m = P.m;
    g.L = P.L;
    g.SL = P.SL;
    g.k = k;
    g.tmax1 = P.tmax1;
    return g;
}

// ---------------------------------------------------------- plan checker
// Closed-form colex rank / unrank of count vectors, written from the
// definition of the order (independent of the tables), against what a tile
// of the plan yields: the host mirror of the device's tile decoding below
// and the 16-bit rank table.
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

struct HostTile {
    uint32_t base_out, kp, low_base;
    std::vector<uint32_t> wbase, wcol;
};

// The device's multi_tile, step for step, on the host.
HostTile host_tile(const MultiPlan &P, int k, uint32_t x) {
    const uint32_t *B = P.blob.data();
    const int mh = P.m - P.L;
    std::vector<uint32_t> h(mh), a(mh), bb(mh), c(mh);
    int q = 0;
    for (int j = 0; j < mh; j++) {
        h[j] = (x / B[P.ohstride + j]) % B[P.ohradix + j];
        q += (int)h[j];
    }
    const int kp = k - q;
    int Pj = kp;
    for (int j = 0; j < mh; j++) {
        Pj += (int)h[j];
        const uint32_t *Gj = B + P.oG + (size_t)j * (P.n + 1) * P.tmax1;
        a[j] = Gj[(size_t)Pj * P.tmax1 + h[j]];
        bb[j] = Pj >= 1 ? Gj[(size_t)(Pj - 1) * P.tmax1 + h[j]] : 0u;
        c[j] = h[j] > 0 ? Gj[(size_t)(Pj - 1) * P.tmax1 + h[j] - 1] : 0u;
    }
    HostTile T;
    uint32_t tot_a = 0, tot_b = 0, pa = 0, pb = 0;
    for (int j = 0; j < mh; j++) {
        tot_a += a[j];
        tot_b += bb[j];
    }
    for (int j = 0; j < mh; j++) {
        pa += a[j];
        pb += bb[j];
        if (h[j] > 0) {
            T.wbase.push_back((pa - a[j]) + c[j] + (tot_b - pb));
            T.wcol.push_back((uint32_t)(P.L + j));
        }
    }
    T.base_out = tot_a;
    T.kp = (uint32_t)kp;
    T.low_base = tot_b;
    return T;
}

int check_plan(const MultiPlan &P, uint64_t *checked) {
    Ranker rk{P.n, P.m, P.mult.data(), prefix_counts(P.n, P.m, P.mult.data())};
    uint64_t all = 0;
    for (int k = 2; k <= P.n; k++) all += P.size[k];
    const bool full = all <= (1ull << 22);
    const uint32_t *B = P.blob.data();
    const uint16_t *lp = (const uint16_t *)(B + P.olp16);
    const uint32_t *kpoff = B + P.okpoff;
    std::vector<int> c(P.m), e(P.m);
    uint64_t done = 0;
    for (int k = 2; k <= P.n; k++) {
        const MultiLayerArgs g = layer_args(P, (const char *)B, k);
        if (g.thin_lo > g.thin_hi || g.thin_hi > g.ntiles)
            return set_error(PERM_EDEVICE, "plan check: layer %d thin split %u..%u of %u tiles", k, g.thin_lo,
                             g.thin_hi, g.ntiles);
        // the tiles of a layer cover its ranks exactly once
        uint64_t covered = 0;
        const uint32_t tstep = (full || g.ntiles <= 512) ? 1 : g.ntiles / 512;
        for (uint32_t bi = 0; bi < g.ntiles; bi++) {
            const HostTile T = host_tile(P, k, B[P.ohlist + g.tile0 + bi]);
            if ((int)T.kp < 0 || (int)T.kp > P.SL)
                return set_error(PERM_EDEVICE, "plan check: layer %d tile %u low sum %d", k, bi, (int)T.kp);
            const uint32_t nout = P.WL[T.kp];
            if ((bi < g.thin_lo || bi >= g.thin_hi) && nout > (uint32_t)kMultiThin)
                return set_error(PERM_EDEVICE, "plan check: layer %d thin tile %u has %u outputs", k, bi, nout);
            covered += nout;
            if (bi % tstep != 0 && bi + 1 != g.ntiles) continue;
            if ((uint64_t)T.base_out + nout > P.size[k])
                return set_error(PERM_EDEVICE, "plan check: layer %d tile %u beyond the layer", k, bi);
            const uint32_t rstep = (full || nout <= 64) ? 1 : nout / 64;
            for (uint32_t r = 0; r < nout; r = (r + rstep < nout || r + 1 == nout) ? r + rstep : nout - 1) {
                const uint64_t rank = (uint64_t)T.base_out + r;
                rk.unrank(k, rank, c);
                int sl = 0;
                for (int i = 0; i < P.L; i++) sl += c[i];
                if ((uint32_t)sl != T.kp)
                    return set_error(PERM_EDEVICE, "plan check: layer %d rank %llu is not in tile %u", k,
                                     (unsigned long long)rank, bi);
                size_t w = 0;
                for (int j = 0; j < P.m; j++) {
                    uint64_t got;
                    if (j < P.L) {
                        const uint32_t q16 = lp[kpoff[T.kp] + (size_t)j * nout + r];
                        if (c[j] == 0) {
                            if (q16 != 0xffff)
                                return set_error(PERM_EDEVICE, "plan check: layer %d rank %llu spurious low %d", k,
                                                 (unsigned long long)rank, j);
                            continue;
                        }
                        if (q16 == 0xffff || T.kp == 0 || q16 >= P.WL[T.kp - 1])
                            return set_error(PERM_EDEVICE, "plan check: layer %d rank %llu low %d", k,
                                             (unsigned long long)rank, j);
                        got = (uint64_t)T.low_base + q16;
                    } else {
                        if (c[j] == 0) continue;
                        if (w >= T.wcol.size() || T.wcol[w] != (uint32_t)j)
                            return set_error(PERM_EDEVICE, "plan check: layer %d rank %llu window of column %d", k,
                                             (unsigned long long)rank, j);
                        got = (uint64_t)T.wbase[w] + r;
                        w++;
                    }
                    e = c;
                    e[j]--;
                    const uint64_t want = rk.rank(e);
                    if (got != want || want >= P.size[k - 1])
                        return set_error(PERM_EDEVICE, "plan check: layer %d rank %llu column %d: %llu != %llu", k,
                                         (unsigned long long)rank, j, (unsigned long long)got,
                                         (unsigned long long)want);
                }
                if (w != T.wcol.size())
                    return set_error(PERM_EDEVICE, "plan check: layer %d rank %llu extra windows", k,
                                     (unsigned long long)rank);
                done++;
                if (r + 1 == nout) break;
            }
        }
        if (covered != P.size[k])
            return set_error(PERM_EDEVICE, "plan check: layer %d tiles cover %llu of %u ranks", k,
                             (unsigned long long)covered, P.size[k]);
    }
    *checked = done;
    return PERM_OK;
}

// ------------------------------------------------------------ plan cache
// Host plans by multiplicity vector, each with its device copies; at most
// kPlanCache plans and kDevPlanBytes of device copies, the oldest unused
// dropped first.
std::mutex g_plan_mu;
std::map<std::vector<int32_t>, std::shared_ptr<const MultiPlan>> g_plans;
std::deque<std::vector<int32_t>> g_plan_order;
size_t g_dev_plan_bytes = 0;
constexpr size_t kPlanCache = 16;
constexpr size_t kDevPlanBytes = (size_t)2 << 30;

// Drops the least recently built plan that no call is using (only the cache
// holds it: a call keeps its plan for its whole duration, so no launch can
// be issued with tables freed here) and that is not `keep`.  Returns false
// when every plan is in use.
bool drop_one_locked(const MultiPlan *keep) {
    for (auto o = g_plan_order.begin(); o != g_plan_order.end(); ++o) {
        auto it = g_plans.find(*o);
        if (it == g_plans.end() || it->second.get() == keep || it->second.use_count() > 1) continue;
        if (!it->second->dev.empty()) {
            // launches already queued on some stream may still read the tables
            (void)hipDeviceSynchronize();
            for (auto &d : it->second->dev) {
                (void)hipFree(d.second);
                g_dev_plan_bytes -= it->second->blob.size() * 4;
            }
            it->second->dev.clear();
        }
        g_plans.erase(it);
        g_plan_order.erase(o);
        return true;
    }
    return false;
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
    while (g_plans.size() >= kPlanCache && drop_one_locked(nullptr)) {
    }
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
    while (g_dev_plan_bytes + bytes > kDevPlanBytes && drop_one_locked(&P)) {
    }
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
        MHIP(launch_multi_layer_c128(prev, next, base + Ly.packed + (size_t)(k - 1) * P.m * 16, g, P.max_window, s),
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

// Layers 1..K whose stored values lie in [-(2^63 - 1), 2^63 - 1]: G(c) has
// one term per distinct column of c, so with R_i = sum_j |a_ij| and
// M_i = max_j |a_ij| over the m columns, |G(c)| for |c| = k is at most
// min(R_{k-1}, min(k, m) M_{k-1}) times the bound of layer k - 1.  Those
// layers run in plain 64-bit arithmetic (sums mod 2^64 recover a value in
// that range exactly).
int plain_int64_layers_multi(const MultiPlan &P, const int64_t *a, int64_t lda) {
    const u128m lim = ((u128m)1 << 63) - 1;
    u128m B = 1;
    int K = 0;
    for (int k = 1; k <= P.n; k++) {
        u128m R = 0, M = 0;
        for (int j = 0; j < P.m; j++) {
            const int64_t v = a[(int64_t)(k - 1) * lda + j];
            const u128m x = v < 0 ? (u128m)((uint64_t)0 - (uint64_t)v) : (u128m)v;
            R += x;
            if (x > M) M = x;
        }
        const u128m f = std::min(R, (u128m)std::min(k, P.m) * M);
        if (f != 0 && B > lim / f) break;
        B *= f;
        K = k;
    }
    return K;
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
    // layers 2..K in plain 64-bit arithmetic ("prime" 0, entries as they are,
    // block Rt of red), then residues
    const int K = Rt < PERM_MAX_PRIMES ? plain_int64_layers_multi(P, a, lda) : 0;
    std::vector<uint64_t> red((Rt + 1) * nm);
    for (int i = 0; i < P.n; i++)
        for (int j = 0; j < P.m; j++) red[Rt * nm + (size_t)i * P.m + j] = (uint64_t)a[(int64_t)i * lda + j];
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
    std::vector<uint64_t> up(ps.begin(), ps.begin() + Rt);
    up.push_back(0);
    const size_t nup = K >= 2 ? up.size() : (size_t)Rt;
    MHIP(hipMemcpyAsync(d_primes, up.data(), nup * 8, hipMemcpyHostToDevice, s), "upload primes");
    MHIP(hipMemcpyAsync(d_red, red.data(), (K >= 2 ? red.size() : Rt * nm) * 8, hipMemcpyHostToDevice, s),
         "upload residues");
    const char *d_plan = nullptr;
    const int rc = device_plan(P, &d_plan);
    if (rc) return rc;
    const bool prof = profiling_on();
    auto layer = [&](const uint64_t *prev, uint64_t *next, int k, const uint64_t *gred, const uint64_t *primes,
                     int cnt) -> int {
        const MultiLayerArgs g = layer_args(P, d_plan, k);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (prof) {
            e0 = profile_event();
            e1 = profile_event();
            if (e0) (void)hipEventRecord(e0, s);
        }
        MHIP(launch_multi_layer_modp(prev, next, plane, gred, primes, cnt, g, P.max_window, s),
             "repeated-column modp layer kernel");
        if (prof && e0 && e1) {
            (void)hipEventRecord(e1, s);
            profile_record(5, e0, e1);
        }
        return PERM_OK;
    };
    for (int s0 = 0; s0 < Rt; s0 += rp) {
        const int cnt = std::min(rp, Rt - s0);
        const uint64_t *gred = d_red + (size_t)s0 * nm;
        uint64_t *prev = buf0, *next = buf1;
        int k0 = 2;
        if (K >= 2) {
            const uint64_t *pred = d_red + (size_t)Rt * nm, *pzero = d_primes + Rt;
            MHIP(launch_multi_init_modp(pred, P.n, P.m, 1, prev, plane, s), "init kernel");
            for (int k = 2; k <= K; k++) {
                const int lrc = layer(prev, next, k, pred, pzero, 1);
                if (lrc) return lrc;
                std::swap(prev, next);
            }
            MHIP(launch_int64_to_modp(prev, next, plane, P.size[K], d_primes + s0, cnt, s),
                 "int64 to residues kernel");
            std::swap(prev, next);
            k0 = K + 1;
        } else {
            MHIP(launch_multi_init_modp(gred, P.n, P.m, cnt, prev, plane, s), "init kernel");
        }
        for (int k = k0; k <= P.n; k++) {
            const int lrc = layer(prev, next, k, gred, d_primes + s0, cnt);
            if (lrc) return lrc;
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

// Repeated rows and columns: per(A) = per(A^T) (property 1 of section 3.1),
// so one side is expanded and the other compressed into count vectors.  The
// side compressed is the one with fewer count vectors, prod(mult + 1) (exact
// 128-bit products: at most 2^64 each); ties compress the columns.
extern "C++" {
namespace {

struct Bunched {
    bool rows;                  // compress the rows (expand the columns of A^T)
    int n, m;                   // expanded rows, compressed columns
    const int32_t *mult;        // multiplicities of the compressed side
};

int bunched_shape(int r, const int32_t *row_mult, int c, const int32_t *col_mult, Bunched *b) {
    if (r < 0 || c < 0 || (r > 0 && !row_mult) || (c > 0 && !col_mult))
        return set_error(PERM_EINVAL, "bad multiplicity arrays");
    int64_t nr = 0, nc = 0;
    unsigned __int128 pr = 1, pc = 1;
    for (int i = 0; i < r; i++) {
        if (row_mult[i] < 1) return set_error(PERM_EINVAL, "row_mult[%d] = %d < 1", i, row_mult[i]);
        nr += row_mult[i];
        if (nr > PERM_MULTI_N_MAX) return set_error(PERM_ERANGE, "n > %d", PERM_MULTI_N_MAX);
        pr *= (unsigned)(row_mult[i] + 1);
    }
    for (int j = 0; j < c; j++) {
        if (col_mult[j] < 1) return set_error(PERM_EINVAL, "col_mult[%d] = %d < 1", j, col_mult[j]);
        nc += col_mult[j];
        if (nc > PERM_MULTI_N_MAX) return set_error(PERM_ERANGE, "n > %d", PERM_MULTI_N_MAX);
        pc *= (unsigned)(col_mult[j] + 1);
    }
    if (nr != nc)
        return set_error(PERM_EINVAL, "row multiplicities sum to %lld, column multiplicities to %lld", (long long)nr,
                         (long long)nc);
    b->rows = pr < pc;
    b->n = (int)nr;
    b->m = b->rows ? r : c;
    b->mult = b->rows ? row_mult : col_mult;
    return PERM_OK;
}

// The expanded n x m matrix (row-major, lda = m) of one orientation.
template <typename T>
std::vector<T> bunched_expand(const Bunched &b, int r, const int32_t *row_mult, int c, const int32_t *col_mult,
                              const T *a, int64_t lda) {
    std::vector<T> e((size_t)b.n * b.m);
    size_t i2 = 0;
    if (!b.rows) {  // rows of A repeated, columns compressed
        for (int i = 0; i < r; i++)
            for (int u = 0; u < row_mult[i]; u++, i2++)
                for (int j = 0; j < c; j++) e[i2 * b.m + j] = a[(int64_t)i * lda + j];
    } else {  // columns of A become repeated rows of A^T, rows compressed
        for (int j = 0; j < c; j++)
            for (int u = 0; u < col_mult[j]; u++, i2++)
                for (int i = 0; i < r; i++) e[i2 * b.m + i] = a[(int64_t)i * lda + j];
    }
    return e;
}

}  // namespace
}  // extern "C++"

size_t perm_bunched_workspace_bytes(perm_dtype_t dt, int r, const int32_t *row_mult, int c, const int32_t *col_mult) {
    Bunched b;
    if (bunched_shape(r, row_mult, c, col_mult, &b) != PERM_OK) return 0;
    return perm_multi_workspace_bytes(dt, b.n, b.m, b.mult);
}

int perm_bunched_orientation(int r, const int32_t *row_mult, int c, const int32_t *col_mult, int *rows) {
    if (!rows) return set_error(PERM_EINVAL, "null pointer");
    Bunched b;
    const int rc = bunched_shape(r, row_mult, c, col_mult, &b);
    if (rc) return rc;
    *rows = b.rows ? 1 : 0;
    return PERM_OK;
}

int perm_solve_bunched(perm_dtype_t dt, int r, const int32_t *row_mult, int c, const int32_t *col_mult, const void *a,
                       int64_t lda, void *result, void *workspace, size_t ws_bytes, void *stream) {
    try {
        if (dt != PERM_INT64 && dt != PERM_COMPLEX128) return set_error(PERM_EINVAL, "bad dtype");
        if (!result || (r > 0 && c > 0 && !a)) return set_error(PERM_EINVAL, "null pointer");
        if (r > 0 && lda < c) return set_error(PERM_EINVAL, "lda = %lld < c = %d", (long long)lda, c);
        Bunched b;
        const int rc = bunched_shape(r, row_mult, c, col_mult, &b);
        if (rc) return rc;
        if (dt == PERM_INT64) {
            const auto e = bunched_expand(b, r, row_mult, c, col_mult, (const int64_t *)a, lda);
            return perm_solve_multi(dt, b.n, b.m, b.mult, e.data(), b.m > 0 ? b.m : 1, result, workspace, ws_bytes,
                                    stream);
        }
        const auto e = bunched_expand(b, r, row_mult, c, col_mult, (const perm_c128_t *)a, lda);
        return perm_solve_multi(dt, b.n, b.m, b.mult, e.data(), b.m > 0 ? b.m : 1, result, workspace, ws_bytes,
                                stream);
    } catch (const std::exception &ex) {
        return set_error(PERM_EDEVICE, "internal error: %s", ex.what());
    }
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

int perm_probe_fp64(double *tflops, void *stream) {
    if (!tflops) return set_error(PERM_EINVAL, "null pointer");
    hipStream_t s = (hipStream_t)stream;
    int dev = 0, cus = 0;
    MHIP(hipGetDevice(&dev), "hipGetDevice");
    MHIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "hipDeviceGetAttribute");
    const int blocks = std::max(1, cus) * 16, iters = 1 << 13;  // about 2 ms per launch
    double *d_out = nullptr;
    MHIP(hipMalloc(&d_out, (size_t)blocks * sizeof(double)), "hipMalloc (probe)");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float ms = 0.f;
    if (e == hipSuccess) e = launch_probe_fma(d_out, blocks, iters, s);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < 5 && e == hipSuccess; r++) e = launch_probe_fma(d_out, blocks, iters, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(d_out);
    if (e != hipSuccess) return hip_error(e, "FP64 probe");
    *tflops = 5.0 * probe_fma_flops(blocks, iters) / (ms * 1e-3) / 1e12;
    return PERM_OK;
}

int perm_probe_int(double *mac_fold_gops, double *add64_gops, void *stream) {
    if (!mac_fold_gops || !add64_gops) return set_error(PERM_EINVAL, "null pointer");
    hipStream_t s = (hipStream_t)stream;
    int dev = 0, cus = 0;
    MHIP(hipGetDevice(&dev), "hipGetDevice");
    MHIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "hipDeviceGetAttribute");
    const int blocks = std::max(1, cus) * 16;
    uint64_t *d_out = nullptr;
    MHIP(hipMalloc(&d_out, (size_t)blocks * sizeof(uint64_t)), "hipMalloc (probe)");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    double rate[2] = {0.0, 0.0};
    for (int mode = 0; mode < 2 && e == hipSuccess; mode++) {
        const int iters = mode == 0 ? (1 << 8) : (1 << 11);  // a few ms per launch
        float ms = 0.f;
        e = launch_probe_int(d_out, blocks, iters, mode, s);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int r = 0; r < 5 && e == hipSuccess; r++) e = launch_probe_int(d_out, blocks, iters, mode, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess) rate[mode] = 5.0 * probe_int_terms(blocks, iters) / (ms * 1e-3) / 1e9;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(d_out);
    if (e != hipSuccess) return hip_error(e, "integer probe");
    *mac_fold_gops = rate[0];
    *add64_gops = rate[1];
    return PERM_OK;
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
