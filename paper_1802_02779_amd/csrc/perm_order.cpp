// Cache-aware tile order of the layer sweep (host side).
//
// A tile of layer k fixes its high part T (m of the nh = n - t high columns)
// and reads the m high windows "T without one column" of layer k-1 (section 4
// of the paper: every stored value F(S) needs F(S \ {j}) for each j in S).
// A window is read by every tile that adds one column to it, so it is fetched
// from HBM once only if those tiles run on one XCD while it is still in that
// XCD's 4 MB L2.  In colexicographic order the tiles that add a low column
// run together but those that add a higher column are spread over the whole
// layer.
//
// This order processes the tiles in families: a family is every not yet
// processed m-subset of one z-set Z of high columns, and the next Z is the one
// with the most unprocessed m-subsets (ties: lowest colex rank).  A family's
// windows are the (m-1)-subsets of Z, each read by up to z - m + 1 of its
// tiles; z is the largest for which C(z, m-1) windows stay within a fixed byte
// budget.  The families are then taken in the colex order of their z-sets
// (so that the eight XCDs work on neighbouring families at any time and share
// the 256 MB MALL) and go whole to the XCD with the fewest tiles so far; the
// per-XCD lists are then evened out to floor or ceil of the group's tiles / 8
// (a few tiles of the longest lists move to the shortest) and interleaved
// so that workgroup b, which the hardware dispatches to XCD b % 8, takes the
// (b / 8)-th tile of that XCD's list.
// Each k' group is padded to a multiple of 8 workgroups with empty slots.
// Where no z fits (m = 0, or m + 2 > nh - 1) the tiles keep colex order in
// runs of `chunk` per XCD, as the unordered sweep does.
#include "perm_host.h"

#include <algorithm>
#include <array>
#include <atomic>
#include <map>
#include <mutex>
#include <queue>
#include <thread>
#include <tuple>

#define OHIP(expr, what)                                  \
    do {                                                  \
        hipError_t _e = (expr);                           \
        if (_e != hipSuccess) return hip_error(_e, what); \
    } while (0)

namespace permgpu {

namespace {

constexpr double kFamilyBytes = 16.0 * 1024 * 1024;  // window bytes of one family

uint32_t colex_unrank(uint32_t r, int z, int nh) {
    uint32_t mask = 0;
    int c = nh - 1;
    for (int i = z; i >= 1; i--) {
        while (binom_host(c, i) > r) c--;
        r -= binom_host(c, i);
        mask |= 1u << c;
        c--;
    }
    return mask;
}

// next mask with the same popcount (Gosper)
uint32_t next_same_pop(uint32_t v) {
    const uint32_t c = v & (0u - v), r = v + c;
    return (((r ^ v) >> 2) / c) | r;
}

// bits of `local` (below 2^cnt) placed on the columns cols[0..cnt-1]
uint32_t deposit(uint32_t local, const int *cols) {
    uint32_t m = 0;
    while (local) {
        m |= 1u << cols[__builtin_ctz(local)];
        local &= local - 1;
    }
    return m;
}

// Decrements cnt[rank(Z)] for every z-subset Z of [0, nh) that contains T,
// walking the columns upwards with the colex rank accumulated on the way
// (column c as the (i+1)-th element of Z adds C(c, i + 1)).
struct SupersetWalk {
    uint32_t T;
    int nh, z;
    int32_t *cnt;
    int free_above[33];  // columns not in T at or above c
    void init() {
        free_above[nh] = 0;
        for (int c = nh - 1; c >= 0; c--) free_above[c] = free_above[c + 1] + !(T >> c & 1);
    }
    void walk(int c, int idx, uint32_t rank, int need) {
        if (c == nh) {
            cnt[rank]--;
            return;
        }
        const uint32_t add = kBinom.v[c][idx + 1];  // c < nh <= 18, idx < z <= 17
        if (T >> c & 1) {
            walk(c + 1, idx + 1, rank + add, need);
            return;
        }
        if (need > 0) walk(c + 1, idx + 1, rank + add, need - 1);
        if (free_above[c + 1] >= need) walk(c + 1, idx, rank, need);
    }
};

// Per-XCD tile lists of one group (m-subsets of [0, nh)).
void group_lists(int nh, int m, int z, int chunk, std::array<std::vector<uint32_t>, 8> &per) {
    const uint32_t cnt = binom_host(nh, m);
    if (z == 0) {
        const uint32_t C = chunk > 0 ? (uint32_t)chunk : 1u;
        uint32_t mask = (1u << m) - 1u;
        for (uint32_t i = 0; i < cnt; i++) {
            per[(i / C) % 8].push_back(mask);
            if (m > 0) mask = next_same_pop(mask);
        }
        return;
    }
    const uint32_t nz = binom_host(nh, z);
    std::vector<int32_t> newc(nz, (int32_t)binom_host(z, m));
    using E = std::pair<int32_t, uint32_t>;  // (unprocessed tiles, ~rank): ties go to the lowest rank
    std::priority_queue<E> pq;
    for (uint32_t r = 0; r < nz; r++) pq.push({newc[r], ~r});
    std::vector<uint8_t> done((size_t)1 << nh, 0);
    std::vector<std::pair<uint32_t, std::vector<uint32_t>>> fams;
    uint32_t left = cnt;
    int zc[32];
    while (left && !pq.empty()) {
        const E e = pq.top();
        pq.pop();
        const uint32_t r = ~e.second;
        if (e.first != newc[r]) {
            if (newc[r] > 0) pq.push({newc[r], e.second});
            continue;
        }
        if (e.first <= 0) continue;
        const uint32_t Z = colex_unrank(r, z, nh);
        fams.push_back({r, {}});
        for (int i = 0, b = (int)Z; b; i++) {
            zc[i] = __builtin_ctz((uint32_t)b);
            b &= b - 1;
        }
        const uint32_t lend = 1u << z;
        for (uint32_t l = (1u << m) - 1u; l < lend; l = next_same_pop(l)) {
            const uint32_t T = deposit(l, zc);
            if (done[T]) continue;
            done[T] = 1;
            fams.back().second.push_back(T);
            left--;
            // every z-superset of T has one unprocessed subset less
            SupersetWalk w{T, nh, z, newc.data(), {}};
            w.init();
            w.walk(0, 0, 0u, z - m);
        }
    }
    std::stable_sort(fams.begin(), fams.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
    std::array<uint32_t, 8> load{};
    for (size_t f = 0; f < fams.size(); f++) {
        int x = 0;
        for (int i = 1; i < 8; i++)
            if (load[i] < load[x]) x = i;
        for (uint32_t T : fams[f].second) per[x].push_back(T);
        load[x] += fams[f].second.size();
    }
}

// Appends the interleaved, padded list of one group to `out`.
void append_group(int nh, int m, int z, int chunk, std::vector<uint32_t> &out) {
    std::array<std::vector<uint32_t>, 8> per;
    group_lists(nh, m, z, chunk, per);
    // even out: the c % 8 longest lists keep floor(c / 8) + 1 tiles, the
    // others floor(c / 8); surplus tails move to the lists that are short
    const size_t c = binom_host(nh, m), lo = c / 8, L = (c + 7) / 8;
    std::array<int, 8> rank{};
    for (int x = 0; x < 8; x++) rank[x] = x;
    std::stable_sort(rank.begin(), rank.end(), [&](int a, int b) { return per[a].size() > per[b].size(); });
    std::array<size_t, 8> target{};
    for (int i = 0; i < 8; i++) target[rank[i]] = lo + ((size_t)i < c % 8 ? 1 : 0);
    std::vector<uint32_t> spill;
    for (int x = 0; x < 8; x++)
        while (per[x].size() > target[x]) {
            spill.push_back(per[x].back());
            per[x].pop_back();
        }
    for (int x = 0; x < 8; x++)
        while (per[x].size() < target[x] && !spill.empty()) {
            per[x].push_back(spill.back());
            spill.pop_back();
        }
    for (size_t i = 0; i < L; i++)
        for (int x = 0; x < 8; x++) out.push_back(i < per[x].size() ? per[x][i] : kNoTile);
}

// The padded lists of every tiled group of layers k0..k1 of (n, t), in
// layer then group order; lists[i] belongs to groups[i] = (k, g).  Groups
// with the same (m, z) share one list, built once; distinct lists are built
// on up to 16 host threads.
struct LayerLists {
    std::vector<std::pair<int, int>> groups;
    std::vector<const std::vector<uint32_t> *> lists;
    std::vector<uint32_t> slots;  // planned slots of each group
    std::vector<std::vector<uint32_t>> store;
};

bool build_lists(int n, int t, uint32_t thin, int chunk, int value_bytes, int k0, int k1, LayerLists &out) {
    const int nh = n - t;
    std::map<std::pair<int, int>, size_t> uniq;
    std::vector<std::pair<int, int>> jobs;  // (m, z)
    std::vector<size_t> job_of;
    for (int k = k0; k <= k1; k++) {
        LayerArgs b;
        plan_layer(n, k, t, chunk, 0, thin, &b, true);
        for (int g = 0; g < b.ngroups; g++) {
            const int m = k - b.kp[g];
            const auto key = std::make_pair(m, order_z(nh, m, b.ck[g], value_bytes));
            auto it = uniq.find(key);
            if (it == uniq.end()) {
                it = uniq.emplace(key, jobs.size()).first;
                jobs.push_back(key);
            }
            out.groups.push_back({k, g});
            out.slots.push_back(b.start[g + 1] - b.start[g]);
            job_of.push_back(it->second);
        }
    }
    out.store.assign(jobs.size(), {});
    std::atomic<size_t> next{0};
    std::atomic<bool> failed{false};
    auto worker = [&]() {
        try {
            for (size_t i; (i = next++) < jobs.size();)
                append_group(nh, jobs[i].first, jobs[i].second, chunk, out.store[i]);
        } catch (...) {
            failed = true;
        }
    };
    const unsigned hw = std::thread::hardware_concurrency();
    const size_t nth = std::min<size_t>(jobs.size(), std::max(1u, std::min(16u, hw)));
    std::vector<std::thread> th;
    for (size_t i = 1; i < nth; i++) th.emplace_back(worker);
    worker();
    for (auto &x : th) x.join();
    if (failed) return false;
    for (size_t i = 0; i < job_of.size(); i++) out.lists.push_back(&out.store[job_of[i]]);
    return true;
}

struct OrderPlan {
    uint32_t *dev = nullptr;
    std::vector<std::array<uint32_t, kMaxGroups>> off;  // off[k][g]
};

std::mutex g_order_mu;
std::map<std::tuple<int, int, int, uint32_t, int, int>, OrderPlan> g_order_plans;

}  // namespace

int order_z(int nh, int m, uint32_t ck, int value_bytes) {
    if (m < 1 || nh > kOrderNhMax) return 0;
    const double w = (double)ck * value_bytes;
    int z = 0;
    for (int c = m + 2; c <= nh - 1; c++)
        if ((double)binom_host(c, m - 1) * w <= kFamilyBytes) z = c;
    return z;
}

bool tile_order_layer(int n, int k, int t, uint32_t thin, int chunk, int value_bytes, std::vector<uint32_t> &out) {
    LayerLists L;
    if (!build_lists(n, t, thin, chunk, value_bytes, k, k, L)) return false;
    for (const auto *v : L.lists) out.insert(out.end(), v->begin(), v->end());
    return true;
}

int apply_tile_order(int n, int k, int t, uint32_t thin, int chunk, int value_bytes, hipStream_t s,
                     LayerArgs *a) {
    int device = 0;
    OHIP(hipGetDevice(&device), "hipGetDevice");
    const auto key = std::make_tuple(device, n, t, thin, chunk, value_bytes);
    const OrderPlan *plan = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_order_mu);
        auto it = g_order_plans.find(key);
        if (it == g_order_plans.end()) {
            OrderPlan p;
            p.off.resize(n + 1);
            std::vector<uint32_t> host;
            LayerLists L;
            if (!build_lists(n, t, thin, chunk, value_bytes, 2, n, L))
                return set_error(PERM_ENOMEM, "building the tile order of order %d failed", n);
            for (size_t i = 0; i < L.groups.size(); i++) {
                const int kk = L.groups[i].first, g = L.groups[i].second;
                p.off[kk][g] = (uint32_t)host.size();
                if (L.lists[i]->size() != L.slots[i])
                    return set_error(PERM_EINVAL, "tile order of layer %d group %d has %zu slots, plan %u", kk, g,
                                     L.lists[i]->size(), L.slots[i]);
                host.insert(host.end(), L.lists[i]->begin(), L.lists[i]->end());
            }
            if (host.empty()) host.push_back(kNoTile);
            OHIP(hipMalloc(&p.dev, host.size() * 4), "hipMalloc tile order");
            hipError_t e = hipMemcpyAsync(p.dev, host.data(), host.size() * 4, hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) {
                (void)hipFree(p.dev);  // nothing launched reads it yet
                return hip_error(e, "upload tile order");
            }
            it = g_order_plans.emplace(key, std::move(p)).first;
        }
        plan = &it->second;
    }
    // std::map nodes stay put, so the plan outlives the lock
    a->zorder = plan->dev;
    for (int g = 0; g < a->ngroups; g++) a->zoff[g] = plan->off[k][g];
    return PERM_OK;
}

}  // namespace permgpu

extern "C" int perm_layer_tile_order(int n, int t, int k, int value_bytes, uint32_t *out, size_t cap,
                                     size_t *len) {
    using namespace permgpu;
    try {
        if (!len) return set_error(PERM_EINVAL, "null len");
        if (n < 2 || n > PERM_N_MAX || t < 1 || t > kTMax || t > n || k < 2 || k > n || value_bytes < 1)
            return set_error(PERM_EINVAL, "n = %d, t = %d, k = %d, value_bytes = %d", n, t, k, value_bytes);
        if (n - t > kOrderNhMax)
            return set_error(PERM_EINVAL, "n - t = %d high columns (the order covers at most %d)", n - t,
                             kOrderNhMax);
        if (cap > 0 && !out) return set_error(PERM_EINVAL, "null out with cap %zu", cap);
        std::vector<uint32_t> v;
        if (!tile_order_layer(n, k, t, tuned_layer_thin(n), tuned_layer_remap(n), value_bytes, v))
            return set_error(PERM_ENOMEM, "building the tile order failed");
        for (size_t i = 0; i < v.size() && i < cap; i++) out[i] = v[i];
        *len = v.size();
        return PERM_OK;
    } catch (...) {
        return set_error(PERM_EDEVICE, "internal error");
    }
}
