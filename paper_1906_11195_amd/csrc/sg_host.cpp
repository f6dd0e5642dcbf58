// Host runtime of the library: instance builder (graph, colouring, sweep
// order, adjacency in sweep order, threshold tables), device memory layout,
// kernel launches and the C ABI declared in include/sg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <tuple>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <stdexcept>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "sg.h"
#include "sg_internal.h"
#include "sg_ledger.h"
#include "sg_split_plan.h"
#include "sg_philox.h"

using namespace sg;

namespace {

struct Fail {
    sg_status code;
};

[[noreturn]] void fail(sg_status s) { throw Fail{s}; }

void hip_check(hipError_t e)
{
    if (e != hipSuccess) {
        if (e == hipErrorOutOfMemory) fail(SG_ENOMEM);
        fail(SG_EDEVICE);
    }
}

// ---------------------------------------------------------------------------
// Thresholds: thr[x] = floor(2^32 exp(-beta dE)), dE = 2 x s (Metropolis).
// ---------------------------------------------------------------------------
#pragma clang fp contract(off)
uint64_t threshold(double T, double s, int64_t x)
{
    const double beta = 1.0 / T;
    const double dE = 2.0 * (double)x * s;
    return (uint64_t)std::floor(std::ldexp(std::exp(-beta * dE), 32));
}

// ---------------------------------------------------------------------------
// VB instance tables.
// ---------------------------------------------------------------------------
struct VbGraph {
    int64_t n = 0;
    std::vector<int32_t> eu, ev;     // edges in acceptance / given order
    std::vector<int8_t> J;
    std::vector<int32_t> colour;     // per vertex
    std::vector<int32_t> order;      // vertex at each position
    std::vector<int32_t> row;        // [n+1], sweep order
    std::vector<uint32_t> ent;       // [2m]
    std::vector<int32_t> eix;        // [2m] edge index of each adjacency entry
    std::vector<int32_t> cls;        // [ncls+1]
    int32_t ncls = 0;
    int32_t max_degree = 0;
};

// G(N, M) from the GRAPH stream (rejecting self-loops and repeated pairs).
void er_generate(VbGraph& g, int64_t m, uint64_t seed, uint32_t graph_id)
{
    const uint64_t n = (uint64_t)g.n;
    g.eu.resize((size_t)m);
    g.ev.resize((size_t)m);
    g.J.resize((size_t)m);
    // accepted pairs in an open-addressing set (linear probing, at most a
    // quarter full; ~0 marks a free slot, no pair key has all bits set)
    size_t cap = 16;
    while (cap < (size_t)m * 4) cap <<= 1;
    std::vector<uint64_t> seen(cap, ~0ull);
    const int shift = 64 - __builtin_ctzll((unsigned long long)cap);
    auto insert = [&](uint64_t key) {
        size_t i = (size_t)((key * 0x9E3779B97F4A7C15ull) >> shift);
        for (;;) {
            if (seen[i] == ~0ull) {
                seen[i] = key;
                return true;
            }
            if (seen[i] == key) return false;
            i = (i + 1) & (cap - 1);
        }
    };
    int64_t k = 0;
    for (uint64_t a = 0; k < m; ++a) {
        const U4 w = philox_stream(seed, (uint32_t)a, (uint32_t)(a >> 32), kDomGraph, 0u, graph_id);
        const uint64_t u = ((uint64_t)w.x * n) >> 32;
        const uint64_t v = ((uint64_t)w.y * n) >> 32;
        if (u == v) continue;
        const uint64_t key = u < v ? (u << 32) | v : (v << 32) | u;
        if (!insert(key)) continue;
        g.eu[(size_t)k] = (int32_t)u;
        g.ev[(size_t)k] = (int32_t)v;
        g.J[(size_t)k] = (w.z & 1u) ? (int8_t)-1 : (int8_t)1;
        ++k;
    }
}

// Greedy colouring, sweep order and the adjacency in sweep order.
void vb_tables(VbGraph& g)
{
    const int64_t n = g.n;
    const size_t m = g.eu.size();
    std::vector<int32_t> deg((size_t)n, 0);
    for (size_t e = 0; e < m; ++e) {
        deg[(size_t)g.eu[e]]++;
        deg[(size_t)g.ev[e]]++;
    }
    std::vector<int64_t> vstart((size_t)n + 1, 0);
    for (int64_t v = 0; v < n; ++v) vstart[(size_t)v + 1] = vstart[(size_t)v] + deg[(size_t)v];
    std::vector<int32_t> vn(2 * m), ve(2 * m);
    std::vector<int8_t> vj(2 * m);
    std::vector<int64_t> fill(vstart.begin(), vstart.end() - 1);
    for (size_t e = 0; e < m; ++e) {
        const int32_t u = g.eu[e], v = g.ev[e];
        ve[(size_t)fill[(size_t)u]] = (int32_t)e;
        vn[(size_t)fill[(size_t)u]] = v;
        vj[(size_t)fill[(size_t)u]++] = g.J[e];
        ve[(size_t)fill[(size_t)v]] = (int32_t)e;
        vn[(size_t)fill[(size_t)v]] = u;
        vj[(size_t)fill[(size_t)v]++] = g.J[e];
    }
    g.max_degree = 0;
    for (int64_t v = 0; v < n; ++v) g.max_degree = std::max(g.max_degree, deg[(size_t)v]);

    // colour(v) = smallest colour absent among neighbours u < v
    g.colour.assign((size_t)n, 0);
    std::vector<int64_t> stamp((size_t)g.max_degree + 2, -1);
    int32_t ncls = 0;
    for (int64_t v = 0; v < n; ++v) {
        for (int64_t a = vstart[(size_t)v]; a < vstart[(size_t)v + 1]; ++a) {
            const int32_t u = vn[(size_t)a];
            if (u < v) {
                const int32_t cu = g.colour[(size_t)u];
                if (cu <= g.max_degree) stamp[(size_t)cu] = v;
            }
        }
        int32_t c = 0;
        while (stamp[(size_t)c] == v) ++c;
        g.colour[(size_t)v] = c;
        ncls = std::max(ncls, c + 1);
    }
    g.ncls = ncls;

    // positions: class by class; inside a class by decreasing degree, ties by
    // increasing id (counting sort on the key (class, max_degree - degree))
    const int32_t nd = g.max_degree + 1;
    std::vector<int32_t> bucket((size_t)ncls * nd + 1, 0);
    auto key = [&](int64_t v) { return (size_t)g.colour[(size_t)v] * nd + (size_t)(g.max_degree - deg[(size_t)v]); };
    for (int64_t v = 0; v < n; ++v) bucket[key(v) + 1]++;
    for (size_t b = 0; b + 1 < bucket.size(); ++b) bucket[b + 1] += bucket[b];
    g.cls.assign((size_t)ncls + 1, 0);
    for (int32_t c = 0; c <= ncls; ++c) g.cls[(size_t)c] = bucket[(size_t)c * nd];
    g.order.assign((size_t)n, 0);
    std::vector<int32_t> pos((size_t)n);
    for (int64_t v = 0; v < n; ++v) {
        const int32_t p = bucket[key(v)]++;
        g.order[(size_t)p] = (int32_t)v;
        pos[(size_t)v] = p;
    }
    g.row.assign((size_t)n + 1, 0);
    g.ent.resize(2 * m);
    g.eix.resize(2 * m);
    int64_t e = 0;
    for (int64_t p = 0; p < n; ++p) {
        const int32_t v = g.order[(size_t)p];
        g.row[(size_t)p] = (int32_t)e;
        for (int64_t a = vstart[(size_t)v]; a < vstart[(size_t)v + 1]; ++a) {
            g.eix[(size_t)e] = ve[(size_t)a];
            g.ent[(size_t)e++] = (uint32_t)pos[(size_t)vn[(size_t)a]] |
                                 (vj[(size_t)a] < 0 ? 0x80000000u : 0u);
        }
    }
    g.row[(size_t)n] = (int32_t)e;
}

bool finite_nonneg_T(double T) { return !(T < 0.0) && !std::isnan(T); }

void check_vb_desc(const sg_vb_desc& d)
{
    if (d.n < 2 || d.n > (1 << 20)) fail(d.n > (1 << 20) ? SG_ENOTSUP : SG_EINVAL);
    if (!finite_nonneg_T(d.T)) fail(SG_EINVAL);
    if (d.n_replicas < 1 || d.n_replicas > kVbMaxChains) fail(SG_EINVAL);
    if (d.start < SG_START_RANDOM || d.start > SG_START_GIVEN) fail(SG_EINVAL);
    if (d.start == SG_START_GIVEN) {
        if (!d.s0) fail(SG_EINVAL);
        for (int64_t i = 0; i < d.n * d.n_replicas; ++i)
            if (d.s0[i] != 1 && d.s0[i] != -1) fail(SG_EINVAL);
    }
    if (d.edges) {
        if (d.n_edges < 0 || !d.J || d.n_edges > d.n * (d.n - 1) / 2) fail(SG_EINVAL);
        std::unordered_set<uint64_t> seen;
        seen.reserve((size_t)d.n_edges * 2 + 1);
        for (int64_t e = 0; e < d.n_edges; ++e) {
            const int64_t u = d.edges[2 * e], v = d.edges[2 * e + 1];
            if (u < 0 || v < 0 || u >= d.n || v >= d.n || u == v) fail(SG_EINVAL);
            if (d.J[e] != 1 && d.J[e] != -1) fail(SG_EINVAL);
            const uint64_t key = u < v ? ((uint64_t)u << 32) | (uint64_t)v
                                       : ((uint64_t)v << 32) | (uint64_t)u;
            if (!seen.insert(key).second) fail(SG_EINVAL);
        }
    } else {
        if (!(d.c >= 0.0) || std::isinf(d.c)) fail(SG_EINVAL);
        const double m = std::floor(d.c * (double)d.n / 2.0);
        if (m > (double)(d.n * (d.n - 1) / 2)) fail(SG_EINVAL);
    }
}

void build_vb_graph(const sg_vb_desc& d, VbGraph& g)
{
    g.n = d.n;
    if (d.edges) {
        g.eu.resize((size_t)d.n_edges);
        g.ev.resize((size_t)d.n_edges);
        g.J.assign(d.J, d.J + d.n_edges);
        for (int64_t e = 0; e < d.n_edges; ++e) {
            g.eu[(size_t)e] = d.edges[2 * e];
            g.ev[(size_t)e] = d.edges[2 * e + 1];
        }
    } else {
        const int64_t m = (int64_t)std::floor(d.c * (double)d.n / 2.0);
        er_generate(g, m, d.seed, d.graph_id);
    }
    vb_tables(g);
    if (g.max_degree >= kVbXMax) fail(SG_ENOTSUP);
}

void check_sk_desc(const sg_sk_desc& d)
{
    if (d.n < 2 || d.n > 32768) fail(d.n > 32768 ? SG_ENOTSUP : SG_EINVAL);
    if (d.Jf) {
        if (d.J) fail(SG_EINVAL);
        if (d.n > 16384) fail(SG_ENOTSUP);   // fields in double stay in one workgroup's LDS
        const int64_t n = d.n;
        for (int64_t i = 0; i < n; ++i) {
            if (d.Jf[i * n + i] != 0.0f) fail(SG_EINVAL);
            for (int64_t j = i + 1; j < n; ++j) {
                const float a = d.Jf[i * n + j];
                if (!std::isfinite(a) || d.Jf[j * n + i] != a) fail(SG_EINVAL);
            }
        }
    }
    if (!finite_nonneg_T(d.T)) fail(SG_EINVAL);
    if (d.n_replicas < 1 || d.n_replicas > kVbMaxChains) fail(SG_EINVAL);
    if (d.start < SG_START_RANDOM || d.start > SG_START_GIVEN) fail(SG_EINVAL);
    if (d.recompute_period < 0) fail(SG_EINVAL);
    if (d.start == SG_START_GIVEN) {
        if (!d.s0) fail(SG_EINVAL);
        for (int64_t i = 0; i < d.n * d.n_replicas; ++i)
            if (d.s0[i] != 1 && d.s0[i] != -1) fail(SG_EINVAL);
    }
    if (d.J) {
        const int64_t n = d.n;
        for (int64_t i = 0; i < n; ++i) {
            if (d.J[i * n + i] != 0) fail(SG_EINVAL);
            for (int64_t j = i + 1; j < n; ++j) {
                const int8_t a = d.J[i * n + j];
                if ((a != 1 && a != -1) || d.J[j * n + i] != a) fail(SG_EINVAL);
            }
        }
    }
}


template <class F>
void parallel_for(size_t count, F&& f)
{
    const size_t hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const size_t nt = std::min(count, hw);
    if (nt <= 1) {
        for (size_t i = 0; i < count; ++i) f(i);
        return;
    }
    std::atomic<size_t> next{0};
    std::atomic<int> err{0};
    std::vector<std::thread> th;
    for (size_t t = 0; t < nt; ++t)
        th.emplace_back([&]() {
            for (;;) {
                const size_t i = next.fetch_add(1);
                if (i >= count) break;
                try {
                    f(i);
                } catch (const Fail& e) {
                    err.store(e.code);
                } catch (...) {
                    err.store(SG_ENOMEM);
                }
            }
        });
    for (auto& x : th) x.join();
    if (err.load() != 0) fail(err.load());
}

// Runs f(0..count-1) on several host threads when `par`, else in order.
template <class F>
void maybe_parallel(bool par, size_t count, F&& f)
{
    if (par) {
        parallel_for(count, f);
    } else {
        for (size_t i = 0; i < count; ++i) f(i);
    }
}

// SK couplings: the upper triangle row by row (one Philox block covers 128
// consecutive idx = i N + j), then the lower triangle mirrored tile by tile;
// both passes on several host threads when `par`.
void sk_generate(int64_t n, uint64_t seed, uint32_t graph_id, int8_t* J, bool par)
{
    maybe_parallel(par, (size_t)n, [&](size_t ii) {
        const int64_t i = (int64_t)ii;
        J[i * n + i] = 0;
        int64_t j = i + 1;
        while (j < n) {
            const uint64_t idx = (uint64_t)i * (uint64_t)n + (uint64_t)j;
            const uint64_t blk = idx >> 7;
            const U4 w = philox_stream(seed, (uint32_t)blk, (uint32_t)(idx >> 39), kDomCoupling, 0u,
                                       graph_id);
            const uint64_t blk_end = (blk + 1) << 7;
            for (; j < n && (uint64_t)i * (uint64_t)n + (uint64_t)j < blk_end; ++j) {
                const uint64_t id2 = (uint64_t)i * (uint64_t)n + (uint64_t)j;
                const uint32_t bit = (word_of(w, (uint32_t)((id2 >> 5) & 3u)) >> (id2 & 31u)) & 1u;
                J[i * n + j] = bit ? (int8_t)-1 : (int8_t)1;
            }
        }
    });
    const int64_t nt = (n + 63) / 64;
    maybe_parallel(par, (size_t)nt, [&](size_t bi) {
        const int64_t r0 = (int64_t)bi * 64, r1 = std::min(n, r0 + 64);
        for (int64_t c0 = 0; c0 < r1; c0 += 64)
            for (int64_t i = r0; i < r1; ++i)
                for (int64_t k = c0; k < std::min(i, c0 + 64); ++k) J[i * n + k] = J[k * n + i];
    });
}

int32_t grid_size(int64_t t_max)
{
    int32_t k = 1;
    for (int64_t t = 1; t <= t_max; t <<= 1) ++k;
    return k;
}

// Device arena: one allocation carved into aligned pieces.
struct Arena {
    size_t size = 0;
    size_t take(size_t bytes)
    {
        const size_t off = size;
        size += (bytes + 255) & ~(size_t)255;
        return off;
    }
};

}  // namespace

namespace {
SplitLedger g_split_ledger;   // split-unit members held per device, all contexts
}  // namespace

struct sg_ctx {
    int kind = 0;   // 0 VB, 1 SK
    int device = 0;
    sg_alloc_fn alloc = nullptr;
    sg_free_fn freef = nullptr;
    void* user = nullptr;
    void* arena = nullptr;
    size_t arena_bytes = 0;
    // every stream a call has put this context's work on (synchronised, with
    // the legacy stream of the set-up work, before the memory is released;
    // never the whole device, so that other contexts keep running)
    std::vector<hipStream_t> streams_used;
    void note_stream(hipStream_t s)
    {
        for (hipStream_t x : streams_used)
            if (x == s) return;
        streams_used.push_back(s);
    }
    void sync_own()
    {
        (void)hipStreamSynchronize(nullptr);
        for (hipStream_t x : streams_used) (void)hipStreamSynchronize(x);
    }
    int32_t count = 0, R = 0, K = 0, n_chains = 0;
    int64_t t_max = 0, t_done = 0;
    int64_t t_start = 0;                  // time of the start configurations (resume)
    int32_t bond_done = 0;   // VB: snapshots whose bond sums bond_d already holds
    // windowed correlation (VB): waiting times, intervals, sums per chain
    int32_t kw = 0, n_bins = 0;
    long long* win_d = nullptr;           // [n_chains][kw][n_bins]
    std::vector<int64_t> times;
    std::vector<int64_t> n_of;            // spins per instance
    // VB
    std::vector<int32_t> group_of_inst;
    std::vector<std::vector<int32_t>> order_of_group;
    std::vector<VbUnit> units;
    VbUnit* units_d = nullptr;
    int32_t* unit_chain_ids_d = nullptr;
    std::vector<std::pair<int32_t, int32_t>> chain_loc;   // chain -> (unit, slot)
    int vb_threads = 64;                  // widest launch group (measurement kernels)
    size_t bond_lds = 0;
    int64_t updates_per_sweep = 0;
    // launch groups: units of one workgroup size, one kernel per sweep chunk
    struct Group {
        int threads = 64;
        size_t lds = 0;
        int32_t first = 0, count = 0;     // range in units_d
        bool split = false;               // members of split units (not autotuned)
        bool multispin = false;           // multispin units: range in vbm_d
        int64_t updates = 0;              // chain-updates per sweep
        hipStream_t stream = nullptr;     // own stream for groups after the first
        hipEvent_t done = nullptr;
    };
    std::vector<Group> groups;
    hipEvent_t fork = nullptr;
    int64_t* t_dev = nullptr;             // device counter of sweeps done
    uint32_t* bars_d = nullptr;           // split units' barrier words, 2 per unit
    int n_bar = 0;
    int split_held = 0;                   // members reserved in the process-wide ledger
    // multispin units (SG_OPT_MULTISPIN): up to 64 chains of one graph per word
    std::vector<VbmUnit> vbm;
    VbmUnit* vbm_d = nullptr;
    int32_t* vbm_ids_d = nullptr;         // [units][64] chain ids
    std::vector<char> chain_ms;           // chain lives in a multispin unit (chain_loc indexes vbm)
    bool use_graph = false;
    hipStream_t capture_stream = nullptr; // for capturing when the caller uses the null stream
    std::vector<std::pair<int64_t, hipGraphExec_t>> graphs;   // chunk length -> executable
    // SK
    std::vector<SkChain> sk;
    SkChain* sk_d = nullptr;
    std::vector<SkSample> sks;
    SkSample* sks_d = nullptr;
    int sk_max_n = 0;
    size_t sk_lds = 0;
    int period = 64;
    int* err_d = nullptr;
    int sk_threads = 256;
    bool sk_real = false;                 // SK with real couplings (sg_skg.hip)
    double* bondr_d = nullptr;            // [n_chains][K] real bond sums
    double* bpart_d = nullptr;            // their partial sums
    // measurement
    MeasureChain* mc_d = nullptr;
    int32_t* pairs_d = nullptr;
    int n_pairs = 0;
    int max_words = 0;
    long long* bond_d = nullptr;
    long long* overlap_d = nullptr;
    long long* gram_d = nullptr;
    unsigned long long* acc_d = nullptr;

    void* dev_alloc(size_t bytes)
    {
        void* p = nullptr;
        if (alloc) {
            p = alloc(bytes, user);
            if (!p) fail(SG_ENOMEM);
        } else {
            hipError_t e = hipMalloc(&p, bytes);
            if (e != hipSuccess) fail(e == hipErrorOutOfMemory ? SG_ENOMEM : SG_EDEVICE);
        }
        return p;
    }
    void release()
    {
        g_split_ledger.release(device, split_held);
        split_held = 0;
        for (auto& gx : graphs) (void)hipGraphExecDestroy(gx.second);
        graphs.clear();
        for (auto& G : groups) {
            if (G.stream) (void)hipStreamDestroy(G.stream);
            if (G.done) (void)hipEventDestroy(G.done);
            G.stream = nullptr;
            G.done = nullptr;
        }
        if (fork) (void)hipEventDestroy(fork);
        fork = nullptr;
        if (capture_stream) (void)hipStreamDestroy(capture_stream);
        capture_stream = nullptr;
        if (arena) {
            if (alloc && freef) freef(arena, arena_bytes, user);
            else if (!alloc) (void)hipFree(arena);
            arena = nullptr;
        }
    }
    void dev_free(void* p, size_t bytes)
    {
        if (!p) return;
        if (alloc && freef) freef(p, bytes, user);
        else if (!alloc) (void)hipFree(p);
    }
    template <class T>
    T* at(size_t off) { return reinterpret_cast<T*>(static_cast<char*>(arena) + off); }
    int32_t k_done() const
    {
        int32_t k = 0;
        for (int64_t t : times)
            if (t <= t_done) ++k;
        return k;
    }
};

namespace {

void setup_common(sg_ctx* c, const sg_opts* o)
{
    c->t_max = o ? o->t_max : 0;
    if (c->t_max < 0 || c->t_max >= (int64_t)1 << 31) fail(SG_EINVAL);
    c->t_start = o ? o->t_start : 0;
    if (c->t_start < 0 || c->t_start >= (int64_t)1 << 32) fail(SG_EINVAL);
    c->t_done = c->t_start;
    c->K = grid_size(c->t_max);
    // slot 0: the start configuration; slot k >= 1: grid time 2^(k-1), not
    // taken (-1) when it is not after t_start
    c->times.push_back(c->t_start);
    for (int64_t t = 1; t <= c->t_max; t <<= 1) c->times.push_back(t > c->t_start ? t : -1);
    if (o) {
        c->alloc = o->alloc;
        c->freef = o->free;
        c->user = o->user;
        if ((o->alloc == nullptr) != (o->free == nullptr)) fail(SG_EINVAL);
        if (o->threads_per_unit != 0 &&
            (o->threads_per_unit < 64 || o->threads_per_unit > 1024 || o->threads_per_unit % 64))
            fail(SG_EINVAL);
        if (o->chains_per_unit < 0 || o->chains_per_unit > kVbMaxChains) fail(SG_EINVAL);
        if (o->flags & SG_OPT_WINDOW) {
            if (c->t_max < 1 || o->window_tw_max < 0) fail(SG_EINVAL);
            if (c->t_start > 0) fail(SG_ENOTSUP);
            c->kw = 0;
            for (int64_t t : c->times)
                if (t <= o->window_tw_max) ++c->kw;
            c->n_bins = vb_window_bin((uint64_t)c->t_max) + 1;
        }
    }
    int dev_count = 0;
    if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count == 0) fail(SG_EDEVICE);
    hip_check(hipGetDevice(&c->device));
    hipDeviceProp_t prop;
    hip_check(hipGetDeviceProperties(&prop, c->device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) fail(SG_EDEVICE);
}

// Enqueues `nsw` sweeps of every launch group on stream s: the groups after
// the first fork onto their own streams and join back; the device sweep
// counter advances after the join (when `advance`).
void vb_launch_chunk(sg_ctx* c, int32_t nsw, hipStream_t s, const int64_t* t0p, bool advance)
{
    const size_t ng = c->groups.size();
    if (ng > 1) {
        hip_check(hipEventRecord(c->fork, s));
        for (size_t gi = 1; gi < ng; ++gi) hip_check(hipStreamWaitEvent(c->groups[gi].stream, c->fork, 0));
    }
    for (size_t gi = 0; gi < ng; ++gi) {
        const sg_ctx::Group& G = c->groups[gi];
        if (G.multispin)
            hip_check(vbm_sweep(c->vbm_d + G.first, G.count, G.threads, G.lds, t0p, nsw, c->t_max,
                                gi == 0 ? s : G.stream));
        else
            hip_check(vb_sweep(c->units_d + G.first, G.count, G.threads, G.lds, t0p, nsw, c->t_max,
                               gi == 0 ? s : G.stream));
    }
    for (size_t gi = 1; gi < ng; ++gi) {
        hip_check(hipEventRecord(c->groups[gi].done, c->groups[gi].stream));
        hip_check(hipStreamWaitEvent(s, c->groups[gi].done, 0));
    }
    if (advance) hip_check(vb_advance(c->t_dev, nsw, c->bars_d, c->n_bar, s));
}

// The sweep chunk of length nsw captured once as a graph (kernels read the
// device sweep counter, so one executable serves every replay).
hipGraphExec_t vb_graph_for(sg_ctx* c, int32_t nsw)
{
    for (auto& gx : c->graphs)
        if (gx.first == nsw) return gx.second;
    if (!c->capture_stream) hip_check(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
    hipStream_t cs = c->capture_stream;
    hip_check(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipGraph_t graph = nullptr;
    try {
        vb_launch_chunk(c, nsw, cs, c->t_dev, true);
    } catch (...) {
        (void)hipStreamEndCapture(cs, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        throw;
    }
    hip_check(hipStreamEndCapture(cs, &graph));
    hipGraphExec_t exec = nullptr;
    const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    hip_check(e);
    if (c->graphs.size() >= 8) {
        (void)hipGraphExecDestroy(c->graphs.front().second);
        c->graphs.erase(c->graphs.begin());
    }
    c->graphs.emplace_back(nsw, exec);
    return exec;
}

// Autotuner: for every launch group, times candidate workgroup sizes (half,
// same, double the heuristic's) on a few trial sweeps and keeps the fastest.
// Trials run at sweep counters >= 2^31, beyond any measurement time, on a
// saved copy of the spins and counters that is restored afterwards, so tuning
// changes no result.  Choices are cached per process by group shape.
struct TuneKey {
    int threads, nlog, rpad, resident;
    bool operator<(const TuneKey& o) const
    {
        return std::tie(threads, nlog, rpad, resident) < std::tie(o.threads, o.nlog, o.rpad, o.resident);
    }
};
std::map<TuneKey, int> g_tuned;
std::mutex g_tuned_mu;

void vb_autotune(sg_ctx* c)
{
    const size_t lds_cap = 160 * 1024 - 1024;
    size_t words = 0;
    for (const auto& U : c->units) words += (size_t)U.state_words;
    const size_t bytes = words * 4 + (size_t)c->n_chains * 8;
    char* save = static_cast<char*>(c->dev_alloc(bytes));
    struct Restore {
        sg_ctx* c;
        char* p;
        size_t bytes;
        ~Restore() { c->dev_free(p, bytes); }
    } guard{c, save, bytes};
    size_t off = 0;
    for (const auto& U : c->units) {
        hip_check(hipMemcpy(save + off, U.state, (size_t)U.state_words * 4, hipMemcpyDeviceToDevice));
        off += (size_t)U.state_words * 4;
    }
    hip_check(hipMemcpy(save + off, c->acc_d, (size_t)c->n_chains * 8, hipMemcpyDeviceToDevice));
    const int64_t trial_t = ((int64_t)1 << 31) + 7;
    hip_check(hipMemcpy(c->t_dev + 1, &trial_t, 8, hipMemcpyHostToDevice));
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0));
    hip_check(hipEventCreate(&e1));
    for (auto& G : c->groups) {
        if (G.split || G.multispin) continue;   // split members meet at barriers; multispin: planned size
        int32_t nmax = 0;
        for (int32_t u = G.first; u < G.first + G.count; ++u) nmax = std::max(nmax, c->units[(size_t)u].n);
        const VbUnit& U0 = c->units[(size_t)G.first];
        int nlog = 0;
        while ((1 << (nlog + 1)) <= nmax) ++nlog;
        const TuneKey key{G.threads, nlog, U0.rpad, U0.resident};
        auto lds_for = [&](int th) {
            size_t l = 0;
            for (int32_t u = G.first; u < G.first + G.count; ++u) {
                const VbUnit& U = c->units[(size_t)u];
                l = std::max(l, vb_lds_bytes(U.n, U.rpad, U.nch, th, U.cpl != 0) +
                                    (U.resident ? vb_resident_bytes(U.n, U.m2) : 0));
            }
            return l;
        };
        int best = -1;
        {
            std::lock_guard<std::mutex> lk(g_tuned_mu);
            auto it = g_tuned.find(key);
            if (it != g_tuned.end()) best = it->second;
        }
        if (best < 0) {
            const int32_t nsw = (int32_t)std::max<int64_t>(1, std::min<int64_t>(32, ((int64_t)1 << 25) / std::max<int64_t>(1, G.updates)));
            float best_ms = 1e30f;
            for (int th : {G.threads / 2, G.threads, G.threads * 2}) {
                if (th < 64 || th > 1024 || lds_for(th) > lds_cap) continue;
                const size_t lds = lds_for(th);
                hip_check(vb_sweep(c->units_d + G.first, G.count, th, lds, c->t_dev + 1, 1, c->t_max, nullptr));
                hip_check(hipEventRecord(e0, nullptr));
                hip_check(vb_sweep(c->units_d + G.first, G.count, th, lds, c->t_dev + 1, nsw, c->t_max, nullptr));
                hip_check(hipEventRecord(e1, nullptr));
                hip_check(hipEventSynchronize(e1));
                float ms = 0.f;
                hip_check(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best_ms) {
                    best_ms = ms;
                    best = th;
                }
            }
            std::lock_guard<std::mutex> lk(g_tuned_mu);
            g_tuned[key] = best;
        }
        if (best > 0) {
            G.threads = best;
            G.lds = lds_for(best);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    off = 0;
    for (const auto& U : c->units) {
        hip_check(hipMemcpy(U.state, save + off, (size_t)U.state_words * 4, hipMemcpyDeviceToDevice));
        off += (size_t)U.state_words * 4;
    }
    hip_check(hipMemcpy(c->acc_d, save + off, (size_t)c->n_chains * 8, hipMemcpyDeviceToDevice));
    hip_check(hipDeviceSynchronize());
    for (const auto& G : c->groups) c->vb_threads = std::max(c->vb_threads, G.threads);
}

std::vector<uint32_t> pack_given(const int8_t* s0, int64_t n, const std::vector<int32_t>* order)
{
    std::vector<uint32_t> bits((size_t)((n + 31) / 32), 0u);
    for (int64_t p = 0; p < n; ++p) {
        const int64_t v = order ? (*order)[(size_t)p] : p;
        if (s0[v] == -1) bits[(size_t)(p >> 5)] |= 1u << (p & 31);
    }
    return bits;
}

void create_vb(sg_ctx* c, const sg_vb_desc* d, int32_t count, const sg_opts* o)
{
    c->kind = 0;
    c->count = count;
    c->R = d[0].n_replicas;
    for (int32_t i = 0; i < count; ++i) {
        check_vb_desc(d[i]);
        if (d[i].n_replicas != c->R) fail(SG_EINVAL);
    }
    setup_common(c, o);
    c->n_chains = count * c->R;

    // group instances that share a generated graph
    struct Key {
        int64_t n;
        uint64_t cbits, seed;
        uint32_t gid;
        bool operator==(const Key& k) const
        {
            return n == k.n && cbits == k.cbits && seed == k.seed && gid == k.gid;
        }
    };
    struct KeyHash {
        size_t operator()(const Key& k) const
        {
            return std::hash<uint64_t>()((uint64_t)k.n * 0x9E3779B97F4A7C15ull ^ k.cbits ^
                                         (k.seed << 1) ^ ((uint64_t)k.gid << 17));
        }
    };
    std::unordered_map<Key, int32_t, KeyHash> gid_of;
    // explicit graphs are shared by the instances that pass the same arrays
    // with the same seed (a unit's chains share one Philox key)
    std::map<std::tuple<int64_t, int64_t, const int32_t*, const int8_t*, uint64_t>, int32_t> explicit_of;
    std::vector<int32_t> first_inst;   // representative desc per group
    c->group_of_inst.resize((size_t)count);
    // Multispin (SG_OPT_MULTISPIN): instances that share a graph -- generated
    // from one key, or passing one edge array with one seed -- whatever their
    // couplings, when they bring at least kVbmMinChains chains and the graph
    // fits (n <= kVbmMaxN), form multispin groups; the others are grouped as
    // usual.
    const bool ms_opt = o && (o->flags & SG_OPT_MULTISPIN);
    if (ms_opt && c->kw > 0) fail(SG_ENOTSUP);
    constexpr int32_t kVbmMinChains = 16;
    std::vector<char> in_ms((size_t)count, 0);
    if (ms_opt) {
        std::map<std::tuple<int64_t, int64_t, const int32_t*, uint64_t, uint64_t, uint32_t>, int32_t> cnt;
        auto mk = [&](int32_t i) {
            uint64_t cb;
            std::memcpy(&cb, &d[i].c, 8);
            return d[i].edges ? std::make_tuple((int64_t)d[i].n, d[i].n_edges, d[i].edges, d[i].seed, (uint64_t)0, 0u)
                              : std::make_tuple((int64_t)d[i].n, (int64_t)-1, (const int32_t*)nullptr, d[i].seed, cb,
                                                d[i].graph_id);
        };
        for (int32_t i = 0; i < count; ++i) cnt[mk(i)] += c->R;
        for (int32_t i = 0; i < count; ++i)
            in_ms[(size_t)i] = cnt[mk(i)] >= kVbmMinChains && d[i].n <= kVbmMaxN;
    }
    for (int32_t i = 0; i < count; ++i) {
        if (d[i].edges) {
            const int8_t* jkey = in_ms[(size_t)i] ? nullptr : d[i].J;   // multispin: couplings per chain
            const auto ek = std::make_tuple((int64_t)d[i].n, d[i].n_edges, d[i].edges, jkey, d[i].seed);
            auto it = explicit_of.find(ek);
            if (it == explicit_of.end()) {
                it = explicit_of.emplace(ek, (int32_t)first_inst.size()).first;
                first_inst.push_back(i);
            }
            c->group_of_inst[(size_t)i] = it->second;
            continue;
        }
        uint64_t cb;
        std::memcpy(&cb, &d[i].c, 8);
        Key k{d[i].n, cb, d[i].seed, d[i].graph_id};
        auto it = gid_of.find(k);
        if (it == gid_of.end()) {
            it = gid_of.emplace(k, (int32_t)first_inst.size()).first;
            first_inst.push_back(i);
        }
        c->group_of_inst[(size_t)i] = it->second;
    }
    const size_t n_groups = first_inst.size();
    std::vector<VbGraph> graphs(n_groups);
    parallel_for(n_groups, [&](size_t gi) { build_vb_graph(d[first_inst[gi]], graphs[gi]); });

    // chains of each group, then work units
    std::vector<std::vector<int32_t>> chains_of(n_groups);
    for (int32_t i = 0; i < count; ++i)
        for (int32_t r = 0; r < c->R; ++r)
            chains_of[(size_t)c->group_of_inst[(size_t)i]].push_back(i * c->R + r);
    const int32_t want = o && o->chains_per_unit ? o->chains_per_unit : kVbMaxChains;
    const size_t lds_cap = 160 * 1024 - 1024;

    struct UnitPlan {
        int32_t group;
        std::vector<int32_t> chains;
        int32_t rpad;
        int threads = 64;
        bool resident = false;
        bool cpl = false;
        int64_t work = 0;
        int members = 1;
    };
    // Workgroup size first: about three 64-position chunks per wavefront in
    // the graph's largest colour class (up to 16 wavefronts).  Then as many
    // chains per unit as fit in LDS at that size; only a graph whose single
    // chain does not fit at that size gets fewer wavefronts.  (Spreading the
    // chains of a large graph over several units keeps each unit's
    // wavefronts busy; packing them at the cost of wavefronts leaves one
    // latency-bound unit that finishes long after the rest.)
    auto rpad_of = [](int32_t k) { return k <= 1 ? 1 : k <= 2 ? 2 : k <= 4 ? 4 : 8; };
    std::vector<char> group_ms(n_groups, 0);
    for (size_t gi = 0; gi < n_groups; ++gi) group_ms[gi] = in_ms[(size_t)first_inst[gi]];
    std::vector<int> graph_threads(n_groups, 64);
    std::vector<UnitPlan> plan;
    for (size_t gi = 0; gi < n_groups; ++gi) {
        if (group_ms[gi]) continue;   // multispin units are planned below
        const VbGraph& g = graphs[gi];
        const int64_t n = g.n;
        int th = 64;
        if (o && o->threads_per_unit) {
            th = o->threads_per_unit;
        } else {
            int32_t maxcls = 0;
            for (int32_t k = 0; k < g.ncls; ++k) maxcls = std::max(maxcls, g.cls[(size_t)k + 1] - g.cls[(size_t)k]);
            const int32_t chunks = (maxcls + 63) / 64;
            int waves = 1;
            while (waves < 16 && waves * 3 < chunks) waves *= 2;
            th = 64 * waves;
            while (th > 64 && vb_lds_bytes((int32_t)n, 1, 1, th) > lds_cap) th /= 2;
        }
        graph_threads[gi] = th;
        int32_t per = std::min<int32_t>(want, (int32_t)chains_of[gi].size());
        while (per > 1 && vb_lds_bytes((int32_t)n, rpad_of(per), per, th) > lds_cap) --per;
        if (vb_lds_bytes((int32_t)n, rpad_of(per), per, th) > lds_cap) fail(SG_ENOTSUP);
        const auto& ch = chains_of[gi];
        for (size_t a = 0; a < ch.size(); a += (size_t)per) {
            UnitPlan u;
            u.group = (int32_t)gi;
            u.chains.assign(ch.begin() + (long)a, ch.begin() + (long)std::min(ch.size(), a + (size_t)per));
            u.rpad = rpad_of((int32_t)u.chains.size());
            plan.push_back(std::move(u));
        }
    }

    // Small graphs keep their adjacency LDS-resident.  Units of one size form
    // one launch group, largest work first inside a group
    // (longest-processing-time order).
    for (auto& u : plan) {
        const VbGraph& g = graphs[(size_t)u.group];
        const int32_t n = (int32_t)g.n;
        const int th = graph_threads[(size_t)u.group];
        if (vb_lds_bytes(n, u.rpad, (int32_t)u.chains.size(), th) > lds_cap) fail(SG_ENOTSUP);
        u.threads = th;
        u.resident = vb_lds_bytes(n, u.rpad, (int32_t)u.chains.size(), th) + vb_resident_bytes(n, (int32_t)g.ent.size()) <= lds_cap;
        u.work = (int64_t)n * (int64_t)u.chains.size();
    }
    // Split units: a unit holding far more than one CU's share of the
    // batch's work is spread over several workgroups (members) that meet at a
    // device-scope barrier after every colour class.  The members of all
    // split units of all contexts of the process on the device use at most
    // half of the CUs (a process-wide ledger), so that they can all be
    // resident at once next to other work, and an automatic plan takes at
    // most a quarter of the CUs, so that two large contexts built at the same
    // time (a server's batches) both split their largest units.
    // Members per unit: plan_split (sg_split_plan.h), by cost n (10 + chains).
    // opts.split_members: 0 automatic, 1 never, k >= 2 every unit that has
    // the chunks for k members (tests, tuning).  No effect on any result.
    {
        int n_cu = 0;
        hip_check(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, c->device));
        const int forced = o ? o->split_members : 0;
        auto cost_of = [&](const UnitPlan& u) {
            return (int64_t)graphs[(size_t)u.group].n * (10 + (int64_t)u.chains.size());
        };
        int64_t total = 0;
        for (const auto& u : plan) total += cost_of(u);
        const int64_t share = std::max<int64_t>(1, total / std::max(1, n_cu));
        // the members of every split unit of the process on this device
        // together stay within half of the CUs (members reserved while their
        // context lives, so that all of them can be resident at once)
        c->split_held = g_split_ledger.reserve(c->device, n_cu / 2, [&](int avail) {
            const int budget = forced == 0 ? std::min(avail, n_cu / 4) : avail;
            std::vector<SplitUnit> su(plan.size());
            for (size_t i = 0; i < plan.size(); ++i) {
                const VbGraph& g = graphs[(size_t)plan[i].group];
                int32_t maxcls = 0;
                for (int32_t k = 0; k < g.ncls; ++k) maxcls = std::max(maxcls, g.cls[(size_t)k + 1] - g.cls[(size_t)k]);
                su[i] = SplitUnit{cost_of(plan[i]), plan[i].resident,
                                  ((maxcls + 63) / 64) / (2 * (plan[i].threads / 64))};
            }
            std::vector<int> members;
            const int used = plan_split(su, share, budget, forced, members);
            for (size_t i = 0; i < plan.size(); ++i) plan[i].members = members[i];
            return used;
        });
    }
    std::stable_sort(plan.begin(), plan.end(), [](const UnitPlan& a, const UnitPlan& b) {
        const bool sa = a.members > 1, sb = b.members > 1;
        if (sa != sb) return sa;
        return a.threads != b.threads ? a.threads > b.threads : a.work > b.work;
    });
    // A unit neither resident nor split keeps a complemented copy of its
    // spin words in LDS when it fits: its adjacency entries then address the
    // neighbour's word, or its complement for J < 0, directly
    const bool plain_lds = o && (o->flags & SG_OPT_PLAIN_LDS);
    for (auto& u : plan) {
        const VbGraph& g = graphs[(size_t)u.group];
        u.cpl = !plain_lds && !u.resident && u.members == 1 &&
                vb_lds_bytes((int32_t)g.n, u.rpad, (int32_t)u.chains.size(), u.threads, true) <= lds_cap;
    }
    int n_split = 0, n_entries = 0;
    for (const auto& u : plan) {
        n_split += u.members > 1 ? 1 : 0;
        n_entries += u.members;
    }

    // device layout
    Arena A;
    std::vector<size_t> off_row(n_groups), off_ent(n_groups), off_cls(n_groups);
    for (size_t gi = 0; gi < n_groups; ++gi) {
        off_row[gi] = A.take(graphs[gi].row.size() * 4);
        off_ent[gi] = A.take((graphs[gi].ent.size() + kVbEntPad) * 4);
        off_cls[gi] = A.take(graphs[gi].cls.size() * 4);
    }
    // entries in the complemented-copy form: one array per graph and slot count
    std::map<std::pair<int32_t, int32_t>, size_t> off_entc;
    for (const auto& u : plan)
        if (u.cpl && !off_entc.count({u.group, u.rpad}))
            off_entc[{u.group, u.rpad}] = A.take((graphs[(size_t)u.group].ent.size() + kVbEntPad) * 4);
    std::vector<size_t> off_state(plan.size());
    for (size_t u = 0; u < plan.size(); ++u) {
        const int64_t n = graphs[(size_t)plan[u].group].n;
        off_state[u] = A.take((size_t)VbLayout(plan[u].rpad).words(n) * 4);
    }
    std::vector<size_t> off_snap((size_t)c->n_chains), off_given((size_t)c->n_chains, 0);
    c->n_of.resize((size_t)count);
    for (int32_t i = 0; i < count; ++i) {
        c->n_of[(size_t)i] = d[i].n;
        const size_t wn = (size_t)((d[i].n + 31) / 32);
        for (int32_t r = 0; r < c->R; ++r) {
            off_snap[(size_t)(i * c->R + r)] = A.take(wn * (size_t)c->K * 4);
            if (d[i].start == SG_START_GIVEN) off_given[(size_t)(i * c->R + r)] = A.take(wn * 4);
        }
        c->max_words = std::max(c->max_words, (int)wn);
    }
    std::vector<size_t> off_wsnap(plan.size(), 0);
    if (c->kw > 0)
        for (size_t u = 0; u < plan.size(); ++u) {
            const int64_t n = graphs[(size_t)plan[u].group].n;
            off_wsnap[u] = A.take((size_t)((VbLayout(plan[u].rpad).words(n) + 3) & ~3) * 4 * (size_t)c->kw);
        }
    const size_t win_per_chain = (size_t)c->kw * (size_t)c->n_bins;
    const size_t off_win = A.take(std::max<size_t>(1, (size_t)c->n_chains * win_per_chain) * 8);
    const size_t off_units = A.take((size_t)n_entries * sizeof(VbUnit));
    const size_t off_ids = A.take((size_t)n_entries * kVbMaxChains * 4);
    const size_t off_bars = A.take((size_t)std::max(1, n_split) * 8);
    const size_t off_err = A.take(8);
    const size_t off_mc = A.take((size_t)c->n_chains * sizeof(MeasureChain));
    c->n_pairs = count * c->R * (c->R - 1) / 2;
    const size_t off_pairs = A.take((size_t)std::max(1, c->n_pairs) * 8);
    const size_t off_bond = A.take((size_t)c->n_chains * c->K * 8);
    const size_t off_ovl = A.take((size_t)std::max(1, c->n_pairs) * c->K * 8);
    const size_t off_gram = A.take((size_t)c->n_chains * c->K * c->K * 8);
    const size_t off_acc = A.take((size_t)c->n_chains * 8);
    const size_t off_t = A.take(16);

    // multispin units: the chains of each multispin group, 64 per unit
    struct MsPlan {
        int32_t group;
        std::vector<int32_t> chains;
    };
    std::vector<MsPlan> ms_plan;
    for (size_t gi = 0; gi < n_groups; ++gi) {
        if (!group_ms[gi]) continue;
        const auto& ch = chains_of[gi];
        for (size_t a = 0; a < ch.size(); a += (size_t)kVbmChains) {
            MsPlan mp;
            mp.group = (int32_t)gi;
            mp.chains.assign(ch.begin() + (long)a, ch.begin() + (long)std::min(ch.size(), a + (size_t)kVbmChains));
            ms_plan.push_back(std::move(mp));
        }
    }
    std::vector<size_t> off_mjw(ms_plan.size()), off_mst(ms_plan.size()), off_mthr(ms_plan.size());
    for (size_t u = 0; u < ms_plan.size(); ++u) {
        const VbGraph& g = graphs[(size_t)ms_plan[u].group];
        off_mjw[u] = A.take((g.ent.size() + kVbEntPad) * 8);
        off_mst[u] = A.take((size_t)g.n * 8);
        off_mthr[u] = A.take((size_t)2 * kVbmChains * kVbXMax * 4);
    }
    const size_t off_vbm = A.take(std::max<size_t>(1, ms_plan.size()) * sizeof(VbmUnit));
    const size_t off_vbm_ids = A.take(std::max<size_t>(1, ms_plan.size()) * kVbmChains * 4);

    c->arena_bytes = A.size;
    c->arena = c->dev_alloc(A.size);

    // uploads
    for (size_t gi = 0; gi < n_groups; ++gi) {
        const VbGraph& g = graphs[gi];
        hip_check(hipMemcpy(c->at<void>(off_row[gi]), g.row.data(), g.row.size() * 4, hipMemcpyHostToDevice));
        std::vector<uint32_t> padded(g.ent.size() + kVbEntPad, 0u);
        std::copy(g.ent.begin(), g.ent.end(), padded.begin());
        hip_check(hipMemcpy(c->at<void>(off_ent[gi]), padded.data(), padded.size() * 4, hipMemcpyHostToDevice));
        hip_check(hipMemcpy(c->at<void>(off_cls[gi]), g.cls.data(), g.cls.size() * 4, hipMemcpyHostToDevice));
    }
    for (const auto& kv : off_entc) {
        const VbGraph& g = graphs[(size_t)kv.first.first];
        std::vector<uint32_t> e(g.ent.size() + kVbEntPad);
        vb_cpl_entries(g.ent.data(), g.ent.size(), kVbEntPad, kv.first.second, (int32_t)g.n, e.data());
        hip_check(hipMemcpy(c->at<void>(kv.second), e.data(), e.size() * 4, hipMemcpyHostToDevice));
    }
    for (int32_t i = 0; i < count; ++i) {
        if (d[i].start != SG_START_GIVEN) continue;
        const VbGraph& g = graphs[(size_t)c->group_of_inst[(size_t)i]];
        for (int32_t r = 0; r < c->R; ++r) {
            const auto bits = pack_given(d[i].s0 + (int64_t)r * d[i].n, d[i].n, &g.order);
            hip_check(hipMemcpy(c->at<void>(off_given[(size_t)(i * c->R + r)]), bits.data(), bits.size() * 4,
                                hipMemcpyHostToDevice));
        }
    }

    c->units.clear();
    c->units.reserve((size_t)n_entries);
    std::vector<int32_t> ids((size_t)n_entries * kVbMaxChains, 0);
    c->bars_d = c->at<uint32_t>(off_bars);
    c->n_bar = 2 * n_split;
    c->err_d = c->at<int>(off_err);
    int split_seen = 0;
    c->chain_loc.resize((size_t)c->n_chains);
    c->updates_per_sweep = 0;
    for (size_t u = 0; u < plan.size(); ++u) {
        const VbGraph& g = graphs[(size_t)plan[u].group];
        VbUnit U;
        std::memset(&U, 0, sizeof(U));
        U.row = c->at<int32_t>(off_row[(size_t)plan[u].group]);
        U.ent = c->at<uint32_t>(off_ent[(size_t)plan[u].group]);
        U.cls = c->at<int32_t>(off_cls[(size_t)plan[u].group]);
        U.resident = plan[u].resident ? 1 : 0;
        U.cpl = plan[u].cpl ? 1 : 0;
        if (U.cpl) U.entc = c->at<uint32_t>(off_entc.at({plan[u].group, plan[u].rpad}));
        U.m2 = (int32_t)g.ent.size();
        // chains of a unit share one graph, hence one seed (graphs are keyed by
        // seed; an explicit edge list belongs to one instance)
        U.key = d[plan[u].chains[0] / c->R].seed;
        for (int32_t ch : plan[u].chains)
            if (d[ch / c->R].seed != U.key) fail(SG_EINVAL);
        U.state = c->at<uint32_t>(off_state[u]);
        U.n = (int32_t)g.n;
        U.ncls = g.ncls;
        if (g.ncls > 64) fail(SG_ENOTSUP);   // the kernel keeps <= 64 class bounds in LDS
        U.nch = (int32_t)plan[u].chains.size();
        U.rpad = plan[u].rpad;
        U.state_words = (int32_t)VbLayout(U.rpad).words(g.n);
        U.words_n = (int32_t)((g.n + 31) / 32);
        U.kw = c->kw;
        U.n_bins = c->n_bins;
        U.wsnap = c->kw > 0 ? c->at<uint32_t>(off_wsnap[u]) : nullptr;
        for (int32_t k = 0; k < U.nch; ++k) {
            const int32_t ch = plan[u].chains[(size_t)k];
            const int32_t i = ch / c->R, r = ch % c->R;
            U.snap[k] = c->at<uint32_t>(off_snap[(size_t)ch]);
            U.accepted[k] = c->at<unsigned long long>(off_acc) + ch;
            U.seed[k] = d[i].seed;
            U.inst[k] = d[i].instance_id;
            U.rep[k] = (uint32_t)r;
            U.init_mode[k] = d[i].start;
            U.given[k] = d[i].start == SG_START_GIVEN ? c->at<uint32_t>(off_given[(size_t)ch]) : nullptr;
            U.win[k] = c->kw > 0 ? c->at<long long>(off_win) + (size_t)ch * win_per_chain : nullptr;
            for (int32_t x = 0; x < kVbXMax; ++x) {
                const uint64_t th = x == 0 ? (uint64_t)1 << 32 : threshold(d[i].T, 1.0, x);
                U.thr_hi[k][x] = (uint32_t)(th >> 16);
                U.thr_lo[k][x] = (uint32_t)(th & 0xffffu);
            }
            c->chain_loc[(size_t)ch] = {(int32_t)c->units.size(), k};
        }
        const int th = plan[u].threads;
        const bool split = plan[u].members > 1;
        U.members = plan[u].members;
        U.err = c->err_d;
        U.bar = split ? c->bars_d + 2 * split_seen++ : nullptr;
        if (c->groups.empty() || c->groups.back().threads != th || c->groups.back().split != split) {
            sg_ctx::Group G;
            G.threads = th;
            G.split = split;
            G.first = (int32_t)c->units.size();
            c->groups.push_back(G);
        }
        sg_ctx::Group& G = c->groups.back();
        for (int m = 0; m < U.members; ++m) {
            U.member = m;
            for (int32_t k = 0; k < U.nch; ++k)
                ids[c->units.size() * kVbMaxChains + (size_t)k] = plan[u].chains[(size_t)k];
            c->units.push_back(U);
            G.count++;
        }
        G.updates += g.n * U.nch;
        G.lds = std::max(G.lds, vb_lds_bytes(U.n, U.rpad, U.nch, th, U.cpl != 0) +
                                    (U.resident ? vb_resident_bytes(U.n, U.m2) : 0));
        c->vb_threads = std::max(c->vb_threads, th);
        c->bond_lds = std::max(c->bond_lds, (size_t)(((U.nch * U.words_n + 1) & ~1) * 4 + kVbMaxChains * 8));
        c->updates_per_sweep += g.n * U.nch;
    }
    // multispin units: descriptors, coupling words (bit k of entry e: the
    // coupling of slot k's chain on that entry is -1) and threshold tables
    c->chain_ms.assign((size_t)c->n_chains, 0);
    std::vector<int32_t> ms_ids(std::max<size_t>(1, ms_plan.size()) * kVbmChains, 0);
    c->vbm.resize(ms_plan.size());
    int ms_threads = 128;
    int64_t ms_updates = 0;
    parallel_for(ms_plan.size(), [&](size_t u) {
        hip_check(hipSetDevice(c->device));   // a worker thread: the context's device
        const MsPlan& mp = ms_plan[u];
        const VbGraph& g = graphs[(size_t)mp.group];
        VbmUnit U;
        std::memset(&U, 0, sizeof(U));
        U.row = c->at<int32_t>(off_row[(size_t)mp.group]);
        U.ent = c->at<uint32_t>(off_ent[(size_t)mp.group]);
        U.cls = c->at<int32_t>(off_cls[(size_t)mp.group]);
        U.jw = c->at<uint64_t>(off_mjw[u]);
        U.state = c->at<uint64_t>(off_mst[u]);
        U.thr = c->at<uint32_t>(off_mthr[u]);
        U.n = (int32_t)g.n;
        U.ncls = g.ncls;
        U.nch = (int32_t)mp.chains.size();
        U.words_n = (int32_t)((g.n + 31) / 32);
        U.key = U.seed = d[mp.chains[0] / c->R].seed;
        if (g.ncls > 64) fail(SG_ENOTSUP);
        std::vector<uint32_t> thr((size_t)2 * kVbmChains * kVbXMax, 0u);   // high halves, then low halves
        std::vector<uint64_t> jw(g.ent.size() + kVbEntPad, 0ull);
        for (int32_t k = 0; k < U.nch; ++k) {
            const int32_t ch = mp.chains[(size_t)k];
            const int32_t i = ch / c->R, r = ch % c->R;
            if (d[i].seed != U.key) fail(SG_EINVAL);
            U.snap[k] = c->at<uint32_t>(off_snap[(size_t)ch]);
            U.accepted[k] = c->at<unsigned long long>(off_acc) + ch;
            U.inst[k] = d[i].instance_id;
            U.rep[k] = (uint32_t)r;
            U.init_mode[k] = d[i].start;
            U.given[k] = d[i].start == SG_START_GIVEN ? c->at<uint32_t>(off_given[(size_t)ch]) : nullptr;
            ms_ids[u * kVbmChains + (size_t)k] = ch;
            for (int32_t x = 1; x < kVbXMax; ++x) {
                const uint64_t th = threshold(d[i].T, 1.0, x);   // up to 2^32 (T = inf)
                thr[(size_t)k * kVbXMax + (size_t)x] = (uint32_t)(th >> 16);
                thr[(size_t)(kVbmChains + k) * kVbXMax + (size_t)x] = (uint32_t)(th & 0xffffu);
            }
            const int8_t* Ji = d[i].edges ? d[i].J : nullptr;
            const uint64_t bit = 1ull << k;
            for (size_t e = 0; e < g.ent.size(); ++e) {
                const bool neg = Ji ? Ji[(size_t)g.eix[e]] < 0 : (g.ent[e] >> 31) != 0u;
                if (neg) jw[e] |= bit;
            }
        }
        hip_check(hipMemcpy(c->at<void>(off_mthr[u]), thr.data(), thr.size() * 4, hipMemcpyHostToDevice));
        hip_check(hipMemcpy(c->at<void>(off_mjw[u]), jw.data(), jw.size() * 8, hipMemcpyHostToDevice));
        c->vbm[u] = U;
    });
    for (size_t u = 0; u < ms_plan.size(); ++u) {
        const MsPlan& mp = ms_plan[u];
        const VbGraph& g = graphs[(size_t)mp.group];
        for (size_t k = 0; k < mp.chains.size(); ++k) {
            c->chain_loc[(size_t)mp.chains[k]] = {(int32_t)u, (int32_t)k};
            c->chain_ms[(size_t)mp.chains[k]] = 1;
        }
        ms_updates += g.n * (int64_t)mp.chains.size();
        // wavefronts: about three 64-position chunks each in the largest
        // colour class (2 to 16), within LDS
        int32_t maxcls = 0;
        for (int32_t k = 0; k < g.ncls; ++k) maxcls = std::max(maxcls, g.cls[(size_t)k + 1] - g.cls[(size_t)k]);
        const int32_t chunks = (maxcls + 63) / 64;
        int waves = 2;
        while (waves < 16 && waves * 3 < chunks) waves *= 2;
        ms_threads = std::max(ms_threads, 64 * waves);
    }
    if (!ms_plan.empty()) {
        const size_t lds_cap = 160 * 1024 - 1024;
        int32_t nmax = 0;
        for (const auto& U : c->vbm) nmax = std::max(nmax, U.n);
        while (ms_threads > 128 && vbm_lds_bytes(nmax, ms_threads) > lds_cap) ms_threads /= 2;
        if (vbm_lds_bytes(nmax, ms_threads) > lds_cap) fail(SG_ENOTSUP);
        sg_ctx::Group G;
        G.threads = ms_threads;
        G.lds = vbm_lds_bytes(nmax, ms_threads);
        G.first = 0;
        G.count = (int32_t)ms_plan.size();
        G.multispin = true;
        G.updates = ms_updates;
        c->groups.push_back(G);
        c->updates_per_sweep += ms_updates;
    }
    c->vbm_d = c->at<VbmUnit>(off_vbm);
    c->vbm_ids_d = c->at<int32_t>(off_vbm_ids);
    if (!ms_plan.empty()) {
        hip_check(hipMemcpy(c->vbm_d, c->vbm.data(), c->vbm.size() * sizeof(VbmUnit), hipMemcpyHostToDevice));
        hip_check(hipMemcpy(c->vbm_ids_d, ms_ids.data(), ms_ids.size() * 4, hipMemcpyHostToDevice));
    }
    c->order_of_group.resize(n_groups);
    for (size_t gi = 0; gi < n_groups; ++gi) c->order_of_group[gi] = std::move(graphs[gi].order);

    std::vector<MeasureChain> mc((size_t)c->n_chains);
    for (int32_t ch = 0; ch < c->n_chains; ++ch) {
        const int64_t n = c->n_of[(size_t)(ch / c->R)];
        mc[(size_t)ch] = MeasureChain{c->at<uint32_t>(off_snap[(size_t)ch]), (int32_t)((n + 31) / 32), (int32_t)n};
    }
    std::vector<int32_t> pairs;
    for (int32_t i = 0; i < count; ++i)
        for (int32_t a = 0; a < c->R; ++a)
            for (int32_t b = a + 1; b < c->R; ++b) {
                pairs.push_back(i * c->R + a);
                pairs.push_back(i * c->R + b);
            }
    c->units_d = c->at<VbUnit>(off_units);
    c->unit_chain_ids_d = c->at<int32_t>(off_ids);
    c->mc_d = c->at<MeasureChain>(off_mc);
    c->pairs_d = c->at<int32_t>(off_pairs);
    c->bond_d = c->at<long long>(off_bond);
    c->overlap_d = c->at<long long>(off_ovl);
    c->gram_d = c->at<long long>(off_gram);
    c->acc_d = c->at<unsigned long long>(off_acc);
    hip_check(hipMemcpy(c->units_d, c->units.data(), c->units.size() * sizeof(VbUnit), hipMemcpyHostToDevice));
    hip_check(hipMemcpy(c->unit_chain_ids_d, ids.data(), ids.size() * 4, hipMemcpyHostToDevice));
    hip_check(hipMemcpy(c->mc_d, mc.data(), mc.size() * sizeof(MeasureChain), hipMemcpyHostToDevice));
    if (!pairs.empty())
        hip_check(hipMemcpy(c->pairs_d, pairs.data(), pairs.size() * 4, hipMemcpyHostToDevice));
    c->t_dev = c->at<int64_t>(off_t);
    c->win_d = c->at<long long>(off_win);
    if (c->kw > 0) {
        hip_check(zero_i64(c->win_d, (size_t)c->n_chains * win_per_chain, nullptr));
        // waiting-time words: rows padded to 16 bytes with zeros
        for (size_t u = 0; u < plan.size(); ++u) {
            const int64_t n = graphs[(size_t)plan[u].group].n;
            const size_t row = (size_t)((VbLayout(plan[u].rpad).words(n) + 3) & ~3);
            hip_check(zero_i64(c->at<long long>(off_wsnap[u]), row * (size_t)c->kw / 2, nullptr));
        }
    }
    hip_check(zero_i64(c->bond_d, (size_t)c->n_chains * c->K, nullptr));
    hip_check(zero_i64((long long*)c->acc_d, (size_t)c->n_chains, nullptr));
    hip_check(zero_i64((long long*)c->t_dev, 2, nullptr));
    if (c->t_start > 0) hip_check(hipMemcpy(c->t_dev, &c->t_start, 8, hipMemcpyHostToDevice));
    hip_check(zero_i64((long long*)c->bars_d, (size_t)std::max(1, n_split), nullptr));
    hip_check(zero_i64((long long*)c->err_d, 1, nullptr));
    hip_check(vb_init(c->units_d, (int)c->units.size(), 256, 0, nullptr));
    hip_check(vb_prepare());
    hip_check(vbm_init(c->vbm_d, (int)c->vbm.size(), nullptr));
    hip_check(vbm_prepare());
    // every launch group after the first runs on a stream of its own, forked
    // from and joined back into the caller's stream
    for (size_t gi = 1; gi < c->groups.size(); ++gi) {
        hip_check(hipStreamCreateWithFlags(&c->groups[gi].stream, hipStreamNonBlocking));
        hip_check(hipEventCreateWithFlags(&c->groups[gi].done, hipEventDisableTiming));
    }
    hip_check(hipEventCreateWithFlags(&c->fork, hipEventDisableTiming));
    c->use_graph = o && (o->flags & SG_OPT_GRAPH);
    // the set-up work ran on the legacy stream: wait for it alone
    hip_check(hipStreamSynchronize(nullptr));
    if (o && (o->flags & SG_OPT_AUTOTUNE) && !o->threads_per_unit) vb_autotune(c);
}

// SK with real couplings: float32 J per distinct array, fields in double.
void create_skg(sg_ctx* c, const sg_sk_desc* d, int32_t count, const sg_opts* o)
{
    c->kind = 1;
    c->sk_real = true;
    c->count = count;
    c->R = d[0].n_replicas;
    c->period = d[0].recompute_period ? d[0].recompute_period : 64;
    for (int32_t i = 0; i < count; ++i) {
        if (!d[i].Jf) fail(SG_EINVAL);   // a context is all real or all binary
        check_sk_desc(d[i]);
        if (d[i].n_replicas != c->R) fail(SG_EINVAL);
        if ((d[i].recompute_period ? d[i].recompute_period : 64) != c->period) fail(SG_EINVAL);
    }
    setup_common(c, o);
    if (c->kw > 0) fail(SG_ENOTSUP);   // the windowed correlation is measured for VB only
    // a resume is exact when the fields start from the direct sums the
    // uninterrupted run also recomputes at that time
    if (c->t_start % c->period != 0) fail(SG_EINVAL);
    c->n_chains = count * c->R;
    c->n_of.resize((size_t)count);
    // instances passing the same array share its device copy
    std::map<std::pair<const float*, int64_t>, int32_t> share;
    std::vector<int32_t> jslot((size_t)count);
    std::vector<int32_t> jrep;
    for (int32_t i = 0; i < count; ++i) {
        c->n_of[(size_t)i] = d[i].n;
        const auto key = std::make_pair(d[i].Jf, d[i].n);
        auto it = share.find(key);
        if (it == share.end()) {
            it = share.emplace(key, (int32_t)jrep.size()).first;
            jrep.push_back(i);
        }
        jslot[(size_t)i] = it->second;
    }
    Arena A;
    std::vector<size_t> off_J(jrep.size());
    for (size_t j = 0; j < jrep.size(); ++j) off_J[j] = A.take((size_t)(d[jrep[j]].n * d[jrep[j]].n) * 4);
    std::vector<size_t> off_state((size_t)c->n_chains), off_H((size_t)c->n_chains), off_snap((size_t)c->n_chains),
        off_given((size_t)c->n_chains, 0);
    for (int32_t i = 0; i < count; ++i) {
        const size_t wn = (size_t)((d[i].n + 31) / 32);
        c->max_words = std::max(c->max_words, (int)wn);
        c->sk_max_n = std::max(c->sk_max_n, (int)d[i].n);
        for (int32_t r = 0; r < c->R; ++r) {
            const size_t ch = (size_t)(i * c->R + r);
            off_state[ch] = A.take(wn * 4);
            off_H[ch] = A.take((size_t)d[i].n * 8);
            off_snap[ch] = A.take(wn * (size_t)c->K * 4);
            if (d[i].start == SG_START_GIVEN) off_given[ch] = A.take(wn * 4);
        }
    }
    const size_t off_chains = A.take((size_t)c->n_chains * sizeof(SkChain));
    const size_t off_samples = A.take((size_t)count * sizeof(SkSample));
    const size_t off_mc = A.take((size_t)c->n_chains * sizeof(MeasureChain));
    c->n_pairs = count * c->R * (c->R - 1) / 2;
    const size_t off_pairs = A.take((size_t)std::max(1, c->n_pairs) * 8);
    const size_t off_bond = A.take((size_t)c->n_chains * c->K * 8);
    const size_t off_ovl = A.take((size_t)std::max(1, c->n_pairs) * c->K * 8);
    const size_t off_gram = A.take((size_t)c->n_chains * c->K * c->K * 8);
    const size_t off_acc = A.take((size_t)c->n_chains * 8);
    const size_t off_err = A.take(8);
    const size_t off_bondr = A.take((size_t)c->n_chains * c->K * 8);
    const size_t off_part = A.take((size_t)count * (size_t)((c->sk_max_n + 15) / 16) * (size_t)c->R * c->K * 8);
    c->arena_bytes = A.size;
    c->arena = c->dev_alloc(A.size);
    for (size_t j = 0; j < jrep.size(); ++j) {
        const int64_t n = d[jrep[j]].n;
        hip_check(hipMemcpy(c->at<void>(off_J[j]), d[jrep[j]].Jf, (size_t)(n * n) * 4, hipMemcpyHostToDevice));
    }
    c->sk.resize((size_t)c->n_chains);
    c->sks.resize((size_t)count);
    for (int32_t i = 0; i < count; ++i) {
        SkSample sm;
        std::memset(&sm, 0, sizeof(sm));
        sm.Jf = c->at<float>(off_J[(size_t)jslot[(size_t)i]]);
        sm.n = (int32_t)d[i].n;
        sm.nch = c->R;
        sm.chain0 = i * c->R;
        c->sks[(size_t)i] = sm;
        for (int32_t r = 0; r < c->R; ++r) {
            const size_t ch = (size_t)(i * c->R + r);
            SkChain S;
            std::memset(&S, 0, sizeof(S));
            S.Jf = sm.Jf;
            S.Hd = c->at<double>(off_H[ch]);
            S.beta = 1.0 / d[i].T;
            S.state = c->at<uint32_t>(off_state[ch]);
            S.snap = c->at<uint32_t>(off_snap[ch]);
            S.accepted = c->at<unsigned long long>(off_acc) + ch;
            S.seed = d[i].seed;
            S.inst = d[i].instance_id;
            S.rep = (uint32_t)r;
            S.n = (int32_t)d[i].n;
            S.words_n = (int32_t)((d[i].n + 31) / 32);
            S.init_mode = d[i].start;
            S.sample = i;
            if (d[i].start == SG_START_GIVEN) {
                const auto bits = pack_given(d[i].s0 + (int64_t)r * d[i].n, d[i].n, nullptr);
                hip_check(hipMemcpy(c->at<void>(off_given[ch]), bits.data(), bits.size() * 4, hipMemcpyHostToDevice));
                S.given = c->at<uint32_t>(off_given[ch]);
            }
            c->sk[ch] = S;
        }
    }
    std::vector<MeasureChain> mc((size_t)c->n_chains);
    for (int32_t ch = 0; ch < c->n_chains; ++ch)
        mc[(size_t)ch] = MeasureChain{c->sk[(size_t)ch].snap, c->sk[(size_t)ch].words_n, c->sk[(size_t)ch].n};
    std::vector<int32_t> pairs;
    for (int32_t i = 0; i < count; ++i)
        for (int32_t a = 0; a < c->R; ++a)
            for (int32_t b = a + 1; b < c->R; ++b) {
                pairs.push_back(i * c->R + a);
                pairs.push_back(i * c->R + b);
            }
    c->sk_d = c->at<SkChain>(off_chains);
    c->sks_d = c->at<SkSample>(off_samples);
    c->mc_d = c->at<MeasureChain>(off_mc);
    c->pairs_d = c->at<int32_t>(off_pairs);
    c->bond_d = c->at<long long>(off_bond);
    c->overlap_d = c->at<long long>(off_ovl);
    c->gram_d = c->at<long long>(off_gram);
    c->acc_d = c->at<unsigned long long>(off_acc);
    c->err_d = c->at<int>(off_err);
    c->bondr_d = c->at<double>(off_bondr);
    c->bpart_d = c->at<double>(off_part);
    hip_check(hipMemcpy(c->sk_d, c->sk.data(), c->sk.size() * sizeof(SkChain), hipMemcpyHostToDevice));
    hip_check(hipMemcpy(c->sks_d, c->sks.data(), c->sks.size() * sizeof(SkSample), hipMemcpyHostToDevice));
    hip_check(hipMemcpy(c->mc_d, mc.data(), mc.size() * sizeof(MeasureChain), hipMemcpyHostToDevice));
    if (!pairs.empty())
        hip_check(hipMemcpy(c->pairs_d, pairs.data(), pairs.size() * 4, hipMemcpyHostToDevice));
    hip_check(zero_i64(c->bond_d, (size_t)c->n_chains * c->K, nullptr));
    hip_check(zero_i64((long long*)c->bondr_d, (size_t)c->n_chains * c->K, nullptr));
    hip_check(zero_i64((long long*)c->acc_d, (size_t)c->n_chains, nullptr));
    hip_check(zero_i64((long long*)c->err_d, 1, nullptr));
    c->sk_lds = skg_lds_bytes(c->sk_max_n);
    hip_check(sk_init(c->sk_d, c->n_chains, 256, nullptr));
    hip_check(skg_recompute(c->sks_d, count, c->sk_d, c->sk_max_n, 0, c->err_d, nullptr));
    hip_check(hipStreamSynchronize(nullptr));
}

void create_sk(sg_ctx* c, const sg_sk_desc* d, int32_t count, const sg_opts* o)
{
    if (d[0].Jf) {
        create_skg(c, d, count, o);
        return;
    }
    c->kind = 1;
    c->count = count;
    c->R = d[0].n_replicas;
    c->period = d[0].recompute_period ? d[0].recompute_period : 64;
    for (int32_t i = 0; i < count; ++i) {
        if (d[i].Jf) fail(SG_EINVAL);    // a context is all real or all binary
        check_sk_desc(d[i]);
        if (d[i].n_replicas != c->R) fail(SG_EINVAL);
        if ((d[i].recompute_period ? d[i].recompute_period : 64) != c->period) fail(SG_EINVAL);
    }
    setup_common(c, o);
    if (c->kw > 0) fail(SG_ENOTSUP);   // the windowed correlation is measured for VB only
    c->n_chains = count * c->R;
    c->n_of.resize((size_t)count);

    // samples sharing a generated coupling matrix
    std::unordered_map<uint64_t, int32_t> share;
    std::vector<int32_t> jslot((size_t)count);
    std::vector<int32_t> jrep;   // representative instance per matrix
    for (int32_t i = 0; i < count; ++i) {
        c->n_of[(size_t)i] = d[i].n;
        if (d[i].J) {
            jslot[(size_t)i] = (int32_t)jrep.size();
            jrep.push_back(i);
            continue;
        }
        const uint64_t key = ((uint64_t)d[i].n * 0x9E3779B97F4A7C15ull) ^ (d[i].seed * 0xC2B2AE3D27D4EB4Full) ^
                             ((uint64_t)d[i].graph_id << 1);
        auto it = share.find(key);
        if (it != share.end()) {
            const sg_sk_desc& r = d[jrep[(size_t)it->second]];
            if (r.n == d[i].n && r.seed == d[i].seed && r.graph_id == d[i].graph_id) {
                jslot[(size_t)i] = it->second;
                continue;
            }
        }
        share[key] = (int32_t)jrep.size();
        jslot[(size_t)i] = (int32_t)jrep.size();
        jrep.push_back(i);
    }

    std::vector<std::vector<uint64_t>> thr((size_t)count);
    for (int32_t i = 0; i < count; ++i) {
        const double s = 1.0 / std::sqrt((double)d[i].n);
        auto& t = thr[(size_t)i];
        t.push_back((uint64_t)1 << 32);
        for (int64_t x = 1; x < d[i].n; ++x) {
            const uint64_t v = threshold(d[i].T, s, x);
            if (v == 0) break;
            t.push_back(v);
        }
    }

    Arena A;
    std::vector<size_t> off_J(jrep.size()), off_Jb(jrep.size()), off_Jt(jrep.size());
    const int tile_words = sk_tile_words();
    for (size_t j = 0; j < jrep.size(); ++j) {
        const int64_t n = d[jrep[j]].n;
        off_J[j] = A.take((size_t)(n * n));
        off_Jb[j] = A.take((size_t)n * (size_t)((n + 31) / 32) * 4);
        off_Jt[j] = A.take((size_t)((n + 63) / 64) * 64 * (size_t)tile_words * 4);
    }
    std::vector<size_t> off_thr((size_t)count);
    for (int32_t i = 0; i < count; ++i) off_thr[(size_t)i] = A.take(thr[(size_t)i].size() * 8);
    std::vector<size_t> off_state((size_t)c->n_chains), off_H((size_t)c->n_chains), off_snap((size_t)c->n_chains),
        off_given((size_t)c->n_chains, 0);
    for (int32_t i = 0; i < count; ++i) {
        const size_t wn = (size_t)((d[i].n + 31) / 32);
        c->max_words = std::max(c->max_words, (int)wn);
        c->sk_max_n = std::max(c->sk_max_n, (int)d[i].n);
        for (int32_t r = 0; r < c->R; ++r) {
            const size_t ch = (size_t)(i * c->R + r);
            off_state[ch] = A.take(wn * 4);
            off_H[ch] = A.take((size_t)d[i].n * 4);
            off_snap[ch] = A.take(wn * (size_t)c->K * 4);
            if (d[i].start == SG_START_GIVEN) off_given[ch] = A.take(wn * 4);
        }
    }
    const size_t off_chains = A.take((size_t)c->n_chains * sizeof(SkChain));
    const size_t off_samples = A.take((size_t)count * sizeof(SkSample));
    const size_t off_mc = A.take((size_t)c->n_chains * sizeof(MeasureChain));
    c->n_pairs = count * c->R * (c->R - 1) / 2;
    const size_t off_pairs = A.take((size_t)std::max(1, c->n_pairs) * 8);
    const size_t off_bond = A.take((size_t)c->n_chains * c->K * 8);
    const size_t off_ovl = A.take((size_t)std::max(1, c->n_pairs) * c->K * 8);
    const size_t off_gram = A.take((size_t)c->n_chains * c->K * c->K * 8);
    const size_t off_acc = A.take((size_t)c->n_chains * 8);
    const size_t off_err = A.take(8);
    c->arena_bytes = A.size;
    c->arena = c->dev_alloc(A.size);

    // couplings: generated on the host in parallel, or copied; int8 rows for
    // the MFMA contractions and bit-packed rows (bit 1 = -1, 8x fewer bytes)
    // for the field updates of the sweep
    // (a few samples: each one's passes run on several threads; many: the
    // samples do)
    const bool inner = jrep.size() < 4;
    maybe_parallel(!inner, jrep.size(), [&](size_t j) {
        const sg_sk_desc& r = d[jrep[j]];
        const int64_t n = r.n, wn = (n + 31) / 32;
        std::vector<int8_t> J;
        const int8_t* src = r.J;
        if (!src) {
            J.resize((size_t)(n * n));
            sk_generate(n, r.seed, r.graph_id, J.data(), inner);
            src = J.data();
        }
        hip_check(hipMemcpy(c->at<void>(off_J[j]), src, (size_t)(n * n), hipMemcpyHostToDevice));
        std::vector<uint32_t> Jb((size_t)(n * wn), 0u);
        maybe_parallel(inner, (size_t)n, [&](size_t ii) {
            const int64_t i = (int64_t)ii;
            for (int64_t k = 0; k < n; ++k)
                if (src[i * n + k] < 0) Jb[(size_t)(i * wn + (k >> 5))] |= 1u << (k & 31);
        });
        hip_check(hipMemcpy(c->at<void>(off_Jb[j]), Jb.data(), Jb.size() * 4, hipMemcpyHostToDevice));
        // the decider's tiles: row 64 b + l, words 2 bb and 2 bb + 1 for
        // bb = b - d (cyclic), d = 0..DW with DW = min(window, blocks - 1)
        const int64_t nb = (n + 63) / 64;
        const int64_t dw = std::min<int64_t>(sk_window(), nb - 1);
        std::vector<uint32_t> Jt((size_t)(nb * 64 * tile_words), 0u);
        for (int64_t b = 0; b < nb; ++b)
            for (int64_t l = 0; l < 64; ++l) {
                const int64_t row = 64 * b + l;
                if (row >= n) continue;
                for (int64_t dd = 0; dd <= dw; ++dd) {
                    const int64_t bb = (b - dd + nb) % nb;
                    for (int64_t h = 0; h < 2; ++h) {
                        const int64_t w = 2 * bb + h;
                        if (w < wn) Jt[(size_t)((b * 64 + l) * tile_words + 2 * dd + h)] = Jb[(size_t)(row * wn + w)];
                    }
                }
            }
        hip_check(hipMemcpy(c->at<void>(off_Jt[j]), Jt.data(), Jt.size() * 4, hipMemcpyHostToDevice));
    });
    for (int32_t i = 0; i < count; ++i)
        hip_check(hipMemcpy(c->at<void>(off_thr[(size_t)i]), thr[(size_t)i].data(), thr[(size_t)i].size() * 8,
                            hipMemcpyHostToDevice));

    c->sk.resize((size_t)c->n_chains);
    c->sks.resize((size_t)count);
    for (int32_t i = 0; i < count; ++i) {
        c->sks[(size_t)i] = SkSample{c->at<int8_t>(off_J[(size_t)jslot[(size_t)i]]), (int32_t)d[i].n, c->R,
                                     i * c->R, 0};
        for (int32_t r = 0; r < c->R; ++r) {
            const size_t ch = (size_t)(i * c->R + r);
            SkChain S;
            std::memset(&S, 0, sizeof(S));
            S.J = c->at<int8_t>(off_J[(size_t)jslot[(size_t)i]]);
            S.Jb = c->at<uint32_t>(off_Jb[(size_t)jslot[(size_t)i]]);
            S.Jt = c->at<uint32_t>(off_Jt[(size_t)jslot[(size_t)i]]);
            S.state = c->at<uint32_t>(off_state[ch]);
            S.H = c->at<int32_t>(off_H[ch]);
            S.snap = c->at<uint32_t>(off_snap[ch]);
            S.accepted = c->at<unsigned long long>(off_acc) + ch;
            // slope of log(thr[x] / 2^32) in x, a starting guess for the
            // kernel's exact search of the largest accepted x
            const double slope = 2.0 / d[i].T / std::sqrt((double)d[i].n);
            S.xslope = std::isinf(d[i].T) ? 0.0f : (d[i].T == 0.0 ? INFINITY : (float)slope);
            S.thr = c->at<uint64_t>(off_thr[(size_t)i]);
            S.seed = d[i].seed;
            S.inst = d[i].instance_id;
            S.rep = (uint32_t)r;
            S.n = (int32_t)d[i].n;
            S.words_n = (int32_t)((d[i].n + 31) / 32);
            S.thr_len = (int32_t)thr[(size_t)i].size();
            S.init_mode = d[i].start;
            S.sample = i;
            if (d[i].start == SG_START_GIVEN) {
                const auto bits = pack_given(d[i].s0 + (int64_t)r * d[i].n, d[i].n, nullptr);
                hip_check(hipMemcpy(c->at<void>(off_given[ch]), bits.data(), bits.size() * 4, hipMemcpyHostToDevice));
                S.given = c->at<uint32_t>(off_given[ch]);
            }
            c->sk[ch] = S;
        }
    }
    std::vector<MeasureChain> mc((size_t)c->n_chains);
    for (int32_t ch = 0; ch < c->n_chains; ++ch)
        mc[(size_t)ch] = MeasureChain{c->sk[(size_t)ch].snap, c->sk[(size_t)ch].words_n, c->sk[(size_t)ch].n};
    std::vector<int32_t> pairs;
    for (int32_t i = 0; i < count; ++i)
        for (int32_t a = 0; a < c->R; ++a)
            for (int32_t b = a + 1; b < c->R; ++b) {
                pairs.push_back(i * c->R + a);
                pairs.push_back(i * c->R + b);
            }
    c->sk_d = c->at<SkChain>(off_chains);
    c->sks_d = c->at<SkSample>(off_samples);
    c->mc_d = c->at<MeasureChain>(off_mc);
    c->pairs_d = c->at<int32_t>(off_pairs);
    c->bond_d = c->at<long long>(off_bond);
    c->overlap_d = c->at<long long>(off_ovl);
    c->gram_d = c->at<long long>(off_gram);
    c->acc_d = c->at<unsigned long long>(off_acc);
    c->err_d = c->at<int>(off_err);
    hip_check(hipMemcpy(c->sk_d, c->sk.data(), c->sk.size() * sizeof(SkChain), hipMemcpyHostToDevice));
    hip_check(hipMemcpy(c->sks_d, c->sks.data(), c->sks.size() * sizeof(SkSample), hipMemcpyHostToDevice));
    hip_check(hipMemcpy(c->mc_d, mc.data(), mc.size() * sizeof(MeasureChain), hipMemcpyHostToDevice));
    if (!pairs.empty())
        hip_check(hipMemcpy(c->pairs_d, pairs.data(), pairs.size() * 4, hipMemcpyHostToDevice));
    hip_check(zero_i64(c->bond_d, (size_t)c->n_chains * c->K, nullptr));
    hip_check(zero_i64((long long*)c->acc_d, (size_t)c->n_chains, nullptr));
    hip_check(zero_i64((long long*)c->err_d, 1, nullptr));
    c->sk_threads = sk_threads();
    c->sk_lds = sk_lds_bytes(c->sk_max_n);
    hip_check(sk_init(c->sk_d, c->n_chains, 256, nullptr));
    hip_check(sk_recompute(c->sks_d, count, c->sk_d, c->sk_max_n, 0, c->err_d, nullptr));
    hip_check(hipStreamSynchronize(nullptr));
}

// Enqueues the measurement kernels of every grid time reached (kd of them)
// on stream s: bond sums into bond[chains][K] (SK: 2 B, halved by the
// caller), overlaps into overlap[pairs][K], Gram matrices into
// gram[chains][K][K] (zeroed first: the kernel accumulates).  VB bond sums
// of the snapshots before k_first are taken as already in `bond` (a
// snapshot never changes once written).
void enqueue_obs(sg_ctx* c, int32_t kd, long long* bond, long long* overlap, long long* gram, hipStream_t s,
                 int32_t k_first = 0)
{
    const int32_t K = c->K;
    if (c->kind == 0) {
        hip_check(vb_bond(c->units_d, (int)c->units.size(), k_first, kd, bond, c->unit_chain_ids_d, K,
                          std::min(1024, c->vb_threads), c->bond_lds, s));
        hip_check(vbm_bond(c->vbm_d, (int)c->vbm.size(), k_first, kd, bond, c->vbm_ids_d, K, s));
    } else if (c->sk_real) {
        hip_check(zero_i64(bond, (size_t)c->n_chains * K, s));
        hip_check(skg_bond(c->sks_d, c->count, c->sk_d, c->sk_max_n, c->R, kd, K, c->bpart_d, c->bondr_d, s));
    } else {
        hip_check(zero_i64(bond, (size_t)c->n_chains * K, s));
        hip_check(sk_bond(c->sks_d, c->count, c->sk_d, c->sk_max_n, c->R, kd, K, bond, s));
    }
    hip_check(measure_overlap(c->mc_d, c->pairs_d, c->n_pairs, kd, K, overlap, s));
    hip_check(zero_i64(gram, (size_t)c->n_chains * K * K, s));
    hip_check(measure_gram(c->mc_d, c->n_chains, kd, K, c->max_words, gram, s));
}

// Number of terms of each windowed sum after the sweeps done so far: the
// times tau = 1 .. min(t_done, t_max) of interval m that exceed the waiting
// time times[k].  m(tau) does not decrease with tau, so interval m is the
// range [first(m), first(m + 1)), first(m) = the smallest tau with m(tau) >=
// m (a binary search; tau < 2^32).
void window_counts(const sg_ctx* c, int64_t* out)
{
    const int64_t T = std::min(c->t_done, c->t_max);
    int64_t first[kWindowBinsMax + 1];   // (no allocation: sg_measure_noalloc uses this too)
    for (int32_t m = 0; m <= c->n_bins; ++m) {
        uint64_t lo = 1, hi = 0xffffffffull;   // m(hi) = 127 >= m
        while (lo < hi) {
            const uint64_t mid = lo + (hi - lo) / 2;
            if (vb_window_bin(mid) >= m) hi = mid;
            else lo = mid + 1;
        }
        first[(size_t)m] = (int64_t)lo;
    }
    for (int32_t k = 0; k < c->kw; ++k)
        for (int32_t m = 0; m < c->n_bins; ++m) {
            const int64_t a = std::max(first[(size_t)m], c->times[(size_t)k] + 1);
            const int64_t b = std::min(first[(size_t)m + 1] - 1, T);
            out[(size_t)k * c->n_bins + m] = b >= a ? b - a + 1 : 0;
        }
}

static_assert(kWindowBinsMax >= 125, "m(t_max) + 1 <= 125 for t_max < 2^31");

// Copies the windowed sums (sg_obs.window, caller's host array, on stream s)
// and fills the counts; the caller synchronises s.
void window_out(sg_ctx* c, sg_obs* out, hipStream_t s)
{
    out->kw = c->kw;
    out->n_bins = c->n_bins;
    if (c->kw == 0) return;
    if (out->window)
        hip_check(hipMemcpyAsync(out->window, c->win_d, (size_t)c->n_chains * c->kw * c->n_bins * 8,
                                 hipMemcpyDeviceToHost, s));
    if (out->window_count) window_counts(c, out->window_count);
}

// Copies the real bond sums (SK with real couplings) into sg_obs.bond_real
// on stream s; grid times not reached yet are zeroed after the caller's
// synchronisation (bond_real_finish).
void bond_real_out(sg_ctx* c, sg_obs* out, hipStream_t s)
{
    if (!c->sk_real || !out->bond_real) return;
    hip_check(hipMemcpyAsync(out->bond_real, c->bondr_d, (size_t)c->n_chains * c->K * 8, hipMemcpyDeviceToHost, s));
}

void bond_real_finish(sg_ctx* c, sg_obs* out, int32_t kd)
{
    if (!c->sk_real || !out->bond_real) return;
    for (size_t i = 0; i < (size_t)c->n_chains * c->K; ++i)
        if ((int32_t)(i % c->K) >= kd) out->bond_real[i] = 0.0;
}

// After a resume (t_start > 0): the entries of the slots not taken (grid
// times not after t_start, times[k] = -1) are 0.  Their snapshot memory was
// never written, so whatever the measurement kernels made of it is dropped.
void mask_untaken(const sg_ctx* c, sg_obs* out)
{
    if (c->t_start == 0) return;
    const size_t K = (size_t)c->K;
    for (size_t k = 0; k < K; ++k) {
        if (c->times[k] >= 0) continue;
        for (size_t ch = 0; ch < (size_t)c->n_chains; ++ch) {
            if (out->bond) out->bond[ch * K + k] = 0;
            if (out->bond_real && c->sk_real) out->bond_real[ch * K + k] = 0.0;
            if (out->gram)
                for (size_t l = 0; l < K; ++l) {
                    out->gram[(ch * K + k) * K + l] = 0;
                    out->gram[(ch * K + l) * K + k] = 0;
                }
        }
        if (out->overlap)
            for (size_t p = 0; p < (size_t)c->n_pairs; ++p) out->overlap[p * K + k] = 0;
    }
}

// Status of a measurement from the context's error word.
sg_status status_of_flag(int err_flag)
{
    // a sweep pipeline stalled, a split unit's barrier timed out, or the VB
    // sweep kernel found its dynamic LDS away from offset 0
    if (err_flag & 14) return SG_EDEVICE;
    return (err_flag & 1) ? SG_EPARITY : SG_OK;
}

template <class F>
sg_status guarded(F&& f)
{
    try {
        f();
        return SG_OK;
    } catch (const Fail& e) {
        return e.code;
    } catch (const std::bad_alloc&) {
        return SG_ENOMEM;
    } catch (...) {
        return SG_EDEVICE;
    }
}

}  // namespace

extern "C" {

const char* sg_strerror(sg_status s)
{
    switch (s) {
        case SG_OK: return "ok";
        case SG_EINVAL: return "invalid argument";
        case SG_ENOMEM: return "out of memory";
        case SG_EDEVICE: return "HIP device error or no gfx950 device";
        case SG_ESTATE: return "invalid state";
        case SG_EPARITY: return "SK incremental fields disagree with the exact recompute";
        case SG_ENOTSUP: return "request outside supported limits";
        default: return "unknown status";
    }
}

sg_status sg_create_vb(const sg_vb_desc* d, int32_t count, const sg_opts* o, sg_ctx** out)
{
    if (!out) return SG_EINVAL;
    *out = nullptr;
    if (!d || count < 1) return SG_EINVAL;
    sg_ctx* c = nullptr;
    sg_status s = guarded([&]() {
        c = new sg_ctx();
        create_vb(c, d, count, o);
    });
    if (s != SG_OK) {
        if (c) {
            (void)hipDeviceSynchronize();
            c->release();
            delete c;
        }
        return s;
    }
    *out = c;
    return SG_OK;
}

sg_status sg_create_sk(const sg_sk_desc* d, int32_t count, const sg_opts* o, sg_ctx** out)
{
    if (!out) return SG_EINVAL;
    *out = nullptr;
    if (!d || count < 1) return SG_EINVAL;
    sg_ctx* c = nullptr;
    sg_status s = guarded([&]() {
        c = new sg_ctx();
        create_sk(c, d, count, o);
    });
    if (s != SG_OK) {
        if (c) {
            (void)hipDeviceSynchronize();
            c->release();
            delete c;
        }
        return s;
    }
    *out = c;
    return SG_OK;
}

sg_status sg_sweep(sg_ctx* c, int64_t n_sweeps, void* stream)
{
    if (!c || n_sweeps < 0) return SG_EINVAL;
    if (c->t_done + n_sweeps >= ((int64_t)1 << 32)) return SG_EINVAL;
    return guarded([&]() {
        hip_check(hipSetDevice(c->device));
        hipStream_t s = (hipStream_t)stream;
        c->note_stream(s);
        if (c->kind == 0) {
            const int64_t cap = std::max<int64_t>(
                1, std::min<int64_t>(4096, ((int64_t)1 << 36) / std::max<int64_t>(1, c->updates_per_sweep)));
            // launches of near-equal length (at most two distinct lengths),
            // so that no short launch trails a call
            const int64_t n_launch = (n_sweeps + cap - 1) / cap;
            int64_t left = n_sweeps;
            for (int64_t li = 0; li < n_launch; ++li) {
                const int64_t chunk = (left + (n_launch - li) - 1) / (n_launch - li);
                if (c->use_graph)
                    hip_check(hipGraphLaunch(vb_graph_for(c, (int32_t)chunk), s));
                else
                    vb_launch_chunk(c, (int32_t)chunk, s, c->t_dev, true);
                c->t_done += chunk;
                left -= chunk;
            }
        } else {
            int64_t left = n_sweeps;
            while (left > 0) {
                const int64_t to_check = c->period - (c->t_done % c->period);
                const int64_t chunk = std::min(left, to_check);
                if (c->sk_real)
                    hip_check(skg_sweep(c->sk_d, c->n_chains, c->sk_lds, c->t_done, (int32_t)chunk, c->t_max, s));
                else
                    hip_check(sk_sweep(c->sk_d, c->n_chains, c->sk_threads, c->sk_lds, c->t_done, (int32_t)chunk,
                                       c->t_max, c->err_d, s));
                c->t_done += chunk;
                left -= chunk;
                if (c->t_done % c->period == 0) {
                    if (c->sk_real)
                        hip_check(skg_recompute(c->sks_d, c->count, c->sk_d, c->sk_max_n, 1, c->err_d, s));
                    else
                        hip_check(sk_recompute(c->sks_d, c->count, c->sk_d, c->sk_max_n, 1, c->err_d, s));
                }
            }
        }
    });
}

sg_status sg_measure(sg_ctx* c, uint32_t flags, sg_obs* out, void* stream)
{
    if (!c || !out) return SG_EINVAL;
    int err_flag = 0;
    sg_status st = guarded([&]() {
        hip_check(hipSetDevice(c->device));
        hipStream_t s = (hipStream_t)stream;
        c->note_stream(s);
        const int32_t kd = c->k_done();
        const int32_t K = c->K, R = c->R;
        out->count = c->count;
        out->n_replicas = R;
        out->k_cap = K;
        out->k_done = kd;
        out->t_done = c->t_done;
        if (flags & SG_MEASURE_OBS) {
            // the context's bond array keeps the sums of earlier measurements
            enqueue_obs(c, kd, c->bond_d, c->overlap_d, c->gram_d, s, c->kind == 0 ? c->bond_done : 0);
            std::vector<long long> bond((size_t)c->n_chains * K), ovl((size_t)std::max(1, c->n_pairs) * K),
                gram((size_t)c->n_chains * K * K);
            std::vector<unsigned long long> acc((size_t)c->n_chains);
            hip_check(hipMemcpyAsync(bond.data(), c->bond_d, bond.size() * 8, hipMemcpyDeviceToHost, s));
            if (c->n_pairs)
                hip_check(hipMemcpyAsync(ovl.data(), c->overlap_d, (size_t)c->n_pairs * K * 8, hipMemcpyDeviceToHost, s));
            hip_check(hipMemcpyAsync(gram.data(), c->gram_d, gram.size() * 8, hipMemcpyDeviceToHost, s));
            hip_check(hipMemcpyAsync(acc.data(), c->acc_d, acc.size() * 8, hipMemcpyDeviceToHost, s));
            hip_check(hipMemcpyAsync(&err_flag, c->err_d, sizeof(int), hipMemcpyDeviceToHost, s));
            window_out(c, out, s);
            bond_real_out(c, out, s);
            hip_check(hipStreamSynchronize(s));
            c->bond_done = kd;
            bond_real_finish(c, out, kd);
            if (out->times)
                for (int32_t k = 0; k < K; ++k) out->times[k] = c->times[(size_t)k];
            if (out->bond)
                for (size_t i = 0; i < bond.size(); ++i)
                    out->bond[i] = (int64_t)i % K < kd ? (int64_t)bond[i] / (c->kind == 1 ? 2 : 1) : 0;
            if (out->overlap && c->n_pairs)
                for (size_t i = 0; i < (size_t)c->n_pairs * K; ++i)
                    out->overlap[i] = (int64_t)i % K < kd ? (int64_t)ovl[i] : 0;
            if (out->gram)
                for (size_t i = 0; i < gram.size(); ++i) out->gram[i] = (int64_t)gram[i];
            if (out->accepted)
                for (size_t i = 0; i < acc.size(); ++i) out->accepted[i] = (int64_t)acc[i];
            mask_untaken(c, out);
        }
        if ((flags & SG_MEASURE_SPINS) && out->spins) {
            hip_check(hipStreamSynchronize(s));
            int64_t base = 0;
            std::vector<int64_t> inst_base((size_t)c->count);
            for (int32_t i = 0; i < c->count; ++i) {
                inst_base[(size_t)i] = base;
                base += (int64_t)R * c->n_of[(size_t)i];
            }
            if (c->kind == 0) {
                std::vector<std::vector<uint32_t>> st(c->units.size());
                for (size_t u = 0; u < c->units.size(); ++u) {
                    st[u].resize((size_t)c->units[u].state_words);
                    hip_check(hipMemcpy(st[u].data(), c->units[u].state, st[u].size() * 4, hipMemcpyDeviceToHost));
                }
                std::vector<std::vector<uint64_t>> stm(c->vbm.size());
                for (size_t u = 0; u < c->vbm.size(); ++u) {
                    stm[u].resize((size_t)c->vbm[u].n);
                    hip_check(hipMemcpy(stm[u].data(), c->vbm[u].state, stm[u].size() * 8, hipMemcpyDeviceToHost));
                }
                for (int32_t ch = 0; ch < c->n_chains; ++ch) {
                    const int32_t u = c->chain_loc[(size_t)ch].first, k = c->chain_loc[(size_t)ch].second;
                    if (c->chain_ms[(size_t)ch]) {
                        const int32_t i = ch / R, r = ch % R;
                        const auto& order = c->order_of_group[(size_t)c->group_of_inst[(size_t)i]];
                        const int32_t nn = c->vbm[(size_t)u].n;
                        int8_t* dst = out->spins + inst_base[(size_t)i] + (int64_t)r * nn;
                        for (int64_t p = 0; p < nn; ++p)
                            dst[order[(size_t)p]] = ((stm[(size_t)u][(size_t)p] >> k) & 1ull) ? (int8_t)-1 : (int8_t)1;
                        continue;
                    }
                    const VbUnit& U = c->units[(size_t)u];
                    const int32_t i = ch / R, r = ch % R;
                    const auto& order = c->order_of_group[(size_t)c->group_of_inst[(size_t)i]];
                    int8_t* dst = out->spins + inst_base[(size_t)i] + (int64_t)r * U.n;
                    const VbLayout lay(U.rpad);
                    for (int64_t p = 0; p < U.n; ++p) {
                        const uint32_t bit =
                            (st[(size_t)u][(size_t)lay.word(p, k)] >> lay.bit(p, k)) & 1u;
                        dst[order[(size_t)p]] = bit ? (int8_t)-1 : (int8_t)1;
                    }
                }
            } else {
                for (int32_t ch = 0; ch < c->n_chains; ++ch) {
                    const SkChain& S = c->sk[(size_t)ch];
                    std::vector<uint32_t> st((size_t)S.words_n);
                    hip_check(hipMemcpy(st.data(), S.state, st.size() * 4, hipMemcpyDeviceToHost));
                    const int32_t i = ch / R, r = ch % R;
                    int8_t* dst = out->spins + inst_base[(size_t)i] + (int64_t)r * S.n;
                    for (int64_t p = 0; p < S.n; ++p)
                        dst[p] = ((st[(size_t)(p >> 5)] >> (p & 31)) & 1u) ? (int8_t)-1 : (int8_t)1;
                }
            }
        }
    });
    if (st != SG_OK) return st;
    return status_of_flag(err_flag);
}

sg_status sg_measure_noalloc(sg_ctx* c, sg_obs* out, void* stream)
{
    if (!c || !out) return SG_EINVAL;
    if (out->spins) return SG_EINVAL;   // spins need host staging: sg_measure only
    const size_t K = (size_t)c->K;
    const size_t n_bond = (size_t)c->n_chains * K, n_ovl = (size_t)c->n_pairs * K;
    const size_t n_gram = (size_t)c->n_chains * K * K;
    if (n_bond + n_ovl + n_gram > kMeasureScratchElems) return SG_ENOTSUP;
    int err_flag = 0;
    sg_status st = guarded([&]() {
        hip_check(hipSetDevice(c->device));
        long long* scr = nullptr;
        hip_check(measure_scratch(&scr));   // this device's copy of the fixed array
        // (the stream is not recorded for sg_free: this call waits for it)
        hipStream_t s = (hipStream_t)stream;
        const int32_t kd = c->k_done();
        out->count = c->count;
        out->n_replicas = c->R;
        out->k_cap = c->K;
        out->k_done = kd;
        out->t_done = c->t_done;
        long long* bond = scr;
        long long* ovl = scr + n_bond;
        long long* gram = ovl + n_ovl;
        enqueue_obs(c, kd, bond, ovl, gram, s);
        // straight into the caller's arrays (int64 on both sides)
        if (out->bond) hip_check(hipMemcpyAsync(out->bond, bond, n_bond * 8, hipMemcpyDeviceToHost, s));
        if (out->overlap && n_ovl)
            hip_check(hipMemcpyAsync(out->overlap, ovl, n_ovl * 8, hipMemcpyDeviceToHost, s));
        if (out->gram) hip_check(hipMemcpyAsync(out->gram, gram, n_gram * 8, hipMemcpyDeviceToHost, s));
        if (out->accepted)
            hip_check(hipMemcpyAsync(out->accepted, c->acc_d, (size_t)c->n_chains * 8, hipMemcpyDeviceToHost, s));
        hip_check(hipMemcpyAsync(&err_flag, c->err_d, sizeof(int), hipMemcpyDeviceToHost, s));
        window_out(c, out, s);
        bond_real_out(c, out, s);
        hip_check(hipStreamSynchronize(s));
        bond_real_finish(c, out, kd);
        if (out->times)
            for (size_t k = 0; k < K; ++k) out->times[k] = c->times[k];
        // entries of grid times not reached hold the previous call's values
        if (out->bond)
            for (size_t i = 0; i < n_bond; ++i)
                out->bond[i] = (int64_t)(i % K) < kd ? out->bond[i] / (c->kind == 1 ? 2 : 1) : 0;
        if (out->overlap)
            for (size_t i = 0; i < n_ovl; ++i)
                if ((int64_t)(i % K) >= kd) out->overlap[i] = 0;
        mask_untaken(c, out);
    });
    if (st != SG_OK) return st;
    return status_of_flag(err_flag);
}

void sg_free(sg_ctx* c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    c->sync_own();
    c->release();
    delete c;
}

sg_status sg_sk_corrupt_field(sg_ctx* c, int32_t instance, int32_t replica, int64_t i, int32_t delta)
{
    if (!c || c->kind != 1 || instance < 0 || instance >= c->count || replica < 0 || replica >= c->R)
        return SG_EINVAL;
    const SkChain& S = c->sk[(size_t)(instance * c->R + replica)];
    if (i < 0 || i >= S.n) return SG_EINVAL;
    return guarded([&]() {
        hip_check(hipSetDevice(c->device));
        c->sync_own();
        if (c->sk_real) {
            double h = 0.0;
            hip_check(hipMemcpy(&h, S.Hd + i, 8, hipMemcpyDeviceToHost));
            h += (double)delta;
            hip_check(hipMemcpy(S.Hd + i, &h, 8, hipMemcpyHostToDevice));
            return;
        }
        int32_t h = 0;
        hip_check(hipMemcpy(&h, S.H + i, 4, hipMemcpyDeviceToHost));
        h += delta;
        hip_check(hipMemcpy(S.H + i, &h, 4, hipMemcpyHostToDevice));
    });
}

sg_status sg_vb_inspect(const sg_vb_desc* d, sg_vb_tables* out)
{
    if (!d || !out) return SG_EINVAL;
    return guarded([&]() {
        check_vb_desc(*d);
        VbGraph g;
        build_vb_graph(*d, g);
        const size_t m = g.eu.size();
        out->n_edges = (int64_t)m;
        out->n_colours = g.ncls;
        out->max_degree = g.max_degree;
        if (out->edges)
            for (size_t e = 0; e < m; ++e) {
                out->edges[2 * e] = g.eu[e];
                out->edges[2 * e + 1] = g.ev[e];
            }
        if (out->J) std::memcpy(out->J, g.J.data(), m);
        if (out->colour) std::memcpy(out->colour, g.colour.data(), g.colour.size() * 4);
        if (out->order) std::memcpy(out->order, g.order.data(), g.order.size() * 4);
        if (out->row_start) std::memcpy(out->row_start, g.row.data(), g.row.size() * 4);
        if (out->entries) std::memcpy(out->entries, g.ent.data(), g.ent.size() * 4);
        if (out->thr)
            for (int32_t x = 0; x < kVbXMax; ++x) out->thr[x] = x == 0 ? (uint64_t)1 << 32 : threshold(d->T, 1.0, x);
    });
}

sg_status sg_sk_inspect(const sg_sk_desc* d, int8_t* J, uint64_t* thr)
{
    if (!d) return SG_EINVAL;
    if (d->Jf) return SG_EINVAL;   // binary couplings only
    return guarded([&]() {
        check_sk_desc(*d);
        const int64_t n = d->n;
        if (J) {
            if (d->J) std::memcpy(J, d->J, (size_t)(n * n));
            else sk_generate(n, d->seed, d->graph_id, J, true);
        }
        if (thr) {
            const double s = 1.0 / std::sqrt((double)n);
            thr[0] = (uint64_t)1 << 32;
            for (int64_t x = 1; x < n; ++x) thr[x] = threshold(d->T, s, x);
        }
    });
}

}  // extern "C"
