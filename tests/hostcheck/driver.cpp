// Runs the library's host runtime under AddressSanitizer / UndefinedBehaviorSanitizer
// against the HIP model (hip_model.cpp): every C ABI call sequence on the join shapes the
// GPU tests use, in recorded-graph, eager and profiling modes, plus the asynchronous
// calls, filter inserts, the filter catalogue and the server. Device columns and
// workspaces are host allocations of exactly the size the runtime asked for, so any
// host access past them is reported. Kernels do not run, so device-side counts read
// back as the zeros the workspace starts with.
//
// Usage: driver [scenario ...]   (no argument: every scenario). Exit status 0 when no
// call failed unexpectedly and the model saw no violation.
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "sievejoin.h"

extern "C" int hipmodel_violations();
extern "C" uint64_t hipmodel_launches();
extern "C" uint64_t hipmodel_graph_launches();
extern "C" uint64_t hipmodel_captures();
// caller-owned streams (declared here with the HIP runtime's C linkage and layout)
extern "C" int hipStreamCreateWithFlags(void **stream, unsigned flags);
extern "C" int hipStreamDestroy(void *stream);

namespace {

int g_fail = 0;

#define EXPECT(cond, ...)                                            \
    do {                                                             \
        if (!(cond)) {                                               \
            std::fprintf(stderr, "FAILED %s:%d: ", __FILE__, __LINE__); \
            std::fprintf(stderr, __VA_ARGS__);                       \
            std::fprintf(stderr, "\n");                              \
            ++g_fail;                                                \
        }                                                            \
    } while (0)

#define OK(ctx, expr)                                                                         \
    do {                                                                                      \
        sj_status s_ = (expr);                                                                \
        EXPECT(s_ == SJ_OK, "%s -> %d (%s)", #expr, s_, (ctx) ? sj_last_error(ctx) : "");     \
    } while (0)

void *dev_alloc(size_t bytes, size_t align = 256) {
    // exact-size allocation (rounded to the alignment only where aligned_alloc needs it)
    const size_t n = (bytes + align - 1) / align * align;
    void *p = std::aligned_alloc(align, n ? n : align);
    std::memset(p, 0, n ? n : align);
    return p;
}

struct Query {
    std::vector<std::vector<int32_t *>> cols;   // per relation, per column
    std::vector<std::vector<const int32_t *>> cptr;
    std::vector<sj_rel> rels;
    std::vector<sj_edge> edges;
    Query() = default;
    Query(const Query &) = delete;
    Query &operator=(const Query &) = delete;
    Query(Query &&o) noexcept
        : cols(std::move(o.cols)), cptr(std::move(o.cptr)), rels(std::move(o.rels)), edges(std::move(o.edges)) {
        o.cols.clear();
    }
    ~Query() {
        for (auto &r : cols)
            for (auto *c : r) std::free(c);
    }
    void add(int64_t rows, int ncols, int pred_col = -1, int32_t lo = 0, int32_t hi = 0) {
        std::vector<int32_t *> cs;
        for (int c = 0; c < ncols; ++c) {
            auto *p = static_cast<int32_t *>(dev_alloc(sizeof(int32_t) * rows, 16));
            for (int64_t i = 0; i < rows; ++i) p[i] = static_cast<int32_t>((i * 2654435761u + c) % 97);
            cs.push_back(p);
        }
        cols.push_back(cs);
        sj_rel r{};
        r.nrows = rows;
        r.ncols = ncols;
        r.pred_col = pred_col;
        r.pred_lo = lo;
        r.pred_hi = hi;
        rels.push_back(r);
    }
    void edge(int a, int ca, int b, int cb) { edges.push_back({a, ca, b, cb}); }
    void finish() {
        cptr.clear();
        for (auto &r : cols) cptr.emplace_back(r.begin(), r.end());
        for (size_t i = 0; i < rels.size(); ++i) rels[i].cols = cptr[i].data();
    }
};

Query tree(const std::vector<int> &parents, const std::vector<int64_t> &rows, int npreds) {
    Query q;
    for (size_t i = 0; i < rows.size(); ++i) {
        const bool pred = i > 0 && static_cast<int>(i) < npreds;
        q.add(rows[i], 2, pred ? 1 : -1, 0, 50);
    }
    for (size_t i = 1; i < rows.size(); ++i) q.edge(parents[i], static_cast<int>(i % 2), static_cast<int>(i), 0);
    q.finish();
    return q;
}

Query chain(int n, int64_t rows) {
    Query q;
    for (int i = 0; i < n; ++i) q.add(rows, 2);
    for (int i = 1; i < n; ++i) q.edge(i - 1, 1, i, 0);
    q.finish();
    return q;
}

Query star(int dims, int64_t fact, int64_t dim_rows) {
    Query q;
    q.add(fact, dims);
    for (int d = 0; d < dims; ++d) q.add(dim_rows, 2, 1, 0, 10);
    for (int d = 0; d < dims; ++d) q.edge(0, d, d + 1, 0);
    q.finish();
    return q;
}

Query cycle(int n, int64_t rows) {
    Query q;
    for (int i = 0; i < n; ++i) q.add(rows, 2);
    for (int i = 0; i < n; ++i) q.edge(i, 1, (i + 1) % n, 0);
    q.finish();
    return q;
}

enum Mode { kGraph, kEager, kProfile };

struct Run {
    sj_ctx *ctx = nullptr;
    sj_plan_t *plan = nullptr;
    void *ws = nullptr;
    uint64_t wsb = 0;
    ~Run() {
        if (plan) sj_plan_destroy(plan);
        if (ctx) sj_ctx_destroy(ctx);
        std::free(ws);
    }
};

sj_status make_plan(Run &r, Query &q, Mode mode, uint32_t passes = 2, uint32_t extra_flags = 0, int root = -1) {
    OK(nullptr, sj_ctx_create(0, nullptr, &r.ctx));
    sj_opts o{};
    o.bits_per_key = 8;
    o.k = 6;
    o.block_bits = 512;
    o.passes = passes;
    o.seed = 7;
    o.root = root;
    o.flags = extra_flags | (mode == kEager ? SJ_FLAG_EAGER : 0u) | (mode == kProfile ? SJ_FLAG_PROFILE : 0u);
    sj_status st = sj_plan(r.ctx, q.rels.data(), static_cast<int32_t>(q.rels.size()), q.edges.data(),
                           static_cast<int32_t>(q.edges.size()), &o, &r.plan, &r.wsb);
    if (st != SJ_OK) return st;
    r.ws = dev_alloc(r.wsb);
    return sj_bind_workspace(r.plan, r.ws, r.wsb);
}

// set while a 4-clique query runs (its count pass also runs asynchronously)
bool g_clique = false;

// plan -> filters -> sieve -> join -> result, `reps` times, then the asynchronous calls
void full_run(const char *name, Query &q, Mode mode, int reps, uint32_t passes = 2, uint32_t flags = 0,
              bool expect_join_ok = true) {
    Run r;
    sj_status st = make_plan(r, q, mode, passes, flags);
    EXPECT(st == SJ_OK, "%s: plan/bind -> %d (%s)", name, st, sj_last_error(r.ctx));
    if (st != SJ_OK) return;
    const size_t nrels = q.rels.size();
    for (int i = 0; i < reps; ++i) {
        OK(r.ctx, sj_build_filters(r.plan));
        std::vector<uint64_t> surv(nrels);
        OK(r.ctx, sj_sieve(r.plan, i == 0 ? surv.data() : nullptr));
        uint64_t cnt = 1, chk = 1;
        st = sj_join(r.plan, &cnt, &chk);
        if (!expect_join_ok) {
            EXPECT(st == SJ_ERR_UNSUPPORTED, "%s: sj_join -> %d, expected SJ_ERR_UNSUPPORTED", name, st);
            return;
        }
        EXPECT(st == SJ_OK, "%s: sj_join -> %d (%s)", name, st, sj_last_error(r.ctx));
        void *rb = dev_alloc(0);
        OK(r.ctx, sj_result(r.plan, static_cast<int32_t *>(rb), 0, SJ_RIDS));
        OK(r.ctx, sj_result(r.plan, static_cast<int32_t *>(rb), 0, SJ_VALUES));
        std::free(rb);
        uint64_t wsb = 0, rbytes = 0;
        int32_t width = 0;
        OK(r.ctx, sj_plan_footprint(r.plan, SJ_VALUES, &wsb, &rbytes, &width));
        int32_t nf = 0;
        OK(r.ctx, sj_filter_count(r.plan, &nf));
        for (int f = 0; f < nf; ++f) {
            int32_t kind, index, rel, col;
            uint32_t nb = 0;
            OK(r.ctx, sj_filter_desc(r.plan, f, &kind, &index, &rel, &col, &nb));
        }
        for (size_t j = 0; j < nrels; ++j) {
            uint64_t n = 0;
            OK(r.ctx, sj_survivors_copy(r.plan, static_cast<int32_t>(j), nullptr, 0, &n));
        }
    }
    const bool cyclic = q.edges.size() >= q.rels.size();
    if (!cyclic || ((nrels == 3 || g_clique) && !(flags & SJ_FLAG_BINARY_CYCLES))) {
        OK(r.ctx, sj_build_filters(r.plan));
        OK(r.ctx, sj_sieve(r.plan, nullptr));
        st = sj_join_async(r.plan);
        EXPECT(st == SJ_OK, "%s: sj_join_async -> %d (%s)", name, st, sj_last_error(r.ctx));
        if (!cyclic) {
            auto *buf = static_cast<int32_t *>(dev_alloc(sizeof(int32_t) * 64 * nrels));
            OK(r.ctx, sj_result_async(r.plan, buf, 64, SJ_RIDS));
            uint64_t c, k;
            sj_status rs = 0;
            OK(r.ctx, sj_join_wait(r.plan, &c, &k, &rs));
            OK(r.ctx, sj_build_filters(r.plan));
            OK(r.ctx, sj_sieve(r.plan, nullptr));
            OK(r.ctx, sj_join_async(r.plan));
            const int32_t proj[4] = {0, 0, static_cast<int32_t>(nrels - 1), 1};
            OK(r.ctx, sj_plan_set_projection(r.plan, proj, 2));
            OK(r.ctx, sj_result_async(r.plan, buf, 32, SJ_VALUES));
            OK(r.ctx, sj_join_wait(r.plan, &c, &k, &rs));
            std::free(buf);
        }
    }
    if (mode == kProfile) {
        OK(r.ctx, sj_profile_collect(r.plan));
        int32_t n = 0;
        OK(r.ctx, sj_profile_count(r.plan, &n));
        EXPECT(n > 0, "%s: no profile entries", name);
        for (int i = 0; i < n; ++i) {
            const char *label;
            double ms;
            uint64_t l, b;
            OK(r.ctx, sj_profile_entry(r.plan, i, &label, &ms, &l, &b));
        }
        OK(r.ctx, sj_profile_reset(r.plan));
    }
}

void all_modes(const char *name, Query &q, uint32_t passes = 2, uint32_t flags = 0, bool join_ok = true) {
    full_run(name, q, kGraph, 3, passes, flags, join_ok);
    full_run(name, q, kEager, 1, passes, flags, join_ok);
    full_run(name, q, kProfile, 1, passes, flags, join_ok);
}

void scenario_chain() {
    Query q = chain(4, 1000);
    all_modes("chain4", q);
    all_modes("chain4 one pass", q, 1);
    all_modes("chain4 sieve in two launches", q, 2, SJ_FLAG_SIEVE_TWO_LAUNCHES);
    Query e = chain(2, 0);   // empty relations
    all_modes("empty chain", e);
}

void scenario_star() {
    Query q = star(7, 6000, 300);
    all_modes("star7", q);
    all_modes("star7 one pass", q, 1);
}

void scenario_bushy() {
    //            0
    //      1     2     3
    //     4 5   6 7   8 9
    Query q = tree({-1, 0, 0, 0, 1, 1, 2, 2, 3, 3}, {3000, 900, 1100, 800, 500, 700, 600, 400, 900, 300}, 6);
    all_modes("bushy tree", q);
}

void scenario_binary_tree() {
    Query q = tree({-1, 0, 0, 1, 1, 2, 2}, {2500, 800, 900, 500, 600, 400, 700}, 4);
    all_modes("binary tree of seven", q);
}

void scenario_chain12() {
    std::vector<int> parents(12);
    for (int i = 0; i < 12; ++i) parents[i] = i - 1;
    Query q = tree(parents, std::vector<int64_t>(12, 400), 0);
    all_modes("twelve-relation chain", q);
}

void scenario_sixteen() {
    std::vector<int> parents(16);
    for (int i = 0; i < 16; ++i) parents[i] = i == 0 ? -1 : (i - 1) / 2;
    Query q = tree(parents, std::vector<int64_t>(16, 300), 8);
    all_modes("sixteen-relation binary tree", q);
}

void scenario_cycles() {
    Query t = cycle(3, 700);
    all_modes("triangle", t);
    all_modes("triangle binary", t, 2, SJ_FLAG_BINARY_CYCLES);
    all_modes("triangle one pass", t, 1);
    Query c4 = cycle(4, 500);
    all_modes("4-cycle", c4);
    // a chain 0-1-2-3 with a closing edge 0-2 (between two relations before the last of
    // the preorder: checked per prefix) and one 1-3 on another column of relation 3
    Query u;
    for (int i = 0; i < 4; ++i) u.add(300, 3);
    u.edge(0, 1, 1, 0);
    u.edge(1, 1, 2, 0);
    u.edge(2, 1, 3, 0);
    u.edge(0, 2, 2, 2);
    u.edge(1, 2, 3, 2);
    u.finish();
    all_modes("general cycles", u);
    // more closing edges than the binary plan takes: refused
    Query w;
    for (int i = 0; i < 3; ++i) w.add(200, 6);
    w.edge(0, 0, 1, 0);
    w.edge(1, 1, 2, 0);
    for (int c = 1; c <= 5; ++c) w.edge(0, c, 2, c);
    w.finish();
    all_modes("too many closing edges", w, 2, 0, false);
    // the 4-clique: relations ab, ac, ad, bc, bd, cd, each variable joining its three
    // relations by two edges; counted and written by intersection (the binary plan
    // refuses it)
    Query k;
    for (int i = 0; i < 6; ++i) k.add(400 + 50 * i, 2);
    const int ke[8][4] = {{0, 0, 1, 0}, {0, 0, 2, 0}, {0, 1, 3, 0}, {0, 1, 4, 0},
                          {1, 1, 3, 1}, {1, 1, 5, 0}, {2, 1, 4, 1}, {2, 1, 5, 1}};
    for (const auto &e : ke) k.edge(e[0], e[1], e[2], e[3]);
    k.finish();
    g_clique = true;
    all_modes("4-clique", k);
    all_modes("4-clique one pass", k, 1);
    g_clique = false;
    all_modes("4-clique binary", k, 2, SJ_FLAG_BINARY_CYCLES);
}

void scenario_updates() {
    Query q = chain(3, 2000);
    Run r;
    OK(r.ctx, make_plan(r, q, kGraph));
    OK(r.ctx, sj_build_filters(r.plan));
    auto *keys = static_cast<int32_t *>(dev_alloc(4 * 100, 16));
    auto *flags = static_cast<uint8_t *>(dev_alloc(100, 16));
    uint64_t miss = 0;
    OK(r.ctx, sj_filter_probe(r.plan, 0, keys, 100, flags, &miss));
    OK(r.ctx, sj_filter_insert(r.plan, 0, keys, 100, flags, &miss));
    EXPECT(sj_filter_insert(r.plan, 3, keys, 100, flags, &miss) == SJ_ERR_STATE, "forward filter before sieve");
    OK(r.ctx, sj_sieve(r.plan, nullptr));
    OK(r.ctx, sj_filter_insert(r.plan, 3, keys, 100, flags, nullptr));
    EXPECT(sj_filter_insert(r.plan, 99, keys, 100, flags, &miss) == SJ_ERR_INVALID, "filter index");
    std::free(keys);
    std::free(flags);
}

void scenario_maintain() {
    Query q = chain(4, 2000);
    Run r;
    OK(r.ctx, make_plan(r, q, kGraph, 1));
    OK(r.ctx, sj_build_filters(r.plan));
    uint64_t bytes = 0;
    OK(r.ctx, sj_filter_propagate_scratch(r.plan, 3, 100, &bytes));
    void *scratch = dev_alloc(bytes);
    std::vector<int32_t *> cols;
    for (int c = 0; c < 2; ++c) cols.push_back(static_cast<int32_t *>(dev_alloc(400, 16)));
    std::vector<const int32_t *> cptr(cols.begin(), cols.end());
    uint64_t ins[4];
    OK(r.ctx, sj_filter_propagate(r.plan, 3, cptr.data(), 100, scratch, bytes, ins));
    EXPECT(sj_filter_propagate(r.plan, 3, cptr.data(), 100, scratch, bytes - 1, ins) == SJ_ERR_NOMEM, "small scratch");
    OK(r.ctx, sj_filter_propagate(r.plan, 0, cptr.data(), 100, scratch, bytes, ins));   // the root: nothing
    int32_t nf = 0;
    OK(r.ctx, sj_filter_count(r.plan, &nf));
    for (int f = 0; f < nf; ++f) {
        // the model's counts read back as zero blocks: a counting filter of one block's worth
        sj_cfilter *cf = nullptr;
        void *counts = dev_alloc(4096);
        const sj_status st = sj_plan_cfilter(r.plan, f, counts, 4096, &cf);
        EXPECT(st == SJ_OK, "sj_plan_cfilter -> %d (%s)", st, sj_last_error(r.ctx));
        if (cf) {
            OK(r.ctx, sj_cfilter_update(cf, cptr[0], 100, +1));
            OK(r.ctx, sj_cfilter_update(cf, cptr[0], 100, -1));
            EXPECT(sj_cfilter_update(cf, cptr[0], 100, 2) == SJ_ERR_INVALID, "sign");
            void *flags = dev_alloc(128);
            uint64_t miss = 0;
            OK(r.ctx, sj_cfilter_probe(cf, cptr[0], 100, static_cast<uint8_t *>(flags), &miss));
            void *words = dev_alloc(4096);
            OK(r.ctx, sj_cfilter_export(cf, static_cast<uint32_t *>(words), 1024));
            OK(r.ctx, sj_cfilter_apply(cf, r.plan, f));
            OK(r.ctx, sj_cfilter_destroy(cf));
            std::free(flags);
            std::free(words);
        }
        std::free(counts);
    }
    for (auto *c : cols) std::free(c);
    std::free(scratch);
}

void scenario_fcache() {
    Query q = chain(4, 1500);
    const uint64_t arena_bytes = 1 << 20;
    void *arena = dev_alloc(arena_bytes);
    sj_fcache *fc = nullptr;
    OK(nullptr, sj_fcache_create(0, arena, arena_bytes, &fc));
    for (Mode m : {kGraph, kEager}) {
        Run a, b;
        OK(a.ctx, make_plan(a, q, m));
        OK(b.ctx, make_plan(b, q, m));
        OK(a.ctx, sj_plan_use_filter_cache(a.plan, fc));
        OK(a.ctx, sj_build_filters(a.plan));
        OK(a.ctx, sj_sieve(a.plan, nullptr));
        uint64_t c, k;
        OK(a.ctx, sj_join(a.plan, &c, &k));
        OK(b.ctx, sj_plan_use_filter_cache(b.plan, fc));
        for (int rep = 0; rep < 2; ++rep) {
            OK(b.ctx, sj_build_filters(b.plan));
            OK(b.ctx, sj_sieve(b.plan, nullptr));
            OK(b.ctx, sj_join(b.plan, &c, &k));
        }
        int32_t how = -1;
        OK(b.ctx, sj_plan_filter_cached(b.plan, 0, &how));
        OK(nullptr, sj_fcache_invalidate(fc, q.rels[3].cols[0]));
        sj_fcache_info info{};
        OK(nullptr, sj_fcache_stats(fc, &info));
        // the context first, then the plan (plans keep their context alive)
        sj_ctx_destroy(a.ctx);
        a.ctx = nullptr;
        sj_plan_destroy(a.plan);
        a.plan = nullptr;
        OK(b.ctx, sj_plan_use_filter_cache(b.plan, nullptr));
    }
    {   // a plan attached to the catalogue outlives its context and the context's stream
        void *stream = nullptr;
        EXPECT(hipStreamCreateWithFlags(&stream, 1) == 0, "stream");
        sj_ctx *ctx = nullptr;
        OK(nullptr, sj_ctx_create(0, stream, &ctx));
        sj_opts o{};
        sj_plan_t *plan = nullptr;
        uint64_t wsb = 0;
        OK(ctx, sj_plan(ctx, q.rels.data(), 4, q.edges.data(), 3, &o, &plan, &wsb));
        void *ws = dev_alloc(wsb);
        OK(ctx, sj_bind_workspace(plan, ws, wsb));
        OK(ctx, sj_plan_use_filter_cache(plan, fc));
        OK(ctx, sj_build_filters(plan));
        OK(ctx, sj_sieve(plan, nullptr));
        sj_ctx_destroy(ctx);
        hipStreamDestroy(stream);
        sj_plan_destroy(plan);
        std::free(ws);
    }
    OK(nullptr, sj_fcache_clear(fc));
    OK(nullptr, sj_fcache_destroy(fc));
    std::free(arena);
}

void scenario_server() {
    const uint64_t arena_bytes = 64ull << 20;
    void *arena = dev_alloc(arena_bytes);
    sj_server *srv = nullptr;
    OK(nullptr, sj_server_create(0, arena, arena_bytes, 3, &srv));
    sj_fcache *fc = nullptr;
    void *fca = dev_alloc(1 << 20);
    OK(nullptr, sj_fcache_create(0, fca, 1 << 20, &fc));
    OK(nullptr, sj_server_use_filter_cache(srv, fc));
    std::vector<Query> qs;
    qs.push_back(chain(3, 3000));
    qs.push_back(star(4, 5000, 200));
    qs.push_back(chain(5, 800));
    qs.push_back(cycle(3, 600));
    std::vector<uint64_t> tickets;
    const int32_t modes[3] = {SJ_RESULT_TUPLES, SJ_RESULT_COUNT, SJ_RESULT_VALUES};
    std::vector<bool> faulty;
    for (int rep = 0; rep < 3; ++rep)
        for (size_t qi = 0; qi < qs.size(); ++qi) {
            Query &q = qs[qi];
            uint64_t t = 0;
            sj_opts o{};
            o.seed = 3;
            const bool fault = rep == 1 && qi == 1;
            if (fault) o.flags = SJ_FLAG_FAULT_SIEVE;
            const sj_status st = sj_server_submit(srv, q.rels.data(), static_cast<int32_t>(q.rels.size()),
                                                  q.edges.data(), static_cast<int32_t>(q.edges.size()), &o,
                                                  modes[rep], &t);
            EXPECT(st == SJ_OK, "server submit -> %d (%s)", st, sj_server_last_error(srv));
            tickets.push_back(t);
            faulty.push_back(fault);
        }
    for (size_t i = 0; i < tickets.size(); ++i) {
        const uint64_t t = tickets[i];
        sj_query_info info{};
        OK(nullptr, sj_server_query(srv, t, 1, &info));
        if (faulty[i])
            EXPECT(info.state == SJ_QUERY_FAILED && info.status == SJ_ERR_DEVICE, "injected failure: state %d",
                   info.state);
        else
            EXPECT(info.state == SJ_QUERY_DONE, "query %llu state %d: %s", static_cast<unsigned long long>(t),
                   info.state, info.error);
        OK(nullptr, sj_server_release(srv, t));
    }
    uint64_t used, peak;
    int32_t queued, running;
    OK(nullptr, sj_server_stats(srv, &used, &peak, &queued, &running));
    OK(nullptr, sj_server_use_filter_cache(srv, nullptr));
    OK(nullptr, sj_server_destroy(srv));
    OK(nullptr, sj_fcache_destroy(fc));
    std::free(arena);
    std::free(fca);
}

void scenario_errors() {
    Query q = chain(3, 100);
    Run r;
    OK(nullptr, sj_ctx_create(0, nullptr, &r.ctx));
    sj_opts o{};
    o.k = 13;
    EXPECT(sj_plan(r.ctx, q.rels.data(), 3, q.edges.data(), 2, &o, &r.plan, &r.wsb) == SJ_ERR_INVALID, "k = 13");
    o.k = 0;
    sj_edge bad[2] = {{0, 1, 0, 0}, {1, 1, 2, 0}};
    EXPECT(sj_plan(r.ctx, q.rels.data(), 3, bad, 2, &o, &r.plan, &r.wsb) == SJ_ERR_GRAPH, "self edge");
    EXPECT(sj_plan(r.ctx, q.rels.data(), 3, q.edges.data(), 1, &o, &r.plan, &r.wsb) == SJ_ERR_GRAPH, "disconnected");
    OK(r.ctx, sj_plan(r.ctx, q.rels.data(), 3, q.edges.data(), 2, &o, &r.plan, &r.wsb));
    EXPECT(sj_build_filters(r.plan) == SJ_ERR_STATE, "filters before bind");
    r.ws = dev_alloc(r.wsb);
    EXPECT(sj_bind_workspace(r.plan, r.ws, r.wsb - 1) == SJ_ERR_NOMEM, "small workspace");
    OK(r.ctx, sj_bind_workspace(r.plan, r.ws, r.wsb));
    EXPECT(sj_join(r.plan, nullptr, nullptr) == SJ_ERR_STATE, "join before sieve");
}

void scenario_static() {
    Query q = chain(3, 20000);
    for (int rep = 0; rep < 2; ++rep) {
        Run r;
        OK(nullptr, sj_ctx_create(0, nullptr, &r.ctx));
        sj_opts o{};
        OK(r.ctx, sj_plan(r.ctx, q.rels.data(), 3, q.edges.data(), 2, &o, &r.plan, &r.wsb));
        OK(r.ctx, sj_bind_static_workspace(r.plan));
        OK(r.ctx, sj_build_filters(r.plan));
        OK(r.ctx, sj_sieve(r.plan, nullptr));
        uint64_t c, k;
        OK(r.ctx, sj_join(r.plan, &c, &k));
    }
    Query big = chain(3, 2000000);
    Run r;
    OK(nullptr, sj_ctx_create(0, nullptr, &r.ctx));
    sj_opts o{};
    OK(r.ctx, sj_plan(r.ctx, big.rels.data(), 3, big.edges.data(), 2, &o, &r.plan, &r.wsb));
    EXPECT(sj_bind_static_workspace(r.plan) == SJ_ERR_NOMEM, "a plan larger than the static workspace");
    EXPECT(sj_build_filters(r.plan) == SJ_ERR_STATE, "nothing was bound");
}

void scenario_batch() {
    std::vector<Query> qs;
    qs.push_back(chain(3, 3000));
    qs.push_back(star(4, 5000, 300));
    qs.push_back(cycle(3, 800));
    qs.push_back(chain(5, 700));
    sj_ctx *ctx = nullptr;
    OK(nullptr, sj_ctx_create(0, nullptr, &ctx));
    std::vector<sj_plan_t *> plans;
    std::vector<void *> mem;
    for (auto &q : qs) {
        sj_opts o{};
        sj_plan_t *p = nullptr;
        uint64_t wsb = 0;
        OK(ctx, sj_plan(ctx, q.rels.data(), static_cast<int32_t>(q.rels.size()), q.edges.data(),
                        static_cast<int32_t>(q.edges.size()), &o, &p, &wsb));
        mem.push_back(dev_alloc(wsb));
        OK(ctx, sj_bind_workspace(p, mem.back(), wsb));
        plans.push_back(p);
    }
    sj_batch *b = nullptr;
    OK(ctx, sj_batch_create(ctx, plans.data(), static_cast<int32_t>(plans.size()), &b));
    std::vector<int32_t *> outs(plans.size(), nullptr);
    std::vector<uint64_t> caps(plans.size(), 64);
    for (size_t i = 0; i < plans.size(); ++i) {
        if (i == 2) continue;   // the 3-cycle: count only
        mem.push_back(dev_alloc(64 * 8 * 4));
        outs[i] = static_cast<int32_t *>(mem.back());
    }
#ifdef SJ_BATCH_ENABLED
    for (int rep = 0; rep < 3; ++rep) {
        OK(ctx, sj_batch_submit(b, outs.data(), caps.data(), rep == 2 ? SJ_VALUES : SJ_RIDS));
        for (auto *p : plans) {
            uint64_t c, k;
            sj_status rs;
            OK(ctx, sj_join_wait(p, &c, &k, &rs));
        }
    }
    OK(ctx, sj_batch_submit(b, nullptr, nullptr, SJ_RIDS));
    EXPECT(sj_batch_submit(b, outs.data(), caps.data(), 5) == SJ_ERR_INVALID, "bad mode");
    outs[2] = outs[0];
    EXPECT(sj_batch_submit(b, outs.data(), caps.data(), SJ_RIDS) == SJ_ERR_UNSUPPORTED, "cyclic tuples");
#else
    EXPECT(sj_batch_submit(b, outs.data(), caps.data(), SJ_RIDS) == SJ_ERR_UNSUPPORTED, "switched off");
#endif
    OK(ctx, sj_batch_destroy(b));
    sj_plan_t *twice[2] = {plans[0], plans[0]};
    EXPECT(sj_batch_create(ctx, twice, 2, &b) == SJ_ERR_INVALID, "a plan twice");
    for (auto *p : plans) sj_plan_destroy(p);
    sj_ctx_destroy(ctx);
    for (void *m : mem) std::free(m);
}

struct Scenario {
    const char *name;
    void (*fn)();
};
const Scenario kScenarios[] = {
    {"chain", scenario_chain},   {"star", scenario_star},       {"bushy", scenario_bushy},
    {"binary", scenario_binary_tree}, {"chain12", scenario_chain12}, {"sixteen", scenario_sixteen},
    {"cycles", scenario_cycles}, {"updates", scenario_updates}, {"fcache", scenario_fcache},
    {"server", scenario_server}, {"errors", scenario_errors}, {"static", scenario_static},
    {"batch", scenario_batch}, {"maintain", scenario_maintain},
};

}  // namespace

int main(int argc, char **argv) {
    for (const auto &s : kScenarios) {
        bool run = argc < 2;
        for (int i = 1; i < argc; ++i) run |= std::strcmp(argv[i], s.name) == 0;
        if (!run) continue;
        const int f0 = g_fail, v0 = hipmodel_violations();
        s.fn();
        std::printf("scenario %-8s failures %d violations %d\n", s.name, g_fail - f0, hipmodel_violations() - v0);
        std::fflush(stdout);
    }
    std::printf("launches %llu graph launches %llu captures %llu\n",
                static_cast<unsigned long long>(hipmodel_launches()),
                static_cast<unsigned long long>(hipmodel_graph_launches()),
                static_cast<unsigned long long>(hipmodel_captures()));
    return (g_fail || hipmodel_violations()) ? 1 : 0;
}
