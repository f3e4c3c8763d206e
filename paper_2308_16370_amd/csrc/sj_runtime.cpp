// Host runtime behind the C ABI in include/sievejoin.h: join-graph validation, the
// spanning tree and filter schedule, the workspace layout, the call-order state
// machine, and the sequencing of the kernels on the context's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "sievejoin.h"
#include "sj_fcache.h"
#include "sj_internal.h"

using namespace sj;

struct sj_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    std::atomic<int> refs{1};   // the creator's reference and one per plan
};

// A context lives until its creator has destroyed it and every plan made on it is gone,
// so plans may be destroyed after their context in any order.
static void ctx_release(sj_ctx *c) {
    if (c && c->refs.fetch_sub(1, std::memory_order_acq_rel) == 1) delete c;
}

namespace {

enum State { kPlanned = 0, kBound = 1, kFiltered = 2, kSieved = 3, kJoined = 4 };
enum Src { kFull = -1 };

struct Rel {
    uint32_t nrows = 0;
    std::vector<const int32_t *> cols;
    int pred_col = -1;
    int32_t lo = 0, hi = 0;
    std::vector<int> jcols;    // distinct join columns, ascending
    int jidx(int col) const {
        for (size_t i = 0; i < jcols.size(); ++i)
            if (jcols[i] == col) return static_cast<int>(i);
        return -1;
    }
};

struct Closing {
    int u, cu, v, cv;
};

struct Filter {
    int kind, index, src_rel, src_col;
    uint64_t max_words = 0;
    uint64_t off = 0;          // workspace offset of the words
    // filter catalogue: words and block count in a catalogue entry instead
    FcEntry *fc = nullptr;
    uint32_t *ext_words = nullptr, *ext_nblocks = nullptr;
    int fc_how = 0;            // 0 workspace, 1 reused, 2 built by this plan into the entry
    bool fc_pending = false;   // fc_how 2 and not built yet
    bool resident() const { return fc_how == 1 || (fc_how == 2 && !fc_pending); }
};

struct StepSpec {
    int phase;                 // 0: build_filters, 1: sieve
    int rel;
    int src;                   // kFull or list buffer 0/1
    int src_step = -1;         // step that wrote the source list
    std::vector<std::pair<int, int>> probes;   // (jcol index, filter)
    std::vector<std::pair<int, int>> builds;
    int out = -1;              // list buffer written, -1: none
    uint64_t off_count = 0;
    uint32_t max_rows = 0;
    std::vector<uint64_t> off_bstatus, off_bcounter, off_btotal;   // per build
    uint64_t off_pstatus = 0, off_pcounter = 0;                   // look-back of the one-launch scan
    int level = 0;             // steps of one phase and level are independent of each other
    int branch = 0;            // its branch stream and scratch set inside the level
    bool alone = false;        // the only step of its level: its builds take a branch each
    int build_set(size_t b) const { return alone ? static_cast<int>(b % 4) : branch; }
};

struct Region {
    uint64_t begin = 0, end = 0;
};

struct Layout {
    uint64_t top = 0;
    uint64_t take(uint64_t bytes) {
        const uint64_t o = top;
        top += (bytes + 255) & ~uint64_t(255);
        return o;
    }
};

}  // namespace

struct sj_plan_s {
    sj_ctx *ctx = nullptr;
    int n = 0;
    std::vector<Rel> rels;
    std::vector<sj_edge> edges;
    sj_opts opts{};
    int logB = 9;
    uint32_t seed32 = 0;
    // tree
    int root = 0;
    std::vector<int> parent, pcol, mycol, preorder, postorder;
    std::vector<std::vector<int>> children;
    std::vector<Closing> closing;
    // filters and steps
    std::vector<Filter> filters;
    std::vector<int> f_bwd, f_fwd;           // per relation, -1 none
    std::vector<int> f_close;                // per closing edge
    std::vector<StepSpec> steps;
    std::vector<int> final_list, final_step; // per relation
    // workspace
    uint64_t ws_bytes = 0;
    char *ws = nullptr;
    Region zero[3];                          // build_filters, sieve, join
    uint64_t off_elig = 0, off_nblocks = 0, off_totals = 0;
    uint64_t off_upd = 0;                    // missing-key counter of sj_filter_probe / sj_filter_insert
    uint32_t region_blocks = 0;
    // probe and build scratch, one set per branch: survivor bits, per-workgroup counts,
    // region histogram, staged keys, kept-key bitmap
    static constexpr int kSets = 4;
    uint64_t off_sbits[kSets] = {}, off_scounts[kSets] = {}, off_bhist[kSets] = {}, off_stage[kSets] = {},
             off_keep[kSets] = {};
    std::vector<std::vector<int>> level_steps[2];   // per phase: the steps of each level
    std::vector<uint64_t> off_list[2];       // per relation: list buffer base
    // join phase
    struct JoinRel {
        uint64_t rid = 0, cols = 0, dir_begin = 0, dir_key = 0, slots = 0, cw = 0, cv = 0, ndir = 0, mask = 0;
        uint32_t slot_cap = 0;
        uint64_t ghist = 0, lb_hist[kRadixPasses] = {}, lb_hist_ctr[kRadixPasses] = {};
        uint64_t lb_dir = 0, lb_dir_ctr = 0;
        // radix-sort and DP scan scratch of its own (relations are bucketed and weighed concurrently)
        uint64_t sklo[2] = {0, 0}, skhi[2] = {0, 0}, svals[2] = {0, 0}, shist = 0, sctl = 0, tsums = 0;
    };
    std::vector<JoinRel> jr;
    uint64_t off_tile_sums = 0;
    uint64_t off_root_cw = 0, off_root_cv = 0;
    std::vector<std::vector<uint64_t>> off_blo, off_bhi;   // [relation][child]
    // cyclic graphs: closing edges all end at L = the last relation of the preorder
    bool cyclic = false, cyc_ok = true;
    int L = -1, cyc_cv = -1;
    uint64_t off_cnt = 0, off_chk = 0, off_off = 0;
    uint32_t cyc_G = 0;
    uint64_t wpre = 0;
    // 3-cycles counted by intersection (sj_tri.hip): root - P - L - root
    bool tri = false;
    bool cyc_counted = false;                // the binary cyclic count pass ran since the last sieve
    int tri_P = -1;
    uint64_t off_tri_w = 0, off_tri_beg = 0, off_tri_off = 0, off_tri_tiles = 0, off_tri_part = 0;
    // 4-cliques counted by intersection (sj_tri.hip): the relations holding the pairs
    // ac, ad, bc, bd, cd of the variables (a, b: the root's join columns) and, per
    // relation, the join-column indices of its earlier and later variable
    bool k4 = false;
    int k4_rel[5] = {-1, -1, -1, -1, -1}, k4_x[5] = {}, k4_y[5] = {};
    static constexpr int kPairs = 5;         // pair hashes: P and L of a 3-cycle, or the five above
    int pair_rel[kPairs] = {-1, -1, -1, -1, -1};
    uint64_t pair_cap[kPairs] = {};
    uint64_t off_pair_slot[kPairs] = {}, off_pair_msum[kPairs] = {}, off_pair_mask[kPairs] = {};
    uint64_t off_pair_sig[kPairs] = {}, off_pair_pos[kPairs] = {};
    uint64_t off_emit_lane = 0, off_emit_block = 0;   // write pass of 3-cycles and 4-cliques
    int state = kPlanned;
    uint64_t count = 0, checksum = 0;
    // event profiling (SJ_FLAG_PROFILE): one event pair per launch group
    bool profile = false;
    struct ProfRec {
        int label;
        hipEvent_t a, b;
        int step;              // sieve step index (probe, compaction, build), -1 otherwise
        int kind;              // ProfKind
    };
    std::vector<ProfRec> prof_pending;
    std::vector<hipEvent_t> prof_free;
    // filter catalogue (sj_plan_use_filter_cache)
    sj_fcache *fcache = nullptr;
    std::vector<hipEvent_t> fc_wait;     // readiness of reused entries not yet seen complete
    // recorded on the context's stream after each call that may read or write catalogue
    // entries, and handed to the catalogue when the plan lets go of them, so that releasing
    // them never touches the stream (which the caller may have destroyed by then)
    FcEventRef fc_last_use;
    bool fc_used = false;
    void fc_detach();
    struct ProfAcc {
        std::string label;
        double ms = 0;
        uint64_t n = 0;
        uint64_t bytes = 0;    // algorithmic bytes of the last launch, 0 if not modelled
    };
    std::vector<ProfAcc> prof_acc;
    // Each launch phase (filter build, sieve, join count pass) is recorded once into a
    // HIP graph on a private stream and replayed on the context's stream afterwards:
    // every grid and argument is fixed once the workspace is bound, and the replay
    // removes the host's per-launch cost between the many short kernels.
    bool eager = false;                  // profiling plans and SJ_FLAG_EAGER launch one by one
    hipStream_t ls = nullptr;            // stream the launch helpers enqueue on
    hipStream_t cap_stream = nullptr;    // capture stream (created on first use)
    hipGraphExec_t gexec[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};   // build, sieve, join, result, 3-cycle count
    // independent launch groups (the relations' bucketings) run on branch streams that
    // fork from and join back into the launch stream through events
    static constexpr int kBranches = 4;
    hipStream_t branch[kBranches] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t fork_ev = nullptr, join_ev[kBranches] = {nullptr, nullptr, nullptr, nullptr};
    static_assert(kBranches == kSets, "one scratch set per branch");
    // asynchronous count / result (sj_join_async, sj_result_async, sj_join_wait)
    bool count_on_host = false;          // p->count / p->checksum hold the last count pass
    bool async_result = false;           // a materialisation with a device-side count is queued
    int32_t *res_out = nullptr;          // its buffer, capacity and mode (the recorded graph uses them)
    uint64_t res_cap = 0;
    int32_t res_mode = SJ_RIDS;
    // columns written per tuple in SJ_VALUES mode (relation, column); empty: every column
    // of every relation, relations in index order
    std::vector<std::pair<int, int>> proj;
    void drop_graphs();
    ~sj_plan_s();
};

void sj_plan_s::drop_graphs() {
    for (auto &g : gexec) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
}

void sj_plan_s::fc_detach() {
    const FcEventRef none;
    for (auto &f : filters) {
        if (f.fc) fc_release(fcache, f.fc, fc_used ? fc_last_use : none);
        f.fc = nullptr;
        f.ext_words = f.ext_nblocks = nullptr;
        f.fc_how = 0;
        f.fc_pending = false;
    }
    fc_wait.clear();
    fcache = nullptr;
    fc_last_use.reset();
    fc_used = false;
}

// After a call that enqueued work which may use catalogue entries: record its end.
static sj_status fc_mark_use(sj_plan_t *p) {
    if (!p->fcache) return SJ_OK;
    if (hipEventRecord(p->fc_last_use->ev, p->ctx->stream) != hipSuccess) {
        // no record of the work: wait for it, so that releasing the entries is safe
        if (hipStreamSynchronize(p->ctx->stream) != hipSuccess) return SJ_ERR_DEVICE;
        return SJ_OK;
    }
    p->fc_used = true;
    return SJ_OK;
}

sj_plan_s::~sj_plan_s() {
    if (fcache) {
        (void)hipSetDevice(ctx->device);
        fc_detach();
    }
    drop_graphs();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (auto &b : branch)
        if (b) (void)hipStreamDestroy(b);
    for (auto &e : join_ev)
        if (e) (void)hipEventDestroy(e);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    for (auto &r : prof_pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : prof_free) (void)hipEventDestroy(e);
    ctx_release(ctx);
}

// ---------------------------------------------------------------- errors

static sj_status fail(sj_ctx *ctx, sj_status code, const char *fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return code;
}

#define SJ_HIP(ctx, expr)                                                                        \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail((ctx), SJ_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));  \
    } while (0)

// ---------------------------------------------------------------- context

extern "C" sj_status sj_ctx_create(int32_t device, void *hip_stream, sj_ctx **out) {
    if (!out) return SJ_ERR_INVALID;
    *out = nullptr;
    if (device < 0) return SJ_ERR_INVALID;
    sj_ctx *c = new (std::nothrow) sj_ctx;
    if (!c) return SJ_ERR_INVALID;
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    *out = c;
    return SJ_OK;
}

extern "C" sj_status sj_ctx_set_stream(sj_ctx *ctx, void *hip_stream) {
    if (!ctx) return SJ_ERR_INVALID;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return SJ_OK;
}

extern "C" sj_status sj_ctx_destroy(sj_ctx *ctx) {
    ctx_release(ctx);
    return SJ_OK;
}

extern "C" const char *sj_last_error(const sj_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

// ---------------------------------------------------------------- planning

static uint32_t tiles_of(uint32_t n, uint32_t tile) { return (n + tile - 1) / tile; }

constexpr uint32_t kCycThreads = 1u << 18;   // threads that share a cyclic join's prefixes

static uint64_t nblocks_for(uint64_t n, uint32_t bpk, uint32_t B) {
    uint64_t nb = (n * bpk + B - 1) / B;
    return nb ? nb : 1;
}

static sj_status build_tree(sj_plan_t *p) {
    const int n = p->n;
    std::vector<std::vector<std::tuple<int, int, int, int>>> adj(n);   // (edge, other, my col, other col)
    for (size_t ei = 0; ei < p->edges.size(); ++ei) {
        const sj_edge &e = p->edges[ei];
        adj[e.rel_a].emplace_back(static_cast<int>(ei), e.rel_b, e.col_a, e.col_b);
        adj[e.rel_b].emplace_back(static_cast<int>(ei), e.rel_a, e.col_b, e.col_a);
    }
    p->parent.assign(n, -1);
    p->pcol.assign(n, -1);
    p->mycol.assign(n, -1);
    p->children.assign(n, {});
    p->preorder.clear();
    std::vector<char> seen(n, 0), tree_edge(p->edges.size(), 0);
    // iterative depth-first search that follows each relation's edges in input order
    std::vector<std::pair<int, size_t>> stack;
    seen[p->root] = 1;
    p->preorder.push_back(p->root);
    stack.emplace_back(p->root, 0);
    while (!stack.empty()) {
        auto &top = stack.back();
        const int u = top.first;
        if (top.second >= adj[u].size()) {
            stack.pop_back();
            continue;
        }
        auto [ei, v, cu, cv] = adj[u][top.second++];
        if (seen[v]) continue;
        seen[v] = 1;
        tree_edge[ei] = 1;
        p->parent[v] = u;
        p->pcol[v] = cu;
        p->mycol[v] = cv;
        p->children[u].push_back(v);
        p->preorder.push_back(v);
        stack.emplace_back(v, 0);
    }
    for (int i = 0; i < n; ++i)
        if (!seen[i]) return fail(p->ctx, SJ_ERR_GRAPH, "join graph is not connected (relation %d unreachable)", i);
    std::vector<int> pos(n);
    for (int i = 0; i < n; ++i) pos[p->preorder[i]] = i;
    p->closing.clear();
    for (size_t ei = 0; ei < p->edges.size(); ++ei) {
        if (tree_edge[ei]) continue;
        const sj_edge &e = p->edges[ei];
        if (pos[e.rel_a] < pos[e.rel_b])
            p->closing.push_back({e.rel_a, e.col_a, e.rel_b, e.col_b});
        else
            p->closing.push_back({e.rel_b, e.col_b, e.rel_a, e.col_a});
    }
    p->postorder.clear();
    // postorder: children (in order) before the parent
    std::vector<std::pair<int, size_t>> st2;
    st2.emplace_back(p->root, 0);
    while (!st2.empty()) {
        auto &t = st2.back();
        if (t.second < p->children[t.first].size()) {
            const int c = p->children[t.first][t.second++];
            st2.emplace_back(c, 0);
        } else {
            p->postorder.push_back(t.first);
            st2.pop_back();
        }
    }
    return SJ_OK;
}

static int add_filter(sj_plan_t *p, int kind, int index, int src_rel, int src_col) {
    Filter f;
    f.kind = kind;
    f.index = index;
    f.src_rel = src_rel;
    f.src_col = src_col;
    const uint64_t nb = nblocks_for(p->rels[src_rel].nrows, p->opts.bits_per_key, p->opts.block_bits);
    f.max_words = nb * (p->opts.block_bits / 32);
    p->filters.push_back(f);
    return static_cast<int>(p->filters.size()) - 1;
}

static sj_status build_schedule(sj_plan_t *p) {
    const int n = p->n;
    const bool two = p->opts.passes == 2;
    p->filters.clear();
    p->f_bwd.assign(n, -1);
    p->f_fwd.assign(n, -1);
    p->f_close.assign(p->closing.size(), -1);
    for (int j : p->postorder)
        if (j != p->root) p->f_bwd[j] = add_filter(p, SJ_FILTER_BACKWARD, j, j, p->mycol[j]);
    if (two)
        for (int x : p->preorder)
            if (x != p->root) p->f_fwd[x] = add_filter(p, SJ_FILTER_FORWARD, x, p->parent[x], p->pcol[x]);
    for (size_t e = 0; e < p->closing.size(); ++e)
        p->f_close[e] = add_filter(p, SJ_FILTER_CLOSING, static_cast<int>(e), p->closing[e].u, p->closing[e].cu);
    if (p->filters.size() > 64) return fail(p->ctx, SJ_ERR_UNSUPPORTED, "more than 64 filters");

    std::vector<int> cur(n, kFull), cur_step(n, -1);
    p->steps.clear();
    auto jx = [&](int rel, int col) { return p->rels[rel].jidx(col); };
    auto push = [&](StepSpec s) -> sj_status {
        if (s.probes.size() > static_cast<size_t>(kMaxProbe) || s.builds.size() > static_cast<size_t>(kMaxBuild))
            return fail(p->ctx, SJ_ERR_UNSUPPORTED, "a relation probes or builds more than 8 filters");
        s.src = cur[s.rel];
        s.src_step = cur_step[s.rel];
        if (s.out >= 0) {
            s.out = (cur[s.rel] == 0) ? 1 : 0;
            cur[s.rel] = s.out;
            cur_step[s.rel] = static_cast<int>(p->steps.size());
        }
        p->steps.push_back(s);
        return SJ_OK;
    };
    // backward pass: leaves toward the root (the pruning phase of Section 2.2)
    for (int j : p->postorder) {
        if (j == p->root) continue;
        StepSpec s;
        s.phase = 0;
        s.rel = j;
        for (int c : p->children[j]) s.probes.emplace_back(jx(j, p->pcol[c]), p->f_bwd[c]);
        s.builds.emplace_back(jx(j, p->mycol[j]), p->f_bwd[j]);
        s.out = (!p->children[j].empty() || !two) ? 0 : -1;
        if (sj_status st = push(s)) return st;
    }
    {   // the root: sieved by its children's filters
        StepSpec s;
        s.phase = 1;
        s.rel = p->root;
        for (int c : p->children[p->root]) s.probes.emplace_back(jx(p->root, p->pcol[c]), p->f_bwd[c]);
        if (two) {
            for (int c : p->children[p->root]) s.builds.emplace_back(jx(p->root, p->pcol[c]), p->f_fwd[c]);
            for (size_t e = 0; e < p->closing.size(); ++e)
                if (p->closing[e].u == p->root) s.builds.emplace_back(jx(p->root, p->closing[e].cu), p->f_close[e]);
        }
        s.out = 0;
        if (sj_status st = push(s)) return st;
    }
    if (!two) {
        // closing edges (Section 2.3): a filter on the earlier end's survivors sieves the later end
        for (size_t e = 0; e < p->closing.size(); ++e) {
            const Closing &c = p->closing[e];
            StepSpec b;
            b.phase = 1;
            b.rel = c.u;
            b.builds.emplace_back(jx(c.u, c.cu), p->f_close[e]);
            if (sj_status st = push(b)) return st;
            StepSpec s;
            s.phase = 1;
            s.rel = c.v;
            s.probes.emplace_back(jx(c.v, c.cv), p->f_close[e]);
            s.out = 0;
            if (sj_status st = push(s)) return st;
        }
    } else {
        // forward pass: root toward the leaves (the dotted arrow of Fig. 2)
        for (int x : p->preorder) {
            if (x == p->root) continue;
            StepSpec s;
            s.phase = 1;
            s.rel = x;
            s.probes.emplace_back(jx(x, p->mycol[x]), p->f_fwd[x]);
            for (size_t e = 0; e < p->closing.size(); ++e)
                if (p->closing[e].v == x) s.probes.emplace_back(jx(x, p->closing[e].cv), p->f_close[e]);
            for (int c : p->children[x]) s.builds.emplace_back(jx(x, p->pcol[c]), p->f_fwd[c]);
            for (size_t e = 0; e < p->closing.size(); ++e)
                if (p->closing[e].u == x) s.builds.emplace_back(jx(x, p->closing[e].cu), p->f_close[e]);
            s.out = 0;
            if (sj_status st = push(s)) return st;
        }
    }
    p->final_list = cur;
    p->final_step = cur_step;
    for (int i = 0; i < n; ++i)
        if (cur[i] == kFull) return fail(p->ctx, SJ_ERR_INVALID, "internal: relation %d has no survivor list", i);
    return SJ_OK;
}

// Dependency levels of each phase's steps: a step follows the step that wrote its
// source list and the steps that build the filters it probes (inside the same phase;
// the previous phase has finished). Steps of one level run on separate branches.
static void schedule_levels(sj_plan_t *p) {
    std::vector<int> builder(p->filters.size(), -1);
    for (int ph = 0; ph < 2; ++ph) {
        p->level_steps[ph].clear();
        for (size_t si = 0; si < p->steps.size(); ++si) {
            StepSpec &st = p->steps[si];
            if (st.phase != ph) continue;
            int lvl = 0;
            if (st.src_step >= 0 && p->steps[st.src_step].phase == ph) lvl = p->steps[st.src_step].level + 1;
            for (auto &pr : st.probes) {
                const int b = builder[pr.second];
                if (b >= 0 && p->steps[b].phase == ph) lvl = std::max(lvl, p->steps[b].level + 1);
            }
            for (auto &bl : st.builds) builder[bl.second] = static_cast<int>(si);
            st.level = lvl;
            if (p->level_steps[ph].size() <= static_cast<size_t>(lvl)) p->level_steps[ph].resize(lvl + 1);
            auto &lv = p->level_steps[ph][lvl];
            st.branch = static_cast<int>(lv.size()) % sj_plan_s::kSets;
            lv.push_back(static_cast<int>(si));
        }
        for (auto &lv : p->level_steps[ph])
            for (int si : lv) p->steps[si].alone = lv.size() == 1;
    }
}

static void build_layout(sj_plan_t *p) {
    Layout L;
    const int n = p->n;
    // phase zero regions first, each contiguous: [build_filters][sieve][join]
    uint32_t max_build_rows[sj_plan_s::kSets] = {}, max_rows[sj_plan_s::kSets] = {};
    uint64_t max_hist[sj_plan_s::kSets] = {1, 1, 1, 1};
    for (int ph = 0; ph < 2; ++ph) {
        p->zero[ph].begin = L.top;
        if (ph == 0) p->off_elig = L.take(sizeof(uint32_t) * SJ_MAX_RELS);
        for (auto &s : p->steps) {
            if (s.phase != ph) continue;
            s.max_rows = p->rels[s.rel].nrows;
            max_rows[s.branch] = std::max(max_rows[s.branch], s.max_rows);
            s.off_count = L.take(4);
            s.off_pstatus = L.take(8ull * kProbeGridMax);
            s.off_pcounter = L.take(4);
            s.off_bstatus.clear();
            s.off_bcounter.clear();
            s.off_btotal.clear();
            for (size_t bi = 0; bi < s.builds.size(); ++bi) {
                const auto &b = s.builds[bi];
                const int set = s.build_set(bi);
                const Filter &f = p->filters[b.second];
                const uint64_t nbm = f.max_words / (p->opts.block_bits / 32);
                const uint64_t nreg = region_count_cap(nbm, p->region_blocks);
                // tiles of any input of up to max_rows keys (build_tile_of keeps them <= kBuildMaxTiles)
                const uint64_t hl = nreg * std::min<uint32_t>(kBuildMaxTiles, tiles_of(s.max_rows, kBuildTileMin));
                max_hist[set] = std::max<uint64_t>(max_hist[set], hl);
                max_build_rows[set] = std::max(max_build_rows[set], s.max_rows);
                s.off_bstatus.push_back(L.take(8ull * std::max<uint64_t>(1, (hl + kScanTile - 1) / kScanTile)));
                s.off_bcounter.push_back(L.take(4));
                s.off_btotal.push_back(L.take(4));
            }
        }
        p->zero[ph].end = L.top;
    }
    for (auto &f : p->filters) f.off = L.take(f.max_words * 4);
    for (int b = 0; b < sj_plan_s::kSets; ++b) {
        const uint32_t br = std::max<uint32_t>(1, max_build_rows[b]);
        p->off_sbits[b] = L.take(max_rows[b] / 8 + 16);
        p->off_scounts[b] = L.take(4ull * kProbeGridMax);
        p->off_bhist[b] = L.take(4 * max_hist[b]);
        p->off_stage[b] = L.take(4ull * br);
        p->off_keep[b] = L.take(8ull * ((uint64_t(br) + 2 * build_tile_of(br)) / 64 + 1));
    }
    p->zero[2].begin = L.top;
    p->off_totals = L.take(16);
    p->jr.assign(n, {});
    uint32_t maxcap = 0;
    for (int j = 0; j < n; ++j) {
        maxcap = std::max(maxcap, p->rels[j].nrows);
        if (j == p->root) continue;
        auto &r = p->jr[j];
        const uint32_t cap = p->rels[j].nrows;
        r.ghist = L.take(4ull * kRadixPasses * kRadixBins);
        const uint32_t htiles = tiles_of(kRadixBins * radix_tiles_max(cap), kScanTile);
        for (int q = 0; q < kRadixPasses; ++q) {
            r.lb_hist[q] = L.take(8ull * std::max<uint32_t>(1, htiles));
            r.lb_hist_ctr[q] = L.take(4);
        }
        r.lb_dir = L.take(8ull * std::max<uint32_t>(1, tiles_of(cap, kSieveTile)));
        r.lb_dir_ctr = L.take(4);
        r.ndir = L.take(4);
    }
    p->zero[2].end = L.top;
    // not cleared
    p->off_nblocks = L.take(4ull * std::max<size_t>(1, p->filters.size()));
    p->off_upd = L.take(8);
    for (int b = 0; b < 2; ++b) p->off_list[b].assign(n, 0);
    for (int j = 0; j < n; ++j) {
        const uint64_t cap = p->rels[j].nrows;
        const uint64_t per = (1 + p->rels[j].jcols.size()) * cap * 4;
        for (int b = 0; b < 2; ++b) p->off_list[b][j] = L.take(per);
    }
    for (int j = 0; j < n; ++j) {
        if (j == p->root) continue;
        auto &r = p->jr[j];
        const uint64_t cap = p->rels[j].nrows;
        r.rid = L.take(4 * cap);
        r.cols = L.take(4 * cap * p->rels[j].jcols.size());
        r.dir_begin = L.take(4 * (cap + 1));
        r.dir_key = L.take(4 * cap);
        uint64_t sc = 16;
        while (sc < 2 * cap + 1) sc <<= 1;
        r.slot_cap = static_cast<uint32_t>(sc);
        r.slots = L.take(8 * sc);
        r.cw = L.take(8 * (cap + 1));
        r.cv = L.take(8 * (cap + 1));
        r.mask = L.take(4);
    }
    for (int j = 0; j < n; ++j) {
        if (j == p->root) continue;
        auto &r = p->jr[j];
        const uint64_t cap = std::max<uint32_t>(1, p->rels[j].nrows);
        // bucketed by two keys: (tree key, closing key) for L of a cyclic join, (key, key)
        // pairs for the relations a 3-cycle or 4-clique walks
        const bool two_word = (p->cyclic && j == p->L) || (p->tri && j == p->tri_P) || p->k4;
        for (int b = 0; b < 2; ++b) {
            r.sklo[b] = L.take(4 * cap);
            r.skhi[b] = two_word ? L.take(4 * cap) : 0;
            r.svals[b] = L.take(4 * cap);
        }
        r.shist = L.take(4ull * kRadixBins * std::max<uint32_t>(1, radix_tiles_max(static_cast<uint32_t>(cap))));
        r.sctl = L.take(4 * 32);
        r.tsums = L.take(16ull * std::max<uint32_t>(1, tiles_of(static_cast<uint32_t>(cap),
                                                                   dp_tile(static_cast<int>(p->children[j].size())))));
    }
    p->off_tile_sums = L.take(16ull * std::max<uint32_t>(
        1, tiles_of(maxcap, dp_tile(static_cast<int>(p->children[p->root].size())))));
    const uint64_t rc = p->rels[p->root].nrows;
    p->off_root_cw = L.take(8 * (rc + 1));
    p->off_root_cv = L.take(8 * (rc + 1));
    p->off_cnt = L.take(8ull * kCycThreads);
    p->off_chk = L.take(8ull * kCycThreads);
    p->off_off = L.take(8ull * kCycThreads);
    p->off_blo.assign(n, {});
    p->off_bhi.assign(n, {});
    for (int j = 0; j < n; ++j) {
        for (size_t c = 0; c < p->children[j].size(); ++c) {
            p->off_blo[j].push_back(L.take(4ull * p->rels[j].nrows));
            p->off_bhi[j].push_back(L.take(4ull * p->rels[j].nrows));
        }
    }
    if (p->tri || p->k4) {
        const uint64_t rn = std::max<uint64_t>(1, rc);
        p->off_tri_w = L.take(4 * rn);
        p->off_tri_beg = L.take(4 * rn);
        p->off_tri_off = L.take(8 * (rc + 1));
        p->off_tri_tiles = L.take(8ull * std::max<uint32_t>(1, tiles_of(static_cast<uint32_t>(rc), kScanTile)));
        p->off_tri_part = L.take(16ull * kTriBlocks);
        if (p->tri) {
            p->pair_rel[0] = p->tri_P;
            p->pair_rel[1] = p->L;
        } else {
            for (int h = 0; h < 5; ++h) p->pair_rel[h] = p->k4_rel[h];
        }
        for (int h = 0; h < sj_plan_s::kPairs; ++h) {
            if (p->pair_rel[h] < 0) continue;
            uint64_t cap = 16;
            while (cap < 2ull * p->rels[p->pair_rel[h]].nrows + 1) cap <<= 1;
            p->pair_cap[h] = cap;
            p->off_pair_slot[h] = L.take(16 * (cap + 1));
            p->off_pair_msum[h] = L.take(8 * (cap + 1));
            p->off_pair_mask[h] = L.take(4);
            p->off_pair_sig[h] = L.take(4 * (cap / 8));
            p->off_pair_pos[h] = L.take(4 * (cap + 1));
        }
        p->off_emit_lane = L.take(8ull * kEmitLanes);
        p->off_emit_block = L.take(8ull * kTriBlocks);
    }
    p->ws_bytes = L.top;
}

// A 4-clique query (Section 3.1.3): six relations that join on two columns each, the
// join columns falling into four variables (the classes of columns the edges make
// equal) so that every relation holds a different pair of them. The root's two join
// columns are the variables a and b; c and d are the other two. Sets p->k4 and the
// roles of the other five relations when the query has that shape.
static void detect_k4(sj_plan_t *p) {
    if (p->n != 6) return;
    for (const Rel &R : p->rels)
        if (R.jcols.size() != 2 || R.nrows >= (1u << 30)) return;
    int up[12];
    for (int i = 0; i < 12; ++i) up[i] = i;   // node: relation * 2 + join-column index
    auto find = [&](int u) {
        while (up[u] != u) u = up[u] = up[up[u]];
        return u;
    };
    for (const sj_edge &e : p->edges) {
        const int u = find(e.rel_a * 2 + p->rels[e.rel_a].jidx(e.col_a));
        const int v = find(e.rel_b * 2 + p->rels[e.rel_b].jidx(e.col_b));
        if (u != v) up[std::max(u, v)] = std::min(u, v);
    }
    int var[12], classes[12], nclass = 0;
    for (int i = 0; i < 12; ++i) {
        var[i] = find(i);
        if (std::find(classes, classes + nclass, var[i]) == classes + nclass) classes[nclass++] = var[i];
    }
    if (nclass != 4) return;
    for (int r = 0; r < 6; ++r) {
        if (var[2 * r] == var[2 * r + 1]) return;
        for (int q = 0; q < r; ++q)
            if (std::min(var[2 * q], var[2 * q + 1]) == std::min(var[2 * r], var[2 * r + 1]) &&
                std::max(var[2 * q], var[2 * q + 1]) == std::max(var[2 * r], var[2 * r + 1]))
                return;   // two relations on the same pair
    }
    const int A = var[2 * p->root], B = var[2 * p->root + 1];
    int others[2], no = 0;
    for (int i = 0; i < 4; ++i)
        if (classes[i] != A && classes[i] != B) others[no++] = classes[i];
    const int C = others[0], D = others[1];
    const int role[5][2] = {{A, C}, {A, D}, {B, C}, {B, D}, {C, D}};
    for (int h = 0; h < 5; ++h) {
        p->k4_rel[h] = -1;
        for (int r = 0; r < 6; ++r) {
            if (var[2 * r] == role[h][0] && var[2 * r + 1] == role[h][1]) {
                p->k4_rel[h] = r;
                p->k4_x[h] = 0;
                p->k4_y[h] = 1;
            } else if (var[2 * r] == role[h][1] && var[2 * r + 1] == role[h][0]) {
                p->k4_rel[h] = r;
                p->k4_x[h] = 1;
                p->k4_y[h] = 0;
            }
        }
        if (p->k4_rel[h] < 0) return;
    }
    p->k4 = true;
}

extern "C" sj_status sj_plan(sj_ctx *ctx, const sj_rel *rels, int32_t nrels, const sj_edge *edges, int32_t nedges,
                             const sj_opts *opts, sj_plan_t **out, uint64_t *workspace_bytes) {
    if (!ctx || !out || !workspace_bytes) return fail(ctx, SJ_ERR_INVALID, "null argument");
    *out = nullptr;
    *workspace_bytes = 0;
    if (!rels || nrels < 1 || nrels > SJ_MAX_RELS) return fail(ctx, SJ_ERR_INVALID, "nrels must be 1..%d", SJ_MAX_RELS);
    if (nedges < 0 || nedges > SJ_MAX_EDGES || (nedges > 0 && !edges))
        return fail(ctx, SJ_ERR_INVALID, "nedges must be 0..%d", SJ_MAX_EDGES);
    sj_opts o{};
    if (opts) o = *opts;
    if (o.bits_per_key == 0) o.bits_per_key = 8;
    if (o.k == 0) o.k = 6;
    if (o.block_bits == 0) o.block_bits = 512;
    if (o.passes == 0) o.passes = 2;
    if (o.root < 0) o.root = 0;
    if (o.k > static_cast<uint32_t>(kMaxK)) return fail(ctx, SJ_ERR_INVALID, "k must be 1..%d", kMaxK);
    if (o.bits_per_key > 1024) return fail(ctx, SJ_ERR_INVALID, "bits_per_key must be <= 1024");
    if (o.block_bits != 256 && o.block_bits != 512 && o.block_bits != 1024)
        return fail(ctx, SJ_ERR_INVALID, "block_bits must be 256, 512 or 1024");
    if (o.passes != 1 && o.passes != 2) return fail(ctx, SJ_ERR_INVALID, "passes must be 1 or 2");
    if (o.root >= nrels) return fail(ctx, SJ_ERR_INVALID, "root out of range");
    if (o.probe_grid == 0) o.probe_grid = kProbeGrid;
    if (o.probe_grid < 64 || o.probe_grid > kProbeGridMax || (o.probe_grid & (o.probe_grid - 1)))
        return fail(ctx, SJ_ERR_INVALID, "probe_grid must be a power of two, 64..%u", kProbeGridMax);
    if (o.probe_lds > 2) return fail(ctx, SJ_ERR_INVALID, "probe_lds must be 0, 1 or 2");
    if (o.flags & ~static_cast<uint32_t>(SJ_FLAG_PROFILE | SJ_FLAG_EAGER | SJ_FLAG_BINARY_CYCLES |
                                         SJ_FLAG_FAULT_FILTERS | SJ_FLAG_FAULT_SIEVE | SJ_FLAG_FAULT_JOIN |
                                         SJ_FLAG_FAULT_RESULT | SJ_FLAG_SIEVE_TWO_LAUNCHES))
        return fail(ctx, SJ_ERR_INVALID, "unknown flags");

    sj_plan_t *p = new (std::nothrow) sj_plan_t;
    if (!p) return fail(ctx, SJ_ERR_INVALID, "out of host memory");
    p->ctx = ctx;
    ctx->refs.fetch_add(1, std::memory_order_relaxed);
    p->n = nrels;
    p->opts = o;
    p->logB = (o.block_bits == 256) ? 8 : (o.block_bits == 512 ? 9 : 10);
    p->root = o.root;
    p->profile = (o.flags & SJ_FLAG_PROFILE) != 0;
    p->eager = p->profile || (o.flags & SJ_FLAG_EAGER) != 0;
    {   // 32-bit filter seed: the low word of SplitMix64's output function of the seed
        uint64_t z = o.seed;
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        z ^= z >> 31;
        p->seed32 = static_cast<uint32_t>(z);
    }
    p->rels.resize(nrels);
    for (int i = 0; i < nrels; ++i) {
        const sj_rel &r = rels[i];
        Rel &R = p->rels[i];
        if (r.nrows < 0 || r.nrows >= (int64_t(1) << 31)) {
            delete p;
            return fail(ctx, SJ_ERR_INVALID, "relation %d: nrows must be in [0, 2^31)", i);
        }
        if (r.ncols < 1 || r.ncols > SJ_MAX_COLS || !r.cols) {
            delete p;
            return fail(ctx, SJ_ERR_INVALID, "relation %d: ncols must be 1..%d", i, SJ_MAX_COLS);
        }
        R.nrows = static_cast<uint32_t>(r.nrows);
        R.cols.assign(r.cols, r.cols + r.ncols);
        for (int c = 0; c < r.ncols; ++c) {
            if (R.nrows > 0 && !R.cols[c]) {
                delete p;
                return fail(ctx, SJ_ERR_INVALID, "relation %d column %d is null", i, c);
            }
            if (reinterpret_cast<uintptr_t>(R.cols[c]) % 16) {
                delete p;
                return fail(ctx, SJ_ERR_INVALID, "relation %d column %d is not 16-byte aligned", i, c);
            }
        }
        if (r.pred_col >= r.ncols || r.pred_col < -1) {
            delete p;
            return fail(ctx, SJ_ERR_GRAPH, "relation %d: bad predicate column %d", i, r.pred_col);
        }
        R.pred_col = r.pred_col;
        R.lo = r.pred_lo;
        R.hi = r.pred_hi;
    }
    p->edges.assign(edges, edges + nedges);
    for (int ei = 0; ei < nedges; ++ei) {
        const sj_edge &e = edges[ei];
        if (e.rel_a < 0 || e.rel_a >= nrels || e.rel_b < 0 || e.rel_b >= nrels) {
            delete p;
            return fail(ctx, SJ_ERR_GRAPH, "edge %d: relation index out of range", ei);
        }
        if (e.rel_a == e.rel_b) {
            delete p;
            return fail(ctx, SJ_ERR_GRAPH, "edge %d joins relation %d with itself", ei, e.rel_a);
        }
        if (e.col_a < 0 || e.col_a >= static_cast<int>(p->rels[e.rel_a].cols.size()) || e.col_b < 0 ||
            e.col_b >= static_cast<int>(p->rels[e.rel_b].cols.size())) {
            delete p;
            return fail(ctx, SJ_ERR_GRAPH, "edge %d: column index out of range", ei);
        }
        for (auto [r, c] : {std::pair<int, int>{e.rel_a, e.col_a}, {e.rel_b, e.col_b}}) {
            auto &jc = p->rels[r].jcols;
            if (std::find(jc.begin(), jc.end(), c) == jc.end()) jc.push_back(c);
        }
    }
    for (int i = 0; i < nrels; ++i) {
        auto &jc = p->rels[i].jcols;
        std::sort(jc.begin(), jc.end());
        if (jc.empty()) jc.push_back(0);
        if (jc.size() > static_cast<size_t>(kMaxJCols)) {
            delete p;
            return fail(ctx, SJ_ERR_UNSUPPORTED, "relation %d joins on more than %d columns", i, kMaxJCols);
        }
    }
    if (sj_status st = build_tree(p)) {
        delete p;
        return st;
    }
    if (sj_status st = build_schedule(p)) {
        delete p;
        return st;
    }
    schedule_levels(p);
    p->L = p->preorder.back();
    p->cyclic = !p->closing.empty();
    // The binary plan enumerates the spanning tree without L (the last relation of the
    // preorder, a leaf) and matches L per prefix: L is sorted by the column of the first
    // closing edge that ends at it, other closing edges at L are checked per entry, and
    // closing edges between two other relations per prefix.
    if (p->closing.size() > static_cast<size_t>(kMaxClose) || (p->cyclic && nrels > 8)) p->cyc_ok = false;
    for (const Closing &c : p->closing)
        if (c.v == p->L && p->cyc_cv < 0) p->cyc_cv = c.cv;
    if (p->cyclic && nrels == 6 && !(o.flags & SJ_FLAG_BINARY_CYCLES)) detect_k4(p);
    if (p->cyclic && p->cyc_ok && nrels == 3 && p->closing.size() == 1 && !(o.flags & SJ_FLAG_BINARY_CYCLES)) {
        // the 3-cycle root - P - L - root: counted by intersection when the pair hashes fit
        const int r = p->root;
        const int P = p->children[r].size() == 1 ? p->children[r][0] : -1;
        if (P >= 0 && p->children[P].size() == 1 && p->children[P][0] == p->L && p->closing[0].u == r &&
            p->closing[0].v == p->L && p->rels[P].nrows < (1u << 30) && p->rels[p->L].nrows < (1u << 30)) {
            p->tri = true;
            p->tri_P = P;
        }
    }
    p->region_blocks = kRegionBytes / (o.block_bits / 8);
    for (auto &f : p->filters) {
        const uint64_t nbm = f.max_words / (o.block_bits / 32);
        if ((nbm + p->region_blocks - 1) / p->region_blocks > 16384) {
            delete p;
            return fail(ctx, SJ_ERR_UNSUPPORTED, "a filter of more than %u blocks", 16384u * p->region_blocks);
        }
    }
    build_layout(p);
    *workspace_bytes = p->ws_bytes;
    *out = p;
    return SJ_OK;
}

extern "C" sj_status sj_bind_workspace(sj_plan_t *p, void *ws, uint64_t bytes) {
    if (!p) return SJ_ERR_INVALID;
    if (!ws && p->ws_bytes) return fail(p->ctx, SJ_ERR_INVALID, "null workspace");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(p->ctx, SJ_ERR_INVALID, "workspace must be 256-byte aligned");
    if (bytes < p->ws_bytes)
        return fail(p->ctx, SJ_ERR_NOMEM, "workspace has %llu bytes, plan needs %llu",
                    static_cast<unsigned long long>(bytes), static_cast<unsigned long long>(p->ws_bytes));
    p->ws = static_cast<char *>(ws);
    p->drop_graphs();   // recorded launches point into the previous workspace
    p->state = kBound;
    return SJ_OK;
}

// ---------------------------------------------------------------- static workspace

// The workspace of sj_bind_static_workspace, for callers that cannot allocate device
// memory: one array per GPU (each device the library runs on holds its own copy until
// the process ends). Host code never uses the array's name as an address: the device
// address comes from hipGetSymbolAddress, once per device.
constexpr uint64_t kStaticWorkspaceBytes = 64ull << 20;
constexpr int kStaticMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kStaticMaxDevices] = {};

extern "C" sj_status sj_bind_static_workspace(sj_plan_t *p) {
    if (!p) return SJ_ERR_INVALID;
    const int dev = p->ctx->device;
    if (dev >= kStaticMaxDevices) return fail(p->ctx, SJ_ERR_INVALID, "device %d: static workspaces exist for devices 0..%d",
                                              dev, kStaticMaxDevices - 1);
    if (p->ws_bytes > kStaticWorkspaceBytes)
        return fail(p->ctx, SJ_ERR_NOMEM,
                    "the plan needs %llu bytes of workspace; the static workspace holds %llu (bind a caller workspace "
                    "with sj_bind_workspace instead)",
                    static_cast<unsigned long long>(p->ws_bytes), static_cast<unsigned long long>(kStaticWorkspaceBytes));
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            int prev = 0;
            SJ_HIP(p->ctx, hipGetDevice(&prev));
            SJ_HIP(p->ctx, hipSetDevice(dev));
            void *addr = nullptr;
            const hipError_t e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
            (void)hipSetDevice(prev);
            if (e != hipSuccess || !addr)
                return fail(p->ctx, SJ_ERR_DEVICE, "hipGetSymbolAddress of the static workspace failed: %s",
                            hipGetErrorString(e));
            g_scratch_ptr[dev] = addr;
        }
        ptr = g_scratch_ptr[dev];
    }
    return sj_bind_workspace(p, ptr, kStaticWorkspaceBytes);
}

extern "C" sj_status sj_plan_destroy(sj_plan_t *p) {
    delete p;
    return SJ_OK;
}

// ---------------------------------------------------------------- execution helpers

template <typename T>
static T *at(sj_plan_t *p, uint64_t off) {
    return reinterpret_cast<T *>(p->ws + off);
}

static uint32_t *list_rid(sj_plan_t *p, int rel, int buf) { return at<uint32_t>(p, p->off_list[buf][rel]); }
static uint32_t *fwords(sj_plan_t *p, int f) {
    const Filter &F = p->filters[f];
    return F.ext_words ? F.ext_words : at<uint32_t>(p, F.off);
}
static uint32_t *fnblocks(sj_plan_t *p, int f) {
    const Filter &F = p->filters[f];
    return F.ext_nblocks ? F.ext_nblocks : at<uint32_t>(p, p->off_nblocks) + f;
}
static int32_t *list_col(sj_plan_t *p, int rel, int buf, int jc) {
    return at<int32_t>(p, p->off_list[buf][rel] + 4ull * p->rels[rel].nrows * (1 + jc));
}

// ---------------------------------------------------------------- profiling

static int prof_label(sj_plan_t *p, const std::string &label) {
    for (size_t i = 0; i < p->prof_acc.size(); ++i)
        if (p->prof_acc[i].label == label) return static_cast<int>(i);
    p->prof_acc.push_back({label, 0.0, 0, 0});
    return static_cast<int>(p->prof_acc.size()) - 1;
}

static hipEvent_t prof_event(sj_plan_t *p) {
    if (!p->prof_free.empty()) {
        hipEvent_t e = p->prof_free.back();
        p->prof_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records an event before the launches of its scope and one after them.
// What a profiled launch group is, for its algorithmic-byte model.
// kProfBuckets and kProfDp carry the relation index in the record's `step` field.
enum ProfKind { kProfOther = 0, kProfProbe = 1, kProfCompact = 2, kProfResult = 3, kProfBuckets = 4, kProfDp = 5,
                kProfScan = 6, kProfBuild0 = 16 };

struct ProfScope {
    sj_plan_t *p;
    long idx = -1;
    ProfScope(sj_plan_t *pp, const std::string &label, int step = -1, int kind = kProfOther) : p(pp) {
        if (!p->profile) return;
        hipEvent_t a = prof_event(p), b = prof_event(p);
        if (!a || !b) return;
        (void)hipEventRecord(a, p->ctx->stream);
        p->prof_pending.push_back({prof_label(p, label), a, b, step, kind});
        idx = static_cast<long>(p->prof_pending.size()) - 1;
    }
    ~ProfScope() {
        if (idx >= 0) (void)hipEventRecord(p->prof_pending[idx].b, p->ctx->stream);
    }
};

static std::string rel_name(int r) { return "R" + std::to_string(r); }

static sj_status fork_streams(sj_plan_t *p, int n, hipStream_t *out);
static sj_status join_streams(sj_plan_t *p, int n);

static sj_status run_step(sj_plan_t *p, StepSpec &st, hipStream_t s) {
    const int set = st.branch;
    {
        const Rel &R = p->rels[st.rel];
        StepArgs a{};
        a.ncol = static_cast<int>(R.jcols.size());
        if (st.src == kFull) {
            a.src_rid = nullptr;
            a.src_count = nullptr;
            a.src_rows = R.nrows;
            for (int c = 0; c < a.ncol; ++c) a.col[c] = R.cols[R.jcols[c]];
            a.pred = R.pred_col >= 0 ? R.cols[R.pred_col] : nullptr;
            a.pred_lo = R.lo;
            a.pred_hi = R.hi;
        } else {
            a.src_rid = list_rid(p, st.rel, st.src);
            a.src_count = at<uint32_t>(p, p->steps[st.src_step].off_count);
            a.src_rows = R.nrows;
            for (int c = 0; c < a.ncol; ++c) a.col[c] = list_col(p, st.rel, st.src, c);
            a.pred = nullptr;
        }
        a.nprobe = static_cast<int>(st.probes.size());
        for (int i = 0; i < a.nprobe; ++i) {
            a.probe_col[i] = static_cast<int8_t>(st.probes[i].first);
            const int f = st.probes[i].second;
            a.probe[i].words = fwords(p, f);
            a.probe[i].nblocks = fnblocks(p, f);
        }
        if (st.out >= 0) {
            a.out_rid = list_rid(p, st.rel, st.out);
            for (int c = 0; c < a.ncol; ++c) a.out_col[c] = list_col(p, st.rel, st.out, c);
            a.out_count = at<uint32_t>(p, st.off_count);
        }
        // LDS for the smallest probed filter that fits (sizes are known on the device only)
        a.lds_words = 0;
        if (p->opts.probe_lds != 1) {
            for (auto &pr : st.probes) {
                const uint64_t mw = p->filters[pr.second].max_words;
                if (p->opts.probe_lds == 2 && mw > kLdsFilterBytes / 4) continue;
                a.lds_words = std::max<uint32_t>(a.lds_words,
                                                 static_cast<uint32_t>(std::min<uint64_t>(mw, kLdsFilterBytes / 4)));
            }
        }
        a.grid = p->opts.probe_grid;
        a.bits = at<uint8_t>(p, p->off_sbits[set]);
        a.counts = at<uint32_t>(p, p->off_scounts[set]);
        a.lb.status = at<uint64_t>(p, st.off_pstatus);
        a.lb.counter = at<uint32_t>(p, st.off_pcounter);
        a.seed = p->seed32;
        a.k = static_cast<int>(p->opts.k);
        a.logB = p->logB;
        const std::string tag = std::string(st.phase == 0 ? "bwd" : "sieve") + ":" + rel_name(st.rel) + ":" +
                                std::to_string(&st - p->steps.data());
        const int si = static_cast<int>(&st - p->steps.data());
        if (st.out >= 0 && !(p->opts.flags & SJ_FLAG_SIEVE_TWO_LAUNCHES)) {
            // probe and survivor list in one launch
            ProfScope ps(p, "probe:" + tag, si, kProfScan);
            SJ_HIP(p->ctx, launch_sieve_fused(a, st.max_rows, s));
        } else if (a.nprobe > 0 || st.out >= 0) {
            {
                ProfScope ps(p, "probe:" + tag, si, kProfProbe);
                SJ_HIP(p->ctx, launch_sieve_probe(a, st.max_rows, s));
            }
            ProfScope ps(p, "compact:" + tag, si, kProfCompact);
            SJ_HIP(p->ctx, launch_sieve_compact(a, st.max_rows, s));
        }
        // a step alone in its level builds its filters side by side, one branch and scratch set each
        int nbuild = 0;
        for (auto &bl : st.builds) nbuild += p->filters[bl.second].resident() ? 0 : 1;
        // (build b uses set b % kSets, as the layout sized them, whether or not others are reused)
        const int nfork = (st.alone && nbuild > 1) ? static_cast<int>(std::min<size_t>(st.builds.size(), sj_plan_s::kSets)) : 0;
        hipStream_t bs[sj_plan_s::kSets];
        if (sj_status e = fork_streams(p, nfork, bs)) return e;
        for (size_t b = 0; b < st.builds.size(); ++b) {
            const int f = st.builds[b].second;
            const int jc = st.builds[b].first;
            if (p->filters[f].resident()) continue;   // reused from the filter catalogue
            const int bset = st.build_set(b);
            const hipStream_t bstream = nfork > 1 ? bs[bset] : s;
            BuildArgs ba{};
            if (st.out >= 0) {          // the step's survivors
                ba.keys = a.out_col[jc];
                ba.n_dev = a.out_count;
            } else if (st.src == kFull) {
                ba.keys = R.cols[R.jcols[jc]];
                ba.n = R.nrows;
                ba.pred = a.pred;
                ba.pred_lo = R.lo;
                ba.pred_hi = R.hi;
                if (R.pred_col >= 0) ba.nkeys_dev = at<uint32_t>(p, p->off_elig) + st.rel;
            } else {
                ba.keys = a.col[jc];
                ba.n_dev = a.src_count;
            }
            ba.n_max = R.nrows;
            ba.words = fwords(p, f);
            ba.nblocks = fnblocks(p, f);
            ba.bits_per_key = p->opts.bits_per_key;
            ba.nblocks_max = static_cast<uint32_t>(p->filters[f].max_words / (p->opts.block_bits / 32));
            ba.region_blocks = p->region_blocks;
            ba.hist = at<uint32_t>(p, p->off_bhist[bset]);
            ba.stage = at<uint32_t>(p, p->off_stage[bset]);
            ba.keep = at<uint64_t>(p, p->off_keep[bset]);
            ba.total_dev = at<uint32_t>(p, st.off_btotal[b]);
            ba.lb.status = at<uint64_t>(p, st.off_bstatus[b]);
            ba.lb.counter = at<uint32_t>(p, st.off_bcounter[b]);
            ba.seed = p->seed32;
            ba.k = static_cast<int>(p->opts.k);
            ba.logB = p->logB;
            static const char *stage_name[kBuildStages] = {"bfb_hist", "bfb_scan", "bfb_scatter", "bfb_region"};
            for (int stg = 0; stg < kBuildStages; ++stg) {
                ProfScope ps(p, std::string(stage_name[stg]) + ":" + tag + ":f" + std::to_string(f), si,
                             kProfBuild0 + kBuildStages * static_cast<int>(b) + stg);
                SJ_HIP(p->ctx, launch_filter_build_stage(ba, stg, bstream));
            }
        }
        if (sj_status e = join_streams(p, nfork)) return e;
    }
    return SJ_OK;
}


// A phase's steps level by level; the steps of one level on branches of their own.
static sj_status run_steps(sj_plan_t *p, int phase) {
    for (const auto &lv : p->level_steps[phase]) {
        const int nb = static_cast<int>(std::min<size_t>(lv.size(), sj_plan_s::kSets));
        hipStream_t br[sj_plan_s::kSets];
        if (sj_status st = fork_streams(p, nb, br)) return st;
        for (int si : lv) {
            StepSpec &st = p->steps[si];
            if (sj_status e = run_step(p, st, br[st.branch])) return e;
        }
        if (sj_status st = join_streams(p, nb)) return st;
    }
    return SJ_OK;
}

static sj_status zero_region(sj_plan_t *p, int ph) {
    const Region &r = p->zero[ph];
    ProfScope ps(p, "zero:" + std::to_string(ph));
    SJ_HIP(p->ctx, launch_zero(p->ws + r.begin, r.end - r.begin, p->ls));
    return SJ_OK;
}

// Failure injection (SJ_FLAG_FAULT_*): the phase fails before it enqueues anything.
static sj_status injected(sj_plan_t *p, uint32_t flag, const char *phase) {
    if (!(p->opts.flags & flag)) return SJ_OK;
    return fail(p->ctx, SJ_ERR_DEVICE, "%s failed: injected failure (SJ_FLAG_FAULT_*)", phase);
}

static sj_status check_exec(sj_plan_t *p, int need) {
    if (!p) return SJ_ERR_INVALID;
    if (p->state < need) {
        static const char *names[] = {"sj_plan", "sj_bind_workspace", "sj_build_filters", "sj_sieve", "sj_join"};
        return fail(p->ctx, SJ_ERR_STATE, "call %s first", names[need]);
    }
    SJ_HIP(p->ctx, hipSetDevice(p->ctx->device));
    // an error left by an earlier, unrelated HIP call would otherwise be reported by the
    // launch checks of this call (sticky device errors still fail the launches)
    (void)hipGetLastError();
    return SJ_OK;
}


// Branch streams and their events, created outside any capture. Only recorded graphs
// fork: an eager plan (one-shot queries, profiling) keeps every launch on one stream,
// where stream creation and the extra event calls would cost more host time than
// the overlap saves.
static sj_status ensure_branches(sj_plan_t *p) {
    if (p->eager || p->fork_ev) return SJ_OK;
    for (auto &b : p->branch) SJ_HIP(p->ctx, hipStreamCreateWithFlags(&b, hipStreamNonBlocking));
    for (auto &e : p->join_ev) SJ_HIP(p->ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    SJ_HIP(p->ctx, hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming));
    return SJ_OK;
}

// Fork: branch i (of n) gets out[i], which starts after everything enqueued on the
// launch stream so far. Eager plans (profiled ones among them, so that each group's
// events time it alone) keep every launch on the launch stream.
static sj_status fork_streams(sj_plan_t *p, int n, hipStream_t *out) {
    if (p->eager || n <= 1) {
        for (int i = 0; i < n; ++i) out[i] = p->ls;
        return SJ_OK;
    }
    if (sj_status st = ensure_branches(p)) return st;
    SJ_HIP(p->ctx, hipEventRecord(p->fork_ev, p->ls));
    for (int i = 0; i < n; ++i) {
        if (i < sj_plan_s::kBranches) SJ_HIP(p->ctx, hipStreamWaitEvent(p->branch[i], p->fork_ev, 0));
        out[i] = p->branch[i % sj_plan_s::kBranches];
    }
    return SJ_OK;
}

// Join: the launch stream continues after every branch of the last fork of n.
static sj_status join_streams(sj_plan_t *p, int n) {
    if (p->eager || n <= 1) return SJ_OK;
    for (int i = 0; i < n && i < sj_plan_s::kBranches; ++i) {
        SJ_HIP(p->ctx, hipEventRecord(p->join_ev[i], p->branch[i]));
        SJ_HIP(p->ctx, hipStreamWaitEvent(p->ls, p->join_ev[i], 0));
    }
    return SJ_OK;
}

// Enqueue one launch phase on the context's stream: eagerly, or by replaying the
// phase's graph, recorded from `enqueue` on the first call.
static sj_status run_phase(sj_plan_t *p, int ph, sj_status (*enqueue)(sj_plan_t *)) {
    if (p->eager) {
        p->ls = p->ctx->stream;
        return enqueue(p);
    }
    if (!p->gexec[ph]) {
        if (!p->cap_stream) SJ_HIP(p->ctx, hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
        if (sj_status st = ensure_branches(p)) return st;
        p->ls = p->cap_stream;
        SJ_HIP(p->ctx, hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
        const sj_status st = enqueue(p);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
        if (st != SJ_OK || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            if (st != SJ_OK) return st;
            SJ_HIP(p->ctx, e);
        }
        const hipError_t ei = hipGraphInstantiate(&p->gexec[ph], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            p->gexec[ph] = nullptr;
            SJ_HIP(p->ctx, ei);
        }
    }
    SJ_HIP(p->ctx, hipGraphLaunch(p->gexec[ph], p->ctx->stream));
    return SJ_OK;
}

// ---------------------------------------------------------------- the pruning phase

static sj_status enqueue_build(sj_plan_t *p) {
    hipStream_t s = p->ls;
    if (sj_status st = zero_region(p, 0)) return st;
    uint32_t *elig = at<uint32_t>(p, p->off_elig);
    std::vector<int> withpred;
    for (int i = 0; i < p->n; ++i)
        if (p->rels[i].pred_col >= 0) withpred.push_back(i);
    const int nb = static_cast<int>(std::min<size_t>(withpred.size(), sj_plan_s::kSets));
    hipStream_t br[sj_plan_s::kSets];
    if (sj_status st = fork_streams(p, nb, br)) return st;
    for (size_t k = 0; k < withpred.size(); ++k) {
        const int i = withpred[k];
        const Rel &R = p->rels[i];
        ProfScope ps(p, std::string("count_pred:") + rel_name(i));
        SJ_HIP(p->ctx, launch_count_pred(R.cols[R.pred_col], R.nrows, R.lo, R.hi, elig + i,
                                         nb ? br[k % sj_plan_s::kSets] : s));
    }
    if (sj_status st = join_streams(p, nb)) return st;
    return run_steps(p, 0);
}

extern "C" sj_status sj_build_filters(sj_plan_t *p) {
    if (sj_status st = check_exec(p, kBound)) return st;
    if (sj_status st = injected(p, SJ_FLAG_FAULT_FILTERS, "sj_build_filters")) return st;
    // reused catalogue entries: wait for their producers' builds (once seen complete, never again)
    for (size_t i = 0; i < p->fc_wait.size();) {
        if (hipEventQuery(p->fc_wait[i]) == hipSuccess) {
            p->fc_wait.erase(p->fc_wait.begin() + static_cast<long>(i));
            continue;
        }
        SJ_HIP(p->ctx, hipStreamWaitEvent(p->ctx->stream, p->fc_wait[i], 0));
        ++i;
    }
    if (sj_status st = run_phase(p, 0, enqueue_build)) return st;
    // filters built into new catalogue entries: publish them; later calls reuse them too
    bool published = false;
    for (auto &F : p->filters) {
        if (!F.fc_pending) continue;
        if (sj_status st = fc_publish(p->fcache, F.fc, p->ctx->stream))
            return fail(p->ctx, st, "could not record a catalogue entry's readiness");
        F.fc_pending = false;
        published = true;
    }
    if (published && p->gexec[0]) {   // the recorded pruning phase still builds them
        (void)hipGraphExecDestroy(p->gexec[0]);
        p->gexec[0] = nullptr;
    }
    if (sj_status st = fc_mark_use(p)) return fail(p->ctx, st, "could not record the use of catalogue entries");
    p->state = kFiltered;
    return SJ_OK;
}

static sj_status enqueue_sieve(sj_plan_t *p) {
    if (sj_status st = zero_region(p, 1)) return st;
    return run_steps(p, 1);
}

extern "C" sj_status sj_sieve(sj_plan_t *p, uint64_t *survivors) {
    if (sj_status st = check_exec(p, kFiltered)) return st;
    if (sj_status st = injected(p, SJ_FLAG_FAULT_SIEVE, "sj_sieve")) return st;
    if (sj_status st = run_phase(p, 1, enqueue_sieve)) return st;
    if (sj_status st = fc_mark_use(p)) return fail(p->ctx, st, "could not record the use of catalogue entries");
    p->state = kSieved;
    if (survivors) {
        std::vector<uint32_t> c(p->n);
        for (int i = 0; i < p->n; ++i)
            SJ_HIP(p->ctx, hipMemcpyAsync(&c[i], at<uint32_t>(p, p->steps[p->final_step[i]].off_count), 4,
                                          hipMemcpyDeviceToHost, p->ctx->stream));
        SJ_HIP(p->ctx, hipStreamSynchronize(p->ctx->stream));
        for (int i = 0; i < p->n; ++i) survivors[i] = c[i];
    }
    return SJ_OK;
}

// ---------------------------------------------------------------- the enumeration phase

static Buckets buckets_of(sj_plan_t *p, int j) {
    auto &r = p->jr[j];
    Buckets b{};
    b.cap = p->rels[j].nrows;
    b.n = at<uint32_t>(p, p->steps[p->final_step[j]].off_count);
    b.rid = at<uint32_t>(p, r.rid);
    b.npay = static_cast<int>(p->rels[j].jcols.size());
    for (int c = 0; c < b.npay; ++c) b.col[c] = at<int32_t>(p, r.cols + 4ull * b.cap * c);
    b.key_jcol = p->rels[j].jidx(p->mycol[j]);
    b.dir_begin = at<uint32_t>(p, r.dir_begin);
    b.dir_key = at<int32_t>(p, r.dir_key);
    b.ndir = at<uint32_t>(p, r.ndir);
    b.slots = at<uint64_t>(p, r.slots);
    b.slot_cap = r.slot_cap;
    b.slot_mask = at<uint32_t>(p, r.mask);
    b.cw = at<uint64_t>(p, r.cw);
    b.cv = at<uint64_t>(p, r.cv);
    return b;
}

// Materialisation arguments for preorder positions 0 .. npos-1 (npos = n: the whole
// tree; npos = n - 1: the prefix tree of a cyclic join, without L).
static MatArgs mat_args(sj_plan_t *p, int npos) {
    MatArgs m{};
    m.nrels = npos;
    std::vector<int> pos(p->n);
    for (int i = 0; i < p->n; ++i) pos[p->preorder[i]] = i;
    const int root = p->root;
    for (int x = 0; x < npos; ++x) {
        const int r = p->preorder[x];
        int nch = 0;
        for (int c : p->children[r])
            if (pos[c] < npos) ++nch;
        m.order[x] = r;
        m.is_leaf[x] = nch == 0 ? 1 : 0;
        m.nchild[x] = nch;
        if (x == 0) {
            m.parent_pos[x] = -1;
            m.rid[x] = list_rid(p, root, p->final_list[root]);
            m.cw[x] = at<uint64_t>(p, p->off_root_cw);
        } else {
            const int par = p->parent[r];
            const size_t c = std::find(p->children[par].begin(), p->children[par].end(), r) - p->children[par].begin();
            m.parent_pos[x] = pos[par];
            const Buckets b = buckets_of(p, r);
            m.rid[x] = b.rid;
            m.cw[x] = b.cw;
            m.blo[x] = at<uint32_t>(p, p->off_blo[par][c]);
            m.bhi[x] = at<uint32_t>(p, p->off_bhi[par][c]);
        }
    }
    m.root_n = at<uint32_t>(p, p->steps[p->final_step[root]].off_count);
    // subtree sizes (preorder: x's subtree is x .. x + subtree[x] - 1) and the tables of
    // the factorised materialisation, in each relation's sort scratch
    for (int x = npos - 1; x >= 0; --x) {
        m.subtree[x] = 1;
        for (int y = x + 1; y < npos; ++y)
            if (m.parent_pos[y] == x) m.subtree[x] += m.subtree[y];
    }
    for (int x = 0; x < npos; ++x) {
        const int r = p->preorder[x];
        m.n_ent[x] = at<uint32_t>(p, p->steps[p->final_step[r]].off_count);
        if (x > 0 && !m.is_leaf[x]) {
            const auto &jr = p->jr[r];
            const uint64_t cap = std::max<uint32_t>(1, p->rels[r].nrows);
            m.tab[x] = at<uint32_t>(p, jr.sklo[0]);
            m.tab_words[x] = (jr.svals[1] + 4 * cap - jr.sklo[0]) / 4;
        }
    }
    return m;
}

// Materialisation of the whole tree: the factorised launches (tables, then the output,
// then the decode, which writes only if some table did not fit) when the tree allows
// them, else the decode alone.
static sj_status launch_result(sj_plan_t *p, MatArgs &m, hipStream_t s) {
    if (!mat_factorisable(m)) {
        ProfScope ps(p, "materialize", -1, kProfResult);
        SJ_HIP(p->ctx, launch_materialize(m, s));
        return SJ_OK;
    }
    m.fact = 1;
    bool tables = false;
    for (int x = m.nrels - 1; x >= 1; --x) {
        if (m.is_leaf[x]) continue;
        tables = true;
        ProfScope ps(p, "mat_table:" + rel_name(p->preorder[x]), -1, kProfOther);
        SJ_HIP(p->ctx, launch_mat_table(m, x, s));
    }
    {
        ProfScope ps(p, "materialize", -1, kProfResult);
        SJ_HIP(p->ctx, launch_mat_output(m, s));
    }
    if (tables) {
        ProfScope ps(p, "mat_fallback", -1, kProfOther);
        SJ_HIP(p->ctx, launch_materialize(m, s));
    }
    return SJ_OK;
}

static CycArgs cyc_args(sj_plan_t *p, int32_t *out) {
    CycArgs c{};
    c.m = mat_args(p, p->n - 1);
    c.nrels = p->n;
    const int L = p->L, P = p->parent[L];
    std::vector<int> pos(p->n);
    for (int i = 0; i < p->n; ++i) pos[p->preorder[i]] = i;
    c.L_rel = L;
    c.pos_P = pos[P];
    const size_t ci = std::find(p->children[P].begin(), p->children[P].end(), L) - p->children[P].begin();
    c.Lblo = at<uint32_t>(p, p->off_blo[P][ci]);
    c.Lbhi = at<uint32_t>(p, p->off_bhi[P][ci]);
    const Buckets bl = buckets_of(p, L);
    c.Lrid = bl.rid;
    c.Lclose = p->cyc_cv >= 0 ? bl.col[p->rels[L].jidx(p->cyc_cv)] : nullptr;
    c.Lcv = bl.cv;
    // a prefix relation's join column, entry-indexed (the root's survivor list, else buckets)
    auto ecol = [&](int rel, int col) -> const int32_t * {
        const int jc = p->rels[rel].jidx(col);
        return rel == p->root ? list_col(p, rel, p->final_list[rel], jc) : buckets_of(p, rel).col[jc];
    };
    for (const Closing &cl : p->closing) {
        if (cl.v == L && cl.cv == p->cyc_cv) {
            c.cpos[c.nclose] = pos[cl.u];
            c.ccol[c.nclose++] = ecol(cl.u, cl.cu);
        } else if (cl.v == L) {
            c.xpos[c.nextra] = pos[cl.u];
            c.xcol[c.nextra] = ecol(cl.u, cl.cu);
            c.xL[c.nextra++] = bl.col[p->rels[L].jidx(cl.cv)];
        } else {
            c.ipos[c.ninner][0] = pos[cl.u];
            c.ipos[c.ninner][1] = pos[cl.v];
            c.icol[c.ninner][0] = ecol(cl.u, cl.cu);
            c.icol[c.ninner++][1] = ecol(cl.v, cl.cv);
        }
    }
    c.wpre = p->wpre;
    c.G = p->cyc_G;
    c.cnt = at<uint64_t>(p, p->off_cnt);
    c.chk = at<uint64_t>(p, p->off_chk);
    c.off = at<uint64_t>(p, p->off_off);
    c.totals = at<uint64_t>(p, p->off_totals);
    c.out = out;
    return c;
}

// Radix-sort scratch and look-back words of relation j's bucketing (the look-back
// words and histogram are cleared with the join phase's zero region). Each relation
// has its own, so that relations are bucketed concurrently.
static SortScratch sort_scratch(sj_plan_t *p, int j) {
    auto &r = p->jr[j];
    SortScratch ss{};
    ss.cap = p->rels[j].nrows;
    for (int q = 0; q < 2; ++q) {
        ss.klo[q] = at<uint32_t>(p, r.sklo[q]);
        ss.khi[q] = r.skhi[q] ? at<uint32_t>(p, r.skhi[q]) : nullptr;
        ss.vals[q] = at<uint32_t>(p, r.svals[q]);
    }
    ss.hist = at<uint32_t>(p, r.shist);
    ss.ghist = at<uint32_t>(p, r.ghist);
    ss.ctl = at<uint32_t>(p, r.sctl);
    for (int q = 0; q < kRadixPasses; ++q) {
        ss.lb[q].status = at<uint64_t>(p, r.lb_hist[q]);
        ss.lb[q].counter = at<uint32_t>(p, r.lb_hist_ctr[q]);
    }
    return ss;
}

static Lookback dir_lookback(sj_plan_t *p, int j) {
    return Lookback{at<uint64_t>(p, p->jr[j].lb_dir), at<uint32_t>(p, p->jr[j].lb_dir_ctr)};
}

// DP arguments of relation j: its own buckets (or the root's survivor list), its
// children's buckets and bounds, and its own scan scratch.
static sj_status dp_args(sj_plan_t *p, int j, DpArgs &d) {
    const int fl = p->final_list[j];
    const Rel &R = p->rels[j];
    const int ncol = static_cast<int>(R.jcols.size());
    d = DpArgs{};
    d.rel = static_cast<uint32_t>(j);
    d.nchild = static_cast<int>(p->children[j].size());
    if (d.nchild > kMaxJCols) return fail(p->ctx, SJ_ERR_UNSUPPORTED, "relation %d has more than %d children", j, kMaxJCols);
    for (int c = 0; c < d.nchild; ++c) {
        const int ch = p->children[j][c];
        d.child_col[c] = R.jidx(p->pcol[ch]);
        d.child[c] = buckets_of(p, ch);
        d.blo[c] = at<uint32_t>(p, p->off_blo[j][c]);
        d.bhi[c] = at<uint32_t>(p, p->off_bhi[j][c]);
        if (p->cyclic && ch == p->L) d.skip_mask |= 1u << c;
    }
    d.tile_sums = at<uint64_t>(p, j == p->root ? p->off_tile_sums : p->jr[j].tsums);
    if (j != p->root) {
        const Buckets b = buckets_of(p, j);
        d.n = b.n;
        d.cap = b.cap;
        d.rid = b.rid;
        for (int c = 0; c < ncol; ++c) d.col[c] = b.col[c];
        d.cw = b.cw;
        d.cv = b.cv;
        d.totals = nullptr;
    } else {
        d.n = at<uint32_t>(p, p->steps[p->final_step[j]].off_count);
        d.cap = R.nrows;
        d.rid = list_rid(p, j, fl);
        for (int c = 0; c < ncol; ++c) d.col[c] = list_col(p, j, fl, c);
        d.cw = at<uint64_t>(p, p->off_root_cw);
        d.cv = at<uint64_t>(p, p->off_root_cv);
        d.totals = at<uint64_t>(p, p->off_totals);
    }
    return SJ_OK;
}

// Count pass of the enumeration: bucket every non-root relation and run the join-tree
// DP from the leaves up; the root's totals land in the workspace.
static sj_status enqueue_join(sj_plan_t *p) {
    hipStream_t s = p->ls;
    if (sj_status st = zero_region(p, 2)) return st;
    // every non-root relation is bucketed on a branch of its own, and a leaf's DP (which
    // reads only its own buckets and scratch) follows there; after the branches join, the
    // other DPs run bottom-up on the launch stream
    std::vector<int> inner;
    for (int j : p->postorder)
        if (j != p->root) inner.push_back(j);
    std::vector<hipStream_t> br(std::max<size_t>(1, inner.size()));
    if (sj_status st = fork_streams(p, static_cast<int>(inner.size()), br.data())) return st;
    for (size_t i = 0; i < inner.size(); ++i) {
        const int j = inner[i];
        const int fl = p->final_list[j];
        const Rel &R = p->rels[j];
        const int ncol = static_cast<int>(R.jcols.size());
        std::vector<const int32_t *> lcols(ncol);
        for (int c = 0; c < ncol; ++c) lcols[c] = list_col(p, j, fl, c);
        const uint32_t *lcount = at<uint32_t>(p, p->steps[p->final_step[j]].off_count);
        Buckets b = buckets_of(p, j);
        int sec = -1;   // L of a cyclic join is ordered by its closing column inside each bucket
        if (p->cyclic && j == p->L && p->cyc_cv >= 0 && p->cyc_cv != p->mycol[j]) sec = R.jidx(p->cyc_cv);
        {
            ProfScope ps(p, std::string("buckets:") + rel_name(j), j, kProfBuckets);
            SJ_HIP(p->ctx, launch_build_buckets(list_rid(p, j, fl), lcols.data(), ncol, lcount, b.key_jcol, sec, b,
                                                sort_scratch(p, j), dir_lookback(p, j), br[i]));
        }
        if (!p->children[j].empty()) continue;
        DpArgs d;
        if (sj_status st = dp_args(p, j, d)) return st;
        ProfScope ps(p, std::string("dp:") + rel_name(j), j, kProfDp);
        SJ_HIP(p->ctx, launch_dp(d, br[i]));
    }
    if (sj_status st = join_streams(p, static_cast<int>(inner.size()))) return st;
    for (int j : p->postorder) {
        if (j != p->root && p->children[j].empty()) continue;   // weighed on its branch
        DpArgs d;
        if (sj_status st = dp_args(p, j, d)) return st;
        ProfScope ps(p, std::string("dp:") + rel_name(j), j, kProfDp);
        SJ_HIP(p->ctx, launch_dp(d, s));
    }
    return SJ_OK;
}

static PairHash pair_hash_of(sj_plan_t *p, int h) {
    PairHash ph{};
    ph.slot = at<PairSlot>(p, p->off_pair_slot[h]);
    ph.rel = static_cast<uint32_t>(p->pair_rel[h]);
    ph.msum = at<uint64_t>(p, p->off_pair_msum[h]);
    ph.cap = static_cast<uint32_t>(p->pair_cap[h]);
    ph.mask = at<uint32_t>(p, p->off_pair_mask[h]);
    ph.sig = at<uint32_t>(p, p->off_pair_sig[h]);
    ph.pos = at<uint32_t>(p, p->off_pair_pos[h]);
    return ph;
}

// The walk's arguments of a 3-cycle root - P - L - root: P grouped by its key toward
// the root (x), L by its closing column (y), each sorted by its (key, z) pairs inside
// the group; bk receives the two relations' buckets.
static TriArgs tri_args(sj_plan_t *p, Buckets bk[2], int key_col[2], int z_col[2]) {
    const int r = p->root, P = p->tri_P, L = p->L;
    const Closing &cl = p->closing[0];
    key_col[0] = p->rels[P].jidx(p->mycol[P]);
    key_col[1] = p->rels[L].jidx(cl.cv);
    z_col[0] = p->rels[P].jidx(p->pcol[L]);
    z_col[1] = p->rels[L].jidx(p->mycol[L]);
    for (int h = 0; h < 2; ++h) {
        bk[h] = buckets_of(p, h == 0 ? P : L);
        bk[h].key_jcol = key_col[h];
    }
    TriArgs a{};
    const Rel &R = p->rels[r];
    const int fl = p->final_list[r];
    a.n_root = at<uint32_t>(p, p->steps[p->final_step[r]].off_count);
    a.root_cap = R.nrows;
    a.root_rid = list_rid(p, r, fl);
    a.root_x = list_col(p, r, fl, R.jidx(p->pcol[P]));
    a.root_y = list_col(p, r, fl, R.jidx(cl.cu));
    a.rel_root = static_cast<uint32_t>(r);
    a.P_slots = bk[0].slots;
    a.P_mask = bk[0].slot_mask;
    a.P_begin = bk[0].dir_begin;
    a.P_rid = bk[0].rid;
    a.P_z = bk[0].col[z_col[0]];
    a.rel_P = static_cast<uint32_t>(P);
    a.L_slots = bk[1].slots;
    a.L_mask = bk[1].slot_mask;
    a.L_begin = bk[1].dir_begin;
    a.L_rid = bk[1].rid;
    a.L_z = bk[1].col[z_col[1]];
    a.rel_L = static_cast<uint32_t>(L);
    a.HP = pair_hash_of(p, 0);
    a.HL = pair_hash_of(p, 1);
    a.lane_cnt = at<uint64_t>(p, p->off_emit_lane);
    a.block_cnt = at<uint64_t>(p, p->off_emit_block);
    a.w = at<uint32_t>(p, p->off_tri_w);
    a.beg = at<uint32_t>(p, p->off_tri_beg);
    a.off = at<uint64_t>(p, p->off_tri_off);
    a.tile_sums = at<uint64_t>(p, p->off_tri_tiles);
    a.part = at<uint64_t>(p, p->off_tri_part);
    a.totals = at<uint64_t>(p, p->off_totals);
    return a;
}

// Count pass of a 3-cycle by intersection: the two relations bucketed and their pair
// hashes built on two branches, then the balanced walk.
static sj_status enqueue_tri(sj_plan_t *p) {
    hipStream_t s = p->ls;
    if (sj_status st = zero_region(p, 2)) return st;
    Buckets bk[2];
    int key_col[2], z_col[2];
    const TriArgs a = tri_args(p, bk, key_col, z_col);
    const int rel[2] = {p->tri_P, p->L};
    hipStream_t br[2];
    if (sj_status st = fork_streams(p, 2, br)) return st;
    for (int h = 0; h < 2; ++h) {
        const int j = rel[h];
        const int fl = p->final_list[j];
        const int ncol = static_cast<int>(p->rels[j].jcols.size());
        std::vector<const int32_t *> lcols(ncol);
        for (int c = 0; c < ncol; ++c) lcols[c] = list_col(p, j, fl, c);
        {
            ProfScope ps(p, std::string("buckets:") + rel_name(j), j, kProfBuckets);
            SJ_HIP(p->ctx, launch_build_buckets(list_rid(p, j, fl), lcols.data(), ncol, bk[h].n, key_col[h],
                                                z_col[h], bk[h], sort_scratch(p, j), dir_lookback(p, j), br[h]));
        }
        ProfScope ps(p, std::string("pairs:") + rel_name(j));
        SJ_HIP(p->ctx, launch_pair_build(pair_hash_of(p, h), bk[h].n, bk[h].cap, bk[h].rid, bk[h].col[key_col[h]],
                                         bk[h].col[z_col[h]], static_cast<uint32_t>(j), br[h]));
    }
    if (sj_status st = join_streams(p, 2)) return st;
    ProfScope ps(p, "tri_count");
    SJ_HIP(p->ctx, launch_tri_count(a, s));
    return SJ_OK;
}

// The walk's arguments of a 4-clique: the five non-root relations grouped by their
// earlier variable and sorted by their (earlier, later) pairs; bk receives their buckets.
static K4Args k4_args(sj_plan_t *p, Buckets bk[5]) {
    K4Args a{};
    a.lane_cnt = at<uint64_t>(p, p->off_emit_lane);
    a.block_cnt = at<uint64_t>(p, p->off_emit_block);
    const int r = p->root;
    const int fl = p->final_list[r];
    a.n_root = at<uint32_t>(p, p->steps[p->final_step[r]].off_count);
    a.root_cap = p->rels[r].nrows;
    a.root_rid = list_rid(p, r, fl);
    a.root_a = list_col(p, r, fl, 0);
    a.root_b = list_col(p, r, fl, 1);
    a.rel_root = static_cast<uint32_t>(r);
    for (int h = 0; h < 5; ++h) {
        bk[h] = buckets_of(p, p->k4_rel[h]);
        bk[h].key_jcol = p->k4_x[h];
        a.g[h].slots = bk[h].slots;
        a.g[h].mask = bk[h].slot_mask;
        a.g[h].begin = bk[h].dir_begin;
        a.g[h].rid = bk[h].rid;
        a.g[h].other = bk[h].col[p->k4_y[h]];
        a.g[h].rel = static_cast<uint32_t>(p->k4_rel[h]);
        a.h[h] = pair_hash_of(p, h);
    }
    a.w = at<uint32_t>(p, p->off_tri_w);
    a.beg = at<uint32_t>(p, p->off_tri_beg);
    a.off = at<uint64_t>(p, p->off_tri_off);
    a.tile_sums = at<uint64_t>(p, p->off_tri_tiles);
    a.part = at<uint64_t>(p, p->off_tri_part);
    a.totals = at<uint64_t>(p, p->off_totals);
    return a;
}

// Count pass of a 4-clique by intersection: the five non-root relations bucketed and
// their pair hashes built on branch streams, then the two-level walk from the root's
// survivors.
static sj_status enqueue_k4(sj_plan_t *p) {
    hipStream_t s = p->ls;
    if (sj_status st = zero_region(p, 2)) return st;
    Buckets bk[5];
    const K4Args a = k4_args(p, bk);
    hipStream_t br[sj_plan_s::kBranches];
    if (sj_status st = fork_streams(p, sj_plan_s::kBranches, br)) return st;
    for (int h = 0; h < 5; ++h) {
        const int j = p->k4_rel[h];
        const int fl = p->final_list[j];
        const int ncol = static_cast<int>(p->rels[j].jcols.size());
        std::vector<const int32_t *> lcols(ncol);
        for (int c = 0; c < ncol; ++c) lcols[c] = list_col(p, j, fl, c);
        hipStream_t bs = br[h % sj_plan_s::kBranches];
        {
            ProfScope ps(p, std::string("buckets:") + rel_name(j), j, kProfBuckets);
            SJ_HIP(p->ctx, launch_build_buckets(list_rid(p, j, fl), lcols.data(), ncol, bk[h].n, p->k4_x[h],
                                                p->k4_y[h], bk[h], sort_scratch(p, j), dir_lookback(p, j), bs));
        }
        ProfScope ps(p, std::string("pairs:") + rel_name(j));
        SJ_HIP(p->ctx, launch_pair_build(pair_hash_of(p, h), bk[h].n, bk[h].cap, bk[h].rid, bk[h].col[p->k4_x[h]],
                                         bk[h].col[p->k4_y[h]], static_cast<uint32_t>(j), bs));
    }
    if (sj_status st = join_streams(p, sj_plan_s::kBranches)) return st;
    ProfScope ps(p, "k4_count");
    SJ_HIP(p->ctx, launch_k4_count(a, s));
    return SJ_OK;
}

// Write pass of a 3-cycle or 4-clique counted by intersection (the count pass's walk,
// buckets and per-lane tuple counts are still in the workspace).
static sj_status clique_write(sj_plan_t *p, int32_t *out, uint64_t capacity, const Projection &pr) {
    CliqueOut o{};
    o.out = out;
    o.capacity = capacity;
    o.nrels = p->n;
    o.proj = pr;
    o.lane_cnt = at<uint64_t>(p, p->off_emit_lane);
    o.block_cnt = at<uint64_t>(p, p->off_emit_block);
    ProfScope ps(p, "clique_write", -1, kProfResult);
    if (p->tri) {
        o.role_rel[0] = p->root;
        o.role_rel[1] = p->tri_P;
        o.role_rel[2] = p->L;
        Buckets bk[2];
        int key_col[2], z_col[2];
        SJ_HIP(p->ctx, launch_tri_emit(tri_args(p, bk, key_col, z_col), o, p->ctx->stream));
    } else {
        o.role_rel[0] = p->root;
        for (int h = 0; h < 5; ++h) o.role_rel[h + 1] = p->k4_rel[h];
        Buckets bk[5];
        SJ_HIP(p->ctx, launch_k4_emit(k4_args(p, bk), o, p->ctx->stream));
    }
    return SJ_OK;
}

// The binary plan's count pass of a cyclic join (tree DP, then the prefixes' matches
// in L). Its per-thread offsets are what the write pass decodes.
static sj_status binary_cyclic_count(sj_plan_t *p, uint64_t tot[2]) {
    hipStream_t s = p->ctx->stream;
    if (sj_status st = run_phase(p, 2, enqueue_join)) return st;
    SJ_HIP(p->ctx, hipMemcpyAsync(tot, at<uint64_t>(p, p->off_totals), 16, hipMemcpyDeviceToHost, s));
    SJ_HIP(p->ctx, hipStreamSynchronize(s));
    // tot[0] counted the prefixes; now count their matches in L
    p->wpre = tot[0];
    uint64_t g = (p->wpre + 31) / 32;
    p->cyc_G = static_cast<uint32_t>(std::min<uint64_t>(g, kCycThreads));
    CycArgs c = cyc_args(p, nullptr);
    {
        ProfScope ps(p, "cyclic_count");
        SJ_HIP(p->ctx, launch_cyclic_count(c, s));
    }
    tot[0] = tot[1] = 0;
    if (p->cyc_G) {
        SJ_HIP(p->ctx, hipMemcpyAsync(tot, at<uint64_t>(p, p->off_totals), 16, hipMemcpyDeviceToHost, s));
        SJ_HIP(p->ctx, hipStreamSynchronize(s));
    }
    p->cyc_counted = true;
    return SJ_OK;
}

extern "C" sj_status sj_join(sj_plan_t *p, uint64_t *count, uint64_t *checksum) {
    if (sj_status st = check_exec(p, kSieved)) return st;
    if (sj_status st = injected(p, SJ_FLAG_FAULT_JOIN, "sj_join")) return st;
    if (!p->cyc_ok && !p->k4)
        return fail(p->ctx, SJ_ERR_UNSUPPORTED, "cyclic join with more than %d closing edges or more than 8 relations",
                    kMaxClose);
    hipStream_t s = p->ctx->stream;
    uint64_t tot[2] = {0, 0};
    p->cyc_counted = false;
    if (p->tri || p->k4) {
        if (sj_status st = run_phase(p, 4, p->tri ? enqueue_tri : enqueue_k4)) return st;
        SJ_HIP(p->ctx, hipMemcpyAsync(tot, at<uint64_t>(p, p->off_totals), 16, hipMemcpyDeviceToHost, s));
        SJ_HIP(p->ctx, hipStreamSynchronize(s));
    } else if (p->cyclic) {
        if (sj_status st = binary_cyclic_count(p, tot)) return st;
    } else {
        if (sj_status st = run_phase(p, 2, enqueue_join)) return st;
        SJ_HIP(p->ctx, hipMemcpyAsync(tot, at<uint64_t>(p, p->off_totals), 16, hipMemcpyDeviceToHost, s));
        SJ_HIP(p->ctx, hipStreamSynchronize(s));
    }
    p->count = tot[0];
    p->checksum = tot[1];
    p->count_on_host = true;
    p->async_result = false;
    if (count) *count = tot[0];
    if (checksum) *checksum = tot[1];
    p->state = kJoined;
    return SJ_OK;
}

extern "C" sj_status sj_join_async(sj_plan_t *p) {
    if (sj_status st = check_exec(p, kSieved)) return st;
    if (sj_status st = injected(p, SJ_FLAG_FAULT_JOIN, "sj_join_async")) return st;
    if (p->cyclic && !p->tri && !p->k4) {
        if (!p->cyc_ok)
            return fail(p->ctx, SJ_ERR_UNSUPPORTED, "cyclic join: this shape is not supported");
        return fail(p->ctx, SJ_ERR_UNSUPPORTED, "this cyclic join counts in two host-driven steps: use sj_join");
    }
    p->cyc_counted = false;
    if (sj_status st = p->tri ? run_phase(p, 4, enqueue_tri)
                              : p->k4 ? run_phase(p, 4, enqueue_k4) : run_phase(p, 2, enqueue_join))
        return st;
    p->count_on_host = false;
    p->async_result = false;
    p->state = kJoined;
    return SJ_OK;
}

// Output words per tuple in `mode`: one row id per relation, or the projection's columns.
static int result_width(const sj_plan_t *p, int32_t mode) {
    if (mode == SJ_RIDS) return p->n;
    if (!p->proj.empty()) return static_cast<int>(p->proj.size());
    int w = 0;
    for (const Rel &R : p->rels) w += static_cast<int>(R.cols.size());
    return w;
}

// The materialisation's output description for `mode` (row ids: proj.n = 0).
static sj_status projection_of(sj_plan_t *p, int32_t mode, Projection &pr) {
    pr = Projection{};
    if (mode == SJ_RIDS) return SJ_OK;
    if (mode != SJ_VALUES) return fail(p->ctx, SJ_ERR_INVALID, "mode must be SJ_RIDS or SJ_VALUES");
    std::vector<std::pair<int, int>> cols = p->proj;
    if (cols.empty())
        for (int r = 0; r < p->n; ++r)
            for (size_t c = 0; c < p->rels[r].cols.size(); ++c) cols.emplace_back(r, static_cast<int>(c));
    if (cols.size() > static_cast<size_t>(kMaxProj))
        return fail(p->ctx, SJ_ERR_UNSUPPORTED, "a value projection of %zu columns (at most %d; see sj_plan_set_projection)",
                    cols.size(), kMaxProj);
    pr.n = static_cast<int>(cols.size());
    for (int q = 0; q < pr.n; ++q) {
        pr.rel[q] = cols[q].first;
        pr.col[q] = p->rels[cols[q].first].cols[cols[q].second];
    }
    return SJ_OK;
}

static sj_status enqueue_result_async(sj_plan_t *p) {
    MatArgs m = mat_args(p, p->n);
    m.count_dev = at<uint64_t>(p, p->off_totals);
    m.capacity = p->res_cap;
    m.out = p->res_out;
    if (sj_status st = projection_of(p, p->res_mode, m.proj)) return st;
    return launch_result(p, m, p->ls);
}

extern "C" sj_status sj_result_async(sj_plan_t *p, int32_t *out, uint64_t capacity, int32_t mode) {
    if (sj_status st = check_exec(p, kJoined)) return st;
    if (sj_status st = injected(p, SJ_FLAG_FAULT_RESULT, "sj_result_async")) return st;
    if (p->cyclic) return fail(p->ctx, SJ_ERR_UNSUPPORTED, "cyclic joins: use sj_result");
    if (mode != SJ_RIDS && mode != SJ_VALUES) return fail(p->ctx, SJ_ERR_INVALID, "mode must be SJ_RIDS or SJ_VALUES");
    if (capacity && !out) return fail(p->ctx, SJ_ERR_INVALID, "null output buffer");
    if (reinterpret_cast<uintptr_t>(out) % 16) return fail(p->ctx, SJ_ERR_INVALID, "output must be 16-byte aligned");
    if (out != p->res_out || capacity != p->res_cap || mode != p->res_mode) {   // the recorded launch names them
        if (p->gexec[3]) (void)hipGraphExecDestroy(p->gexec[3]);
        p->gexec[3] = nullptr;
        p->res_out = out;
        p->res_cap = capacity;
        p->res_mode = mode;
    }
    if (sj_status st = run_phase(p, 3, enqueue_result_async)) return st;
    p->async_result = true;
    return SJ_OK;
}

extern "C" sj_status sj_join_wait(sj_plan_t *p, uint64_t *count, uint64_t *checksum, sj_status *result_status) {
    if (sj_status st = check_exec(p, kJoined)) return st;
    if (!p->count_on_host) {
        uint64_t tot[2] = {0, 0};
        SJ_HIP(p->ctx, hipMemcpyAsync(tot, at<uint64_t>(p, p->off_totals), 16, hipMemcpyDeviceToHost, p->ctx->stream));
        SJ_HIP(p->ctx, hipStreamSynchronize(p->ctx->stream));
        p->count = tot[0];
        p->checksum = tot[1];
        p->count_on_host = true;
    } else {
        SJ_HIP(p->ctx, hipStreamSynchronize(p->ctx->stream));
    }
    if (count) *count = p->count;
    if (checksum) *checksum = p->checksum;
    if (result_status)
        *result_status = !p->async_result ? SJ_OK : (p->count > p->res_cap ? SJ_ERR_CAPACITY : SJ_OK);
    return SJ_OK;
}

extern "C" sj_status sj_result(sj_plan_t *p, int32_t *out, uint64_t capacity, int32_t mode) {
    if (sj_status st = check_exec(p, kJoined)) return st;
    if (sj_status st = injected(p, SJ_FLAG_FAULT_RESULT, "sj_result")) return st;
    Projection pr;
    if (sj_status st = projection_of(p, mode, pr)) return st;
    if (!p->count_on_host) return fail(p->ctx, SJ_ERR_STATE, "call sj_join_wait first (the count is on the device)");
    if (capacity < p->count)
        return fail(p->ctx, SJ_ERR_CAPACITY, "result has %llu tuples, buffer holds %llu",
                    static_cast<unsigned long long>(p->count), static_cast<unsigned long long>(capacity));
    if (p->count == 0) return SJ_OK;
    if (!out) return fail(p->ctx, SJ_ERR_INVALID, "null output buffer");
    if (reinterpret_cast<uintptr_t>(out) % 16) return fail(p->ctx, SJ_ERR_INVALID, "output must be 16-byte aligned");
    if (p->tri || p->k4) return clique_write(p, out, capacity, pr);
    if (p->cyclic) {
        if (!p->cyc_counted) {
            // the binary count pass has not run since the last sieve: the write pass
            // decodes its per-thread offsets, and it must reach the same total
            uint64_t tot[2] = {0, 0};
            if (sj_status st = binary_cyclic_count(p, tot)) return st;
            if (tot[0] != p->count || tot[1] != p->checksum)
                return fail(p->ctx, SJ_ERR_DEVICE, "internal: the two cyclic count passes disagree");
        }
        CycArgs c = cyc_args(p, out);
        c.m.proj = pr;
        ProfScope ps(p, "cyclic_write", -1, kProfResult);
        SJ_HIP(p->ctx, launch_cyclic_write(c, p->ctx->stream));
        return SJ_OK;
    }
    MatArgs m = mat_args(p, p->n);
    m.count = p->count;
    m.capacity = capacity;
    m.out = out;
    m.proj = pr;
    p->res_mode = mode;   // for the profile's byte model
    return launch_result(p, m, p->ctx->stream);
}

extern "C" sj_status sj_plan_set_projection(sj_plan_t *p, const int32_t *rel_col, int32_t n) {
    if (!p) return SJ_ERR_INVALID;
    if (n < 0 || n > kMaxProj || (n > 0 && !rel_col))
        return fail(p->ctx, SJ_ERR_INVALID, "a projection has 0..%d columns", kMaxProj);
    std::vector<std::pair<int, int>> cols;
    for (int q = 0; q < n; ++q) {
        const int r = rel_col[2 * q], c = rel_col[2 * q + 1];
        if (r < 0 || r >= p->n || c < 0 || c >= static_cast<int>(p->rels[r].cols.size()))
            return fail(p->ctx, SJ_ERR_GRAPH, "projection column %d: relation %d column %d does not exist", q, r, c);
        cols.emplace_back(r, c);
    }
    p->proj = cols;
    if (p->gexec[3] && p->res_mode == SJ_VALUES) {   // the recorded materialisation names the columns
        (void)hipGraphExecDestroy(p->gexec[3]);
        p->gexec[3] = nullptr;
    }
    return SJ_OK;
}

extern "C" sj_status sj_plan_footprint(const sj_plan_t *p, int32_t mode, uint64_t *workspace_bytes,
                                       uint64_t *result_bytes, int32_t *width) {
    if (!p || (mode != SJ_RIDS && mode != SJ_VALUES)) return SJ_ERR_INVALID;
    if (workspace_bytes) *workspace_bytes = p->ws_bytes;
    if (width) *width = result_width(p, mode);
    if (result_bytes) {
        if (p->state < kJoined || !p->count_on_host) return fail(p->ctx, SJ_ERR_STATE, "the count is not known yet");
        *result_bytes = p->count * 4ull * static_cast<uint64_t>(result_width(p, mode));
    }
    return SJ_OK;
}

// ---------------------------------------------------------------- batches

#ifndef SJ_BATCH_ENABLED
#define SJ_BATCH_ENABLED 0
#endif
constexpr bool kBatchEnabled = SJ_BATCH_ENABLED != 0;

// A batch records the whole query of every plan it holds (pruning, count pass, and the
// materialisation with the count read on the device) into one HIP graph, the plans
// side by side on lanes forked from one capture stream, and replays it on the
// context's stream. Recorded on the first submit and again when the outputs change.
struct sj_batch {
    sj_ctx *ctx = nullptr;
    std::vector<sj_plan_t *> plans;
    std::vector<int32_t *> outs;
    std::vector<uint64_t> caps;
    int32_t mode = SJ_RIDS;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
    static constexpr int kLanes = 8;
    hipStream_t lane[kLanes] = {};
    hipEvent_t fork = nullptr, join[kLanes] = {};
    ~sj_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (cap) (void)hipStreamDestroy(cap);
        for (auto &l : lane)
            if (l) (void)hipStreamDestroy(l);
        for (auto &e : join)
            if (e) (void)hipEventDestroy(e);
        if (fork) (void)hipEventDestroy(fork);
        ctx_release(ctx);
    }
};

extern "C" sj_status sj_batch_create(sj_ctx *ctx, sj_plan_t *const *plans, int32_t n, sj_batch **out) {
    if (!ctx || !out || n < 1 || n > SJ_MAX_BATCH || !plans) return fail(ctx, SJ_ERR_INVALID, "a batch holds 1..%d plans", SJ_MAX_BATCH);
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
        sj_plan_t *p = plans[i];
        if (!p) return fail(ctx, SJ_ERR_INVALID, "plan %d is null", i);
        if (p->ctx != ctx) return fail(ctx, SJ_ERR_INVALID, "plan %d was made on another context", i);
        if (p->state < kBound) return fail(ctx, SJ_ERR_STATE, "plan %d has no workspace (sj_bind_workspace first)", i);
        if (p->profile || p->fcache)
            return fail(ctx, SJ_ERR_UNSUPPORTED, "plan %d: profiling plans and plans attached to a filter catalogue "
                                                 "are not batched", i);
        if (!p->cyc_ok || (p->cyclic && !p->tri))
            return fail(ctx, SJ_ERR_UNSUPPORTED, "plan %d: this cyclic join counts in two host-driven steps", i);
        if (p->opts.flags & (SJ_FLAG_FAULT_FILTERS | SJ_FLAG_FAULT_SIEVE | SJ_FLAG_FAULT_JOIN | SJ_FLAG_FAULT_RESULT))
            return fail(ctx, SJ_ERR_DEVICE, "plan %d: injected failure (SJ_FLAG_FAULT_*)", i);
        for (int j = 0; j < i; ++j) {
            if (plans[j] == p) return fail(ctx, SJ_ERR_INVALID, "plan %d appears twice", i);
            const char *a0 = p->ws, *a1 = p->ws + p->ws_bytes, *b0 = plans[j]->ws, *b1 = plans[j]->ws + plans[j]->ws_bytes;
            if (p->ws_bytes && plans[j]->ws_bytes && a0 < b1 && b0 < a1)
                return fail(ctx, SJ_ERR_INVALID, "plans %d and %d share workspace memory (they run at the same time)",
                            j, i);
        }
    }
    sj_batch *b = new (std::nothrow) sj_batch;
    if (!b) return fail(ctx, SJ_ERR_INVALID, "out of host memory");
    b->ctx = ctx;
    ctx->refs.fetch_add(1, std::memory_order_relaxed);
    b->plans.assign(plans, plans + n);
    *out = b;
    return SJ_OK;
}

// Record every plan's query into one graph (called with b->outs, caps, mode set).
static sj_status batch_record(sj_batch *b) {
    sj_ctx *ctx = b->ctx;
    if (!b->cap) {
        SJ_HIP(ctx, hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
        for (auto &l : b->lane) SJ_HIP(ctx, hipStreamCreateWithFlags(&l, hipStreamNonBlocking));
        for (auto &e : b->join) SJ_HIP(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
        SJ_HIP(ctx, hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
    }
    for (sj_plan_t *p : b->plans)
        if (sj_status st = ensure_branches(p)) return st;
    SJ_HIP(ctx, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    sj_status st = SJ_OK;
    const int nl = static_cast<int>(std::min<size_t>(b->plans.size(), sj_batch::kLanes));
    if (hipEventRecord(b->fork, b->cap) != hipSuccess) st = fail(ctx, SJ_ERR_DEVICE, "batch fork record failed");
    for (int l = 0; st == SJ_OK && l < nl; ++l)
        if (hipStreamWaitEvent(b->lane[l], b->fork, 0) != hipSuccess) st = fail(ctx, SJ_ERR_DEVICE, "batch fork failed");
    for (size_t i = 0; st == SJ_OK && i < b->plans.size(); ++i) {
        sj_plan_t *p = b->plans[i];
        p->ls = b->lane[i % sj_batch::kLanes];
        p->res_out = b->outs[i];
        p->res_cap = b->caps[i];
        p->res_mode = b->mode;
        if ((st = enqueue_build(p)) != SJ_OK) break;
        if ((st = enqueue_sieve(p)) != SJ_OK) break;
        if ((st = p->tri ? enqueue_tri(p) : enqueue_join(p)) != SJ_OK) break;
        if (!p->cyclic && b->outs[i] && (st = enqueue_result_async(p)) != SJ_OK) break;
    }
    for (int l = 0; st == SJ_OK && l < nl; ++l) {
        if (hipEventRecord(b->join[l], b->lane[l]) != hipSuccess ||
            hipStreamWaitEvent(b->cap, b->join[l], 0) != hipSuccess)
            st = fail(ctx, SJ_ERR_DEVICE, "batch join failed");
    }
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (st != SJ_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        if (st != SJ_OK) return st;
        SJ_HIP(ctx, e);
    }
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
        b->exec = nullptr;
        SJ_HIP(ctx, ei);
    }
    return SJ_OK;
}

extern "C" sj_status sj_batch_submit(sj_batch *b, int32_t *const *out_dev, const uint64_t *capacity_tuples,
                                     int32_t mode) {
    if (!b) return SJ_ERR_INVALID;
    sj_ctx *ctx = b->ctx;
    // Switched off: recording a batch (17 plans on lanes forked from one capture stream)
    // crashed the host process inside this call on MI355X. The capture is legal under
    // the stream-capture rules the host checker models and the host code is clean under
    // AddressSanitizer, so no cause in this code is known; until one is, the call refuses.
    if (!kBatchEnabled)
        return fail(ctx, SJ_ERR_UNSUPPORTED, "batched submission is switched off in this build (see sievejoin.h)");
    if (mode != SJ_RIDS && mode != SJ_VALUES) return fail(ctx, SJ_ERR_INVALID, "mode must be SJ_RIDS or SJ_VALUES");
    const size_t n = b->plans.size();
    std::vector<int32_t *> outs(n, nullptr);
    std::vector<uint64_t> caps(n, 0);
    for (size_t i = 0; i < n; ++i) {
        if (out_dev && out_dev[i]) {
            if (b->plans[i]->cyclic)
                return fail(ctx, SJ_ERR_UNSUPPORTED, "plan %zu is cyclic: its tuples need sj_result", i);
            if (reinterpret_cast<uintptr_t>(out_dev[i]) % 16)
                return fail(ctx, SJ_ERR_INVALID, "output %zu must be 16-byte aligned", i);
            outs[i] = out_dev[i];
            caps[i] = capacity_tuples ? capacity_tuples[i] : 0;
        }
        if (b->plans[i]->state < kBound) return fail(ctx, SJ_ERR_STATE, "plan %zu lost its workspace", i);
    }
    SJ_HIP(ctx, hipSetDevice(ctx->device));
    (void)hipGetLastError();
    if (!b->exec || outs != b->outs || caps != b->caps || mode != b->mode) {
        b->outs = outs;
        b->caps = caps;
        b->mode = mode;
        if (sj_status st = batch_record(b)) {
            if (b->exec) (void)hipGraphExecDestroy(b->exec);
            b->exec = nullptr;
            return st;
        }
    }
    SJ_HIP(ctx, hipGraphLaunch(b->exec, ctx->stream));
    for (size_t i = 0; i < n; ++i) {   // each plan now holds a device-side count (sj_join_wait)
        sj_plan_t *p = b->plans[i];
        p->cyc_counted = false;
        p->count_on_host = false;
        p->async_result = outs[i] != nullptr;
        p->res_out = outs[i];
        p->res_cap = caps[i];
        p->res_mode = mode;
        if (p->gexec[3]) {   // the plan's own recorded materialisation may name other outputs
            (void)hipGraphExecDestroy(p->gexec[3]);
            p->gexec[3] = nullptr;
        }
        p->state = kJoined;
    }
    return SJ_OK;
}

extern "C" sj_status sj_batch_destroy(sj_batch *b) {
    delete b;
    return SJ_OK;
}

// ---------------------------------------------------------------- filter catalogue

// Canonical signature of relation j's backward filter: everything its bits depend on.
// Its rows (count, build column, predicate), then each child's probe column with the
// child's own signature, sorted, since the order of probes does not change the
// survivors. `cols` collects the columns read, for invalidation.
static std::string fc_sig(const sj_plan_t *p, int j, std::vector<const void *> &cols) {
    const Rel &R = p->rels[j];
    char buf[128];
    std::snprintf(buf, sizeof buf, "n%u:k%p", R.nrows, static_cast<const void *>(R.cols[p->mycol[j]]));
    std::string s = buf;
    cols.push_back(R.cols[p->mycol[j]]);
    if (R.pred_col >= 0) {
        std::snprintf(buf, sizeof buf, ":p%p:%d:%d", static_cast<const void *>(R.cols[R.pred_col]), R.lo, R.hi);
        s += buf;
        cols.push_back(R.cols[R.pred_col]);
    }
    std::vector<std::string> kids;
    for (int c : p->children[j]) {
        std::snprintf(buf, sizeof buf, "%p", static_cast<const void *>(R.cols[p->pcol[c]]));
        cols.push_back(R.cols[p->pcol[c]]);
        kids.push_back(std::string(buf) + "(" + fc_sig(p, c, cols) + ")");
    }
    std::sort(kids.begin(), kids.end());
    s += "[";
    for (auto &k : kids) s += k + ";";
    return s + "]";
}

extern "C" sj_status sj_plan_use_filter_cache(sj_plan_t *p, sj_fcache *cache) {
    if (!p) return SJ_ERR_INVALID;
    if (cache && fc_device(cache) != p->ctx->device)
        return fail(p->ctx, SJ_ERR_INVALID, "the filter catalogue is on device %d, the plan on %d", fc_device(cache),
                    p->ctx->device);
    if (p->fcache) {
        SJ_HIP(p->ctx, hipSetDevice(p->ctx->device));
        p->fc_detach();
    }
    p->drop_graphs();   // recorded launches name the previous filter locations
    if (p->state > kBound) p->state = kBound;
    if (!cache) return SJ_OK;
    SJ_HIP(p->ctx, hipSetDevice(p->ctx->device));
    p->fc_last_use = std::make_shared<FcEvent>();
    SJ_HIP(p->ctx, hipEventCreateWithFlags(&p->fc_last_use->ev, hipEventDisableTiming));
    p->fc_used = false;
    p->fcache = cache;
    char opt[96];
    std::snprintf(opt, sizeof opt, "b%u,k%u,B%u,s%08x,p%u|", p->opts.bits_per_key, p->opts.k, p->opts.block_bits,
                  p->seed32, p->opts.passes);
    for (int j : p->postorder) {
        if (j == p->root) continue;
        Filter &F = p->filters[p->f_bwd[j]];
        std::vector<const void *> cols;
        const std::string sig = opt + fc_sig(p, j, cols);
        const FcGrant g = fc_acquire(cache, sig, F.max_words, cols);
        if (!g.entry) continue;   // no room: built in the workspace
        F.fc = g.entry;
        F.ext_words = g.words;
        F.ext_nblocks = g.nblocks;
        F.fc_how = g.hit ? 1 : 2;
        F.fc_pending = !g.hit;
        if (g.hit && g.ready) p->fc_wait.push_back(g.ready);
    }
    return SJ_OK;
}

extern "C" sj_status sj_plan_filter_cached(const sj_plan_t *p, int32_t f, int32_t *how) {
    if (!p || !how || f < 0 || f >= static_cast<int32_t>(p->filters.size())) return SJ_ERR_INVALID;
    *how = p->filters[f].fc_how;
    return SJ_OK;
}

// ---------------------------------------------------------------- introspection

extern "C" sj_status sj_filter_count(const sj_plan_t *p, int32_t *nf) {
    if (!p || !nf) return SJ_ERR_INVALID;
    *nf = static_cast<int32_t>(p->filters.size());
    return SJ_OK;
}

extern "C" sj_status sj_filter_desc(sj_plan_t *p, int32_t f, int32_t *kind, int32_t *index, int32_t *src_rel,
                                    int32_t *src_col, uint32_t *nblocks) {
    if (!p || f < 0 || f >= static_cast<int32_t>(p->filters.size())) return SJ_ERR_INVALID;
    const Filter &F = p->filters[f];
    if (kind) *kind = F.kind;
    if (index) *index = F.index;
    if (src_rel) *src_rel = F.src_rel;
    if (src_col) *src_col = F.src_col;
    if (nblocks) {
        if (sj_status st = check_exec(p, kFiltered)) return st;
        uint32_t nb = 0;
        SJ_HIP(p->ctx, hipMemcpyAsync(&nb, fnblocks(p, f), 4, hipMemcpyDeviceToHost, p->ctx->stream));
        SJ_HIP(p->ctx, hipStreamSynchronize(p->ctx->stream));
        *nblocks = nb;
    }
    return SJ_OK;
}

extern "C" sj_status sj_filter_copy(sj_plan_t *p, int32_t f, uint32_t *dst, uint64_t capacity_words) {
    if (!p || f < 0 || f >= static_cast<int32_t>(p->filters.size()) || !dst) return SJ_ERR_INVALID;
    if (sj_status st = check_exec(p, kFiltered)) return st;
    uint32_t nb = 0;
    if (sj_status st = sj_filter_desc(p, f, nullptr, nullptr, nullptr, nullptr, &nb)) return st;
    const uint64_t words = static_cast<uint64_t>(nb) * (p->opts.block_bits / 32);
    if (capacity_words < words) return fail(p->ctx, SJ_ERR_CAPACITY, "filter has %llu words", static_cast<unsigned long long>(words));
    SJ_HIP(p->ctx, hipMemcpyAsync(dst, fwords(p, f), words * 4, hipMemcpyDeviceToDevice,
                                  p->ctx->stream));
    if (sj_status st = fc_mark_use(p)) return fail(p->ctx, st, "could not record the use of catalogue entries");
    return SJ_OK;
}

// Section 2.4: a new tuple's key goes into a relation's filter only if the filter does
// not contain it already; the keys that were missing are the ones to propagate.
static sj_status filter_update(sj_plan_t *p, int32_t f, const int32_t *keys, uint64_t n, uint8_t *contained,
                               uint64_t *missing, bool set) {
    if (!p || f < 0 || f >= static_cast<int32_t>(p->filters.size())) return SJ_ERR_INVALID;
    const Filter &F = p->filters[f];
    // backward filters exist after sj_build_filters, forward and closing ones after sj_sieve
    if (sj_status st = check_exec(p, F.kind == SJ_FILTER_BACKWARD ? kFiltered : kSieved)) return st;
    if (n > 0 && (!keys || !contained)) return fail(p->ctx, SJ_ERR_INVALID, "null keys or flags");
    if (set && F.fc_how != 0)
        return fail(p->ctx, SJ_ERR_STATE, "filter %d is held in a filter catalogue and shared with other plans", f);
    FilterUpdate u{};
    u.words = fwords(p, f);
    u.nblocks = fnblocks(p, f);
    u.keys = keys;
    u.n = n;
    u.contained = contained;
    u.missing = at<unsigned long long>(p, p->off_upd);
    u.seed = p->seed32;
    u.k = static_cast<int>(p->opts.k);
    u.logB = p->logB;
    hipStream_t s = p->ctx->stream;
    SJ_HIP(p->ctx, launch_zero(u.missing, 8, s));
    SJ_HIP(p->ctx, launch_filter_update(u, set, s));
    if (sj_status st = fc_mark_use(p)) return fail(p->ctx, st, "could not record the use of catalogue entries");
    if (missing) {
        SJ_HIP(p->ctx, hipMemcpyAsync(missing, u.missing, 8, hipMemcpyDeviceToHost, s));
        SJ_HIP(p->ctx, hipStreamSynchronize(s));
    }
    return SJ_OK;
}

extern "C" sj_status sj_filter_probe(sj_plan_t *p, int32_t f, const int32_t *keys, uint64_t n, uint8_t *contained,
                                     uint64_t *missing) {
    return filter_update(p, f, keys, n, contained, missing, false);
}

extern "C" sj_status sj_filter_insert(sj_plan_t *p, int32_t f, const int32_t *keys, uint64_t n, uint8_t *contained,
                                      uint64_t *inserted) {
    return filter_update(p, f, keys, n, contained, inserted, true);
}

// ---------------------------------------------------------------- counting filters (Section 2.4)

// The counting twin of a plan's filter: one 4-bit counter per bit position (the filter's
// blocks, k, seed and bit pattern), in caller memory, followed by 256 bytes for the
// probe's missing-key count.
struct sj_cfilter {
    sj_ctx *ctx = nullptr;
    uint32_t *counts = nullptr;
    uint32_t nblocks = 0, k = 0, seed32 = 0;
    int logB = 9;
    uint64_t bytes() const { return (static_cast<uint64_t>(nblocks) << logB) / 2; }
    unsigned long long *missing() const {
        return reinterpret_cast<unsigned long long *>(reinterpret_cast<char *>(counts) + bytes());
    }
    CfArgs args(const int32_t *keys, uint64_t n) const {
        CfArgs a{};
        a.counts = counts;
        a.nblocks = nblocks;
        a.keys = keys;
        a.n = n;
        a.seed = seed32;
        a.k = static_cast<int>(k);
        a.logB = logB;
        return a;
    }
    ~sj_cfilter() { ctx_release(ctx); }
};

// The keys a plan inserted into filter f, with their multiplicity: what its build reads.
struct FilterSource {
    const int32_t *keys = nullptr;
    const uint32_t *n_dev = nullptr;
    uint32_t n = 0, n_max = 0;
    const int32_t *pred = nullptr;
    int32_t lo = 0, hi = 0;
};

static bool filter_source(sj_plan_t *p, int f, FilterSource &src) {
    for (const StepSpec &st : p->steps) {
        for (const auto &bl : st.builds) {
            if (bl.second != f) continue;
            const Rel &R = p->rels[st.rel];
            const int jc = bl.first;
            src.n_max = R.nrows;
            if (st.out >= 0) {
                src.keys = list_col(p, st.rel, st.out, jc);
                src.n_dev = at<uint32_t>(p, st.off_count);
            } else if (st.src == kFull) {
                src.keys = R.cols[R.jcols[jc]];
                src.n = R.nrows;
                if (R.pred_col >= 0) {
                    src.pred = R.cols[R.pred_col];
                    src.lo = R.lo;
                    src.hi = R.hi;
                }
            } else {
                src.keys = list_col(p, st.rel, st.src, jc);
                src.n_dev = at<uint32_t>(p, p->steps[st.src_step].off_count);
            }
            return true;
        }
    }
    return false;
}

extern "C" sj_status sj_plan_cfilter(sj_plan_t *p, int32_t f, void *counts_dev, uint64_t bytes, sj_cfilter **out) {
    if (!p || !out || f < 0 || f >= static_cast<int32_t>(p->filters.size())) return SJ_ERR_INVALID;
    *out = nullptr;
    const Filter &F = p->filters[f];
    if (sj_status st = check_exec(p, F.kind == SJ_FILTER_BACKWARD ? kFiltered : kSieved)) return st;
    if (reinterpret_cast<uintptr_t>(counts_dev) % 256) return fail(p->ctx, SJ_ERR_INVALID, "counters must be 256-byte aligned");
    uint32_t nb = 0;
    SJ_HIP(p->ctx, hipMemcpyAsync(&nb, fnblocks(p, f), 4, hipMemcpyDeviceToHost, p->ctx->stream));
    SJ_HIP(p->ctx, hipStreamSynchronize(p->ctx->stream));
    const uint64_t need = (static_cast<uint64_t>(nb) << p->logB) / 2 + 256;
    if (!counts_dev || bytes < need)
        return fail(p->ctx, SJ_ERR_NOMEM, "the counting filter of filter %d needs %llu bytes", f,
                    static_cast<unsigned long long>(need));
    FilterSource src;
    if (!filter_source(p, f, src)) return fail(p->ctx, SJ_ERR_INVALID, "internal: filter %d has no build", f);
    sj_cfilter *c = new (std::nothrow) sj_cfilter;
    if (!c) return fail(p->ctx, SJ_ERR_INVALID, "out of host memory");
    c->ctx = p->ctx;
    p->ctx->refs.fetch_add(1, std::memory_order_relaxed);
    c->counts = static_cast<uint32_t *>(counts_dev);
    c->nblocks = nb;
    c->k = p->opts.k;
    c->seed32 = p->seed32;
    c->logB = p->logB;
    CfArgs a = c->args(src.keys, src.n);
    a.pred = src.pred;
    a.pred_lo = src.lo;
    a.pred_hi = src.hi;
    hipStream_t s = p->ctx->stream;
    hipError_t e = launch_zero(c->counts, need, s);
    if (e == hipSuccess) e = launch_cf_update(a, src.n_dev, src.n_max, +1, s);
    if (e != hipSuccess) {
        delete c;
        return fail(p->ctx, SJ_ERR_DEVICE, "counting filter build failed: %s", hipGetErrorString(e));
    }
    *out = c;
    return SJ_OK;
}

extern "C" sj_status sj_cfilter_update(sj_cfilter *c, const int32_t *keys_dev, uint64_t n, int32_t sign) {
    if (!c) return SJ_ERR_INVALID;
    if ((sign != 1 && sign != -1) || (n && !keys_dev))
        return fail(c->ctx, SJ_ERR_INVALID, "sign must be +1 (insert) or -1 (delete), keys non-null");
    SJ_HIP(c->ctx, hipSetDevice(c->ctx->device));
    SJ_HIP(c->ctx, launch_cf_update(c->args(keys_dev, n), nullptr, 0, sign, c->ctx->stream));
    return SJ_OK;
}

extern "C" sj_status sj_cfilter_probe(sj_cfilter *c, const int32_t *keys_dev, uint64_t n, uint8_t *contained_dev,
                                      uint64_t *missing) {
    if (!c) return SJ_ERR_INVALID;
    if (n && (!keys_dev || !contained_dev)) return fail(c->ctx, SJ_ERR_INVALID, "null keys or flags");
    SJ_HIP(c->ctx, hipSetDevice(c->ctx->device));
    hipStream_t s = c->ctx->stream;
    SJ_HIP(c->ctx, launch_zero(c->missing(), 8, s));
    SJ_HIP(c->ctx, launch_cf_probe(c->args(keys_dev, n), contained_dev, c->missing(), s));
    if (missing) {
        SJ_HIP(c->ctx, hipMemcpyAsync(missing, c->missing(), 8, hipMemcpyDeviceToHost, s));
        SJ_HIP(c->ctx, hipStreamSynchronize(s));
    }
    return SJ_OK;
}

extern "C" sj_status sj_cfilter_export(sj_cfilter *c, uint32_t *words_dev, uint64_t capacity_words) {
    if (!c) return SJ_ERR_INVALID;
    const uint64_t words = static_cast<uint64_t>(c->nblocks) << (c->logB - 5);
    if (!words_dev || capacity_words < words)
        return fail(c->ctx, SJ_ERR_CAPACITY, "the filter has %llu words", static_cast<unsigned long long>(words));
    SJ_HIP(c->ctx, hipSetDevice(c->ctx->device));
    SJ_HIP(c->ctx, launch_cf_export(c->counts, words, words_dev, c->ctx->stream));
    return SJ_OK;
}

extern "C" sj_status sj_cfilter_apply(sj_cfilter *c, sj_plan_t *p, int32_t f) {
    if (!c || !p || f < 0 || f >= static_cast<int32_t>(p->filters.size())) return SJ_ERR_INVALID;
    const Filter &F = p->filters[f];
    if (sj_status st = check_exec(p, F.kind == SJ_FILTER_BACKWARD ? kFiltered : kSieved)) return st;
    if (F.fc_how != 0)
        return fail(p->ctx, SJ_ERR_STATE, "filter %d is held in a filter catalogue and shared with other plans", f);
    if (c->ctx->device != p->ctx->device || c->k != p->opts.k || c->logB != p->logB || c->seed32 != p->seed32)
        return fail(p->ctx, SJ_ERR_INVALID, "the counting filter does not twin filter %d (device, k, block, seed)", f);
    uint32_t nb = 0;
    SJ_HIP(p->ctx, hipMemcpyAsync(&nb, fnblocks(p, f), 4, hipMemcpyDeviceToHost, p->ctx->stream));
    SJ_HIP(p->ctx, hipStreamSynchronize(p->ctx->stream));
    if (nb != c->nblocks) return fail(p->ctx, SJ_ERR_INVALID, "filter %d has %u blocks, the counting filter %u", f, nb, c->nblocks);
    SJ_HIP(p->ctx, launch_cf_export(c->counts, static_cast<uint64_t>(nb) << (c->logB - 5), fwords(p, f),
                                    p->ctx->stream));
    return SJ_OK;
}

extern "C" sj_status sj_cfilter_destroy(sj_cfilter *c) {
    delete c;
    return SJ_OK;
}

// ---------------------------------------------------------------- propagation (Section 2.4)

// Scratch of sj_filter_propagate for n new rows of relation rel: a 256-byte counter
// area, flags and keys for the largest key batch on the path to the root, and a key set
// of twice that many slots (a power of two).
static uint64_t propagate_rows_max(const sj_plan_t *p, int rel, uint64_t n) {
    uint64_t m = n;
    for (int j = p->parent[rel]; j >= 0 && j != p->root; j = p->parent[j]) m = std::max<uint64_t>(m, p->rels[j].nrows);
    return m;
}
static uint64_t set_cap(uint64_t m) {
    uint64_t c = 16;
    while (c < 2 * m + 1) c <<= 1;
    return c;
}

extern "C" sj_status sj_filter_propagate_scratch(const sj_plan_t *p, int32_t rel, uint64_t n, uint64_t *bytes) {
    if (!p || !bytes || rel < 0 || rel >= p->n) return SJ_ERR_INVALID;
    const uint64_t m = propagate_rows_max(p, rel, n);
    *bytes = 256 + ((m + 255) & ~uint64_t(255)) + ((4 * m + 255) & ~uint64_t(255)) + 8 * set_cap(m);
    return SJ_OK;
}

extern "C" sj_status sj_filter_propagate(sj_plan_t *p, int32_t rel, const int32_t *const *cols, uint64_t n,
                                         void *scratch, uint64_t scratch_bytes, uint64_t *inserted) {
    if (!p || rel < 0 || rel >= p->n) return SJ_ERR_INVALID;
    if (sj_status st = check_exec(p, kFiltered)) return st;
    if (n > 0x7fffffffull) return fail(p->ctx, SJ_ERR_INVALID, "at most 2^31 - 1 new rows");
    if (n && !cols) return fail(p->ctx, SJ_ERR_INVALID, "null columns");
    if (inserted)
        for (int i = 0; i < p->n; ++i) inserted[i] = 0;
    if (n == 0 || rel == p->root) return SJ_OK;   // the root has no backward filter
    uint64_t need = 0;
    (void)sj_filter_propagate_scratch(p, rel, n, &need);
    if (!scratch || scratch_bytes < need || reinterpret_cast<uintptr_t>(scratch) % 256)
        return fail(p->ctx, SJ_ERR_NOMEM, "propagation needs %llu bytes of 256-byte aligned scratch",
                    static_cast<unsigned long long>(need));
    for (int j = rel; j >= 0 && j != p->root; j = p->parent[j])
        if (p->filters[p->f_bwd[j]].fc_how != 0)
            return fail(p->ctx, SJ_ERR_STATE, "the backward filter of relation %d is held in a filter catalogue", j);
    const uint64_t m = propagate_rows_max(p, rel, n);
    char *base = static_cast<char *>(scratch);
    uint32_t *counter = reinterpret_cast<uint32_t *>(base);                       // [0]: keys out, [2..3]: missing
    uint8_t *flags = reinterpret_cast<uint8_t *>(base + 256);
    int32_t *keys = reinterpret_cast<int32_t *>(base + 256 + ((m + 255) & ~uint64_t(255)));
    KeySet set{reinterpret_cast<uint64_t *>(base + 256 + ((m + 255) & ~uint64_t(255)) + ((4 * m + 255) & ~uint64_t(255))),
               static_cast<uint32_t>(set_cap(m) - 1)};
    hipStream_t s = p->ctx->stream;
    const Rel &R0 = p->rels[rel];
    int j = rel, from = -1;
    for (;;) {
        // the rows of j that now pass: the new rows (first level), or the rows whose key
        // toward the child `from` is among the keys that child's filter newly holds
        const Rel &R = p->rels[j];
        const bool first = from < 0;
        const int32_t *const *jc = first ? cols : R.cols.data();
        PropArgs a{};
        a.nrows = first ? n : R.nrows;
        a.match_col = first ? nullptr : jc[p->pcol[from]];
        a.set = first ? KeySet{nullptr, 0} : set;
        a.pred = R.pred_col >= 0 ? jc[R.pred_col] : nullptr;
        a.pred_lo = R.lo;
        a.pred_hi = R.hi;
        for (int c : p->children[j]) {
            if (c == from) continue;   // those rows match it by construction
            a.probe_col[a.nprobe] = jc[p->pcol[c]];
            a.probe[a.nprobe].words = fwords(p, p->f_bwd[c]);
            a.probe[a.nprobe].nblocks = fnblocks(p, p->f_bwd[c]);
            ++a.nprobe;
        }
        a.out_col = jc[p->mycol[j]];
        a.out = keys;
        a.out_n = counter;
        a.seed = p->seed32;
        a.k = static_cast<int>(p->opts.k);
        a.logB = p->logB;
        SJ_HIP(p->ctx, launch_zero(counter, 256, s));
        SJ_HIP(p->ctx, launch_propagate_rows(a, s));
        uint32_t got = 0;
        SJ_HIP(p->ctx, hipMemcpyAsync(&got, counter, 4, hipMemcpyDeviceToHost, s));
        SJ_HIP(p->ctx, hipStreamSynchronize(s));
        if (got == 0) break;
        // insert them into j's filter; the ones it did not hold go up to j's parent
        FilterUpdate u{};
        const int f = p->f_bwd[j];
        u.words = fwords(p, f);
        u.nblocks = fnblocks(p, f);
        u.keys = keys;
        u.n = got;
        u.contained = flags;
        u.missing = reinterpret_cast<unsigned long long *>(counter + 2);
        u.seed = p->seed32;
        u.k = static_cast<int>(p->opts.k);
        u.logB = p->logB;
        SJ_HIP(p->ctx, launch_filter_update(u, true, s));
        unsigned long long miss = 0;
        SJ_HIP(p->ctx, hipMemcpyAsync(&miss, counter + 2, 8, hipMemcpyDeviceToHost, s));
        SJ_HIP(p->ctx, hipStreamSynchronize(s));
        if (inserted) inserted[j] = miss;
        const int par = p->parent[j];
        if (miss == 0 || par == p->root) break;
        SJ_HIP(p->ctx, launch_zero(set.slots, 8 * (static_cast<uint64_t>(set.mask) + 1), s));
        SJ_HIP(p->ctx, launch_set_insert(set, keys, flags, got, s));
        from = j;
        j = par;
    }
    (void)R0;
    return SJ_OK;
}

extern "C" sj_status sj_survivors_copy(sj_plan_t *p, int32_t rel, uint32_t *dst, uint64_t capacity, uint64_t *n) {
    if (!p || rel < 0 || rel >= p->n || !n) return SJ_ERR_INVALID;
    if (sj_status st = check_exec(p, kSieved)) return st;
    uint32_t c = 0;
    SJ_HIP(p->ctx, hipMemcpyAsync(&c, at<uint32_t>(p, p->steps[p->final_step[rel]].off_count), 4,
                                  hipMemcpyDeviceToHost, p->ctx->stream));
    SJ_HIP(p->ctx, hipStreamSynchronize(p->ctx->stream));
    *n = c;
    if (c == 0 || !dst) return SJ_OK;
    if (capacity < c) return fail(p->ctx, SJ_ERR_CAPACITY, "relation %d has %u survivors", rel, c);
    SJ_HIP(p->ctx, hipMemcpyAsync(dst, list_rid(p, rel, p->final_list[rel]), 4ull * c, hipMemcpyDeviceToDevice,
                                  p->ctx->stream));
    return SJ_OK;
}

// ---------------------------------------------------------------- profiling ABI

extern "C" sj_status sj_profile_collect(sj_plan_t *p) {
    if (!p) return SJ_ERR_INVALID;
    if (p->prof_pending.empty()) return SJ_OK;
    SJ_HIP(p->ctx, hipStreamSynchronize(p->ctx->stream));
    std::vector<uint32_t> nb(p->filters.size());
    for (size_t f = 0; f < nb.size(); ++f)
        SJ_HIP(p->ctx, hipMemcpy(&nb[f], fnblocks(p, static_cast<int>(f)), 4, hipMemcpyDeviceToHost));
    for (auto &r : p->prof_pending) {
        float ms = 0;
        SJ_HIP(p->ctx, hipEventElapsedTime(&ms, r.a, r.b));
        auto &acc = p->prof_acc[r.label];
        acc.ms += ms;
        acc.n += 1;
        if (r.kind == kProfBuckets || r.kind == kProfDp) {
            // the join's byte models (per sieved entry n of relation j): bucketing reads and
            // writes an 8-byte (key, index) pair per active radix pass, gathers the row id and
            // join columns into bucket order (read and written once), reads each key for the
            // directory and writes each distinct key's directory entry and hash slot (16 B);
            // a DP reads each entry's row id, per child its key, the child's bucket bounds
            // and the two prefix pairs at them (28 B), writes the bounds (8 B per child) and
            // the entry's two prefix weights (16 B)
            const int j = r.step;
            const uint64_t ncol = p->rels[j].jcols.size();
            uint32_t n = 0;
            SJ_HIP(p->ctx, hipMemcpy(&n, at<uint32_t>(p, p->steps[p->final_step[j]].off_count), 4,
                                     hipMemcpyDeviceToHost));
            if (r.kind == kProfBuckets && j != p->root) {
                uint32_t ctl[kRadixPasses] = {}, ndir = 0;
                SJ_HIP(p->ctx, hipMemcpy(ctl, at<uint32_t>(p, p->jr[j].sctl), sizeof ctl, hipMemcpyDeviceToHost));
                SJ_HIP(p->ctx, hipMemcpy(&ndir, at<uint32_t>(p, p->jr[j].ndir), 4, hipMemcpyDeviceToHost));
                uint64_t passes = 0;
                for (uint32_t c : ctl) passes += c ? 1 : 0;
                acc.bytes = uint64_t(n) * (16 * passes + 8 * (1 + ncol) + 4) + uint64_t(ndir) * 16;
            } else if (r.kind == kProfDp) {
                const uint64_t nch = p->children[j].size();
                acc.bytes = uint64_t(n) * (4 + nch * (4 + 28 + 8) + 16);
            }
        } else if (r.step >= 0) {
            const StepSpec &st = p->steps[r.step];
            const Rel &R = p->rels[st.rel];
            const uint64_t ncol = R.jcols.size();
            const bool listsrc = st.src != kFull;
            uint32_t nin = R.nrows, nout = 0;
            if (listsrc)
                SJ_HIP(p->ctx, hipMemcpy(&nin, at<uint32_t>(p, p->steps[st.src_step].off_count), 4, hipMemcpyDeviceToHost));
            if (st.out >= 0) SJ_HIP(p->ctx, hipMemcpy(&nout, at<uint32_t>(p, st.off_count), 4, hipMemcpyDeviceToHost));
            const uint64_t fbytes = p->opts.block_bits / 8;
            uint64_t bytes = 0;
            // the probe: probed columns (+ the predicate column of a full scan) read, each
            // probed filter read once; the survivor list: each survivor's columns (+ row id
            // of a list source) read and its row id and columns written; between the two
            // launches of the two-launch form, one survivor bit per row written and read
            uint32_t used = 0;
            for (auto &pr : st.probes) used |= 1u << pr.first;
            const uint64_t pcols = __builtin_popcount(used) + (!listsrc && R.pred_col >= 0 ? 1 : 0);
            uint64_t probe_bytes = uint64_t(nin) * 4 * pcols;
            for (auto &pr : st.probes) probe_bytes += uint64_t(nb[pr.second]) * fbytes;
            const uint64_t list_bytes = uint64_t(nout) * 4 * (ncol + (listsrc ? 1 : 0)) + uint64_t(nout) * 4 * (ncol + 1);
            const uint64_t bit_bytes = (uint64_t(nin) + 7) / 8;
            if (r.kind == kProfProbe) {
                bytes = probe_bytes + bit_bytes;
            } else if (r.kind == kProfCompact) {
                bytes = bit_bytes + list_bytes;
            } else if (r.kind == kProfScan) {
                bytes = probe_bytes + list_bytes;
            } else if (r.kind >= kProfBuild0) {
                // keys read once (with the predicate column of a full scan): by the count and
                // the scatter stages; the staged keys: written by the scatter, read by the
                // region stage, which writes the filter once
                const int bi = (r.kind - kProfBuild0) / kBuildStages, stg = (r.kind - kProfBuild0) % kBuildStages;
                const auto &bl = st.builds[static_cast<size_t>(bi)];
                const uint64_t n = st.out >= 0 ? nout : nin;
                const uint64_t keys = n * 4 * (1 + (!listsrc && st.out < 0 && R.pred_col >= 0 ? 1 : 0));
                uint32_t staged = 0;
                SJ_HIP(p->ctx, hipMemcpy(&staged, at<uint32_t>(p, st.off_btotal[static_cast<size_t>(bi)]), 4,
                                         hipMemcpyDeviceToHost));
                if (stg == 0) bytes = keys;
                else if (stg == 2) bytes = keys + uint64_t(staged) * 4;
                else if (stg == 3) bytes = uint64_t(staged) * 4 + uint64_t(nb[bl.second]) * fbytes;
            }
            acc.bytes = bytes;
        } else if (r.kind == kProfResult) {
            acc.bytes = p->count * 4ull * static_cast<uint64_t>(result_width(p, p->res_mode));   // result written
        }
        p->prof_free.push_back(r.a);
        p->prof_free.push_back(r.b);
    }
    p->prof_pending.clear();
    return SJ_OK;
}

extern "C" sj_status sj_profile_count(const sj_plan_t *p, int32_t *n) {
    if (!p || !n) return SJ_ERR_INVALID;
    *n = static_cast<int32_t>(p->prof_acc.size());
    return SJ_OK;
}

extern "C" sj_status sj_profile_entry(const sj_plan_t *p, int32_t i, const char **label, double *total_ms,
                                      uint64_t *launches, uint64_t *alg_bytes) {
    if (!p || i < 0 || i >= static_cast<int32_t>(p->prof_acc.size())) return SJ_ERR_INVALID;
    const auto &a = p->prof_acc[i];
    if (label) *label = a.label.c_str();
    if (total_ms) *total_ms = a.ms;
    if (launches) *launches = a.n;
    if (alg_bytes) *alg_bytes = a.bytes;
    return SJ_OK;
}

extern "C" sj_status sj_profile_reset(sj_plan_t *p) {
    if (!p) return SJ_ERR_INVALID;
    if (sj_status st = sj_profile_collect(p)) return st;
    for (auto &a : p->prof_acc) {
        a.ms = 0;
        a.n = 0;
    }
    return SJ_OK;
}
