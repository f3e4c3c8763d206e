// Serving: continuous admission of join queries onto one GPU (the serving extension
// of include/sievejoin.h).
//
// The server owns a caller-provided device arena and `slots` worker threads, each with
// its own context and stream. A worker takes the oldest queued query whose workspace
// fits in the free arena (a later query may pass one that does not fit yet), runs the
// pruning and count phases on its stream, reserves the result's bytes once the exact
// count is known, materialises, and frees the workspace. Queries on different slots
// overlap on the device; a query waits only for memory and a free slot. Every arena
// region is 256-byte aligned.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "sievejoin.h"
#include "sj_arena.h"

using sj::Arena;
using sj::round256;

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Request {
    uint64_t ticket = 0;
    std::vector<sj_rel> rels;
    std::vector<std::vector<const int32_t *>> cols;   // the rels' column pointer arrays
    std::vector<sj_edge> edges;
    sj_opts opts{};
    int32_t mode = SJ_RESULT_TUPLES;
    sj_query_info info{};
    uint64_t ws_off = 0, res_off = 0, res_bytes = 0;
    bool has_result = false, released = false;
};

constexpr int64_t kResultWaitNs = 2000000000;   // a result waits at most 2 s for arena memory
// execute()'s answer when the query gave its workspace back to let others finish: the
// worker queues it again (not an sj_status; never reported to the caller)
constexpr sj_status kRequeue = 1;
// With nothing running and no queued query fitting, memory can only come back from
// results the caller releases; after this long the oldest queued query fails.
constexpr int64_t kAdmitStallNs = 2000000000;

}  // namespace

struct sj_server {
    int device = 0;
    char *base = nullptr;
    Arena arena{0};
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::shared_ptr<Request>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> all;
    std::vector<std::thread> workers;
    sj_ctx *plan_ctx = nullptr;   // validates queries at submit (planning is host-only)
    uint64_t next_ticket = 1;
    int running = 0;
    // running queries waiting for arena memory for their result; no query is admitted
    // while one waits, so that memory freed goes to results first
    std::vector<Request *> result_waiters;
    uint64_t requeues = 0;
    int64_t stall_since = 0;      // when admission last found nothing running and nothing fitting
    bool stop = false;
    sj_status init_status = SJ_OK;
    sj_fcache *fcache = nullptr;  // filter catalogue every admitted query attaches to
};

namespace {

void fail_request(Request &r, sj_status st, const char *msg) {
    r.info.state = SJ_QUERY_FAILED;
    r.info.status = st;
    std::snprintf(r.info.error, sizeof r.info.error, "%s", msg);
}

// Runs an admitted query on the worker's context. Called without the server lock.
sj_status execute(sj_server *s, Request &r, sj_ctx *ctx, hipStream_t stream, std::string &err) {
    sj_plan_t *plan = nullptr;
    uint64_t wsb = 0;
    sj_opts o = r.opts;
    o.flags |= SJ_FLAG_EAGER;   // one call per phase: recording a graph would cost more than it saves
    // the library's message for a failed call, or `msg`
    auto done = [&](sj_status code, const std::string &msg = std::string()) {
        if (code != SJ_OK) err = msg.empty() ? std::string(sj_last_error(ctx)) : msg;
        if (plan) sj_plan_destroy(plan);
        return code;
    };
    sj_status st = sj_plan(ctx, r.rels.data(), static_cast<int32_t>(r.rels.size()), r.edges.data(),
                           static_cast<int32_t>(r.edges.size()), &o, &plan, &wsb);
    if (st != SJ_OK) return done(st);
    if ((st = sj_bind_workspace(plan, s->base + r.ws_off, r.info.workspace_bytes)) != SJ_OK) return done(st);
    sj_fcache *fc = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        fc = s->fcache;
    }
    if (fc && (st = sj_plan_use_filter_cache(plan, fc)) != SJ_OK) return done(st);
    if ((st = sj_build_filters(plan)) != SJ_OK) return done(st);
    if ((st = sj_sieve(plan, nullptr)) != SJ_OK) return done(st);
    uint64_t count = 0, checksum = 0;
    if ((st = sj_join(plan, &count, &checksum)) != SJ_OK) return done(st);
    r.info.count = count;
    r.info.checksum = checksum;
    const int32_t rmode = r.mode == SJ_RESULT_VALUES ? SJ_VALUES : SJ_RIDS;
    if (r.mode != SJ_RESULT_COUNT && count > 0) {
        uint64_t need = 0;
        if ((st = sj_plan_footprint(plan, rmode, nullptr, &need, nullptr)) != SJ_OK) return done(st);
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (round256(need) > s->arena.size() - round256(r.info.workspace_bytes))
                return done(SJ_ERR_CAPACITY, "result of " + std::to_string(count) + " tuples does not fit the arena");
            // wait for memory that running queries or released results free up, for a bounded time
            const auto deadline = std::chrono::steady_clock::now() + std::chrono::nanoseconds(kResultWaitNs);
            bool got = s->arena.alloc(need, &r.res_off);
            if (!got) {
                s->result_waiters.push_back(&r);
                s->cv.notify_all();   // the other waiters re-check whether everyone now waits
                auto leave = [&] {
                    s->result_waiters.erase(std::find(s->result_waiters.begin(), s->result_waiters.end(), &r));
                    s->cv.notify_all();
                };
                while (!got) {
                    // Every running query waits for result memory, so none can finish and free
                    // its workspace: the one admitted last gives its workspace back and is
                    // queued again (its result is the same when it runs later).
                    if (s->running >= 2 && s->result_waiters.size() == static_cast<size_t>(s->running)) {
                        const Request *young = s->result_waiters.front();
                        for (const Request *w : s->result_waiters)
                            if (w->info.t_admit_ns > young->info.t_admit_ns ||
                                (w->info.t_admit_ns == young->info.t_admit_ns && w->ticket > young->ticket))
                                young = w;
                        if (young == &r) {
                            leave();
                            return done(kRequeue, "requeued");
                        }
                    }
                    const auto now = std::chrono::steady_clock::now();
                    s->cv.wait_until(lk, std::min(deadline, now + std::chrono::milliseconds(20)));
                    got = s->arena.alloc(need, &r.res_off);
                    if (!got && std::chrono::steady_clock::now() >= deadline) {
                        leave();
                        return done(SJ_ERR_NOMEM,
                                    "no arena memory for the result (" + std::to_string(need) + " bytes) within 2 s");
                    }
                }
                leave();
            }
            r.res_bytes = need;
            r.has_result = true;
        }
        if ((st = sj_result(plan, reinterpret_cast<int32_t *>(s->base + r.res_off), count, rmode)) != SJ_OK)
            return done(st);
        r.info.result_offset = r.res_off;
    }
    if (hipStreamSynchronize(stream) != hipSuccess) return done(SJ_ERR_DEVICE, "stream synchronisation failed");
    return done(SJ_OK);
}

void worker(sj_server *s, int slot) {
    hipStream_t stream = nullptr;
    sj_ctx *ctx = nullptr;
    const bool ok = hipSetDevice(s->device) == hipSuccess &&
                    hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess &&
                    sj_ctx_create(s->device, stream, &ctx) == SJ_OK;
    for (;;) {
        std::shared_ptr<Request> r;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            for (;;) {
                if (!ok && !s->queue.empty()) {   // a worker without a stream fails what it takes
                    r = s->queue.front();
                    s->queue.pop_front();
                    break;
                }
                // while a running query waits for result memory, nothing is admitted
                for (auto it = s->queue.begin(); s->result_waiters.empty() && it != s->queue.end(); ++it) {
                    if (s->arena.alloc((*it)->info.workspace_bytes, &(*it)->ws_off)) {
                        r = *it;
                        s->queue.erase(it);
                        break;
                    }
                }
                if (r || s->stop) break;
                if (s->running == 0 && !s->queue.empty()) {
                    const int64_t t = now_ns();
                    if (s->stall_since == 0) {
                        s->stall_since = t;
                    } else if (t - s->stall_since > kAdmitStallNs) {
                        auto head = s->queue.front();
                        s->queue.pop_front();
                        fail_request(*head, SJ_ERR_NOMEM,
                                     "workspace does not fit: the arena is held by results that are not released");
                        head->info.t_done_ns = t;
                        s->stall_since = 0;
                        s->cv.notify_all();
                        continue;
                    }
                } else {
                    s->stall_since = 0;
                }
                s->cv.wait_for(lk, std::chrono::milliseconds(50));
            }
            if (!r) break;
            if (!ok) {
                fail_request(*r, SJ_ERR_DEVICE, "worker could not create its stream");
                r->info.t_done_ns = now_ns();
                s->cv.notify_all();
                continue;
            }
            r->info.state = SJ_QUERY_RUNNING;
            r->info.slot = slot;
            r->info.t_admit_ns = now_ns();
            ++s->running;
        }
        std::string err;
        const sj_status st = execute(s, *r, ctx, stream, err);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->arena.release(r->ws_off, r->info.workspace_bytes);
            if (st == kRequeue) {   // back to the head of the queue, as if never admitted
                r->info.state = SJ_QUERY_QUEUED;
                r->info.slot = -1;
                r->info.t_admit_ns = 0;
                r->info.count = r->info.checksum = 0;
                ++r->info.requeues;
                ++s->requeues;
                --s->running;
                if (s->stop) {
                    fail_request(*r, SJ_ERR_STATE, "server destroyed before the query was admitted again");
                    r->info.t_done_ns = now_ns();
                } else {
                    s->queue.push_front(r);
                }
                s->cv.notify_all();
                continue;
            }
            if (st != SJ_OK) {
                if (r->has_result) {
                    s->arena.release(r->res_off, r->res_bytes);
                    r->has_result = false;
                }
                fail_request(*r, st, err.c_str());
            } else {
                r->info.state = SJ_QUERY_DONE;
                r->info.status = SJ_OK;
            }
            r->info.t_done_ns = now_ns();
            --s->running;
            s->cv.notify_all();
        }
    }
    if (ctx) sj_ctx_destroy(ctx);
    if (stream) (void)hipStreamDestroy(stream);
}

}  // namespace

extern "C" sj_status sj_server_create(int32_t device, void *arena_dev, uint64_t arena_bytes, int32_t slots,
                                      sj_server **out) {
    if (!out) return SJ_ERR_INVALID;
    *out = nullptr;
    if (device < 0 || slots < 1 || slots > SJ_MAX_SLOTS || (!arena_dev && arena_bytes)) return SJ_ERR_INVALID;
    if (reinterpret_cast<uintptr_t>(arena_dev) % 256) return SJ_ERR_INVALID;
    sj_server *s = new (std::nothrow) sj_server;
    if (!s) return SJ_ERR_INVALID;
    s->device = device;
    s->base = static_cast<char *>(arena_dev);
    s->arena = Arena(arena_bytes & ~uint64_t(255));
    if (sj_ctx_create(device, nullptr, &s->plan_ctx) != SJ_OK) {
        delete s;
        return SJ_ERR_INVALID;
    }
    for (int i = 0; i < slots; ++i) s->workers.emplace_back(worker, s, i);
    *out = s;
    return SJ_OK;
}

extern "C" sj_status sj_server_submit(sj_server *s, const sj_rel *rels, int32_t nrels, const sj_edge *edges,
                                      int32_t nedges, const sj_opts *opts, int32_t result_mode, uint64_t *ticket) {
    if (!s || !ticket ||
        (result_mode != SJ_RESULT_TUPLES && result_mode != SJ_RESULT_COUNT && result_mode != SJ_RESULT_VALUES))
        return SJ_ERR_INVALID;
    if (nrels < 0 || nrels > SJ_MAX_RELS || nedges < 0 || nedges > SJ_MAX_EDGES || (nrels && !rels) ||
        (nedges && !edges))
        return SJ_ERR_INVALID;
    auto r = std::make_shared<Request>();
    r->rels.assign(rels, rels + nrels);
    r->cols.resize(nrels);
    for (int i = 0; i < nrels; ++i) {
        if (rels[i].ncols < 0 || rels[i].ncols > SJ_MAX_COLS || (rels[i].ncols && !rels[i].cols)) return SJ_ERR_INVALID;
        r->cols[i].assign(rels[i].cols, rels[i].cols + rels[i].ncols);
        r->rels[i].cols = r->cols[i].data();
    }
    r->edges.assign(edges, edges + nedges);
    if (opts) r->opts = *opts;
    else r->opts.root = -1;
    r->mode = result_mode;
    // validate and size the workspace now (host-only); the worker plans again on its stream
    sj_plan_t *plan = nullptr;
    uint64_t wsb = 0;
    sj_opts o = r->opts;
    o.flags |= SJ_FLAG_EAGER;
    std::lock_guard<std::mutex> lk(s->mu);
    const sj_status st = sj_plan(s->plan_ctx, r->rels.data(), nrels, r->edges.data(), nedges, &o, &plan, &wsb);
    if (st != SJ_OK) return st;
    sj_plan_destroy(plan);
    if (round256(wsb) > s->arena.size()) return SJ_ERR_NOMEM;
    if (s->stop) return SJ_ERR_STATE;
    r->ticket = s->next_ticket++;
    r->info.state = SJ_QUERY_QUEUED;
    r->info.status = SJ_OK;
    r->info.slot = -1;
    r->info.workspace_bytes = wsb;
    r->info.t_submit_ns = now_ns();
    s->all[r->ticket] = r;
    s->queue.push_back(r);
    s->cv.notify_all();
    *ticket = r->ticket;
    return SJ_OK;
}

extern "C" const char *sj_server_last_error(const sj_server *s) {
    return s ? sj_last_error(s->plan_ctx) : "null server";
}

extern "C" sj_status sj_server_query(sj_server *s, uint64_t ticket, int32_t wait, sj_query_info *info) {
    if (!s || !info) return SJ_ERR_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return SJ_ERR_INVALID;
    auto r = it->second;
    if (wait)
        s->cv.wait(lk, [&] { return r->info.state == SJ_QUERY_DONE || r->info.state == SJ_QUERY_FAILED; });
    *info = r->info;
    return SJ_OK;
}

extern "C" sj_status sj_server_release(sj_server *s, uint64_t ticket) {
    if (!s) return SJ_ERR_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return SJ_ERR_INVALID;
    auto r = it->second;
    if (r->info.state != SJ_QUERY_DONE && r->info.state != SJ_QUERY_FAILED) return SJ_ERR_STATE;
    if (r->has_result) s->arena.release(r->res_off, r->res_bytes);
    r->has_result = false;
    s->all.erase(it);
    s->cv.notify_all();
    return SJ_OK;
}

extern "C" sj_status sj_server_stats(sj_server *s, uint64_t *arena_used, uint64_t *arena_peak, int32_t *queued,
                                     int32_t *running) {
    if (!s) return SJ_ERR_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    if (arena_used) *arena_used = s->arena.used();
    if (arena_peak) *arena_peak = s->arena.peak();
    if (queued) *queued = static_cast<int32_t>(s->queue.size());
    if (running) *running = s->running;
    return SJ_OK;
}

extern "C" sj_status sj_server_use_filter_cache(sj_server *s, sj_fcache *cache) {
    if (!s) return SJ_ERR_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    s->fcache = cache;
    return SJ_OK;
}

extern "C" sj_status sj_server_destroy(sj_server *s) {
    if (!s) return SJ_ERR_INVALID;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (auto &r : s->queue) {
            fail_request(*r, SJ_ERR_STATE, "server destroyed before the query was admitted");
            r->info.t_done_ns = now_ns();
        }
        s->queue.clear();
        s->cv.notify_all();
    }
    for (auto &t : s->workers) t.join();
    sj_ctx_destroy(s->plan_ctx);
    delete s;
    return SJ_OK;
}
