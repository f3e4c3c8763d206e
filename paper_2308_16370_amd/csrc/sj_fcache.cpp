// Filter catalogue: backward filters kept resident and reused across queries (the
// filter reuse extension of include/sievejoin.h; Section 2.3 of the paper).
//
// Entries live in a caller-provided device arena: a 256-byte header holding the
// filter's block count, then its words. An entry is referenced by every plan that
// uses it and is visible to lookups once its producer has enqueued the build
// ("published"). Unreferenced published entries are evicted least recently used
// first when an allocation fails. Entries that are no longer visible (invalidated,
// cleared, or private duplicates) are freed once unreferenced and once the device
// work of every plan that used them has finished (each release hands over an event the
// releasing plan recorded after its last use of the entry).
#include "sj_fcache.h"

#include <algorithm>
#include <mutex>
#include <unordered_map>

#include "sj_arena.h"

namespace sj {

struct FcEntry {
    std::string sig;
    uint64_t off = 0, bytes = 0, max_words = 0;
    std::vector<const void *> cols;
    int refs = 0;
    bool published = false;
    hipEvent_t ready = nullptr;
    std::vector<FcEventRef> done;   // releasing plans' last uses of the entry
    uint64_t last_use = 0;
};

}  // namespace sj

using sj::FcEntry;

struct sj_fcache {
    int device = 0;
    char *base = nullptr;
    sj::Arena arena{0};
    std::mutex mu;
    std::unordered_map<std::string, FcEntry *> map;   // published entries by signature
    std::vector<FcEntry *> all;                       // every entry not yet freed
    uint64_t clock = 0;
    uint64_t hits = 0, misses = 0, uncached = 0, evictions = 0;
};

namespace {

constexpr uint64_t kHeader = 256;

// Called with the lock held. `wait`: block until the entry's users are done; otherwise
// free only if they already are. Returns whether the entry was freed.
bool free_entry(sj_fcache *c, FcEntry *e, bool wait) {
    for (const sj::FcEventRef &ev : e->done)
        if (!wait && hipEventQuery(ev->ev) == hipErrorNotReady) return false;
    for (const sj::FcEventRef &ev : e->done) (void)hipEventSynchronize(ev->ev);
    e->done.clear();
    if (e->ready) {
        (void)hipEventSynchronize(e->ready);
        (void)hipEventDestroy(e->ready);
    }
    if (e->published) c->map.erase(e->sig);
    c->arena.release(e->off, e->bytes);
    c->all.erase(std::find(c->all.begin(), c->all.end(), e));
    delete e;
    return true;
}

// Free unreferenced, unpublished entries (all of them with `wait`, else those whose
// users have finished).
void reap(sj_fcache *c, bool wait) {
    std::vector<FcEntry *> dead;
    for (FcEntry *e : c->all)
        if (e->refs == 0 && !e->published) dead.push_back(e);
    for (FcEntry *e : dead) free_entry(c, e, wait);
}

void unpublish(sj_fcache *c, FcEntry *e) {
    if (!e->published) return;
    c->map.erase(e->sig);
    e->published = false;
}

}  // namespace

namespace sj {

int fc_device(const sj_fcache *c) { return c->device; }

FcGrant fc_acquire(sj_fcache *c, const std::string &sig, uint64_t max_words, const std::vector<const void *> &cols) {
    std::lock_guard<std::mutex> lk(c->mu);
    FcGrant g;
    auto it = c->map.find(sig);
    if (it != c->map.end() && it->second->max_words == max_words) {
        FcEntry *e = it->second;
        ++e->refs;
        e->last_use = ++c->clock;
        ++c->hits;
        g.entry = e;
        g.hit = true;
        g.nblocks = reinterpret_cast<uint32_t *>(c->base + e->off);
        g.words = reinterpret_cast<uint32_t *>(c->base + e->off + kHeader);
        g.ready = e->ready;
        return g;
    }
    reap(c, false);
    const uint64_t bytes = kHeader + max_words * 4;
    uint64_t off = 0;
    bool got = c->arena.alloc(bytes, &off);
    if (!got) {
        reap(c, true);
        got = c->arena.alloc(bytes, &off);
    }
    while (!got) {
        FcEntry *victim = nullptr;
        for (FcEntry *e : c->all)
            if (e->refs == 0 && e->published && (!victim || e->last_use < victim->last_use)) victim = e;
        if (!victim) {
            ++c->uncached;
            return g;
        }
        unpublish(c, victim);
        free_entry(c, victim, true);
        ++c->evictions;
        got = c->arena.alloc(bytes, &off);
    }
    FcEntry *e = new FcEntry;
    e->sig = sig;
    e->off = off;
    e->bytes = bytes;
    e->max_words = max_words;
    e->cols = cols;
    e->refs = 1;
    e->last_use = ++c->clock;
    c->all.push_back(e);
    ++c->misses;
    g.entry = e;
    g.nblocks = reinterpret_cast<uint32_t *>(c->base + off);
    g.words = reinterpret_cast<uint32_t *>(c->base + off + kHeader);
    return g;
}

sj_status fc_publish(sj_fcache *c, FcEntry *e, hipStream_t stream) {
    std::lock_guard<std::mutex> lk(c->mu);
    if (!e->ready && hipEventCreateWithFlags(&e->ready, hipEventDisableTiming) != hipSuccess) {
        e->ready = nullptr;
        return SJ_ERR_DEVICE;
    }
    if (hipEventRecord(e->ready, stream) != hipSuccess) return SJ_ERR_DEVICE;
    if (c->map.find(e->sig) == c->map.end()) {
        c->map[e->sig] = e;
        e->published = true;
    }
    return SJ_OK;
}

void fc_release(sj_fcache *c, FcEntry *e, const FcEventRef &last_use) {
    std::lock_guard<std::mutex> lk(c->mu);
    if (last_use && std::find(e->done.begin(), e->done.end(), last_use) == e->done.end()) e->done.push_back(last_use);
    // keep only the uses still in flight
    auto keep = std::remove_if(e->done.begin(), e->done.end(),
                               [](const FcEventRef &x) { return hipEventQuery(x->ev) == hipSuccess; });
    e->done.erase(keep, e->done.end());
    --e->refs;
    if (e->refs == 0 && !e->published) free_entry(c, e, false);
}

}  // namespace sj

extern "C" sj_status sj_fcache_create(int32_t device, void *arena_dev, uint64_t arena_bytes, sj_fcache **out) {
    if (!out) return SJ_ERR_INVALID;
    *out = nullptr;
    if (!arena_dev || arena_bytes < 512 || reinterpret_cast<uintptr_t>(arena_dev) % 256) return SJ_ERR_INVALID;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) return SJ_ERR_DEVICE;
    if (device < 0 || device >= ndev) return SJ_ERR_INVALID;
    sj_fcache *c = new (std::nothrow) sj_fcache;
    if (!c) return SJ_ERR_INVALID;
    c->device = device;
    c->base = static_cast<char *>(arena_dev);
    c->arena = sj::Arena(arena_bytes & ~uint64_t(255));
    *out = c;
    return SJ_OK;
}

extern "C" sj_status sj_fcache_invalidate(sj_fcache *c, const void *column_dev) {
    if (!c) return SJ_ERR_INVALID;
    std::lock_guard<std::mutex> lk(c->mu);
    for (FcEntry *e : c->all)
        if (std::find(e->cols.begin(), e->cols.end(), column_dev) != e->cols.end()) unpublish(c, e);
    reap(c, false);
    return SJ_OK;
}

extern "C" sj_status sj_fcache_clear(sj_fcache *c) {
    if (!c) return SJ_ERR_INVALID;
    std::lock_guard<std::mutex> lk(c->mu);
    for (FcEntry *e : c->all) unpublish(c, e);
    reap(c, false);
    return SJ_OK;
}

extern "C" sj_status sj_fcache_stats(sj_fcache *c, sj_fcache_info *info) {
    if (!c || !info) return SJ_ERR_INVALID;
    std::lock_guard<std::mutex> lk(c->mu);
    info->capacity_bytes = c->arena.size();
    info->used_bytes = c->arena.used();
    info->entries = c->map.size();
    info->pinned = static_cast<uint64_t>(std::count_if(c->all.begin(), c->all.end(), [](FcEntry *e) { return e->refs > 0; }));
    info->hits = c->hits;
    info->misses = c->misses;
    info->uncached = c->uncached;
    info->evictions = c->evictions;
    return SJ_OK;
}

extern "C" sj_status sj_fcache_destroy(sj_fcache *c) {
    if (!c) return SJ_OK;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        for (FcEntry *e : c->all)
            if (e->refs > 0) return SJ_ERR_STATE;
        (void)hipSetDevice(c->device);
        for (FcEntry *e : c->all) unpublish(c, e);
        reap(c, true);
    }
    delete c;
    return SJ_OK;
}
