// Internal interface between the plan runtime and the filter catalogue
// (sj_fcache.cpp). The runtime computes each backward filter's signature; the
// catalogue owns the entries, their arena memory and their readiness events.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "sievejoin.h"

namespace sj {

struct FcEntry;

// An event shared between a plan, which records its last use of catalogue entries on
// it, and the entries the plan has released, which keep it until that work is done.
struct FcEvent {
    hipEvent_t ev = nullptr;
    FcEvent() = default;
    FcEvent(const FcEvent &) = delete;
    FcEvent &operator=(const FcEvent &) = delete;
    ~FcEvent() {
        if (ev) (void)hipEventDestroy(ev);
    }
};
using FcEventRef = std::shared_ptr<FcEvent>;

struct FcGrant {
    FcEntry *entry = nullptr;   // null: not cached (no room)
    bool hit = false;           // true: resident, reuse; false: the plan builds into it
    uint32_t *words = nullptr;  // max_words uint32 in the arena
    uint32_t *nblocks = nullptr;
    hipEvent_t ready = nullptr; // hit: recorded after the producer's build
};

// Find the resident entry for `sig` (a hit, referenced) or reserve a new unpublished
// one of `max_words` words (a miss, referenced). `cols` lists every column the
// filter's sub-tree reads, for invalidation.
FcGrant fc_acquire(sj_fcache *c, const std::string &sig, uint64_t max_words, const std::vector<const void *> &cols);
// The producing plan has enqueued the build on `stream`: record readiness and make the
// entry visible to later lookups (unless an equal entry was published meanwhile, in
// which case it stays private to the producer).
sj_status fc_publish(sj_fcache *c, FcEntry *e, hipStream_t stream);
// Drop a plan's reference. `last_use` (recorded after the plan's last work that may read
// the entry; null if it enqueued none) must complete before the entry's memory is reused.
// No stream is touched: the plan's stream may be gone by now.
void fc_release(sj_fcache *c, FcEntry *e, const FcEventRef &last_use);
int fc_device(const sj_fcache *c);

}  // namespace sj
