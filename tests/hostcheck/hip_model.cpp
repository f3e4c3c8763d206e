// Host-only model of the HIP runtime calls the library makes, for running the host
// runtime (plan, schedule, stream forks and joins, graph capture, serving, filter
// catalogue) under AddressSanitizer and UndefinedBehaviorSanitizer on a machine
// without a GPU. Test infrastructure only: it is linked into the checker executable,
// never into the library.
//
// "Device" memory is ordinary host memory, so the sanitizers see every host access the
// runtime makes to it (copies of counts, for instance). Kernels are not executed:
// a launch is checked (grid and block limits, the stream's state) and recorded as a node
// of the capture graph when its stream is capturing.
//
// Streams, events and graphs follow the capture rules of the HIP programming model:
//   - a launch, copy or event wait on a capturing stream adds to that capture;
//   - an event recorded on a capturing stream stands for the stream's last nodes, and a
//     stream that waits on it joins the capture (a fork) or gains those dependencies;
//   - waiting on an event of another capture, or on an event recorded outside any
//     capture while capturing, is an isolation error;
//   - ending the capture needs every stream that joined it to have been joined back
//     into the origin stream (each joined stream's last nodes are ancestors of the
//     origin's last nodes), else the capture is unjoined;
//   - synchronising a capturing stream, querying or synchronising a captured event,
//     and launching a graph into a capturing stream are errors.
// Objects are deleted when destroyed, so a later use is a heap use-after-free that
// AddressSanitizer reports. Every violation is printed and counted; the checker fails
// if the count is not zero (hipmodel_violations()).
#include <hip/hip_runtime.h>

#include <atomic>
#include <memory>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <set>
#include <string>
#include <vector>

namespace {

struct Graph {
    std::vector<std::vector<int>> deps;   // node -> its predecessors
    std::vector<std::string> what;
    int add(const std::set<int> &d, const std::string &w) {
        deps.emplace_back(d.begin(), d.end());
        what.push_back(w);
        return static_cast<int>(deps.size()) - 1;
    }
    // every node that reaches one of `from` (inclusive)
    std::set<int> ancestors(const std::set<int> &from) const {
        std::set<int> seen(from.begin(), from.end());
        std::vector<int> st(from.begin(), from.end());
        while (!st.empty()) {
            const int n = st.back();
            st.pop_back();
            for (int d : deps[n])
                if (seen.insert(d).second) st.push_back(d);
        }
        return seen;
    }
};

struct Capture {
    Graph g;
    hipStream_t origin;
    std::vector<hipStream_t> joined;   // streams that joined the capture by waiting on its events
    bool ended = false;
    int id;
};

std::recursive_mutex g_mu;
// capture records live until exit: events recorded into a capture keep pointing at it
std::vector<std::unique_ptr<Capture>> g_all_captures;
std::atomic<int> g_violations{0};
std::atomic<uint64_t> g_launches{0}, g_graph_launches{0}, g_captures{0};
int g_next_capture = 1;
thread_local int t_capturing = 0;   // captures begun on this thread and not ended

void violation(const char *fmt, const char *a = "", long b = 0) {
    char buf[512];
    std::snprintf(buf, sizeof buf, fmt, a, b);
    std::fprintf(stderr, "HIPMODEL VIOLATION: %s\n", buf);
    g_violations.fetch_add(1);
}

}  // namespace

struct ihipStream_t {
    uint32_t magic = 0x5354524d;
    Capture *cap = nullptr;
    std::set<int> tail;
};

struct ihipEvent_t {
    uint32_t magic = 0x4556454e;
    Capture *cap = nullptr;     // the capture it was last recorded into, or nullptr
    std::set<int> nodes;
    bool recorded = false;
    unsigned flags = 0;
};

struct ihipGraph {
    Capture *cap = nullptr;     // owns the captured nodes
};

struct hipGraphExec {
    size_t nodes = 0;
};

namespace {

thread_local struct {
    dim3 grid, block;
    size_t shmem = 0;
    hipStream_t stream = nullptr;
    int pushed = 0;
} t_cfg;

// A stream operation: added to the stream's capture, or nothing (the model runs no kernels).
hipError_t stream_op(hipStream_t s, const std::string &what) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (s && s->magic != 0x5354524d) {
        violation("%s on a destroyed or invalid stream", what.c_str());
        return hipErrorInvalidResourceHandle;
    }
    if (!s) {
        if (t_capturing) {
            violation("%s on the null stream while this thread captures", what.c_str());
            return hipErrorStreamCaptureImplicit;
        }
        return hipSuccess;
    }
    if (s->cap) {
        const int n = s->cap->g.add(s->tail, what);
        s->tail = {n};
    }
    return hipSuccess;
}

bool in_capture(hipStream_t s) { return s && s->cap; }

}  // namespace

extern "C" {

int hipmodel_violations() { return g_violations.load(); }
uint64_t hipmodel_launches() { return g_launches.load(); }
uint64_t hipmodel_graph_launches() { return g_graph_launches.load(); }
uint64_t hipmodel_captures() { return g_captures.load(); }

hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDevice(int *d) {
    if (d) *d = 0;
    return hipSuccess;
}
hipError_t hipGetDeviceCount(int *n) {
    if (n) *n = 1;
    return hipSuccess;
}
hipError_t hipGetLastError(void) { return hipSuccess; }
hipError_t hipPeekAtLastError(void) { return hipSuccess; }
const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "hipSuccess" : "hip model error"; }
const char *hipGetErrorName(hipError_t e) { return hipGetErrorString(e); }

hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int) {
    if (!s) return hipErrorInvalidValue;
    *s = new ihipStream_t;
    return hipSuccess;
}
hipError_t hipStreamCreate(hipStream_t *s) { return hipStreamCreateWithFlags(s, 0); }

hipError_t hipStreamDestroy(hipStream_t s) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (!s) return hipErrorInvalidResourceHandle;
    if (s->cap) violation("%s", "hipStreamDestroy of a capturing stream");
    for (auto &c : g_all_captures)   // no ended capture refers to a freed stream
        for (auto &t : c->joined)
            if (t == s) t = nullptr;
    s->magic = 0;
    delete s;
    return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t s) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (in_capture(s)) {
        violation("%s", "hipStreamSynchronize of a capturing stream");
        return hipErrorStreamCaptureUnsupported;
    }
    if (!s && t_capturing) {
        violation("%s", "hipStreamSynchronize(null) while this thread captures");
        return hipErrorStreamCaptureImplicit;
    }
    return hipSuccess;
}

hipError_t hipDeviceSynchronize(void) {
    if (t_capturing) violation("%s", "hipDeviceSynchronize while this thread captures");
    return hipSuccess;
}

hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned flags) {
    if (!e) return hipErrorInvalidValue;
    *e = new ihipEvent_t;
    (*e)->flags = flags;
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e) { return hipEventCreateWithFlags(e, 0); }

hipError_t hipEventDestroy(hipEvent_t e) {
    if (!e) return hipErrorInvalidResourceHandle;
    e->magic = 0;
    delete e;
    return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (!e || e->magic != 0x4556454e) {
        violation("%s", "hipEventRecord of a destroyed or invalid event");
        return hipErrorInvalidResourceHandle;
    }
    if (s && s->magic != 0x5354524d) {
        violation("%s", "hipEventRecord on a destroyed or invalid stream");
        return hipErrorInvalidResourceHandle;
    }
    if (!s && t_capturing) {
        violation("%s", "hipEventRecord on the null stream while this thread captures");
        return hipErrorStreamCaptureImplicit;
    }
    e->recorded = true;
    if (in_capture(s)) {
        e->cap = s->cap;
        e->nodes = s->tail;
    } else {
        e->cap = nullptr;
        e->nodes.clear();
    }
    return hipSuccess;
}

hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (!e || e->magic != 0x4556454e) {
        violation("%s", "hipStreamWaitEvent on a destroyed or invalid event");
        return hipErrorInvalidResourceHandle;
    }
    if (s && s->magic != 0x5354524d) {
        violation("%s", "hipStreamWaitEvent on a destroyed or invalid stream");
        return hipErrorInvalidResourceHandle;
    }
    if (e->cap && e->cap->ended) {
        violation("%s", "hipStreamWaitEvent on an event recorded in a capture that has ended");
        return hipErrorStreamCaptureIsolation;
    }
    if (e->cap) {
        if (!s) {
            violation("%s", "the null stream waits on a captured event");
            return hipErrorStreamCaptureIsolation;
        }
        if (!s->cap) {          // fork: the stream joins the capture
            s->cap = e->cap;
            s->tail = e->nodes;
            e->cap->joined.push_back(s);
        } else if (s->cap != e->cap) {
            violation("%s", "a stream waits on an event of another capture");
            return hipErrorStreamCaptureIsolation;
        } else {
            s->tail.insert(e->nodes.begin(), e->nodes.end());
        }
        return hipSuccess;
    }
    if (in_capture(s)) {
        violation("%s", "a capturing stream waits on an event recorded outside the capture");
        return hipErrorStreamCaptureIsolation;
    }
    return hipSuccess;
}

hipError_t hipEventQuery(hipEvent_t e) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (!e || e->magic != 0x4556454e) {
        violation("%s", "hipEventQuery of a destroyed or invalid event");
        return hipErrorInvalidResourceHandle;
    }
    if (e->cap) {
        violation("%s", "hipEventQuery of a captured event");
        return hipErrorCapturedEvent;
    }
    return hipSuccess;
}

hipError_t hipEventSynchronize(hipEvent_t e) { return hipEventQuery(e); }

hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) {
    if (hipEventQuery(a) != hipSuccess || hipEventQuery(b) != hipSuccess) return hipErrorInvalidResourceHandle;
    if (!a->recorded || !b->recorded) {
        violation("%s", "hipEventElapsedTime of an event never recorded");
        return hipErrorInvalidResourceHandle;
    }
    if (ms) *ms = 0.001f;
    return hipSuccess;
}

hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (!s) {
        violation("%s", "capture of the null stream");
        return hipErrorStreamCaptureUnsupported;
    }
    if (s->cap) {
        violation("%s", "hipStreamBeginCapture of a stream that already captures");
        return hipErrorIllegalState;
    }
    g_all_captures.emplace_back(new Capture);
    Capture *c = g_all_captures.back().get();
    c->origin = s;
    c->id = g_next_capture++;
    s->cap = c;
    s->tail.clear();
    ++t_capturing;
    g_captures.fetch_add(1);
    return hipSuccess;
}

// Streams that are part of a capture are found through this registry of live captures'
// streams: every stream that joined a capture keeps a pointer to it.
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (!s || !s->cap) {
        violation("%s", "hipStreamEndCapture of a stream that does not capture");
        return hipErrorIllegalState;
    }
    Capture *c = s->cap;
    if (c->origin != s) {
        violation("%s", "hipStreamEndCapture on a stream that did not begin the capture");
        return hipErrorStreamCaptureUnmatched;
    }
    c->ended = true;
    s->cap = nullptr;
    for (hipStream_t t : c->joined)   // the capture ends on every stream that joined it
        if (t && t->cap == c) t->cap = nullptr;
    --t_capturing;
    ihipGraph *graph = new ihipGraph;
    graph->cap = c;
    const std::set<int> done = c->g.ancestors(s->tail);
    // a node that is not an ancestor of the origin's last nodes belongs to an unjoined fork
    for (size_t n = 0; n < c->g.deps.size(); ++n)
        if (!done.count(static_cast<int>(n))) {
            violation("unjoined capture: node '%s' (%ld) does not lead back to the origin stream",
                      c->g.what[n].c_str(), static_cast<long>(n));
            if (g) *g = graph;
            return hipErrorStreamCaptureUnjoined;
        }
    if (g) *g = graph;
    return hipSuccess;
}

hipError_t hipStreamIsCapturing(hipStream_t s, hipStreamCaptureStatus *st) {
    if (st) *st = in_capture(s) ? hipStreamCaptureStatusActive : hipStreamCaptureStatusNone;
    return hipSuccess;
}

hipError_t hipGraphDestroy(hipGraph_t g) {
    if (!g) return hipErrorInvalidValue;
    // the capture record stays allocated: events recorded into it still point at it
    delete g;
    return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t *ex, hipGraph_t g, hipGraphNode_t *, char *, size_t) {
    if (!ex || !g) return hipErrorInvalidValue;
    *ex = new hipGraphExec;
    (*ex)->nodes = g->cap ? g->cap->g.deps.size() : 0;
    return hipSuccess;
}

hipError_t hipGraphExecDestroy(hipGraphExec_t ex) {
    if (!ex) return hipErrorInvalidValue;
    delete ex;
    return hipSuccess;
}

hipError_t hipGraphLaunch(hipGraphExec_t ex, hipStream_t s) {
    if (!ex) {
        violation("%s", "hipGraphLaunch of a null graph");
        return hipErrorInvalidValue;
    }
    volatile size_t n = ex->nodes;   // a destroyed exec is a use-after-free here
    (void)n;
    if (in_capture(s)) violation("%s", "hipGraphLaunch into a capturing stream");
    g_graph_launches.fetch_add(1);
    return stream_op(s, "graph launch");
}

hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind, hipStream_t s) {
    if (bytes && (!dst || !src)) {
        violation("%s", "hipMemcpyAsync with a null pointer");
        return hipErrorInvalidValue;
    }
    const bool cap = in_capture(s);
    if (hipError_t e = stream_op(s, "memcpy")) return e;
    if (!cap && bytes) std::memmove(dst, src, bytes);   // memory is host memory here
    return hipSuccess;
}

hipError_t hipMemcpy(void *dst, const void *src, size_t bytes, hipMemcpyKind) {
    if (t_capturing) violation("%s", "synchronous hipMemcpy while this thread captures");
    if (bytes && (!dst || !src)) return hipErrorInvalidValue;
    if (bytes) std::memmove(dst, src, bytes);
    return hipSuccess;
}

hipError_t hipMemsetAsync(void *dst, int v, size_t bytes, hipStream_t s) {
    if (in_capture(s)) violation("%s", "hipMemsetAsync recorded into a capture");
    if (hipError_t e = stream_op(s, "memset")) return e;
    if (!in_capture(s) && bytes) std::memset(dst, v, bytes);
    return hipSuccess;
}

// A __device__ variable's address: in a host-only build the variable itself is the
// host-side stand-in, so its own address serves as the "device" memory.
hipError_t hipGetSymbolAddress(void **ptr, const void *symbol) {
    if (!ptr || !symbol) return hipErrorInvalidValue;
    *ptr = const_cast<void *>(symbol);
    return hipSuccess;
}

hipError_t hipMalloc(void **, size_t) {
    violation("%s", "hipMalloc called");
    return hipErrorOutOfMemory;
}
hipError_t hipFree(void *) {
    violation("%s", "hipFree called");
    return hipErrorInvalidValue;
}

hipError_t __hipPushCallConfiguration(dim3 grid, dim3 block, size_t shmem, hipStream_t stream) {
    t_cfg.grid = grid;
    t_cfg.block = block;
    t_cfg.shmem = shmem;
    t_cfg.stream = stream;
    t_cfg.pushed = 1;
    return hipSuccess;
}

hipError_t __hipPopCallConfiguration(dim3 *grid, dim3 *block, size_t *shmem, hipStream_t *stream) {
    if (!t_cfg.pushed) violation("%s", "launch configuration popped without a push");
    *grid = t_cfg.grid;
    *block = t_cfg.block;
    *shmem = t_cfg.shmem;
    *stream = t_cfg.stream;
    t_cfg.pushed = 0;
    return hipSuccess;
}

hipError_t hipLaunchKernel(const void *fn, dim3 grid, dim3 block, void **args, size_t shmem, hipStream_t s) {
    g_launches.fetch_add(1);
    if (!fn || !args) violation("%s", "kernel launch without a function or arguments");
    const uint64_t threads = uint64_t(block.x) * block.y * block.z;
    if (grid.x == 0 || grid.y == 0 || grid.z == 0 || grid.x > 0x7fffffffu || grid.y > 65535 || grid.z > 65535)
        violation("kernel grid out of range (x = %ld)", "", static_cast<long>(grid.x));
    if (threads == 0 || threads > 1024) violation("kernel block of %ld threads", "", static_cast<long>(threads));
    if (shmem > 160 * 1024) violation("kernel with %ld bytes of dynamic LDS", "", static_cast<long>(shmem));
    return stream_op(s, "kernel");
}

// module registration emitted by the compiler for each translation unit
void **__hipRegisterFatBinary(const void *) {
    static void *handle = nullptr;
    return &handle;
}
void __hipRegisterFunction(void **, const void *, char *, const char *, unsigned int, void *, void *, void *,
                           void *, int *) {}
void __hipRegisterVar(void **, void *, char *, const char *, int, size_t, int, int) {}
void __hipRegisterManagedVar(void *, void **, void *, const char *, size_t, unsigned) {}
void __hipUnregisterFatBinary(void **) {}

}  // extern "C"
