// A CPU stand-in for the HIP runtime calls the library's host code makes,
// for running that host code (plans, workspace, streams, events, graph
// capture, cache, replay and eviction) under AddressSanitizer and
// UndefinedBehaviorSanitizer on a machine without a GPU.  Kernels do not
// run: a launch is checked (grid, block, LDS size) and, on a capturing
// stream, recorded.  Device memory is host memory (zero-filled), so copies
// of the control blocks read zeros.
//
// It also checks the rules of stream capture that the library relies on,
// and reports each breach (mock_violations() > 0):
//   * no synchronisation, copy or allocation on a capturing stream;
//   * a stream joins a capture only by waiting on an event recorded in it;
//   * every stream forked into a capture is joined back before it ends;
//   * no use of a destroyed stream, event or graph (destroyed objects are
//     freed, so AddressSanitizer reports a later use).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <set>
#include <vector>

namespace {
std::mutex g_mu;
int g_violations = 0;
long g_launches = 0, g_graph_launches = 0, g_captures = 0;
hipError_t g_last = hipSuccess;

void violation(const char *what)
{
    std::fprintf(stderr, "[mock hip] violation: %s\n", what);
    ++g_violations;
}

struct Capture;
}  // namespace

struct ihipStream_t {
    Capture *cap = nullptr;
    unsigned long long ops = 0;     // operations enqueued while capturing
    unsigned long long joined = 0;  // ops of this stream that the origin has waited on
};
struct ihipEvent_t {
    Capture *cap = nullptr;          // the capture it was recorded in (if any)
    ihipStream_t *stream = nullptr;  // ... on this stream
    unsigned long long at = 0;       // ... after this many ops
};
struct ihipGraph {
    long nodes = 0;
};
struct hipGraphExec {
    long nodes = 0;
};

namespace {
struct Capture {
    ihipStream_t *origin = nullptr;
    std::set<ihipStream_t *> members;
    ihipGraph *graph = nullptr;
    bool broken = false;
};
ihipStream_t g_null_stream;
ihipStream_t *S(hipStream_t s) { return s ? s : &g_null_stream; }

struct Config {
    dim3 grid, block;
    size_t shmem;
    hipStream_t stream;
};
thread_local std::vector<Config> g_configs;

void note_op(ihipStream_t *s)
{
    if (s->cap) {
        ++s->ops;
        ++s->cap->graph->nodes;
    }
}
}  // namespace

extern "C" int mock_violations() { return g_violations; }
extern "C" long mock_launches() { return g_launches; }
extern "C" long mock_graph_launches() { return g_graph_launches; }
extern "C" long mock_captures() { return g_captures; }

// ---- device, errors -------------------------------------------------------
hipError_t hipGetDeviceCount(int *count)
{
    *count = 1;
    return hipSuccess;
}
hipError_t hipGetDevice(int *dev)
{
    *dev = 0;
    return hipSuccess;
}
hipError_t hipSetDevice(int dev) { return dev == 0 ? hipSuccess : hipErrorInvalidDevice; }
hipError_t hipGetLastError(void)
{
    hipError_t e = g_last;
    g_last = hipSuccess;
    return e;
}
const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "mock error"; }

// ---- memory ---------------------------------------------------------------
static hipError_t alloc(void **p, size_t n)
{
    std::lock_guard<std::mutex> lk(g_mu);
    *p = std::calloc(1, n ? n : 1);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
static bool any_capture_active();
hipError_t hipMalloc(void **p, size_t n)
{
    if (any_capture_active()) violation("hipMalloc during a stream capture");
    return alloc(p, n);
}
hipError_t hipFree(void *p)
{
    if (any_capture_active()) violation("hipFree during a stream capture");
    std::free(p);
    return hipSuccess;
}
hipError_t hipHostMalloc(void **p, size_t n, unsigned int) { return alloc(p, n); }
hipError_t hipHostFree(void *p)
{
    std::free(p);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind, hipStream_t s)
{
    if (S(s)->cap) violation("hipMemcpyAsync on a capturing stream");
    if (n) std::memmove(dst, src, n);
    return hipSuccess;
}
hipError_t hipGetSymbolAddress(void **p, const void *symbol)
{
    *p = const_cast<void *>(symbol);  // the host shadow of the device array
    return hipSuccess;
}

// ---- streams and events ---------------------------------------------------
static std::set<Capture *> g_caps;
static bool any_capture_active() { return !g_caps.empty(); }

hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int)
{
    *s = new ihipStream_t();
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s)
{
    if (s && s->cap) violation("hipStreamDestroy of a capturing stream");
    delete s;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s)
{
    if (S(s)->cap) violation("hipStreamSynchronize on a capturing stream");
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e)
{
    *e = new ihipEvent_t();
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e)
{
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s)
{
    ihipStream_t *st = S(s);
    note_op(st);
    e->cap = st->cap;
    e->stream = st;
    e->at = st->ops;
    return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int)
{
    ihipStream_t *st = S(s);
    if (e->cap) {
        if (!g_caps.count(e->cap)) {
            violation("wait on an event recorded in a capture that has ended");
            return hipErrorStreamCaptureInvalidated;
        }
        if (!st->cap) {  // a fork: the stream joins the capture
            st->cap = e->cap;
            st->ops = 0;
            st->joined = 0;
            e->cap->members.insert(st);
        } else if (st->cap != e->cap) {
            violation("wait across two captures");
            return hipErrorStreamCaptureIsolation;
        }
        // a join: the origin now depends on e's stream up to e
        if (st == st->cap->origin && e->stream != st && e->stream->joined < e->at) e->stream->joined = e->at;
    } else if (st->cap) {
        violation("a capturing stream waits on an event from outside the capture");
    }
    note_op(st);
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e)
{
    if (e->cap && g_caps.count(e->cap)) violation("hipEventSynchronize on an event of an active capture");
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b)
{
    if (a->cap || b->cap) violation("hipEventElapsedTime on captured events");
    *ms = 1.0f;
    return hipSuccess;
}

// ---- capture and graphs ---------------------------------------------------
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode)
{
    if (!s) {
        violation("capture of the null stream");
        return hipErrorStreamCaptureUnsupported;
    }
    if (s->cap) {
        violation("hipStreamBeginCapture on a capturing stream");
        return hipErrorIllegalState;
    }
    Capture *c = new Capture();
    c->origin = s;
    c->graph = new ihipGraph();
    c->members.insert(s);
    s->cap = c;
    s->ops = 0;
    s->joined = 0;
    g_caps.insert(c);
    ++g_captures;
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g)
{
    if (!s || !s->cap || s->cap->origin != s) {
        violation("hipStreamEndCapture on a stream that did not begin the capture");
        return hipErrorIllegalState;
    }
    Capture *c = s->cap;
    hipError_t r = hipSuccess;
    for (ihipStream_t *m : c->members) {
        if (m != s && m->joined != m->ops) {
            violation("a stream forked into the capture was not joined back");
            r = hipErrorStreamCaptureUnjoined;
        }
        m->cap = nullptr;
    }
    g_caps.erase(c);
    *g = c->graph;
    if (r != hipSuccess) {
        delete c->graph;
        *g = nullptr;
    }
    delete c;
    return r;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *ex, hipGraph_t g, hipGraphNode_t *, char *, size_t)
{
    *ex = new hipGraphExec();
    (*ex)->nodes = g->nodes;
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g)
{
    delete g;
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t ex)
{
    delete ex;
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t ex, hipStream_t s)
{
    if (S(s)->cap) violation("hipGraphLaunch on a capturing stream");
    volatile long n = ex->nodes;  // a freed graph is reported here
    (void)n;
    ++g_graph_launches;
    return hipSuccess;
}

// ---- kernel launches ------------------------------------------------------
hipError_t __hipPushCallConfiguration(dim3 grid, dim3 block, size_t shmem, hipStream_t stream)
{
    g_configs.push_back(Config{grid, block, shmem, stream});
    return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3 *grid, dim3 *block, size_t *shmem, hipStream_t *stream)
{
    if (g_configs.empty()) return hipErrorInvalidConfiguration;
    Config c = g_configs.back();
    g_configs.pop_back();
    *grid = c.grid;
    *block = c.block;
    *shmem = c.shmem;
    *stream = c.stream;
    return hipSuccess;
}
hipError_t hipLaunchKernel(const void *, dim3 grid, dim3 block, void **, size_t shmem, hipStream_t s)
{
    const unsigned long long threads = (unsigned long long)block.x * block.y * block.z;
    if (grid.x == 0 || grid.y == 0 || grid.z == 0 || grid.y > 65535 || grid.z > 65535 ||
        grid.x > 0x7fffffffu || threads == 0 || threads > 1024 || shmem > 160 * 1024) {
        char buf[160];
        std::snprintf(buf, sizeof(buf), "launch grid (%u,%u,%u) block (%u,%u,%u) LDS %zu out of range", grid.x,
                      grid.y, grid.z, block.x, block.y, block.z, shmem);
        violation(buf);
        g_last = hipErrorInvalidConfiguration;
        return hipErrorInvalidConfiguration;
    }
    note_op(S(s));
    ++g_launches;
    return hipSuccess;
}

// ---- code object registration (nothing to register) ---------------------
extern "C" void **__hipRegisterFatBinary(const void *)
{
    static void *handle = nullptr;
    return &handle;
}
extern "C" void __hipUnregisterFatBinary(void **) {}
extern "C" void __hipRegisterFunction(void **, const void *, char *, const char *, unsigned int, uint3 *, uint3 *,
                                      dim3 *, dim3 *, int *)
{
}
extern "C" void __hipRegisterVar(void **, void *, char *, char *, int, size_t, int, int) {}

// ---- used by the driver -----------------------------------------------------
hipError_t hipMemcpy(void *dst, const void *src, size_t n, hipMemcpyKind)
{
    if (any_capture_active()) violation("hipMemcpy during a stream capture");
    if (n) std::memmove(dst, src, n);
    return hipSuccess;
}
hipError_t hipDeviceSynchronize(void)
{
    if (any_capture_active()) violation("hipDeviceSynchronize during a stream capture");
    return hipSuccess;
}
