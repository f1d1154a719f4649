// A recording stand-in for the HIP runtime, for host-only checks of the
// stream, event, copy and graph calls the library makes.  No device work
// runs: device memory is host memory, kernel launches are recorded, copies
// outside a capture are done at once.  Stream capture is modelled the way the
// HIP and CUDA programming guides describe it: a stream joins the capture of
// an event it waits on, captured work becomes a node depending on the
// stream's last nodes, and at the end of the capture every node must have
// been joined back into the origin stream.
//
// Every rule broken is recorded as a violation (hiprec_report prints them):
//   - allocation, free, stream or event creation/destruction, or a host wait
//     while a capture is active;
//   - work on a stream outside the active capture (it would run at once and
//     be missing from the graph), or on the null stream;
//   - a wait, inside the capture, on an event not recorded in it;
//   - a stream of the capture not joined back into the origin at the end;
//   - a copy whose host or device range runs past its allocation, or whose
//     host side is pageable memory inside a capture;
//   - a buffer freed while a graph that copies to or from it still exists,
//     and a graph launched after such a free;
//   - a launch with an invalid grid or block shape.
#include <hip/hip_runtime_api.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

namespace {

struct Alloc {
    size_t bytes;
    bool pinned; // hipHostMalloc
    bool live;
};

struct Stream {
    int capture = 0;           // id of the capture it belongs to, 0: none
    std::vector<int> last;     // its last nodes in that capture
    bool destroyed = false;
};

struct Event {
    int capture = 0;           // capture it was last recorded in (0: outside any)
    std::vector<int> nodes;    // the recording stream's last nodes then
    bool recorded = false;
};

struct Copy {
    uintptr_t host; // pinned host range copied to or from, 0: none
    uintptr_t dev;  // device range
};

struct Capture {
    int id = 0;
    hipStream_t origin = nullptr;
    std::vector<std::vector<int>> deps; // node -> its dependencies
    std::vector<Copy> copies;
    int kernels = 0, memcpys = 0;
};

struct Graph {
    std::vector<Copy> copies;
    int nodes = 0;
};

std::mutex mu;
std::map<uintptr_t, Alloc> allocs; // base -> allocation
std::map<hipStream_t, Stream> streams;
std::map<hipEvent_t, Event> events;
std::map<hipGraph_t, Graph> graphs;
std::map<hipGraphExec_t, Graph> execs;
std::vector<std::string> violations;
Capture cap;       // the active capture (id 0: none)
int next_capture = 1;
long n_launch = 0, n_copy = 0, n_captures = 0, n_graph_launch = 0, max_nodes = 0;
struct Config {
    dim3 grid, block;
    size_t shmem;
    hipStream_t stream;
};
thread_local std::vector<Config> configs;
std::map<const void *, size_t> symbols; // registered device variables: host shadow -> bytes

void violation(const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (violations.size() < 200)
        violations.emplace_back(buf);
}

bool capturing() { return cap.id != 0; }

void forbid_in_capture(const char *what)
{
    if (capturing())
        violation("%s while a stream capture is active", what);
}

// The allocation holding [p, p + bytes), or nullptr.
const std::pair<const uintptr_t, Alloc> *find(uintptr_t p)
{
    auto it = allocs.upper_bound(p);
    if (it == allocs.begin())
        return nullptr;
    --it;
    if (p >= it->first && p < it->first + it->second.bytes + (it->second.bytes == 0))
        return &*it;
    return nullptr;
}

Stream &stream_of(hipStream_t s)
{
    auto it = streams.find(s);
    if (it == streams.end()) {
        if (s != nullptr)
            violation("work on an unknown stream %p", (void *)s);
        return streams[s];
    }
    if (it->second.destroyed)
        violation("work on a destroyed stream %p", (void *)s);
    return it->second;
}

// Work submitted to stream s: a node of the active capture, or eager work.
// Returns true if it was captured.
bool submit(hipStream_t s, const char *what)
{
    Stream &st = stream_of(s);
    if (!capturing()) {
        if (st.capture)
            violation("%s on stream %p of an ended capture", what, (void *)s);
        return false;
    }
    if (s == nullptr) {
        violation("%s on the null stream while a capture is active", what);
        return false;
    }
    if (st.capture != cap.id) {
        violation("%s on stream %p, which is not part of the active capture (it would run "
                  "at once and be missing from the graph)",
                  what, (void *)s);
        return false;
    }
    const int node = (int)cap.deps.size();
    cap.deps.push_back(st.last);
    st.last.assign(1, node);
    return true;
}

// One side of a copy: bounds, and pinned memory inside a capture.  Returns
// false if the range must not be touched (past its allocation, or freed).
bool check_range(const void *p, size_t bytes, bool host, bool captured, const char *what,
                 std::vector<Copy> *refs)
{
    const uintptr_t a = (uintptr_t)p;
    const auto *al = find(a);
    if (!al) {
        if (!host) {
            violation("%s: device pointer %p is not in any allocation", what, p);
            return false;
        }
        if (captured)
            violation("%s: host pointer %p is pageable memory inside a capture", what, p);
        return true;
    }
    bool ok = true;
    if (!al->second.live) {
        violation("%s: pointer %p lies in a freed allocation", what, p);
        ok = false;
    }
    if (a + bytes > al->first + al->second.bytes) {
        violation("%s: %zu bytes at %p run %zu bytes past the end of its allocation", what,
                  bytes, p, (size_t)(a + bytes - al->first - al->second.bytes));
        ok = false;
    }
    if (host && !al->second.pinned && captured)
        violation("%s: host pointer %p is device memory used as host memory", what, p);
    if (captured && refs)
        refs->push_back(host ? Copy{al->first, 0} : Copy{0, al->first});
    return ok;
}

// Whether the destination (dst = true) or source side of a copy is host
// memory: from the kind, or for hipMemcpyDefault from the allocation.
bool is_host(const void *p, hipMemcpyKind kind, bool dst)
{
    if (kind == hipMemcpyDefault) {
        const auto *al = find((uintptr_t)p);
        return !al || al->second.pinned;
    }
    return dst ? (kind == hipMemcpyDeviceToHost || kind == hipMemcpyHostToHost)
               : (kind == hipMemcpyHostToDevice || kind == hipMemcpyHostToHost);
}

void copy(void *dst, const void *src, size_t bytes, hipMemcpyKind kind, hipStream_t s,
          const char *what)
{
    ++n_copy;
    const bool captured = submit(s, what);
    const bool dhost = is_host(dst, kind, true), shost = is_host(src, kind, false);
    std::vector<Copy> refs;
    const bool ok = check_range(dst, bytes, dhost, captured, what, &refs) &
                    check_range(src, bytes, shost, captured, what, &refs);
    if (captured) {
        ++cap.memcpys;
        cap.copies.insert(cap.copies.end(), refs.begin(), refs.end());
    } else if (bytes && ok) {
        std::memmove(dst, src, bytes);
    }
}

template <class T> T handle()
{
    static uintptr_t next = 0x1000;
    next += 0x10;
    return reinterpret_cast<T>(next);
}

void end_capture_checks()
{
    // every node must reach the origin's last nodes: mark the ancestors of
    // the origin's frontier and require every node to be among them
    std::vector<char> joined(cap.deps.size(), 0);
    std::vector<int> stack = streams[cap.origin].last;
    while (!stack.empty()) {
        const int v = stack.back();
        stack.pop_back();
        if (joined[v])
            continue;
        joined[v] = 1;
        for (int d : cap.deps[v])
            stack.push_back(d);
    }
    int unjoined = 0;
    for (char j : joined)
        unjoined += !j;
    if (unjoined)
        violation("capture %d: %d of %zu nodes are not joined back into the origin stream",
                  cap.id, unjoined, cap.deps.size());
    for (auto &kv : streams)
        if (kv.second.capture == cap.id) {
            kv.second.capture = 0;
            kv.second.last.clear();
        }
}

} // namespace

extern "C" {

// ---- registration (no device code is loaded) ----
void **__hipRegisterFatBinary(const void *) { return handle<void **>(); }
void __hipUnregisterFatBinary(void **) {}
void __hipRegisterFunction(void **, const void *, char *, const char *, unsigned int, void *,
                           void *, void *, void *, int *)
{
}
void __hipRegisterVar(void **, void *var, char *, char *, int, size_t size, int, int)
{
    std::lock_guard<std::mutex> g(mu);
    symbols[var] = size;
}

// ---- device ----
hipError_t hipGetDeviceCount(int *n)
{
    *n = 1;
    return hipSuccess;
}
hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_tR0600 *p, int dev)
{
    if (dev != 0)
        return hipErrorInvalidDevice;
    std::memset(p, 0, sizeof(*p));
    std::strcpy(p->name, "recording stand-in");
    std::strcpy(p->gcnArchName, "gfx950:sramecc+:xnack-");
    p->multiProcessorCount = 256;
    p->totalGlobalMem = (size_t)288 << 30;
    p->warpSize = 64;
    p->maxThreadsPerBlock = 1024;
    p->sharedMemPerBlock = 160 * 1024;
    return hipSuccess;
}
hipError_t hipSetDevice(int dev) { return dev == 0 ? hipSuccess : hipErrorInvalidDevice; }
hipError_t hipGetLastError(void) { return hipSuccess; }
const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "error"; }

// ---- memory ----
// Device memory starts filled with one 8-byte pattern that reads as a
// finite double (1 + 2^-21 or so) and, at 8-byte aligned offsets, as the int
// 0x7fffffff: so the host logic that follows the launches (which do not
// run) sees finite results and a completed factorisation, and takes the same
// paths as after a successful evaluation.
constexpr uint64_t DEVICE_FILL = 0x3ff000007fffffffull;

hipError_t hipMalloc(void **p, size_t bytes)
{
    std::lock_guard<std::mutex> g(mu);
    forbid_in_capture("hipMalloc");
    *p = std::malloc(bytes ? bytes : 1);
    if (!*p)
        return hipErrorOutOfMemory;
    uint64_t *q = static_cast<uint64_t *>(*p);
    for (size_t i = 0; i < bytes / 8; ++i)
        q[i] = DEVICE_FILL;
    allocs[(uintptr_t)*p] = {bytes, false, true};
    return hipSuccess;
}
hipError_t hipHostMalloc(void **p, size_t bytes, unsigned int)
{
    std::lock_guard<std::mutex> g(mu);
    forbid_in_capture("hipHostMalloc");
    *p = std::calloc(1, bytes ? bytes : 1);
    if (!*p)
        return hipErrorOutOfMemory;
    allocs[(uintptr_t)*p] = {bytes, true, true};
    return hipSuccess;
}
static hipError_t release(void *p, bool pinned, const char *what)
{
    std::lock_guard<std::mutex> g(mu);
    forbid_in_capture(what);
    if (!p)
        return hipSuccess;
    auto it = allocs.find((uintptr_t)p);
    if (it == allocs.end() || !it->second.live || it->second.pinned != pinned) {
        violation("%s(%p): not a live allocation of that kind", what, p);
        return hipErrorInvalidValue;
    }
    for (auto &kv : graphs)
        for (const Copy &c : kv.second.copies)
            if (c.host == (uintptr_t)p || c.dev == (uintptr_t)p)
                violation("%s(%p) while graph %p still copies to or from it", what, p,
                          (void *)kv.first);
    for (auto &kv : execs)
        for (const Copy &c : kv.second.copies)
            if (c.host == (uintptr_t)p || c.dev == (uintptr_t)p)
                violation("%s(%p) while executable graph %p still copies to or from it", what,
                          p, (void *)kv.first);
    it->second.live = false; // kept (not freed) so later uses are recognised
    return hipSuccess;
}
hipError_t hipFree(void *p) { return release(p, false, "hipFree"); }
hipError_t hipHostFree(void *p) { return release(p, true, "hipHostFree"); }

hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind kind,
                          hipStream_t s)
{
    std::lock_guard<std::mutex> g(mu);
    copy(dst, src, bytes, kind, s, "hipMemcpyAsync");
    return hipSuccess;
}
hipError_t hipMemcpy2DAsync(void *dst, size_t dpitch, const void *src, size_t spitch, size_t width,
                            size_t height, hipMemcpyKind kind, hipStream_t s)
{
    std::lock_guard<std::mutex> g(mu);
    if (height == 0 || width == 0)
        return hipSuccess;
    if (width > dpitch || width > spitch)
        violation("hipMemcpy2DAsync: width %zu exceeds a pitch (%zu, %zu)", width, dpitch, spitch);
    // bounds of the whole strided ranges; the rows are then copied one by one
    const size_t dspan = dpitch * (height - 1) + width, sspan = spitch * (height - 1) + width;
    const bool captured = submit(s, "hipMemcpy2DAsync");
    std::vector<Copy> refs;
    const bool dhost = is_host(dst, kind, true), shost = is_host(src, kind, false);
    const bool ok = check_range(dst, dspan, dhost, captured, "hipMemcpy2DAsync", &refs) &
                    check_range(src, sspan, shost, captured, "hipMemcpy2DAsync", &refs);
    ++n_copy;
    if (captured) {
        ++cap.memcpys;
        cap.copies.insert(cap.copies.end(), refs.begin(), refs.end());
    } else if (ok) {
        for (size_t r = 0; r < height; ++r)
            std::memmove((char *)dst + r * dpitch, (const char *)src + r * spitch, width);
    }
    return hipSuccess;
}
hipError_t hipGetSymbolAddress(void **p, const void *sym)
{
    std::lock_guard<std::mutex> g(mu);
    forbid_in_capture("hipGetSymbolAddress");
    // the host shadow of the device variable stands for it
    *p = const_cast<void *>(sym);
    auto it = symbols.find(sym);
    const size_t bytes = it == symbols.end() ? 0 : it->second;
    if (!allocs.count((uintptr_t)sym))
        allocs[(uintptr_t)sym] = {bytes, false, true};
    return hipSuccess;
}

// ---- streams and events ----
// used by the persistent round execution (not captured)
hipError_t hipStreamCreate(hipStream_t *s)
{
    std::lock_guard<std::mutex> g(mu);
    forbid_in_capture("hipStreamCreate");
    *s = handle<hipStream_t>();
    streams[*s] = Stream();
    return hipSuccess;
}
hipError_t hipMemcpy(void *dst, const void *src, size_t bytes, hipMemcpyKind kind)
{
    std::lock_guard<std::mutex> g(mu);
    forbid_in_capture("hipMemcpy");
    copy(dst, src, bytes, kind, nullptr, "hipMemcpy");
    return hipSuccess;
}
hipError_t hipMemsetAsync(void *dst, int v, size_t bytes, hipStream_t)
{
    std::lock_guard<std::mutex> g(mu);
    forbid_in_capture("hipMemsetAsync");
    std::memset(dst, v, bytes);
    return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t, int)
{
    *v = 100000;
    return hipSuccess;
}
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int *nb, const void *, int, size_t)
{
    *nb = 2;
    return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int)
{
    std::lock_guard<std::mutex> g(mu);
    forbid_in_capture("hipStreamCreateWithFlags");
    *s = handle<hipStream_t>();
    streams[*s] = Stream();
    return hipSuccess;
}
hipError_t hipExtStreamCreateWithCUMask(hipStream_t *s, uint32_t cuMaskSize, const uint32_t *)
{
    std::lock_guard<std::mutex> g(mu);
    forbid_in_capture("hipExtStreamCreateWithCUMask");
    if (cuMaskSize == 0)
        violation("hipExtStreamCreateWithCUMask with an empty mask");
    *s = handle<hipStream_t>();
    streams[*s] = Stream();
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s)
{
    std::lock_guard<std::mutex> g(mu);
    forbid_in_capture("hipStreamDestroy");
    Stream &st = stream_of(s);
    st.destroyed = true;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s)
{
    std::lock_guard<std::mutex> g(mu);
    forbid_in_capture("hipStreamSynchronize");
    (void)stream_of(s);
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e)
{
    std::lock_guard<std::mutex> g(mu);
    forbid_in_capture("hipEventCreate");
    *e = handle<hipEvent_t>();
    events[*e] = Event();
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned int)
{
    std::lock_guard<std::mutex> g(mu);
    forbid_in_capture("hipEventCreateWithFlags");
    *e = handle<hipEvent_t>();
    events[*e] = Event();
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e)
{
    std::lock_guard<std::mutex> g(mu);
    forbid_in_capture("hipEventDestroy");
    if (!events.erase(e))
        violation("hipEventDestroy(%p): unknown event", (void *)e);
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s)
{
    std::lock_guard<std::mutex> g(mu);
    auto it = events.find(e);
    if (it == events.end()) {
        violation("hipEventRecord(%p): unknown event", (void *)e);
        return hipErrorInvalidValue;
    }
    Stream &st = stream_of(s);
    Event &ev = it->second;
    ev.recorded = true;
    if (capturing() && st.capture == cap.id) {
        ev.capture = cap.id;
        ev.nodes = st.last;
    } else {
        if (capturing())
            violation("hipEventRecord on stream %p outside the active capture", (void *)s);
        ev.capture = 0;
        ev.nodes.clear();
    }
    return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int)
{
    std::lock_guard<std::mutex> g(mu);
    auto it = events.find(e);
    if (it == events.end()) {
        violation("hipStreamWaitEvent on unknown event %p", (void *)e);
        return hipErrorInvalidValue;
    }
    Stream &st = stream_of(s);
    const Event &ev = it->second;
    if (capturing()) {
        if (ev.capture == cap.id) {
            if (st.capture == 0) { // the stream joins the capture
                st.capture = cap.id;
                st.last = ev.nodes;
            } else if (st.capture == cap.id) {
                st.last.insert(st.last.end(), ev.nodes.begin(), ev.nodes.end());
            } else {
                violation("stream %p of another capture waits on an event of capture %d",
                          (void *)s, cap.id);
            }
        } else if (st.capture == cap.id) {
            violation("a stream of capture %d waits on event %p, which was %s", cap.id, (void *)e,
                      ev.recorded ? (ev.capture ? "recorded in an earlier capture"
                                                : "recorded outside the capture")
                                  : "never recorded");
        } else if (ev.capture) {
            violation("stream %p outside the capture waits on event %p of capture %d", (void *)s,
                      (void *)e, ev.capture);
        }
    } else if (ev.capture) {
        violation("stream %p waits, after the capture, on event %p recorded inside capture %d",
                  (void *)s, (void *)e, ev.capture);
    }
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t)
{
    std::lock_guard<std::mutex> g(mu);
    forbid_in_capture("hipEventElapsedTime");
    *ms = 0.f;
    return hipSuccess;
}

// ---- launches ----
hipError_t __hipPushCallConfiguration(dim3 grid, dim3 block, size_t shmem, hipStream_t s)
{
    configs.push_back({grid, block, shmem, s});
    return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3 *grid, dim3 *block, size_t *shmem, hipStream_t *s)
{
    if (configs.empty())
        return hipErrorInvalidConfiguration;
    const Config c = configs.back();
    configs.pop_back();
    *grid = c.grid;
    *block = c.block;
    *shmem = c.shmem;
    *s = c.stream;
    return hipSuccess;
}
hipError_t hipLaunchKernel(const void *fn, dim3 grid, dim3 block, void **, size_t shmem,
                           hipStream_t s)
{
    std::lock_guard<std::mutex> g(mu);
    ++n_launch;
    if (grid.x == 0 || grid.y == 0 || grid.z == 0 || grid.y > 65535 || grid.z > 65535 ||
        (uint64_t)grid.x * block.x > 0xffffffffull)
        violation("launch of %p with grid (%u, %u, %u)", fn, grid.x, grid.y, grid.z);
    if (block.x * block.y * block.z == 0 || block.x * block.y * block.z > 1024)
        violation("launch of %p with block (%u, %u, %u)", fn, block.x, block.y, block.z);
    if (shmem > 160 * 1024)
        violation("launch of %p with %zu bytes of dynamic LDS", fn, shmem);
    if (submit(s, "kernel launch"))
        ++cap.kernels;
    return hipSuccess;
}

// ---- capture and graphs ----
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode)
{
    std::lock_guard<std::mutex> g(mu);
    if (capturing()) {
        violation("hipStreamBeginCapture while capture %d is active", cap.id);
        return hipErrorIllegalState;
    }
    Stream &st = stream_of(s);
    if (s == nullptr)
        violation("capture of the null stream");
    cap = Capture();
    cap.id = next_capture++;
    cap.origin = s;
    st.capture = cap.id;
    st.last.clear();
    ++n_captures;
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *out)
{
    std::lock_guard<std::mutex> g(mu);
    if (!capturing() || s != cap.origin) {
        violation("hipStreamEndCapture on stream %p, which is not the origin of a capture",
                  (void *)s);
        *out = nullptr;
        return hipErrorIllegalState;
    }
    end_capture_checks();
    Graph gr;
    gr.copies = cap.copies;
    gr.nodes = (int)cap.deps.size();
    if (gr.nodes > max_nodes)
        max_nodes = gr.nodes;
    *out = handle<hipGraph_t>();
    graphs[*out] = gr;
    cap = Capture();
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *ge, hipGraph_t gr, hipGraphNode_t *, char *, size_t)
{
    std::lock_guard<std::mutex> g(mu);
    forbid_in_capture("hipGraphInstantiate");
    auto it = graphs.find(gr);
    if (it == graphs.end()) {
        violation("hipGraphInstantiate of an unknown graph");
        return hipErrorInvalidValue;
    }
    *ge = handle<hipGraphExec_t>();
    execs[*ge] = it->second;
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t ge, hipStream_t s)
{
    std::lock_guard<std::mutex> g(mu);
    forbid_in_capture("hipGraphLaunch");
    auto it = execs.find(ge);
    if (it == execs.end()) {
        violation("hipGraphLaunch of an unknown executable graph");
        return hipErrorInvalidValue;
    }
    (void)stream_of(s);
    for (const Copy &c : it->second.copies) {
        const uintptr_t p = c.host ? c.host : c.dev;
        auto a = allocs.find(p);
        if (a == allocs.end() || !a->second.live)
            violation("hipGraphLaunch: the graph copies to or from freed memory at %p", (void *)p);
    }
    ++n_graph_launch;
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t gr)
{
    std::lock_guard<std::mutex> g(mu);
    forbid_in_capture("hipGraphDestroy");
    if (!graphs.erase(gr))
        violation("hipGraphDestroy of an unknown graph");
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t ge)
{
    std::lock_guard<std::mutex> g(mu);
    forbid_in_capture("hipGraphExecDestroy");
    if (!execs.erase(ge))
        violation("hipGraphExecDestroy of an unknown executable graph");
    return hipSuccess;
}

// ---- report ----
int hiprec_report(FILE *f)
{
    std::lock_guard<std::mutex> g(mu);
    fprintf(f, "launches %ld, copies %ld, captures %ld (largest %ld nodes), graph launches %ld\n",
            n_launch, n_copy, n_captures, max_nodes, n_graph_launch);
    for (const std::string &v : violations)
        fprintf(f, "VIOLATION: %s\n", v.c_str());
    return (int)violations.size();
}
long hiprec_violation_count(void)
{
    std::lock_guard<std::mutex> g(mu);
    return (long)violations.size();
}
long hiprec_captures(void) { return n_captures; }
long hiprec_graph_launches(void) { return n_graph_launch; }
long hiprec_launches(void) { return n_launch; }

} // extern "C"
