// Host-only stand-in for the HIP runtime, used to run the library's host code
// (planner, executor, batch task graphs, C ABI) without a GPU, under
// AddressSanitizer and UndefinedBehaviorSanitizer.
//
// Device memory is host memory from aligned_alloc; kernels are not executed.
// Instead every stage-kernel launch is checked: thread count and LDS bytes
// against the gfx950 limits, and the element range that the lines of the tile
// read and write (from the launch arguments, following each kernel's
// addressing) against the allocation it starts in.  Streams, events and graph
// capture are modelled closely enough to reject what the real runtime rejects
// or what would be wrong on it: work on a destroyed stream or event, a
// synchronisation inside a capture, a capture that ends with a forked stream
// not joined back, destroying a stream that is still capturing.
//
// Violations are counted; hostsim_violations() reports them to the driver.
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <set>
#include <vector>

#include "../../paper_2601_12209_amd/csrc/fft_lengths.hpp"
#include "../../paper_2601_12209_amd/csrc/kernels.hpp"
#include "../../paper_2601_12209_amd/csrc/plane_list.hpp"
#include "../../paper_2601_12209_amd/csrc/stage_args.hpp"

namespace {

constexpr unsigned kStreamMagic = 0x57524541u;
constexpr unsigned kEventMagic = 0x45564e54u;
constexpr unsigned kGraphMagic = 0x47524150u;
constexpr unsigned kExecMagic = 0x45584543u;

std::map<uintptr_t, size_t> g_allocs;  // base -> bytes
int g_violations = 0;
long g_launches = 0;
int g_next_capture = 1;

void violation(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    fprintf(stderr, "hostsim violation: ");
    vfprintf(stderr, fmt, ap);
    fprintf(stderr, "\n");
    va_end(ap);
    ++g_violations;
}

}  // namespace

struct ihipStream_t {
    unsigned magic = kStreamMagic;
    int capture = 0;                 // id of the capture this stream takes part in
    ihipStream_t* origin = nullptr;  // the stream the capture began on
    long ops = 0;                    // work items enqueued so far
};

struct ihipEvent_t {
    unsigned magic = kEventMagic;
    ihipStream_t* stream = nullptr;
    long ops = -1;
    int capture = 0;
};

struct hipGraphNode {
    ihipGraph* owner = nullptr;
};

struct ihipGraph {
    unsigned magic = kGraphMagic;
    std::vector<hipGraphNode*> nodes;  // built node by node (hipGraphAdd*Node)
    ~ihipGraph()
    {
        for (hipGraphNode* n : nodes) delete n;
    }
};

struct hipGraphExec {
    unsigned magic = kExecMagic;
};

namespace {

struct WaitEdge {
    ihipStream_t* waiter;
    ihipStream_t* target;
    long target_ops;
};
std::map<int, std::vector<ihipStream_t*>> g_members;  // capture id -> streams in it
std::map<int, std::vector<WaitEdge>> g_edges;         // capture id -> cross-stream waits

bool stream_ok(hipStream_t s, const char* what)
{
    if (s == nullptr) return true;  // the null stream
    if (s->magic != kStreamMagic) {
        violation("%s: invalid or destroyed stream", what);
        return false;
    }
    return true;
}

bool event_ok(hipEvent_t e, const char* what)
{
    if (!e || e->magic != kEventMagic) {
        violation("%s: invalid or destroyed event", what);
        return false;
    }
    return true;
}

// Allocation containing [p, p + bytes), or violation.
bool in_alloc(const void* p, size_t bytes, const char* what)
{
    const uintptr_t a = (uintptr_t)p;
    auto it = g_allocs.upper_bound(a);
    if (it == g_allocs.begin()) {
        violation("%s: %p is not in any allocation", what, p);
        return false;
    }
    --it;
    if (a + bytes > it->first + it->second) {
        violation("%s: [%p, +%zu) runs past its allocation [%p, +%zu)", what, p, bytes, (void*)it->first,
                  it->second);
        return false;
    }
    return true;
}

void enqueue(hipStream_t s) { if (s) ++s->ops; }

}  // namespace

// streams that took part in the most recently ended capture
size_t g_last_capture_members = 0;
extern "C" size_t hostsim_last_capture_members() { return g_last_capture_members; }
extern "C" int hostsim_violations() { return g_violations; }
extern "C" long hostsim_launches() { return g_launches; }
extern "C" size_t hostsim_live_allocations() { return g_allocs.size(); }

// ------------------------------------------------------------------- runtime

hipError_t hipGetDevice(int* d)
{
    *d = 0;
    return hipSuccess;
}

hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidDevice; }

hipError_t hipGetLastError() { return hipSuccess; }

const char* hipGetErrorString(hipError_t e)
{
    static char buf[64];
    snprintf(buf, sizeof buf, "stub error %d", (int)e);
    return buf;
}

hipError_t hipMalloc(void** p, size_t bytes)
{
    if (!p) return hipErrorInvalidValue;
    if (bytes == 0) {
        *p = nullptr;
        return hipSuccess;
    }
    const size_t r = (bytes + 255) & ~(size_t)255;
    void* m = aligned_alloc(256, r);
    if (!m) return hipErrorOutOfMemory;
    g_allocs[(uintptr_t)m] = bytes;
    *p = m;
    return hipSuccess;
}

hipError_t hipFree(void* p)
{
    if (!p) return hipSuccess;
    auto it = g_allocs.find((uintptr_t)p);
    if (it == g_allocs.end()) {
        violation("hipFree of %p, not an allocation base", p);
        return hipErrorInvalidValue;
    }
    g_allocs.erase(it);
    free(p);
    return hipSuccess;
}

hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind)
{
    if (kind == hipMemcpyHostToDevice || kind == hipMemcpyDeviceToDevice) in_alloc(dst, bytes, "hipMemcpy dst");
    if (kind == hipMemcpyDeviceToHost || kind == hipMemcpyDeviceToDevice) in_alloc(src, bytes, "hipMemcpy src");
    memcpy(dst, src, bytes);
    return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int)
{
    *s = new ihipStream_t();
    return hipSuccess;
}

hipError_t hipStreamDestroy(hipStream_t s)
{
    if (!s) return hipErrorInvalidHandle;
    if (!stream_ok(s, "hipStreamDestroy")) return hipErrorInvalidHandle;
    if (s->capture) violation("hipStreamDestroy of a stream that is capturing");
    s->magic = 0;
    delete s;
    return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t s)
{
    if (!stream_ok(s, "hipStreamSynchronize")) return hipErrorInvalidHandle;
    if (s && s->capture) {
        violation("hipStreamSynchronize inside a capture");
        return hipErrorStreamCaptureUnsupported;
    }
    return hipSuccess;
}

hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned)
{
    *e = new ihipEvent_t();
    return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t* e) { return hipEventCreateWithFlags(e, 0); }

hipError_t hipEventDestroy(hipEvent_t e)
{
    if (!event_ok(e, "hipEventDestroy")) return hipErrorInvalidHandle;
    e->magic = 0;
    delete e;
    return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t e, hipStream_t s)
{
    if (!event_ok(e, "hipEventRecord") || !stream_ok(s, "hipEventRecord")) return hipErrorInvalidHandle;
    e->stream = s;
    e->ops = s ? s->ops : 0;
    e->capture = s ? s->capture : 0;
    return hipSuccess;
}

hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int)
{
    if (!event_ok(e, "hipStreamWaitEvent") || !stream_ok(s, "hipStreamWaitEvent")) return hipErrorInvalidHandle;
    if (e->capture) {
        if (!s) {
            violation("the null stream waits on an event recorded in a capture");
            return hipErrorStreamCaptureIsolation;
        }
        if (s->capture && s->capture != e->capture) {
            violation("stream of one capture waits on an event of another");
            return hipErrorStreamCaptureIsolation;
        }
        if (!s->capture) {  // fork: s joins the capture
            s->capture = e->capture;
            s->origin = e->stream->origin;
            g_members[s->capture].push_back(s);
        }
        if (e->stream && e->stream != s) g_edges[s->capture].push_back({s, e->stream, e->ops});
    }
    enqueue(s);
    return hipSuccess;
}

hipError_t hipEventSynchronize(hipEvent_t e)
{
    if (!event_ok(e, "hipEventSynchronize")) return hipErrorInvalidHandle;
    if (e->capture) violation("hipEventSynchronize on an event recorded in a capture");
    return hipSuccess;
}

hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b)
{
    if (!event_ok(a, "hipEventElapsedTime") || !event_ok(b, "hipEventElapsedTime")) return hipErrorInvalidHandle;
    if (a->ops < 0 || b->ops < 0) return hipErrorNotReady;
    *ms = 0.001f;
    return hipSuccess;
}

hipError_t hipStreamIsCapturing(hipStream_t s, hipStreamCaptureStatus* st)
{
    if (!stream_ok(s, "hipStreamIsCapturing")) return hipErrorInvalidHandle;
    *st = (s && s->capture) ? hipStreamCaptureStatusActive : hipStreamCaptureStatusNone;
    return hipSuccess;
}

hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode)
{
    if (!s) return hipErrorStreamCaptureUnsupported;
    if (!stream_ok(s, "hipStreamBeginCapture")) return hipErrorInvalidHandle;
    if (s->capture) return hipErrorIllegalState;
    s->capture = g_next_capture++;
    s->origin = s;
    g_members[s->capture].push_back(s);
    return hipSuccess;
}

hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g)
{
    if (!stream_ok(s, "hipStreamEndCapture") || !s) return hipErrorInvalidHandle;
    if (!s->capture || s->origin != s) return hipErrorIllegalState;
    // a forked stream is joined when a joined stream (first the origin) waited
    // on an event recorded after its last work item
    std::set<ihipStream_t*> joined{s};
    for (bool grew = true; grew;) {
        grew = false;
        for (const WaitEdge& w : g_edges[s->capture])
            if (joined.count(w.waiter) && !joined.count(w.target) && w.target_ops == w.target->ops) {
                joined.insert(w.target);
                grew = true;
            }
    }
    hipError_t r = hipSuccess;
    for (ihipStream_t* m : g_members[s->capture]) {
        if (!joined.count(m)) {
            violation("capture ends with a forked stream not joined back");
            r = hipErrorStreamCaptureUnjoined;
        }
    }
    g_edges.erase(s->capture);
    g_last_capture_members = g_members[s->capture].size();
    for (ihipStream_t* m : g_members[s->capture]) {
        m->capture = 0;
        m->origin = nullptr;
    }
    g_members.erase(s->capture);
    *g = r == hipSuccess ? new ihipGraph() : nullptr;
    return r;
}

hipError_t hipGraphCreate(hipGraph_t* g, unsigned int flags)
{
    if (!g || flags != 0) return hipErrorInvalidValue;
    *g = new ihipGraph();
    return hipSuccess;
}

namespace {
hipError_t add_node(hipGraphNode_t* n, hipGraph_t g, const hipGraphNode_t* deps, size_t nd, const char* what)
{
    if (!n || !g || g->magic != kGraphMagic) {
        violation("%s on an invalid graph", what);
        return hipErrorInvalidValue;
    }
    for (size_t i = 0; i < nd; ++i) {
        if (!deps || !deps[i] || deps[i]->owner != g) {
            violation("%s with a dependency outside the graph", what);
            return hipErrorInvalidValue;
        }
    }
    hipGraphNode* node = new hipGraphNode();
    node->owner = g;
    g->nodes.push_back(node);
    *n = node;
    return hipSuccess;
}
}  // namespace

hipError_t hipGraphAddKernelNode(hipGraphNode_t* n, hipGraph_t g, const hipGraphNode_t* deps, size_t nd,
                                 const hipKernelNodeParams* kp)
{
    // the stage kernels take one StageArgs: the node must carry it
    if (!kp || !kp->func || !kp->kernelParams || !kp->kernelParams[0] || kp->extra) {
        violation("kernel node without a function or its StageArgs argument");
        return hipErrorInvalidValue;
    }
    const unsigned threads = kp->blockDim.x * kp->blockDim.y * kp->blockDim.z;
    if (threads == 0 || threads > 1024 || kp->sharedMemBytes > fft3d::kMaxLdsBytes)
        violation("kernel node shape over the limits");
    ++g_launches;
    return add_node(n, g, deps, nd, "hipGraphAddKernelNode");
}

hipError_t hipGraphAddEmptyNode(hipGraphNode_t* n, hipGraph_t g, const hipGraphNode_t* deps, size_t nd)
{
    return add_node(n, g, deps, nd, "hipGraphAddEmptyNode");
}

namespace fft3d {
void check_grouped(const void* f, dim3 grid, const StageArgs& a);  // below, with the kernel stand-ins
}

hipError_t hipLaunchKernel(const void* f, dim3 grid, dim3, void** args, size_t, hipStream_t s)
{
    if (!f || !args || !args[0]) violation("kernel launch without a function or arguments");
    if (!stream_ok(s, "kernel launch")) return hipErrorInvalidHandle;
    if (args && args[0]) {
        const fft3d::StageArgs& a = *static_cast<const fft3d::StageArgs*>(args[0]);
        if (!a.in || !a.out) violation("kernel launch without its buffers");
        fft3d::check_grouped(f, grid, a);
    }
    enqueue(s);
    ++g_launches;
    return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t)
{
    if (!g || g->magic != kGraphMagic) {
        violation("hipGraphInstantiate of an invalid graph");
        return hipErrorInvalidValue;
    }
    *x = new hipGraphExec();
    return hipSuccess;
}

hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s)
{
    if (!x || x->magic != kExecMagic) {
        violation("hipGraphLaunch of an invalid or destroyed graph");
        return hipErrorInvalidValue;
    }
    if (!stream_ok(s, "hipGraphLaunch")) return hipErrorInvalidHandle;
    enqueue(s);
    return hipSuccess;
}

hipError_t hipGraphExecDestroy(hipGraphExec_t x)
{
    if (!x || x->magic != kExecMagic) {
        violation("hipGraphExecDestroy of an invalid graph");
        return hipErrorInvalidValue;
    }
    x->magic = 0;
    delete x;
    return hipSuccess;
}

hipError_t hipGraphDestroy(hipGraph_t g)
{
    if (!g || g->magic != kGraphMagic) {
        violation("hipGraphDestroy of an invalid graph");
        return hipErrorInvalidValue;
    }
    g->magic = 0;
    delete g;
    return hipSuccess;
}

// ------------------------------------------------------------ stage kernels

namespace fft3d {

namespace {

constexpr int kMaxThreads = 1024;

bool has_variants(int n)
{
    return n == 64 || n == 128 || n == 256 || n == 512 || n == 1024 || n == 2048 || n == 4096 || n == 840;
}

size_t table_entries(int n, int ord = 0) { return (size_t)pass_table_size(radix_plan(n, ord)); }

size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }

// Element range [lo, hi] (in units of `es` bytes) of a lines x len tile:
// line (a, b) covers off + a*sa + b*sb + e*se, e < len.
void check_range(const void* base, size_t es, int64_t off, int64_t A, int64_t sa, int64_t B, int64_t sb, int64_t len,
                 int64_t se, const char* what)
{
    // no buffer yet: a launch recorded for a grouped launch, whose buffers
    // come at issue (hipLaunchKernel rejects a launch without them, and
    // check_grouped checks every tile against them)
    if (!base) return;
    const int64_t lo = off;
    const int64_t hi = off + (A - 1) * sa + (B - 1) * sb + (len - 1) * se;
    if (lo < 0) {
        violation("%s: negative element offset %lld", what, (long long)lo);
        return;
    }
    in_alloc((const char*)base + lo * es, (size_t)(hi - lo + 1) * es, what);
}

void check_tables(const StageArgs& a, int n, size_t es, const char* what, int ord = 0)
{
    const size_t s = table_entries(n, ord);
    if (s) in_alloc(a.twp, s * es, what);
}

// Stand-in kernel functions: one per kernel kind, length(s) and precision,
// as the GPU build has one instantiation per such set.  A grouped launch
// (StageArgs::tiles) names one of them; check_grouped re-runs its checks on
// every tile of the table.
struct StubKernel {
    int kind, n, n2, dtype;
};
std::map<std::vector<int>, StubKernel> g_kernels;  // node addresses stay put
bool g_checking = false;  // re-checking a tile of a grouped launch: launch nothing

// The checked launch goes through the library's launch hook, which launches
// (hipLaunchKernel above) or records the launch for a grouped one.
hipError_t launched(const fft3d::StageArgs& a, hipStream_t s, int kind, int n, int n2, int dtype)
{
    if (g_checking) return hipSuccess;
    const StubKernel& k = g_kernels.emplace(std::vector<int>{kind, n, n2, dtype}, StubKernel{kind, n, n2, dtype}).first->second;
    return fft3d::launch_stage_kernel(&k, dim3(1), dim3(64), a, 0, s);
}

}  // namespace

bool c2c_order_available(int n, int tdiv, int split)
{
    return length_supported(n) && radix_order_distinct(n) && tdiv == 1 && !split;
}

bool c2c_variant_available(int n, int tdiv, int split)
{
    if (tdiv == 1 && !split) return length_supported(n);
    if (!has_variants(n)) return false;
    const int tpl = radix_plan(n).tpl;
    return tdiv == 1 || (tdiv == 2 && tpl % 2 == 0) || (tdiv == 4 && tpl % 4 == 0);
}

hipError_t launch_c2c(int n, int dtype, const StageArgs& a, hipStream_t s)
{
    if (!length_supported(n)) return hipErrorInvalidValue;
    const int tdiv = a.tdiv < 1 ? 1 : a.tdiv;
    if (!c2c_variant_available(n, tdiv, a.split)) return hipErrorInvalidValue;
    if (a.order != 0 && (a.order != 1 || !c2c_order_available(n, tdiv, a.split) || a.nt != 0))
        return hipErrorInvalidValue;
    const size_t es = dtype == DT_F64 ? 16 : 8;
    const int threads = a.lw * (radix_plan(n).tpl / tdiv);
    const size_t line = a.strided ? (size_t)n : (size_t)(n + a.pad * (n / 8));
    const size_t lds = align16((size_t)a.lw * line * (a.split ? es / 2 : es)) + table_entries(n, a.order) * es;
    const int64_t blocks = a.strided ? (a.A + (a.align > 1 ? a.align - 1 : 0) + a.lw - 1) / a.lw
                                     : (a.A * a.B + a.lw - 1) / a.lw;
    if (a.align > 1 && (!a.strided || a.lw % a.align != 0)) violation("c2c align without a strided tile of whole lines");
    if (blocks == 0 || (a.strided && a.B == 0)) return hipSuccess;
    if (threads > kMaxThreads || lds > kMaxLdsBytes) return hipErrorInvalidConfiguration;
    if (a.strided && (a.sa != 1 || a.B > 65535)) violation("c2c strided tile with sa != 1 or too many rows");
    if (blocks > 0x7fffffff) violation("c2c grid too large");
    if (a.strided) {
        if (a.sa_o != 1) violation("c2c strided tile with sa_o != 1");
        check_range(a.in, es, a.off, a.A, 1, a.B, a.sb, n, a.se, "c2c strided load");
        check_range(a.out, es, a.off_o, a.A, 1, a.B, a.sb_o, n, a.se_o, "c2c strided store");
    } else {
        if (a.se != 1 || a.se_o != 1) violation("c2c contiguous tile with element stride != 1");
        check_range(a.in, es, a.off, a.A, a.sa, a.B, a.sb, n, 1, "c2c load");
        check_range(a.out, es, a.off_o, a.A, a.sa_o, a.B, a.sb_o, n, 1, "c2c store");
    }
    check_tables(a, n, es, "c2c pass table", a.order);
    return launched(a, s, K_C2C, n, a.order, dtype);
}

static hipError_t launch_real(bool r2c, int n, int dtype, const StageArgs& a, hipStream_t s)
{
    if (n % 2 != 0 || !length_supported(n / 2)) return hipErrorInvalidValue;
    const int h = n / 2;
    const size_t es = dtype == DT_F64 ? 16 : 8;
    const int threads = a.lw * radix_plan(h).tpl;
    const size_t lds = align16((size_t)a.lw * (h + 1 + (a.pad ? h / 8 : 0)) * es) + table_entries(h) * es;
    if ((a.A * a.B + a.lw - 1) / a.lw == 0) return hipSuccess;
    if (threads > kMaxThreads || lds > kMaxLdsBytes) violation("real kernel shape over the limits");
    // complex-pair side has h values per line, half-spectrum side h + 1
    const int64_t lin = r2c ? h : h + 1, lout = r2c ? h + 1 : h;
    check_range(a.in, es, a.off, a.A, a.sa, a.B, a.sb, lin, 1, r2c ? "r2c load" : "c2r load");
    check_range(a.out, es, a.off_o, a.A, a.sa_o, a.B, a.sb_o, lout, 1, r2c ? "r2c store" : "c2r store");
    in_alloc(a.tw, (size_t)(h + 1) * es, "real kernel root table");
    check_tables(a, h, es, "real kernel pass table");
    return launched(a, s, r2c ? K_R2C_X : K_C2R_X, n, 0, dtype);
}

hipError_t launch_r2c_x(int n, int dtype, const StageArgs& a, hipStream_t s) { return launch_real(true, n, dtype, a, s); }

hipError_t launch_c2r_x(int n, int dtype, const StageArgs& a, hipStream_t s) { return launch_real(false, n, dtype, a, s); }

hipError_t launch_c2c_xy(int nx, int ny, int dtype, const StageArgs& a, hipStream_t s)
{
    const size_t es = dtype == DT_F64 ? 16 : 8;
    if (!plane_available(nx, ny, es)) return hipErrorInvalidValue;
    if (a.B == 0) return hipSuccess;
    if (plane_threads(nx, ny) > kMaxThreads || plane_threads(nx, ny) % 64) violation("plane kernel threads");
    // plane b: rows of nx values sa apart, planes sb apart
    check_range(a.in, es, a.off, ny, a.sa, a.B, a.sb, nx, 1, "plane load");
    check_range(a.out, es, a.off_o, ny, a.sa_o, a.B, a.sb_o, nx, 1, "plane store");
    if (a.twp) check_tables(a, nx, es, "plane x pass table");
    const size_t sy = table_entries(ny);
    if (sy) in_alloc(a.twp2, sy * es, "plane y pass table");
    return launched(a, s, K_C2C_XY, nx, ny, dtype);
}

hipError_t launch_poisson_z(int n, int dtype, const StageArgs& a, hipStream_t s)
{
    if (!length_supported(n)) return hipErrorInvalidValue;
    const size_t es = dtype == DT_F64 ? 16 : 8;
    const int threads = a.lw * radix_plan(n).tpl;
    const size_t lds = align16((size_t)a.lw * n * es) + table_entries(n) * es;
    if ((a.A + a.lw - 1) / a.lw == 0 || a.B == 0) return hipSuccess;
    if (threads > kMaxThreads || lds > kMaxLdsBytes) violation("poisson kernel shape over the limits");
    if (a.sa != 1 || a.sa_o != 1) violation("poisson tile with sa != 1");
    check_range(a.in, es, a.off, a.A, 1, a.B, a.sb, n, a.se, "poisson load");
    check_range(a.out, es, a.off_o, a.A, 1, a.B, a.sb_o, n, a.se_o, "poisson store");
    check_tables(a, n, es, "poisson pass table");
    return launched(a, s, K_POISSON_Z, n, 0, dtype);
}

hipError_t launch_r2r_z(int n, int dtype, const StageArgs& a, hipStream_t s)
{
    if (!length_supported(n) || a.r2r < R2R_DCT2 || a.r2r > R2R_POISSON_D) return hipErrorInvalidValue;
    const size_t es = dtype == DT_F64 ? 16 : 8;
    const int threads = a.lw * radix_plan(n).tpl;
    const size_t lds = align16((size_t)a.lw * n * es) + table_entries(n) * es + (size_t)n * es;
    if ((a.A + a.lw - 1) / a.lw == 0 || a.B == 0) return hipSuccess;
    if (threads > kMaxThreads || lds > kMaxLdsBytes) violation("r2r kernel shape over the limits");
    if (a.sa != 1 || a.sa_o != 1) violation("r2r tile with sa != 1");
    check_range(a.in, es, a.off, a.A, 1, a.B, a.sb, n, a.se, "r2r load");
    check_range(a.out, es, a.off_o, a.A, 1, a.B, a.sb_o, n, a.se_o, "r2r store");
    check_tables(a, n, es, "r2r pass table");
    in_alloc(a.tw, (size_t)n * es, "r2r W_4n roots");
    return launched(a, s, K_R2R_Z, n, 0, dtype);
}

// A grouped launch: the table lies in one allocation and holds grid.x / gmax
// tiles, each with no more workgroups than gmax, and every tile passes the
// checks of a launch of its own (the launch's buffers where the entry has
// none).
void check_grouped(const void* f, dim3 grid, const StageArgs& a)
{
    if (!a.tiles) return;
    const StubKernel* k = nullptr;
    for (const auto& kv : g_kernels)
        if (&kv.second == f) k = &kv.second;
    if (!k) {
        violation("grouped launch of an unknown kernel");
        return;
    }
    if (a.gmax < 1 || grid.x % a.gmax != 0 || grid.y != 1 || grid.z != 1) {
        violation("grouped launch grid %u x %u x %u with gmax %lld", grid.x, grid.y, grid.z, (long long)a.gmax);
        return;
    }
    const int64_t count = grid.x / a.gmax;
    if (!in_alloc(a.tiles, (size_t)count * sizeof(TileEntry), "tile table")) return;
    if (a.ntiles < 0 || (a.ntiles > 0 && count % a.ntiles != 0))
        violation("interleaved grouped launch with runs of %lld for %lld tiles", (long long)a.ntiles, (long long)count);
    {
        // the device's workgroup -> (tile, local workgroup) map, tile-major or
        // interleaved, hits every workgroup of every tile exactly once
        std::vector<int64_t> hits((size_t)grid.x, 0);
        for (uint32_t w = 0; w < grid.x; ++w) {
            uint32_t t, local;
            if (a.ntiles > 0) {
                const uint32_t nt = (uint32_t)a.ntiles, span = nt * (uint32_t)a.gmax, run = w / span,
                               r = w - run * span;
                local = r / nt;
                t = run * nt + (r - local * nt);
            } else {
                t = w / (uint32_t)a.gmax;
                local = w - t * (uint32_t)a.gmax;
            }
            if ((int64_t)t >= count || (int64_t)local >= a.gmax) {
                violation("workgroup %u maps outside the grouped launch", w);
                break;
            }
            if (local < a.tiles[t].gx * a.tiles[t].gy) ++hits[(size_t)t * a.gmax + local];
        }
        for (int64_t t = 0; t < count; ++t)
            for (int64_t l = 0; l < a.tiles[t].gx * a.tiles[t].gy && l < a.gmax; ++l)
                if (hits[(size_t)(t * a.gmax + l)] != 1) {
                    violation("tile %lld workgroup %lld mapped %lld times", (long long)t, (long long)l,
                              (long long)hits[(size_t)(t * a.gmax + l)]);
                    t = count;
                    break;
                }
    }
    g_checking = true;
    for (int64_t i = 0; i < count; ++i) {
        const TileEntry& e = a.tiles[i];
        if (e.gx < 1 || e.gy < 1 || e.gx * e.gy > a.gmax) violation("tile %lld of a grouped launch has %lld x %lld workgroups, gmax %lld", (long long)i, (long long)e.gx, (long long)e.gy, (long long)a.gmax);
        StageArgs b = a;
        b.tiles = nullptr;
        b.gmax = 0;
        b.ntiles = 0;
        if (e.in) b.in = e.in;
        if (e.out) b.out = e.out;
        b.off = e.off;
        b.off_o = e.off_o;
        b.A = e.A;
        b.B = e.B;
        b.kx0 = e.kx0;
        b.ky0 = e.ky0;
        hipError_t r = hipSuccess;
        switch (k->kind) {
        case K_C2C: r = launch_c2c(k->n, k->dtype, b, nullptr); break;
        case K_R2C_X: r = launch_r2c_x(k->n, k->dtype, b, nullptr); break;
        case K_C2R_X: r = launch_c2r_x(k->n, k->dtype, b, nullptr); break;
        case K_C2C_XY: r = launch_c2c_xy(k->n, k->n2, k->dtype, b, nullptr); break;
        case K_POISSON_Z: r = launch_poisson_z(k->n, k->dtype, b, nullptr); break;
        case K_R2R_Z: r = launch_r2r_z(k->n, k->dtype, b, nullptr); break;
        default: violation("grouped launch of kernel kind %d", k->kind);
        }
        if (r != hipSuccess) violation("tile %lld of a grouped launch fails its own launch checks", (long long)i);
    }
    g_checking = false;
}

// The library's static device scratch: one stand-in allocation made before
// main (so it is not counted as a leak), like the array the GPU build holds
// from code-object load until the process ends.
namespace {
void* const g_scratch = [] {
    void* m = nullptr;
    hipMalloc(&m, kScratchBytes);
    return m;
}();
}  // namespace

hipError_t scratch_address(int device, void** out)
{
    *out = nullptr;
    if (device != 0) return hipErrorInvalidDevice;
    if (!g_scratch) return hipErrorOutOfMemory;
    *out = g_scratch;
    return hipSuccess;
}

}  // namespace fft3d
