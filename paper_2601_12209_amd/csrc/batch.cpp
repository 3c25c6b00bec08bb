// C ABI of batched transforms: many independent, unevenly sized 3D FFTs.
// Every transform runs the stage kernels of the single-transform plan of its
// shape.  A call issues, stage by stage, one grouped launch per shape: the
// stage-s tiles of every transform of that shape in one kernel launch whose
// workgroups find their transform's buffers and tile in a device table (the
// paper's FFT tasks over uneven work, Sec. III-C and IV-D, released a stage at
// a time; shapes largest first, the order of Alg. 3's placement).  The tables
// of a pointer set are built on its first call and cached.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/fft3d.h"
#include "fft_lengths.hpp"
#include "kernels.hpp"
#include "plan.hpp"
#include "stage_args.hpp"

namespace fft3d {
fft3d_status set_error(fft3d_status st, const std::string& msg);  // runtime.cpp
fft3d_status set_hip_error(hipError_t e, const char* what);       // runtime.cpp
fft3d_status record_stage(fft3d_plan_s* p, int op, int stage, const void* in, void* out,
                          std::vector<KernelLaunch>* launches);  // runtime.cpp
int stage_count(fft3d_plan_s* p, int op);                        // runtime.cpp
}  // namespace fft3d

using namespace fft3d;

namespace {

constexpr size_t kMaxCached = 8;  // pointer sets with launch tables kept per batch

using Shape = std::tuple<int64_t, int64_t, int64_t>;

constexpr int kDefaultStreams = 4;

// The launches of one operation on one pointer set: one chain per stream
// (the shapes placed on it, each shape's stages in order); grouped launches
// point at the set's device table.
struct CachedIssue {
    int op;
    std::vector<const void*> in;
    std::vector<void*> out;
    std::vector<std::vector<KernelLaunch>> chains;
    TileEntry* dev = nullptr;
    bool captured = false;  // issued into a caller's capture: its graph refers to dev
};

}  // namespace

struct fft3d_batch_s {
    std::mutex mu;  // calls and setters on one batch are serialised
    std::vector<PlanDesc> ffts;
    int dtype = 0;
    int device = 0;
    std::map<Shape, fft3d_plan_t> plans;  // one single-stream plan per distinct shape
    std::vector<int> order;               // transforms in decreasing cost (issue order)
    std::vector<CachedIssue> cache;
    std::vector<TileEntry*> retired;  // tables of captured issues, kept until the batch is destroyed
    int nstreams = kDefaultStreams;  // shapes run concurrently on this many streams
    std::vector<hipStream_t> streams;  // created on the first call that forks
    std::vector<hipEvent_t> joins;
    hipEvent_t fork = nullptr;
    hipEvent_t done = nullptr;  // recorded on the caller's stream after each call
};

namespace {

Shape shape_of(const PlanDesc& d) { return Shape(d.nx, d.ny, d.nz); }

std::vector<double> batch_costs(const std::vector<PlanDesc>& ffts);

// Wait for the work of the last call (the caller's stream itself may be gone).
void wait_done(fft3d_batch_s* b)
{
    if (b->done) hipEventSynchronize(b->done);
}

// Drop the cached launch tables (after the last call); tables that a
// caller's captured graph may still use stay allocated until the batch is
// destroyed.
void drop_cache(fft3d_batch_s* b)
{
    wait_done(b);
    for (auto& c : b->cache) {
        if (!c.dev) continue;
        if (c.captured) b->retired.push_back(c.dev);
        else hipFree(c.dev);
    }
    b->cache.clear();
}

void release(fft3d_batch_s* b)
{
    drop_cache(b);
    for (TileEntry* t : b->retired) hipFree(t);
    for (hipStream_t st : b->streams)
        if (st) hipStreamDestroy(st);
    for (hipEvent_t ev : b->joins)
        if (ev) hipEventDestroy(ev);
    if (b->fork) hipEventDestroy(b->fork);
    if (b->done) hipEventDestroy(b->done);
    for (auto& kv : b->plans) fft3d_destroy(kv.second);
    delete b;
}

bool overlap(const void* a, size_t na, const void* c, size_t nc)
{
    const char* pa = (const char*)a;
    const char* pc = (const char*)c;
    return pa < pc + nc && pc < pa + na;
}

// Build the launches of operation op on this pointer set.  Each distinct
// shape gets one chain: per stage, the stage tiles of all its transforms as
// one grouped launch (or one by one where they cannot be grouped).  Shapes
// are placed on the batch's streams by Alg. 3's rule on their total cost
// (count x N log2 N), largest first; with one stream every chain runs in
// order on the caller's stream.
fft3d_status build_issue(fft3d_batch_t b, int op, const void* const* in, void* const* out, CachedIssue* c)
{
    const int pop = op == 0 ? OP_FORWARD : OP_INVERSE;
    std::vector<Shape> shapes;
    for (int f : b->order) {
        const Shape sh = shape_of(b->ffts[f]);
        if (std::find(shapes.begin(), shapes.end(), sh) == shapes.end()) shapes.push_back(sh);
    }
    const std::vector<double> fcost = batch_costs(b->ffts);
    std::vector<double> scost(shapes.size(), 0.0);
    for (size_t f = 0; f < b->ffts.size(); ++f)
        scost[std::find(shapes.begin(), shapes.end(), shape_of(b->ffts[f])) - shapes.begin()] += fcost[f];
    const int ns = std::max(1, std::min<int>(b->nstreams, (int)shapes.size()));
    const std::vector<std::vector<int>> placed = place_batch(scost, ns);
    // launch groups of each shape's chain, in stage order
    std::vector<std::vector<std::vector<KernelLaunch>>> groups(shapes.size());
    std::vector<std::vector<char>> grouped(shapes.size());
    size_t total = 0;
    for (size_t k = 0; k < shapes.size(); ++k) {
        fft3d_plan_t p = b->plans[shapes[k]];
        for (int st = 0; st < stage_count(p, pop); ++st) {
            std::vector<KernelLaunch> v, one;
            for (int f : b->order) {
                if (shape_of(b->ffts[f]) != shapes[k]) continue;
                const fft3d_status r = record_stage(p, pop, st, in[f], out[f], &one);
                if (r != FFT3D_OK) return r;
                v.insert(v.end(), one.begin(), one.end());
            }
            if (can_group(v.data(), v.size())) {
                total += v.size();
                groups[k].push_back(v);
                grouped[k].push_back(1);
            } else {
                for (const KernelLaunch& kl : v) {
                    groups[k].push_back({kl});
                    grouped[k].push_back(0);
                }
            }
        }
    }
    std::vector<TileEntry> host(total);
    std::vector<std::vector<size_t>> at(shapes.size());  // table offset of each launch of a chain
    std::vector<std::vector<KernelLaunch>> launches(shapes.size());
    size_t pos = 0;
    for (size_t k = 0; k < shapes.size(); ++k)
        for (size_t g = 0; g < groups[k].size(); ++g) {
            at[k].push_back(pos);
            if (!grouped[k][g]) {
                launches[k].push_back(groups[k][g][0]);
                continue;
            }
            KernelLaunch kl;
            make_group(groups[k][g].data(), groups[k][g].size(), true, 0, host.data() + pos, &kl);
            pos += groups[k][g].size();
            launches[k].push_back(kl);
        }
    c->dev = nullptr;
    if (total > 0) {
        hipError_t e = hipMalloc(&c->dev, total * sizeof(TileEntry));
        if (e == hipSuccess) e = hipMemcpy(c->dev, host.data(), total * sizeof(TileEntry), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            if (c->dev) hipFree(c->dev);
            c->dev = nullptr;
            return set_hip_error(e, "batch tile table upload");
        }
    }
    c->chains.assign(ns, {});
    for (int q = 0; q < ns; ++q)
        for (int k : placed[q])
            for (size_t g = 0; g < launches[k].size(); ++g) {
                KernelLaunch kl = launches[k][g];
                if (grouped[k][g]) kl.args.tiles = c->dev + at[k][g];
                c->chains[q].push_back(kl);
            }
    return FFT3D_OK;
}

// The batch's streams and events, created on the first call that forks.
hipError_t ensure_streams(fft3d_batch_t b, int ns)
{
    if ((int)b->streams.size() >= ns) return hipSuccess;
    hipError_t e = hipSuccess;
    if (!b->fork) {
        e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
        if (e != hipSuccess) {
            b->fork = nullptr;
            return e;
        }
    }
    while ((int)b->streams.size() < ns) {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            hipStreamDestroy(st);
            return e;
        }
        b->streams.push_back(st);
        b->joins.push_back(ev);
    }
    return hipSuccess;
}

fft3d_status run_batch(fft3d_batch_t b, int op, const void* const* in, void* const* out, void* stream)
{
    if (!b) return set_error(FFT3D_ERR_INVALID_ARG, "null batch plan");
    std::lock_guard<std::mutex> lock(b->mu);
    if (!in || !out) return set_error(FFT3D_ERR_INVALID_ARG, "null pointer array");
    const int count = (int)b->ffts.size();
    const size_t es = b->dtype == DT_F64 ? 16 : 8;
    std::vector<size_t> bytes(count);
    for (int f = 0; f < count; ++f) {
        if (!in[f] || !out[f]) return set_error(FFT3D_ERR_INVALID_ARG, "null buffer");
        bytes[f] = (size_t)b->ffts[f].nx * b->ffts[f].ny * b->ffts[f].nz * es;
        if (in[f] != out[f] && overlap(in[f], bytes[f], out[f], bytes[f]))
            return set_error(FFT3D_ERR_ALIAS, "in and out of one transform partially overlap");
    }
    for (int f = 0; f < count; ++f)
        for (int g = 0; g < count; ++g)
            if (f != g && (overlap(out[f], bytes[f], out[g], bytes[g]) || overlap(out[f], bytes[f], in[g], bytes[g])))
                return set_error(FFT3D_ERR_ALIAS, "buffers of two transforms of the batch overlap");
    hipError_t e = hipSetDevice(b->device);
    if (e != hipSuccess) return set_hip_error(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (s != nullptr) {  // the legacy default stream cannot be captured
        e = hipStreamIsCapturing(s, &cap);
        if (e != hipSuccess) return set_hip_error(e, "hipStreamIsCapturing");
    }
    CachedIssue* hit = nullptr;
    for (auto& c : b->cache) {
        if (c.op != op) continue;
        bool same = true;
        for (int f = 0; same && f < count; ++f) same = c.in[f] == in[f] && c.out[f] == out[f];
        if (same) {
            hit = &c;
            break;
        }
    }
    if (cap != hipStreamCaptureStatusNone) {
        // a stream the caller is capturing.  With launch tables already built
        // for this pointer set (an earlier call), their grouped launches go in
        // order onto the capturing stream, and the tables are kept until the
        // batch is destroyed (the caller's graph refers to them).  Otherwise
        // (building tables would allocate and copy during the capture) every
        // transform goes in order onto it, each plan issuing its stages in
        // order.
        if (hit) {
            hit->captured = true;
            for (const auto& chain : hit->chains)
                for (const KernelLaunch& kl : chain) {
                    e = launch_stage_kernel(kl.func, kl.grid, kl.block, kl.args, kl.lds, s);
                    if (e != hipSuccess) return set_hip_error(e, "batch kernel launch");
                }
            return FFT3D_OK;
        }
        for (int f : b->order) {
            fft3d_plan_t p = b->plans[shape_of(b->ffts[f])];
            fft3d_status st = op == 0 ? fft3d_forward(p, in[f], out[f], s) : fft3d_inverse(p, in[f], out[f], s);
            if (st != FFT3D_OK) return st;
        }
        return FFT3D_OK;
    }
    if (!hit) {
        if (b->cache.size() >= kMaxCached) drop_cache(b);
        CachedIssue c;
        c.op = op;
        c.in.assign(in, in + count);
        c.out.assign(out, out + count);
        const fft3d_status st = build_issue(b, op, in, out, &c);
        if (st != FFT3D_OK) return st;
        b->cache.push_back(c);
        hit = &b->cache.back();
    }
    const int ns = (int)hit->chains.size();
    if (ns == 1) {
        for (const KernelLaunch& kl : hit->chains[0]) {
            e = launch_stage_kernel(kl.func, kl.grid, kl.block, kl.args, kl.lds, s);
            if (e != hipSuccess) return set_hip_error(e, "batch kernel launch");
        }
    } else {
        // fork the chains from the caller's stream onto the batch's streams
        // and join them back
        e = ensure_streams(b, ns);
        if (e != hipSuccess) return set_hip_error(e, "batch streams");
        e = hipEventRecord(b->fork, s);
        if (e != hipSuccess) return set_hip_error(e, "hipEventRecord(fork)");
        for (int q = 0; q < ns; ++q) {
            e = hipStreamWaitEvent(b->streams[q], b->fork, 0);
            if (e != hipSuccess) return set_hip_error(e, "hipStreamWaitEvent(fork)");
            for (const KernelLaunch& kl : hit->chains[q]) {
                e = launch_stage_kernel(kl.func, kl.grid, kl.block, kl.args, kl.lds, b->streams[q]);
                if (e != hipSuccess) return set_hip_error(e, "batch kernel launch");
            }
            e = hipEventRecord(b->joins[q], b->streams[q]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, b->joins[q], 0);
            if (e != hipSuccess) return set_hip_error(e, "batch join");
        }
    }
    if (!b->done) {
        e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
        if (e != hipSuccess) {
            b->done = nullptr;
            return set_hip_error(e, "hipEventCreate");
        }
    }
    e = hipEventRecord(b->done, s);
    return e == hipSuccess ? FFT3D_OK : set_hip_error(e, "hipEventRecord");
}

std::vector<double> batch_costs(const std::vector<PlanDesc>& ffts)
{
    std::vector<double> c;
    for (const PlanDesc& d : ffts) {
        const double n = (double)d.nx * d.ny * d.nz;
        c.push_back(n * log2(std::max(2.0, n)));
    }
    return c;
}

}  // namespace

extern "C" {

fft3d_status fft3d_plan_batch(fft3d_batch_t* out, int count, const int64_t* dims, int dtype)
{
    if (!out) return set_error(FFT3D_ERR_INVALID_ARG, "null plan pointer");
    *out = nullptr;
    if (count < 1 || !dims) return set_error(FFT3D_ERR_INVALID_ARG, "count >= 1 and dims required");
    if (dtype != DT_F32 && dtype != DT_F64) return set_error(FFT3D_ERR_INVALID_ARG, "dtype must be 0 or 1");
    fft3d_batch_s* b = new fft3d_batch_s();
    b->dtype = dtype;
    for (int f = 0; f < count; ++f) {
        PlanDesc d{};
        d.nx = dims[3 * f]; d.ny = dims[3 * f + 1]; d.nz = dims[3 * f + 2];
        d.dtype = dtype; d.p1 = 1; d.p2 = 1; d.r2c = 0;
        b->ffts.push_back(d);
        const Shape sh = shape_of(d);
        if (b->plans.count(sh)) continue;
        fft3d_plan_t p = nullptr;
        fft3d_status st = fft3d_plan(&p, d.nx, d.ny, d.nz, dtype, 1, 1, 0);
        if (st == FFT3D_OK) st = fft3d_set_streams(p, 1);
        // transforms of one shape share the plan: no workspace (fused x-y
        // planes where the plane fits in LDS, else in place)
        if (st == FFT3D_OK && fft3d_set_staging(p, FFT3D_STAGING_FUSED_XY) != FFT3D_OK)
            st = fft3d_set_staging(p, FFT3D_STAGING_IN_PLACE);
        if (st != FFT3D_OK) {
            if (p) fft3d_destroy(p);
            release(b);
            return st;
        }
        b->plans[sh] = p;
    }
    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) {
        release(b);
        return set_hip_error(e, "hipGetDevice");
    }
    b->order = place_batch(batch_costs(b->ffts), 1)[0];
    *out = b;
    return FFT3D_OK;
}

fft3d_status fft3d_forward_batch(fft3d_batch_t b, const void* const* in, void* const* out, void* stream)
{
    return run_batch(b, 0, in, out, stream);
}

fft3d_status fft3d_inverse_batch(fft3d_batch_t b, const void* const* in, void* const* out, void* stream)
{
    return run_batch(b, 1, in, out, stream);
}

fft3d_status fft3d_batch_set_stage_config(fft3d_batch_t b, int64_t nx, int64_t ny, int64_t nz, int axis, int lw,
                                          int tdiv, int split, int pad)
{
    if (!b) return set_error(FFT3D_ERR_INVALID_ARG, "null batch plan");
    std::lock_guard<std::mutex> lock(b->mu);
    auto it = b->plans.find(Shape(nx, ny, nz));
    if (it == b->plans.end()) return set_error(FFT3D_ERR_INVALID_ARG, "no transform of that shape in the batch");
    drop_cache(b);  // launch shapes are baked into the cached launches
    return fft3d_set_stage_config(it->second, axis, lw, tdiv, split, pad);
}

fft3d_status fft3d_batch_set_radix_order(fft3d_batch_t b, int64_t nx, int64_t ny, int64_t nz, int axis, int order)
{
    if (!b) return set_error(FFT3D_ERR_INVALID_ARG, "null batch plan");
    std::lock_guard<std::mutex> lock(b->mu);
    auto it = b->plans.find(Shape(nx, ny, nz));
    if (it == b->plans.end()) return set_error(FFT3D_ERR_INVALID_ARG, "no transform of that shape in the batch");
    drop_cache(b);  // the radix order is baked into the cached launches
    return fft3d_set_radix_order(it->second, axis, order);
}

fft3d_status fft3d_batch_set_staging(fft3d_batch_t b, int64_t nx, int64_t ny, int64_t nz, int staging)
{
    if (!b) return set_error(FFT3D_ERR_INVALID_ARG, "null batch plan");
    std::lock_guard<std::mutex> lock(b->mu);
    auto it = b->plans.find(Shape(nx, ny, nz));
    if (it == b->plans.end()) return set_error(FFT3D_ERR_INVALID_ARG, "no transform of that shape in the batch");
    if (staging != FFT3D_STAGING_IN_PLACE && staging != FFT3D_STAGING_FUSED_XY)
        return set_error(FFT3D_ERR_INVALID_ARG, "a batch stages in place or in fused x-y planes (no workspace)");
    drop_cache(b);  // the stage lists are baked into the cached launches
    return fft3d_set_staging(it->second, staging);
}

fft3d_status fft3d_batch_set_streams(fft3d_batch_t b, int nstreams)
{
    if (!b) return set_error(FFT3D_ERR_INVALID_ARG, "null batch plan");
    std::lock_guard<std::mutex> lock(b->mu);
    if (nstreams < 1 || nstreams > 16) return set_error(FFT3D_ERR_INVALID_ARG, "nstreams must be 1..16");
    drop_cache(b);  // the chains are placed per stream count
    b->nstreams = nstreams;
    return FFT3D_OK;
}

int fft3d_batch_get_staging(fft3d_batch_t b, int64_t nx, int64_t ny, int64_t nz)
{
    if (!b) {
        set_error(FFT3D_ERR_INVALID_ARG, "null batch plan");
        return -1;
    }
    std::lock_guard<std::mutex> lock(b->mu);
    auto it = b->plans.find(Shape(nx, ny, nz));
    if (it == b->plans.end()) {
        set_error(FFT3D_ERR_INVALID_ARG, "no transform of that shape in the batch");
        return -1;
    }
    return fft3d_get_staging(it->second);
}

fft3d_status fft3d_batch_destroy(fft3d_batch_t b)
{
    if (b) release(b);
    return FFT3D_OK;
}

int64_t fft3d_query_batch_placement(int count, const int64_t* dims, int nstreams, int64_t* out, int64_t cap)
{
    if (count < 1 || !dims || nstreams < 1) return -1;
    std::vector<PlanDesc> ffts;
    for (int f = 0; f < count; ++f) {
        PlanDesc d{};
        d.nx = dims[3 * f]; d.ny = dims[3 * f + 1]; d.nz = dims[3 * f + 2];
        if (d.nx < 1 || d.ny < 1 || d.nz < 1) return -1;
        ffts.push_back(d);
    }
    const auto per = place_batch(batch_costs(ffts), nstreams);
    std::vector<int64_t> v;
    v.push_back((int64_t)per.size());
    for (const auto& p : per) {
        v.push_back((int64_t)p.size());
        v.insert(v.end(), p.begin(), p.end());
    }
    if (out && cap >= (int64_t)v.size()) memcpy(out, v.data(), v.size() * sizeof(int64_t));
    return (int64_t)v.size();
}

}  // extern "C"
