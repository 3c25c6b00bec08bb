// C ABI of batched transforms: many independent, unevenly sized 3D FFTs in
// one persistent launch (work queue + per-stage completion counters, see
// k_batch.hip), captured once into a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "../../include/fft3d.h"
#include "batch_args.hpp"
#include "fft_lengths.hpp"
#include "kernels.hpp"
#include "plan.hpp"
#include "stage_args.hpp"

namespace fft3d {
fft3d_status set_error(fft3d_status st, const std::string& msg);  // runtime.cpp
fft3d_status set_hip_error(hipError_t e, const char* what);       // runtime.cpp
}  // namespace fft3d

using namespace fft3d;

namespace {

constexpr int kSpinLimit = 1 << 24;  // ~10^7 sleeps of 128 clocks: about half a second

struct OpState {
    std::vector<BatchSegDesc> q;
    std::vector<BatchSeg> hsegs;
    BatchSeg* dsegs = nullptr;
    int* ctl = nullptr;  // [0] head, [1] error, [2..] one counter per segment
    size_t lds = 0;
    int grid = 0;
    int64_t total = 0;
    int64_t stage_end[3] = {0, 0, 0};  // one past the last queue index of each stage
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<const void*> in_ptrs;
    std::vector<void*> out_ptrs;
    bool uploaded = false;
};

}  // namespace

struct fft3d_batch_s {
    std::vector<PlanDesc> ffts;
    int device = 0;
    int cus = 1;
    int mode = 0;
    std::map<int, void*> twp;  // length -> device per-pass twiddle table (complex64)
    std::map<std::pair<int, int>, int> lw_override;
    OpState ops[2];
    hipStream_t last_stream = nullptr;
    bool used = false;
};

namespace {

int lw_for(void* ctx, int n, int strided)
{
    const fft3d_batch_s* b = (const fft3d_batch_s*)ctx;
    auto it = b->lw_override.find({n, strided});
    return it != b->lw_override.end() ? it->second : batch_default_lw(n, strided);
}

size_t seg_lds(int n, int lw)
{
    const size_t data = ((size_t)(lw + 1) * n * 8 + 15) & ~(size_t)15;
    return data + (size_t)pass_table_size(radix_plan(n)) * 8;
}

void free_op(OpState& o)
{
    if (o.exec) hipGraphExecDestroy(o.exec);
    if (o.graph) hipGraphDestroy(o.graph);
    if (o.dsegs) hipFree(o.dsegs);
    if (o.ctl) hipFree(o.ctl);
    o = OpState();
}

// (Re)build the queue of one operation and its device tables.
fft3d_status prepare_op(fft3d_batch_s* b, int opi)
{
    OpState& o = b->ops[opi];
    free_op(o);
    o.q = build_batch_queue(b->ffts, opi == 0 ? OP_FORWARD : OP_INVERSE, lw_for, b);
    o.hsegs.assign(o.q.size(), BatchSeg());
    size_t lds = 0;
    for (size_t i = 0; i < o.q.size(); ++i) {
        const BatchSegDesc& d = o.q[i];
        BatchSeg& s = o.hsegs[i];
        memset(&s, 0, sizeof s);
        s.twp = b->twp[d.n];
        s.first = d.first;
        s.items = d.items;
        s.A = d.A; s.B = d.B; s.off = d.off; s.sa = d.sa; s.sb = d.sb; s.se = d.se;
        s.blocks_a = d.blocks_a;
        s.n = d.n; s.strided = d.strided; s.lw = d.lw; s.conj = d.conj;
        s.dep = d.dep;
        s.done_idx = d.done_idx;
        s.dep_count = d.dep_count;
        s.scale = (float)d.scale;
        lds = std::max(lds, seg_lds(d.n, d.lw));
        o.total = d.first + d.items;
        o.stage_end[d.stage] = std::max(o.stage_end[d.stage], d.first + d.items);
    }
    if (lds > kMaxLdsBytes) return set_error(FFT3D_ERR_INVALID_ARG, "lines per item exceed the LDS limit");
    o.lds = lds;
    o.grid = b->cus * batch_max_blocks_per_cu(lds);
    hipError_t e = hipMalloc(&o.dsegs, sizeof(BatchSeg) * o.hsegs.size());
    if (e == hipSuccess) e = hipMalloc(&o.ctl, sizeof(int) * (2 + o.hsegs.size()));
    if (e != hipSuccess) {
        free_op(o);
        return set_hip_error(e, "batch table allocation");
    }
    return FFT3D_OK;
}

BatchCtl make_ctl(const OpState& o, int64_t base, int64_t end, int ignore)
{
    BatchCtl c;
    memset(&c, 0, sizeof c);
    c.head = o.ctl;
    c.error = o.ctl + 1;
    c.done = o.ctl + 2;
    c.segs = o.dsegs;
    c.nsegs = (int)o.hsegs.size();
    c.spin_limit = kSpinLimit;
    c.item_base = base;
    c.total = end;
    c.ignore_deps = ignore;
    return c;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb)
{
    const char* pa = (const char*)a;
    const char* pb = (const char*)b;
    return pa < pb + nb && pb < pa + na;
}

fft3d_status run_batch(fft3d_batch_t b, int opi, const void* const* in, void* const* out, void* stream)
{
    if (!b) return set_error(FFT3D_ERR_INVALID_ARG, "null batch plan");
    if (!in || !out) return set_error(FFT3D_ERR_INVALID_ARG, "null pointer array");
    const int count = (int)b->ffts.size();
    std::vector<size_t> bytes(count);
    for (int f = 0; f < count; ++f) {
        if (!in[f] || !out[f]) return set_error(FFT3D_ERR_INVALID_ARG, "null buffer");
        bytes[f] = (size_t)b->ffts[f].nx * b->ffts[f].ny * b->ffts[f].nz * 8;
        if (in[f] != out[f] && overlap(in[f], bytes[f], out[f], bytes[f]))
            return set_error(FFT3D_ERR_ALIAS, "in and out of one transform partially overlap");
    }
    for (int f = 0; f < count; ++f)
        for (int g = 0; g < count; ++g)
            if (f != g && (overlap(out[f], bytes[f], out[g], bytes[g]) || overlap(out[f], bytes[f], in[g], bytes[g])))
                return set_error(FFT3D_ERR_ALIAS, "buffers of two transforms of the batch overlap");
    hipError_t e = hipSetDevice(b->device);
    if (e != hipSuccess) return set_hip_error(e, "hipSetDevice");
    OpState& o = b->ops[opi];
    hipStream_t s = (hipStream_t)stream;
    bool same = o.uploaded && (int)o.in_ptrs.size() == count;
    for (int f = 0; same && f < count; ++f) same = o.in_ptrs[f] == in[f] && o.out_ptrs[f] == out[f];
    if (!same) {
        for (size_t i = 0; i < o.q.size(); ++i) {
            const BatchSegDesc& d = o.q[i];
            o.hsegs[i].in = d.src == BUF_IN ? in[d.fft] : out[d.fft];
            o.hsegs[i].out = out[d.fft];
        }
        // the table may still be read by work enqueued earlier on this stream
        e = hipStreamSynchronize(s);
        if (e == hipSuccess)
            e = hipMemcpy(o.dsegs, o.hsegs.data(), sizeof(BatchSeg) * o.hsegs.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return set_hip_error(e, "batch table upload");
        o.in_ptrs.assign(in, in + count);
        o.out_ptrs.assign(out, out + count);
        o.uploaded = true;
    }
    const int nd = (int)o.hsegs.size();
    b->last_stream = s;
    b->used = true;
    if (b->mode == 2) {  // one launch per stage: the stream orders the stages
        int64_t base = 0;
        for (int st = 0; st < 3; ++st) {
            e = launch_batch(make_ctl(o, base, o.stage_end[st], 1), nd, o.grid, o.lds, s);
            if (e != hipSuccess) return set_hip_error(e, "batch launch");
            base = o.stage_end[st];
        }
        return FFT3D_OK;
    }
    const BatchCtl c = make_ctl(o, 0, o.total, 0);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    e = hipStreamIsCapturing(s, &cap);
    if (e != hipSuccess) return set_hip_error(e, "hipStreamIsCapturing");
    if (b->mode == 1 || cap != hipStreamCaptureStatusNone || s == nullptr) {
        // direct launch (also when the caller is capturing this stream itself)
        e = launch_batch(c, nd, o.grid, o.lds, s);
        return e == hipSuccess ? FFT3D_OK : set_hip_error(e, "batch launch");
    }
    if (!o.exec) {
        e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return set_hip_error(e, "hipStreamBeginCapture");
        hipError_t le = launch_batch(c, nd, o.grid, o.lds, s);
        e = hipStreamEndCapture(s, &o.graph);
        if (le != hipSuccess) return set_hip_error(le, "batch launch (capture)");
        if (e != hipSuccess) return set_hip_error(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&o.exec, o.graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            o.exec = nullptr;
            return set_hip_error(e, "hipGraphInstantiate");
        }
    }
    e = hipGraphLaunch(o.exec, s);
    return e == hipSuccess ? FFT3D_OK : set_hip_error(e, "hipGraphLaunch");
}

}  // namespace

extern "C" {

fft3d_status fft3d_plan_batch(fft3d_batch_t* out, int count, const int64_t* dims, int dtype)
{
    if (!out) return set_error(FFT3D_ERR_INVALID_ARG, "null plan pointer");
    *out = nullptr;
    if (count < 1 || !dims) return set_error(FFT3D_ERR_INVALID_ARG, "count >= 1 and dims required");
    if (dtype != DT_F32) return set_error(FFT3D_ERR_UNSUPPORTED_SIZE, "batched transforms are complex64 only");
    fft3d_batch_s* b = new fft3d_batch_s();
    for (int f = 0; f < count; ++f) {
        PlanDesc d{};
        d.nx = dims[3 * f]; d.ny = dims[3 * f + 1]; d.nz = dims[3 * f + 2];
        d.dtype = dtype; d.p1 = 1; d.p2 = 1; d.r2c = 0;
        if (!batch_length_supported(d.nx) || !batch_length_supported(d.ny) || !batch_length_supported(d.nz)) {
            delete b;
            return set_error(FFT3D_ERR_UNSUPPORTED_SIZE, "batched lengths must be supported lengths <= 512");
        }
        b->ffts.push_back(d);
    }
    hipError_t e = hipGetDevice(&b->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, b->device);
    if (e != hipSuccess) {
        delete b;
        return set_hip_error(e, "device query");
    }
    for (const PlanDesc& d : b->ffts) {
        for (int64_t n : {d.nx, d.ny, d.nz}) {
            if (b->twp.count((int)n)) continue;
            const int64_t entries = std::max<int64_t>(1, pass_twiddles_f32(n, nullptr));
            std::vector<float> h((size_t)(2 * entries), 0.f);
            pass_twiddles_f32(n, h.data());
            void* p = nullptr;
            e = hipMalloc(&p, h.size() * sizeof(float));
            if (e == hipSuccess) e = hipMemcpy(p, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                if (p) hipFree(p);
                fft3d_batch_destroy(b);
                return set_hip_error(e, "twiddle upload");
            }
            b->twp[(int)n] = p;
        }
    }
    for (int opi = 0; opi < 2; ++opi) {
        fft3d_status st = prepare_op(b, opi);
        if (st != FFT3D_OK) {
            fft3d_batch_destroy(b);
            return st;
        }
    }
    *out = b;
    return FFT3D_OK;
}

fft3d_status fft3d_batch_forward(fft3d_batch_t b, const void* const* in, void* const* out, void* stream)
{
    return run_batch(b, 0, in, out, stream);
}

fft3d_status fft3d_batch_inverse(fft3d_batch_t b, const void* const* in, void* const* out, void* stream)
{
    return run_batch(b, 1, in, out, stream);
}

fft3d_status fft3d_batch_set_lines(fft3d_batch_t b, int64_t n, int strided, int lw)
{
    if (!b) return set_error(FFT3D_ERR_INVALID_ARG, "null batch plan");
    if (!batch_length_supported(n) || strided < 0 || strided > 1 || lw < 0)
        return set_error(FFT3D_ERR_INVALID_ARG, "bad length, layout or lines per item");
    const int tpl = radix_plan((int)n).tpl;
    if (lw > 0 && (lw * tpl > kBatchThreadsPerBlock || seg_lds((int)n, lw) > kMaxLdsBytes))
        return set_error(FFT3D_ERR_INVALID_ARG, "lines per item exceed 256 threads or the LDS limit");
    if (b->last_stream || b->used) hipStreamSynchronize(b->last_stream);
    if (lw == 0) b->lw_override.erase({(int)n, strided});
    else b->lw_override[{(int)n, strided}] = lw;
    for (int opi = 0; opi < 2; ++opi) {
        fft3d_status st = prepare_op(b, opi);
        if (st != FFT3D_OK) return st;
    }
    return FFT3D_OK;
}

fft3d_status fft3d_batch_set_mode(fft3d_batch_t b, int mode)
{
    if (!b) return set_error(FFT3D_ERR_INVALID_ARG, "null batch plan");
    if (mode < 0 || mode > 2) return set_error(FFT3D_ERR_INVALID_ARG, "mode must be 0, 1 or 2");
    b->mode = mode;
    return FFT3D_OK;
}

fft3d_status fft3d_batch_check(fft3d_batch_t b)
{
    if (!b) return set_error(FFT3D_ERR_INVALID_ARG, "null batch plan");
    if (!b->used) return FFT3D_OK;
    hipError_t e = hipStreamSynchronize(b->last_stream);
    if (e != hipSuccess) return set_hip_error(e, "hipStreamSynchronize");
    for (int opi = 0; opi < 2; ++opi) {
        int flag = 0;
        if (!b->ops[opi].ctl) continue;
        e = hipMemcpy(&flag, b->ops[opi].ctl + 1, sizeof flag, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return set_hip_error(e, "error flag read");
        if (flag) return set_error(FFT3D_ERR_HIP, "a batched transform gave up waiting on a dependency");
    }
    return FFT3D_OK;
}

fft3d_status fft3d_batch_destroy(fft3d_batch_t b)
{
    if (!b) return FFT3D_OK;
    if (b->used) hipStreamSynchronize(b->last_stream);
    for (OpState& o : b->ops) free_op(o);
    for (auto& kv : b->twp) hipFree(kv.second);
    delete b;
    return FFT3D_OK;
}

int64_t fft3d_query_batch_queue(int count, const int64_t* dims, int op, int64_t* out, int64_t cap)
{
    if (count < 1 || !dims || (op != 0 && op != 1)) return -1;
    std::vector<PlanDesc> ffts;
    for (int f = 0; f < count; ++f) {
        PlanDesc d{};
        d.nx = dims[3 * f]; d.ny = dims[3 * f + 1]; d.nz = dims[3 * f + 2];
        if (!batch_length_supported(d.nx) || !batch_length_supported(d.ny) || !batch_length_supported(d.nz))
            return -1;
        ffts.push_back(d);
    }
    const auto q = build_batch_queue(ffts, op == 0 ? OP_FORWARD : OP_INVERSE, nullptr, nullptr);
    std::vector<int64_t> v;
    v.push_back((int64_t)q.size());
    for (const auto& s : q) {
        int64_t rec[11] = {s.fft, s.stage, s.axis, s.n, s.strided, s.lw, s.items, s.first, s.dep, s.dep_count,
                           s.done_idx};
        v.insert(v.end(), rec, rec + 11);
    }
    if (out && cap >= (int64_t)v.size()) memcpy(out, v.data(), v.size() * sizeof(int64_t));
    return (int64_t)v.size();
}

}  // extern "C"
