// C ABI of the library: plan objects, argument checks, and the issue of
// pencil-tile tasks onto HIP streams (paper Alg. 1 stages, Sec. IV-D per-tile
// dependencies, Alg. 3 placement; see plan.cpp for the graph itself).
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fft3d.h"
#include "fft_lengths.hpp"
#include "kernels.hpp"
#include "plan.hpp"
#include "plane_list.hpp"
#include "stage_args.hpp"

using namespace fft3d;

namespace {

thread_local std::string g_last_error;

fft3d_status fail(fft3d_status st, const std::string& msg)
{
    g_last_error = msg;
    return st;
}

fft3d_status hip_fail(hipError_t e, const char* what)
{
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    g_last_error = buf;
    return e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation ? FFT3D_ERR_ALLOC
                                                                     : FFT3D_ERR_HIP;
}

constexpr int kMaxStreams = 16;
// Tiles per stage a plan may have: the planner's dependency search is
// quadratic in it and a plan creates five events per tile.
constexpr int64_t kMaxTiles = 1024;
// C2C plans of at least this many bytes, and R2C plans whose half spectrum is
// at least this large, default to the swapped-y/z staging (measured on MI355X:
// faster at 512^3, slower at 256^3, whose 128-256 MiB field stays in the
// 256 MB Infinity Cache)
constexpr size_t kSwapStagingMinBytes = (size_t)512 << 20;
constexpr size_t kR2CSwapMaxBytes = (size_t)2 << 30;  // R2C: half spectra from here stage in place

}  // namespace

namespace fft3d {
namespace {
thread_local KernelLaunch* t_recorder = nullptr;
thread_local bool* t_recorded = nullptr;
}  // namespace

void set_launch_recorder(KernelLaunch* rec, bool* recorded)
{
    t_recorder = rec;
    t_recorded = recorded;
}

hipError_t launch_stage_kernel(const void* func, dim3 grid, dim3 block, const StageArgs& a, size_t lds,
                               hipStream_t s)
{
    if (t_recorder) {
        t_recorder->func = func;
        t_recorder->grid = grid;
        t_recorder->block = block;
        t_recorder->lds = lds;
        t_recorder->args = a;
        *t_recorded = true;
        return hipSuccess;
    }
    StageArgs arg = a;
    void* args[] = {&arg};
    return hipLaunchKernel(func, grid, block, args, lds, s);
}

// The tile launches of one stage of one call of `p` (operation op, in ->
// out, the plan's workspace), recorded instead of issued; tiles with nothing
// to launch are left out.  Used by the batch to group the stage launches of
// its transforms.
fft3d_status record_stage(fft3d_plan_s* p, int op, int stage, const void* in, void* out,
                          std::vector<KernelLaunch>* launches);
int stage_count(fft3d_plan_s* p, int op);

namespace {
// StageArgs with the per-tile fields cleared, for comparing launches.
StageArgs without_tile_fields(StageArgs a)
{
    a.in = nullptr;
    a.out = nullptr;
    a.off = a.off_o = a.A = a.B = a.kx0 = a.ky0 = 0;
    a.tiles = nullptr;
    a.gmax = 0;
    return a;
}
}  // namespace

bool can_group(const KernelLaunch* v, size_t n)
{
    if (n < 2) return false;
    const StageArgs a0 = without_tile_fields(v[0].args);
    uint64_t gmax = 1;
    for (size_t i = 0; i < n; ++i) gmax = std::max<uint64_t>(gmax, (uint64_t)v[i].grid.x * v[i].grid.y);
    // the grouped grid (gmax * n workgroups along x) must fit the dispatch's 32-bit work-item count
    if (gmax * n > 0x7fffffffu || gmax * n * v[0].block.x > 0xffffffffu) return false;
    for (size_t i = 0; i < n; ++i) {
        if (v[i].func != v[0].func || v[i].lds != v[0].lds || v[i].block.x != v[0].block.x ||
            v[i].block.y != v[0].block.y || v[i].block.z != v[0].block.z || v[i].grid.z != 1 ||
            v[i].args.tiles != nullptr)
            return false;
        const StageArgs ai = without_tile_fields(v[i].args);
        if (memcmp(&ai, &a0, sizeof ai) != 0) return false;
    }
    return true;
}

void make_group(const KernelLaunch* v, size_t n, bool own_buffers, int64_t ntiles, TileEntry* entries,
                KernelLaunch* common)
{
    int64_t gmax = 1;
    for (size_t i = 0; i < n; ++i) {
        const StageArgs& a = v[i].args;
        TileEntry& e = entries[i];
        e.in = own_buffers ? a.in : nullptr;
        e.out = own_buffers ? a.out : nullptr;
        e.off = a.off;
        e.off_o = a.off_o;
        e.A = a.A;
        e.B = a.B;
        e.kx0 = a.kx0;
        e.ky0 = a.ky0;
        e.gx = v[i].grid.x;
        e.gy = v[i].grid.y;
        gmax = std::max<int64_t>(gmax, e.gx * e.gy);
    }
    *common = v[0];
    common->args.gmax = gmax;
    common->args.ntiles = ntiles > 0 && n % (size_t)ntiles == 0 ? ntiles : 0;
    common->grid = dim3((unsigned)(gmax * (int64_t)n), 1, 1);
}

// error reporting shared with the batch entry points (batch.cpp)
fft3d_status set_error(fft3d_status st, const std::string& msg) { return fail(st, msg); }
fft3d_status set_hip_error(hipError_t e, const char* what) { return hip_fail(e, what); }
}  // namespace fft3d

namespace {
constexpr int kDefaultStreams = 4;

}  // namespace

// Launch shape of one stage kernel.
struct KConf {
    int lw = 0;      // lines per workgroup (0: use the default shape)
    int tdiv = 1;    // threads-per-line divisor
    int split = 0;   // split re/im LDS exchange
    int pad = 0;     // padded contiguous LDS lines
};

struct fft3d_plan_s {
    PlanDesc d{};
    int device = 0;
    int nstreams = kDefaultStreams;
    std::vector<hipStream_t> streams;  // kMaxStreams slots, created when a multi-stream issue needs them
    std::vector<hipEvent_t> events;    // one per task of the largest pipeline
    hipEvent_t fork = nullptr;
    void* tw[3] = {nullptr, nullptr, nullptr};   // per-axis forward root tables
    void* twp[3] = {nullptr, nullptr, nullptr};  // per-axis per-pass tables of the kernel length
    void* twp_rev[3] = {nullptr, nullptr, nullptr};  // the same for the reverse radix order (C2C axes)
    void* ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_owned = false;
    Pipeline pipes[OP_COUNT];
    bool pipe_ok[OP_COUNT] = {};
    std::vector<char> needs_event[OP_COUNT];
    KConf conf_override[3];  // per axis; lw == 0: default
    int order_override[3] = {0, 0, 0};  // per axis: radix order of the C2C line kernels
    // Completion of the last call issued outside a stream capture, recorded on
    // that call's stream.  A call on another stream first waits on it, so two
    // streams never use the plan's workspace at once; the destructor and the
    // setters wait on it before they free or rebuild anything.
    hipEvent_t call_done = nullptr;
    hipStream_t last_stream = nullptr;
    bool called = false;
    std::mutex mu;  // one host thread at a time inside a call or setter
    // per-stage timing (tracing): events around every stage of the last call
    bool timing = false;
    std::vector<hipEvent_t> tev;  // 6 timing events (up to 5 stages)
    int timed_stages = 0;
    // issue of tiled plans (fft3d_set_issue): one launch per tile on the
    // plan's streams, or one grouped launch per stage
    int issue = FFT3D_ISSUE_STAGES;
    struct StageGroup {
        bool grouped = false;  // one launch for all tiles of the stage
        KernelLaunch launch;   // that launch (args.in/out set per call)
    };
    struct OpGroups {
        bool valid = false;
        std::vector<StageGroup> stages;
        TileEntry* dev = nullptr;  // the grouped stages' tile tables
    };
    OpGroups groups[OP_COUNT];
};

namespace {

size_t elem_bytes(int dtype) { return dtype == DT_F64 ? 16 : 8; }

int64_t next_pow2(int64_t v)
{
    int64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

int kernel_length(const Stage& st)
{
    const bool real = st.kind == K_R2C_X || st.kind == K_C2R_X;
    return real ? st.n / 2 : st.n;
}

// Threads and LDS bytes a configuration needs, or false if it cannot run.
bool conf_fits(const Stage& st, int dtype, const KConf& c, bool strided)
{
    if (st.kind == K_C2C_XY) return true;  // fixed launch shape
    const int nk = kernel_length(st);
    const RadixPlan rp = radix_plan(nk);
    if (c.lw < 1 || c.tdiv < 1 || rp.tpl % c.tdiv != 0) return false;
    const bool real_x = st.kind == K_R2C_X || st.kind == K_C2R_X;
    if (st.kind != K_C2C && (c.tdiv != 1 || c.split || (c.pad && !real_x))) return false;
    if (st.kind == K_C2C && !c2c_variant_available(nk, c.tdiv, c.split)) return false;
    const int threads = c.lw * (rp.tpl / c.tdiv);
    const size_t s = elem_bytes(dtype) / (c.split ? 2 : 1);
    const size_t line = strided ? (size_t)nk : (size_t)(nk + 1 + (c.pad ? nk / 8 : 0));
    size_t tw = (size_t)pass_table_size(rp) * elem_bytes(dtype) + 16;
    if (st.kind == K_R2R_Z) tw += (size_t)nk * elem_bytes(dtype);  // the W_4n roots
    return threads <= 1024 && (size_t)c.lw * line * s + tw <= kMaxLdsBytes;
}

// Default launch shape (chosen from measured sweeps on MI355X at 512^3).
// Strided stages (y, z): 16 neighbouring lines per workgroup (128-byte row
// segments for complex64, 256 for complex128), more for short lines so a
// workgroup has >= 256 threads, threads per line divided down to fit 1024,
// split re/im exchange (half the LDS).  Contiguous stages (x): ~128 threads,
// split exchange and padded LDS lines.
KConf default_conf(const PlanDesc& d, const Stage& st, const Box& b)
{
    const int nk = kernel_length(st);
    const int tpl = radix_plan(nk).tpl;
    KConf c;
    const bool c2c = st.kind == K_C2C;
    const bool pow2_tpl = (tpl & (tpl - 1)) == 0;
    if (st.axis != 0) {
        // threads per line that are not a power of two leave the lines'
        // wavefronts partly idle; there 8-line tiles (more workgroups per CU)
        // measured fastest on MI355X: complex64 840^3 y/z 2.51-2.57 ms against
        // 2.97-3.15 for 16 lines, 720^3 1.63-1.66 against 1.95, complex128
        // 840^3 3.76-3.79 against 4.63-4.68
        int lw = pow2_tpl ? 16 : 8;
        while (lw * tpl < 256 && lw < 64) lw *= 2;
        const int64_t a = b.hi[0] - b.lo[0];
        lw = (int)std::min<int64_t>(lw, next_pow2(a));
        // too many threads for lw lines: fewer threads per line (2 or 4) where
        // the kernel has the variant
        int tdiv = 1;
        if (c2c && lw * tpl > 1024) {
            for (int td : {2, 4})
                if (tpl % td == 0 && c2c_variant_available(nk, td, 1) && lw * (tpl / td) <= 1024) {
                    tdiv = td;
                    break;
                }
            if (tdiv == 1)  // none fits 1024 threads: the largest divisor, lw shrinks below
                for (int td : {4, 2})
                    if (tpl % td == 0 && c2c_variant_available(nk, td, 1)) {
                        tdiv = td;
                        break;
                    }
        }
        c.lw = lw;
        c.tdiv = tdiv;
        c.split = c2c && c2c_variant_available(nk, tdiv, 1) ? 1 : 0;
        // complex64 lines of 64-256 points: the full complex LDS tile (at most
        // 32 KiB for 16 lines) runs faster than the split exchange (autotuner
        // at 256^3 on MI355X: y and z 3-5 % faster; the batch's 64^3 and
        // 100x120x128 z stages chose it too)
        if (c2c && d.dtype == DT_F32 && nk <= 256 && pow2_tpl && (nk & (nk - 1)) == 0) c.split = 0;
        // complex64 lines of 512 with a full complex LDS tile (no split
        // exchange).  In whole 32-line tiles: 32 lines per workgroup
        // (256-byte row segments) with half the threads per line: fwd+inv
        // 2.42 ms at 512^3 on MI355X against 2.43 for 16-line tiles and 2.46
        // with the split exchange.  Otherwise (the R2C half spectrum's 257
        // columns) 16 lines, one thread per butterfly.
        // (decided per plan, not per tile, so that every tile of a stage runs
        // the same kernel and the stage stays one grouped launch)
        if (c2c && d.dtype == DT_F32 && nk == 512 && d.nxc() >= 16) {
            KConf w;
            const bool whole32 = !d.r2c && d.nx % 32 == 0 && c2c_variant_available(nk, 2, 0);
            w.lw = whole32 ? 32 : 16;
            w.tdiv = whole32 ? 2 : 1;
            w.split = 0;
            if (conf_fits(st, d.dtype, w, true)) c = w;
        }
        // complex64 lines of 1024 over an R2C half spectrum: 16 lines with a
        // full complex LDS tile as well (1024^3 z stage 2.52 ms against 2.74
        // with the split exchange, MI355X)
        if (c2c && d.dtype == DT_F32 && nk == 1024 && d.r2c && d.nxc() >= 16) {
            KConf w;
            w.lw = 16;
            w.tdiv = 1;
            w.split = 0;
            if (conf_fits(st, d.dtype, w, true)) c = w;
        }
    } else {
        int lw = 1;
        while (2 * lw * tpl <= 128) lw *= 2;
        // thread counts per line that are not a power of two leave the lines'
        // wavefronts partly idle, so take more lines: below 32 threads per
        // line >= 256 threads (the rule for all such lengths before the
        // radix-15 pass: 480^3 complex64 with 60 threads per line went from
        // 0.38 ms on 2 lines to 0.33 on 8), from 32 up >= 128 (840^3 with 56
        // threads per line: 1.85 ms on 4 lines against 1.98 on 8; 720^3, 45
        // per line: 1.43 against 1.48; MI355X)
        if (!pow2_tpl)
            while (lw * tpl < (tpl >= 32 ? 128 : 256)) lw *= 2;
        // the complex64 real kernels at half lengths 256 and 512 run fastest
        // with more lines per workgroup on MI355X: R2C 512 threads (512^3:
        // 16 lines, 237 -> 195 us; 1024^3: 8 lines), C2R 8 lines (512^3: 241
        // -> 233 us); the complex128 ones are best at the default
        if (d.dtype == DT_F32 && (nk == 256 || nk == 512)) {
            if (st.kind == K_R2C_X) lw = 512 / tpl;
            if (st.kind == K_C2R_X) lw = 8;
        }
        c.lw = lw;
        c.split = c2c && c2c_variant_available(nk, 1, 1) ? 1 : 0;
        c.pad = 1;
    }
    // the hard limits (1024 threads, 160 KiB of LDS) always hold
    while (c.lw > 1 && !conf_fits(st, d.dtype, c, st.axis != 0)) c.lw /= 2;
    return c;
}

// Row pitch (complex elements) of a complex buffer: the workspace rows are
// padded to 128 bytes, caller buffers are dense.
int64_t row_pitch(const PlanDesc& d, int buf) { return buf == BUF_WS ? d.wpitch() : d.nxc(); }

// Element strides (x, y, z) of a complex buffer in a layout.
void layout_strides(const PlanDesc& d, int buf, int lay, int64_t st[3])
{
    const int64_t pitch = row_pitch(d, buf);
    st[0] = 1;
    if (lay == LAY_SWAP_YZ) {
        st[1] = pitch * d.nz;
        st[2] = pitch;
    } else {
        st[1] = pitch;
        st[2] = pitch * d.ny;
    }
}

// Cache policy of a C2C launch (StageArgs::nt), from measurements at 512^3 on
// MI355X.  Non-temporal stores: complex128 C2C stages 2-3 % faster, in-place
// R2C y stages 11-19 %; complex64 stages writing another buffer along y or z
// ran 1-2 % slower with them and keep plain stores.  Non-temporal loads as
// well where the tile reads whole cache lines of another buffer (complex128
// stages a further 1-3 %, the complex64 x stage 3-4 %); where neighbouring
// tiles share lines (misaligned rows) or the stage works in place, plain
// loads (non-temporal ones there measured 4-25 % slower).  Fields that fit
// the 256 MB Infinity Cache next to their workspace keep plain accesses, so
// one stage's output stays cached for the next.
int c2c_cache_policy(const PlanDesc& d, const Stage& st, const StageArgs& a, int64_t per_line)
{
    if (st.kind != K_C2C) return 0;
    if ((size_t)d.nxc() * d.ny * d.nz * elem_bytes(d.dtype) < kSwapStagingMinBytes) return 0;
    const bool in_place = st.src == st.dst;
    // complex64 C2C plans' y/z stages writing another buffer keep plain stores
    // (1-2 % slower with them at 512^3); the R2C half spectrum's gain (R2C y
    // and z stages 252 -> 234 us mean at 512^3)
    if (d.dtype == DT_F32 && a.strided && !in_place && !d.r2c) return 0;
    bool whole_lines;
    if (a.strided)  // row segments of lw lines at off + b*sb + e*se
        whole_lines = a.align <= 1 && a.lw % per_line == 0 && a.A % per_line == 0 && a.off % per_line == 0 &&
                      a.sb % per_line == 0 && a.se % per_line == 0;
    else  // lanes along each line: lines of st.n contiguous values at off + a*sa + b*sb
        whole_lines = a.se == 1 && st.n % per_line == 0 && a.off % per_line == 0 && a.sa % per_line == 0 &&
                      a.sb % per_line == 0;
    return !in_place && whole_lines ? 2 : 1;
}

StageArgs make_args(const fft3d_plan_s* p, const Stage& st, const Box& b, void* const bufs[3])
{
    const PlanDesc& d = p->d;
    const int64_t ny = d.ny;
    StageArgs a;
    memset(&a, 0, sizeof a);
    a.in = bufs[st.src];
    a.out = bufs[st.dst];
    a.tw = p->tw[st.axis];
    a.twp = p->twp[st.axis];
    a.twp2 = p->twp[1];
    a.conj = st.conj;
    a.weight = st.weight;
    a.scale = st.scale;
    // the tile's lines run along st.axis; they form an A x B grid over the
    // other two axes (x first when it is one of them)
    const int ax_a = st.axis == 0 ? 1 : 0;
    const int ax_b = st.axis == 2 ? 1 : 2;
    a.A = b.hi[ax_a] - b.lo[ax_a];
    a.B = b.hi[ax_b] - b.lo[ax_b];
    if (st.kind == K_R2C_X || st.kind == K_C2R_X) {
        // real rows: nx reals = nx/2 complex pairs per row (dense, natural
        // order); complex rows: the buffer's pitch and layout (row (y, z) at
        // y*st[1] + z*st[2])
        const int64_t h = d.nx / 2;
        int64_t sc[3];
        layout_strides(d, st.kind == K_R2C_X ? st.dst : st.src, st.kind == K_R2C_X ? st.lay_dst : st.lay_src, sc);
        const int64_t ry = st.kind == K_R2C_X ? h : sc[1], rz = st.kind == K_R2C_X ? h * ny : sc[2];
        const int64_t wy = st.kind == K_R2C_X ? sc[1] : h, wz = st.kind == K_R2C_X ? sc[2] : h * ny;
        a.off = b.lo[1] * ry + b.lo[2] * rz; a.sa = ry; a.sb = rz; a.se = 1;
        a.off_o = b.lo[1] * wy + b.lo[2] * wz; a.sa_o = wy; a.sb_o = wz; a.se_o = 1;
        a.strided = 0;
    } else {
        int64_t si[3], so[3];
        layout_strides(d, st.src, st.lay_src, si);
        layout_strides(d, st.dst, st.lay_dst, so);
        a.off = b.lo[0] * si[0] + b.lo[1] * si[1] + b.lo[2] * si[2];
        a.sa = si[ax_a]; a.sb = si[ax_b]; a.se = si[st.axis];
        a.off_o = b.lo[0] * so[0] + b.lo[1] * so[1] + b.lo[2] * so[2];
        a.sa_o = so[ax_a]; a.sb_o = so[ax_b]; a.se_o = so[st.axis];
        a.strided = st.axis != 0 ? 1 : 0;
    }
    if (st.kind == K_C2C_XY) {
        // whole planes: rows of nx values (pitch sa), planes sb apart, B planes
        a.A = 1;
        a.B = b.hi[2] - b.lo[2];
        int64_t si[3], so[3];
        layout_strides(d, st.src, st.lay_src, si);
        layout_strides(d, st.dst, st.lay_dst, so);
        a.sa = si[1]; a.sb = si[2]; a.sa_o = so[1]; a.sb_o = so[2];
        a.strided = 0;
        return a;
    }
    if (st.kind == K_POISSON_Z || st.kind == K_R2R_Z) {
        a.pnx = d.nx; a.pny = d.ny; a.pnz = d.nz;
        a.kx0 = b.lo[0];
        a.ky0 = b.lo[1];
        a.r2r = st.r2r;
    }
    KConf c = default_conf(d, st, b);
    const KConf& ov = p->conf_override[st.axis];
    if (ov.lw > 0) {
        KConf o = ov;
        if (conf_fits(st, d.dtype, o, st.axis != 0)) c = o;
    }
    // the reverse radix order where the axis asks for it: its kernel takes one
    // thread per butterfly and the plain exchange, so the shape gives way
    // (fewer lines where the threads no longer fit)
    bool reverse = false;
    if (st.kind == K_C2C && p->order_override[st.axis] == 1 && p->twp_rev[st.axis] &&
        radix_order_distinct(kernel_length(st))) {
        KConf o = c;
        o.tdiv = 1;
        o.split = 0;
        while (o.lw > 1 && !conf_fits(st, d.dtype, o, st.axis != 0)) o.lw /= 2;
        if (conf_fits(st, d.dtype, o, st.axis != 0) && c2c_order_available(kernel_length(st), 1, 0)) {
            c = o;
            reverse = true;
        }
    }
    a.lw = c.lw;
    a.tdiv = c.tdiv;
    a.split = c.split;
    a.pad = c.pad;
    // strided C2C tiles writing rows that do not start on cache lines: shift
    // each row's tiles so the stores cover whole lines (partial-line stores
    // cost about as much again on MI355X)
    const int64_t per_line = 128 / (int64_t)elem_bytes(d.dtype);
    if (st.kind == K_C2C && a.strided && c.lw % per_line == 0 && a.sb_o % per_line != 0 && a.se_o % per_line == 0)
        a.align = (int)per_line;
    // complex128 strided tiles in XCD-grouped order: 2.5-5 % faster per y/z
    // stage at 512^3 on MI355X (C2C and R2C); complex64 stages ran 3-5 % slower
    // with it (C2C, and the R2C z stages at 512^3), so they keep the plain
    // order, except in R2C plans of half spectra from 512 MiB: the y stages
    // (512^3: 2-6 % faster) and, from 2 GiB, the z stages (1024^3: 3-5 %
    // faster); and tiles narrower than a cache line, whose neighbours share
    // every line they read and write (8-line complex64 tiles of the lengths
    // with 45 or 56 threads per line: 720^3 y/z stages 1.66 -> 1.51 ms)
    const size_t half = d.r2c ? (size_t)d.nxc() * d.ny * d.nz * elem_bytes(d.dtype) : 0;
    const bool r2c_xcd = half >= kR2CSwapMaxBytes || (half >= kSwapStagingMinBytes && st.axis == 1);
    const bool narrow = a.lw * (int64_t)elem_bytes(d.dtype) < 128;
    if (a.strided && (d.dtype == DT_F64 || r2c_xcd || narrow)) a.xcd = 1;
    a.nt = c2c_cache_policy(d, st, a, per_line);
    // the FP64 C2R x kernel streams its real output rows (whole cache lines)
    // with non-temporal stores past the Infinity Cache: 512^3 C2R x 0.415-0.420
    // -> 0.403-0.414 ms and the next forward's R2C x 1-2 % faster; FP32 was
    // unchanged and keeps plain stores
    if (st.kind == K_C2R_X && d.dtype == DT_F64 &&
        (size_t)d.nxc() * d.ny * d.nz * elem_bytes(d.dtype) >= kSwapStagingMinBytes)
        a.nt = 1;
    if (reverse) {
        a.order = 1;
        a.twp = p->twp_rev[st.axis];
        a.nt = 0;  // the reverse-order kernel has plain accesses only
    }
    return a;
}

hipError_t launch_task(const fft3d_plan_s* p, const Stage& st, const StageArgs& a, hipStream_t s)
{
    switch (st.kind) {
    case K_C2C: return launch_c2c(st.n, p->d.dtype, a, s);
    case K_R2C_X: return launch_r2c_x(st.n, p->d.dtype, a, s);
    case K_C2R_X: return launch_c2r_x(st.n, p->d.dtype, a, s);
    case K_POISSON_Z: return launch_poisson_z(st.n, p->d.dtype, a, s);
    case K_R2R_Z: return launch_r2r_z(st.n, p->d.dtype, a, s);
    case K_C2C_XY: return launch_c2c_xy((int)p->d.nx, (int)p->d.ny, p->d.dtype, a, s);
    default: return hipErrorInvalidValue;
    }
}

fft3d_status validate_desc(const PlanDesc& d)
{
    if (d.dtype != DT_F32 && d.dtype != DT_F64) return fail(FFT3D_ERR_INVALID_ARG, "dtype must be 0 (c64) or 1 (c128)");
    if (d.nx < 1 || d.ny < 1 || d.nz < 1) return fail(FFT3D_ERR_INVALID_ARG, "dimensions must be >= 1");
    if (d.r2c != 0 && d.r2c != 1) return fail(FFT3D_ERR_INVALID_ARG, "r2c must be 0 or 1");
    if (d.zbc != Z_PERIODIC && d.zbc != Z_NEUMANN && d.zbc != Z_DIRICHLET)
        return fail(FFT3D_ERR_INVALID_ARG, "z boundary must be 1 (Neumann) or 2 (Dirichlet)");
    if (d.zbc != Z_PERIODIC && !d.r2c) return fail(FFT3D_ERR_INVALID_ARG, "a bounded z axis needs an R2C plan");
    if (!length_supported(d.ny) || !length_supported(d.nz))
        return fail(FFT3D_ERR_UNSUPPORTED_SIZE, "ny or nz has no compiled kernel");
    if (d.r2c) {
        if (d.nx % 2 != 0 || !length_supported(d.nx / 2) || !length_supported(d.nx))
            return fail(FFT3D_ERR_UNSUPPORTED_SIZE, "r2c needs an even nx with nx and nx/2 supported");
    } else if (!length_supported(d.nx)) {
        return fail(FFT3D_ERR_UNSUPPORTED_SIZE, "nx has no compiled kernel");
    }
    if (d.p1 < 1 || d.p2 < 1 || d.p1 > std::min(d.ny, d.nxc()) || d.p2 > std::min(d.nz, d.ny))
        return fail(FFT3D_ERR_INVALID_ARG, "pencil grid must satisfy 1<=p1<=min(ny,nxc), 1<=p2<=min(nz,ny)");
    if ((int64_t)d.p1 * d.p2 > kMaxTiles) return fail(FFT3D_ERR_INVALID_ARG, "at most 1024 tiles per stage (p1*p2)");
    return FFT3D_OK;
}

bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb)
{
    const char* pa = (const char*)a;
    const char* pb = (const char*)b;
    return pa < pb + nb && pb < pa + na;
}

const Pipeline& get_pipeline(fft3d_plan_s* p, int op)
{
    if (!p->pipe_ok[op] || p->pipes[op].nstreams != p->nstreams) {
        p->pipes[op] = build_pipeline(p->d, op, p->nstreams);
        const Pipeline& pl = p->pipes[op];
        std::vector<char> need(pl.tasks.size(), 0);
        std::vector<int> last(p->nstreams, -1);
        for (size_t i = 0; i < pl.tasks.size(); ++i) {
            for (int w : pl.tasks[i].waits) need[w] = 1;
            last[pl.tasks[i].stream] = (int)i;
        }
        for (int s = 0; s < p->nstreams; ++s)
            if (last[s] >= 0) need[last[s]] = 1;
        p->needs_event[op] = need;
        p->pipe_ok[op] = true;
    }
    return p->pipes[op];
}

// Whether calls fork onto the plan's streams: only with more than one stream
// and more than one tile per stage (a 1x1 grid issues straight onto the
// caller's stream, in task order).
bool forks(const fft3d_plan_s* p) { return p->nstreams > 1 && (int64_t)p->d.p1 * p->d.p2 > 1; }

// Create the first `count` streams if they do not exist yet.
hipError_t ensure_streams(fft3d_plan_s* p, int count)
{
    for (int s = 0; s < count; ++s) {
        if (p->streams[s]) continue;
        hipError_t e = hipStreamCreateWithFlags(&p->streams[s], hipStreamNonBlocking);
        if (e != hipSuccess) {
            p->streams[s] = nullptr;
            return e;
        }
    }
    return hipSuccess;
}

fft3d_status build_groups(fft3d_plan_s* p, int op, const Pipeline& pl);
fft3d_status issue_stage(fft3d_plan_s* p, int op, const Pipeline& pl, int stage, void* const bufs[3],
                         hipStream_t s, bool group);
bool stage_groups(const fft3d_plan_s* p);

// Timed issue: every stage is its own region on the caller's stream (its
// grouped launch, or its tiles forked onto the plan's streams and joined),
// with a timing event after it, so stage durations can be read back.
fft3d_status run_timed(fft3d_plan_s* p, int op, const Pipeline& pl, void* const bufs[3], hipStream_t user)
{
    const bool grouped = stage_groups(p);
    if (grouped && !p->groups[op].valid) {
        const fft3d_status r = build_groups(p, op, pl);
        if (r != FFT3D_OK) return r;
    }
    hipError_t e = hipEventRecord(p->tev[0], user);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord(timing)");
    for (int st = 0; st < (int)pl.stages.size(); ++st) {
        if (grouped) {
            const fft3d_status r = issue_stage(p, op, pl, st, bufs, user, true);
            if (r != FFT3D_OK) return r;
            e = hipEventRecord(p->tev[st + 1], user);
            if (e != hipSuccess) return hip_fail(e, "hipEventRecord(timing)");
            continue;
        }
        const bool fork = forks(p);
        if (fork) {
            e = hipEventRecord(p->fork, user);
            if (e != hipSuccess) return hip_fail(e, "hipEventRecord(fork)");
        }
        std::vector<char> used(p->nstreams, 0);
        std::vector<int> last(p->nstreams, -1);
        for (size_t i = 0; i < pl.tasks.size(); ++i) {
            const Task& t = pl.tasks[i];
            if (t.stage != st) continue;
            hipStream_t s = fork ? p->streams[t.stream] : user;
            if (fork && !used[t.stream]) {
                e = hipStreamWaitEvent(s, p->fork, 0);
                if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent(fork)");
                used[t.stream] = 1;
            }
            const Stage& sg = pl.stages[t.stage];
            e = launch_task(p, sg, make_args(p, sg, t.box, bufs), s);
            if (e != hipSuccess) return hip_fail(e, "kernel launch");
            last[t.stream] = (int)i;
        }
        if (fork) {
            for (int s = 0; s < p->nstreams; ++s) {
                if (last[s] < 0) continue;
                e = hipEventRecord(p->events[last[s]], p->streams[s]);
                if (e == hipSuccess) e = hipStreamWaitEvent(user, p->events[last[s]], 0);
                if (e != hipSuccess) return hip_fail(e, "stage join");
            }
        }
        e = hipEventRecord(p->tev[st + 1], user);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord(timing)");
    }
    p->timed_stages = (int)pl.stages.size();
    return FFT3D_OK;
}

// Wait until the last call has finished (its work may still use the
// workspace); the caller's stream may be gone by now, the plan's own event
// is not.
void wait_last_call(fft3d_plan_s* p)
{
    if (p->called) hipEventSynchronize(p->call_done);
}

fft3d_status issue_forked(fft3d_plan_s* p, int op, const Pipeline& pl, void* const bufs[3], hipStream_t user);

// Record the launch of every tile of stage `stage` (in task order) instead
// of issuing it; tiles with nothing to launch are left out.
hipError_t record_tiles(fft3d_plan_s* p, const Pipeline& pl, int stage, void* const bufs[3],
                        std::vector<KernelLaunch>* launches, std::vector<Box>* boxes = nullptr)
{
    launches->clear();
    if (boxes) boxes->clear();
    for (const Task& t : pl.tasks) {
        if (t.stage != stage) continue;
        const Stage& st = pl.stages[t.stage];
        KernelLaunch kl;
        bool recorded = false;
        set_launch_recorder(&kl, &recorded);
        const hipError_t e = launch_task(p, st, make_args(p, st, t.box, bufs), nullptr);
        set_launch_recorder(nullptr, nullptr);
        if (e != hipSuccess) return e;
        if (recorded) {
            launches->push_back(kl);
            if (boxes) boxes->push_back(t.box);
        }
    }
    return hipSuccess;
}

// Puts the tiles of a stage that share their rows (the same range of the
// second index of their line grids) next to each other, in x order within a
// row of tiles, and returns the tiles per row of tiles; 0 (order kept) when
// the rows of tiles do not all hold the same number.
int64_t order_tile_rows(std::vector<KernelLaunch>& v, std::vector<Box>& b, int axis)
{
    if (v.size() != b.size() || v.empty()) return 0;
    const int s1 = axis == 0 ? 1 : 0, s2 = axis == 2 ? 1 : 2;
    std::vector<size_t> idx(v.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](size_t x, size_t y) {
        return b[x].lo[s2] != b[y].lo[s2] ? b[x].lo[s2] < b[y].lo[s2] : b[x].lo[s1] < b[y].lo[s1];
    });
    std::vector<KernelLaunch> v2;
    std::vector<Box> b2;
    for (size_t i : idx) {
        v2.push_back(v[i]);
        b2.push_back(b[i]);
    }
    int64_t g = 0;
    while (g < (int64_t)b2.size() && b2[g].lo[s2] == b2[0].lo[s2]) ++g;
    if ((int64_t)b2.size() % g != 0) return 0;
    for (size_t k = 0; k < b2.size(); ++k)
        if (b2[k].lo[s2] != b2[k - k % g].lo[s2] || (k % g == 0 && k > 0 && b2[k].lo[s2] == b2[k - g].lo[s2]))
            return 0;
    v.swap(v2);
    b.swap(b2);
    return g;
}

// A grouped strided stage whose output rows do not start on cache lines (the
// tiles shift their lines so that every stored segment is a whole line) runs
// each row of tiles as one tile spanning the row: between two tiles of a row
// the shifted tiles would store partial lines from both sides of the border.
// Merges the recorded tiles of stage `stage` that way; false (unchanged)
// where the stage has no such tiles or its rows of tiles are not contiguous.
bool merge_row_tiles(fft3d_plan_s* p, const Pipeline& pl, int stage, std::vector<KernelLaunch>& v,
                     std::vector<Box>& b)
{
    if (v.size() < 2 || v.size() != b.size()) return false;
    for (const KernelLaunch& k : v)
        if (!k.args.strided || k.args.align <= 1) return false;
    const Stage& st = pl.stages[stage];
    const int s1 = st.axis == 0 ? 1 : 0, s2 = st.axis == 2 ? 1 : 2;
    if (s1 != 0) return false;
    std::vector<Box> rows;
    for (const Box& x : b) {
        bool found = false;
        for (Box& r : rows)
            if (r.lo[s2] == x.lo[s2] && r.hi[s2] == x.hi[s2] && r.lo[st.axis] == x.lo[st.axis] &&
                r.hi[st.axis] == x.hi[st.axis]) {
                r.lo[s1] = std::min(r.lo[s1], x.lo[s1]);
                r.hi[s1] = std::max(r.hi[s1], x.hi[s1]);
                found = true;
            }
        if (!found) rows.push_back(x);
    }
    // every row of tiles must cover one contiguous x range (its tiles' total)
    for (const Box& r : rows) {
        int64_t covered = 0;
        for (const Box& x : b)
            if (x.lo[s2] == r.lo[s2] && x.hi[s2] == r.hi[s2]) covered += x.hi[s1] - x.lo[s1];
        if (covered != r.hi[s1] - r.lo[s1]) return false;
    }
    if (rows.size() == b.size()) return false;
    void* const none[3] = {nullptr, nullptr, nullptr};
    std::vector<KernelLaunch> v2;
    for (const Box& r : rows) {
        KernelLaunch kl;
        bool recorded = false;
        set_launch_recorder(&kl, &recorded);
        const hipError_t e = launch_task(p, st, make_args(p, st, r, none), nullptr);
        set_launch_recorder(nullptr, nullptr);
        if (e != hipSuccess || !recorded) return false;
        v2.push_back(kl);
    }
    v.swap(v2);
    b.swap(rows);
    return true;
}

// Free the grouped launches' tables after the last call has finished.
void drop_groups(fft3d_plan_s* p)
{
    wait_last_call(p);
    for (auto& g : p->groups) {
        if (g.dev) hipFree(g.dev);
        g = fft3d_plan_s::OpGroups();
    }
}

// Decide, per stage of operation op, whether its tiles go out as one
// grouped launch, and upload the tile tables of the grouped stages.
fft3d_status build_groups(fft3d_plan_s* p, int op, const Pipeline& pl)
{
    fft3d_plan_s::OpGroups& G = p->groups[op];
    G = fft3d_plan_s::OpGroups();
    void* const none[3] = {nullptr, nullptr, nullptr};
    std::vector<std::vector<KernelLaunch>> rec(pl.stages.size());
    std::vector<std::vector<Box>> boxes(pl.stages.size());
    size_t total = 0;
    for (size_t st = 0; st < pl.stages.size(); ++st) {
        hipError_t e = record_tiles(p, pl, (int)st, none, &rec[st], &boxes[st]);
        if (e != hipSuccess) return hip_fail(e, "recording tile launches");
        if (can_group(rec[st].data(), rec[st].size())) merge_row_tiles(p, pl, (int)st, rec[st], boxes[st]);
        if (can_group(rec[st].data(), rec[st].size())) total += rec[st].size();
    }
    std::vector<TileEntry> host(total);
    G.stages.resize(pl.stages.size());
    size_t pos = 0;
    for (size_t st = 0; st < pl.stages.size(); ++st) {
        std::vector<KernelLaunch>& v = rec[st];
        if (!can_group(v.data(), v.size())) continue;
        G.stages[st].grouped = true;
        // C2C plans, and the contiguous x stages of R2C plans: the tiles of each
        // row of tiles (the tiles sharing their rows) interleaved workgroup by
        // workgroup, so the workgroups in flight cover every tile's slice of the
        // same rows, as on one tile (MI355X, fwd+inv: 256^3 complex128 on 4x4
        // tiles 0.586 -> 0.552 ms, 512^3 complex64 on 4x4 2.67 -> 2.44 ms,
        // 256^3 complex64 unchanged, every tile of the stage interleaved gave
        // 0.559 and 2.54 ms; 512^3 R2C on 4x4 1.41 -> 1.37 ms, 1024^3 on 8x8
        // 12.6 -> 12.45 ms).  The strided stages of R2C plans keep the tiles
        // one after another: 1024^3 on 8x8 tiles ran 6 % slower with either
        // interleave.
        int64_t ntiles = 0;
        if (!p->d.r2c || !v[0].args.strided) {
            const int64_t g = order_tile_rows(v, boxes[st], pl.stages[st].axis);
            ntiles = g > 0 ? g : (int64_t)v.size();
        }
        make_group(v.data(), v.size(), false, ntiles, host.data() + pos, &G.stages[st].launch);
        G.stages[st].launch.args.tiles = reinterpret_cast<const TileEntry*>(pos);  // offset until uploaded
        pos += v.size();
    }
    if (total > 0) {
        hipError_t e = hipMalloc(&G.dev, total * sizeof(TileEntry));
        if (e == hipSuccess) e = hipMemcpy(G.dev, host.data(), total * sizeof(TileEntry), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            if (G.dev) hipFree(G.dev);
            G = fft3d_plan_s::OpGroups();
            return hip_fail(e, "tile table upload");
        }
        for (auto& sg : G.stages)
            if (sg.grouped) sg.launch.args.tiles = G.dev + reinterpret_cast<size_t>(sg.launch.args.tiles);
    }
    G.valid = true;
    return FFT3D_OK;
}

// Issue stage `stage` of a call on `s`: its grouped launch, or its tiles in
// task order.
fft3d_status issue_stage(fft3d_plan_s* p, int op, const Pipeline& pl, int stage, void* const bufs[3],
                         hipStream_t s, bool group)
{
    const fft3d_plan_s::OpGroups& G = p->groups[op];
    if (group && G.valid && G.stages[stage].grouped) {
        const KernelLaunch& kl = G.stages[stage].launch;
        StageArgs a = kl.args;
        a.in = bufs[pl.stages[stage].src];
        a.out = bufs[pl.stages[stage].dst];
        const hipError_t e = launch_stage_kernel(kl.func, kl.grid, kl.block, a, kl.lds, s);
        return e == hipSuccess ? FFT3D_OK : hip_fail(e, "grouped kernel launch");
    }
    for (const Task& t : pl.tasks) {
        if (t.stage != stage) continue;
        const Stage& st = pl.stages[t.stage];
        const hipError_t e = launch_task(p, st, make_args(p, st, t.box, bufs), s);
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
    }
    return FFT3D_OK;
}

}  // namespace

fft3d_status fft3d::record_stage(fft3d_plan_s* p, int op, int stage, const void* in, void* out,
                                 std::vector<KernelLaunch>* launches)
{
    if (!p || op < 0 || op >= OP_COUNT) return fail(FFT3D_ERR_INVALID_ARG, "invalid plan or operation");
    const Pipeline& pl = get_pipeline(p, op);
    if (stage < 0 || stage >= (int)pl.stages.size()) return fail(FFT3D_ERR_INVALID_ARG, "invalid stage");
    void* bufs[3] = {const_cast<void*>(in), out, p->ws};
    const hipError_t e = record_tiles(p, pl, stage, bufs, launches);
    return e == hipSuccess ? FFT3D_OK : hip_fail(e, "recording tile launches");
}

int fft3d::stage_count(fft3d_plan_s* p, int op)
{
    if (!p || op < 0 || op >= OP_COUNT) return 0;
    return (int)get_pipeline(p, op).stages.size();
}

namespace {

// Whether tiled calls of this plan go out as one grouped launch per stage.
bool stage_groups(const fft3d_plan_s* p)
{
    return p->issue == FFT3D_ISSUE_STAGES && (int64_t)p->d.p1 * p->d.p2 > 1;
}

fft3d_status issue(fft3d_plan_s* p, int op, const Pipeline& pl, void* const bufs[3], hipStream_t user,
                   bool capturing)
{
    if (p->timing && !capturing) return run_timed(p, op, pl, bufs, user);
    // One grouped launch per stage, in order on the caller's stream (not into
    // a capture: a captured launch would keep the plan's tile table in use)
    if (stage_groups(p) && !capturing) {
        if (!p->groups[op].valid) {
            const fft3d_status st = build_groups(p, op, pl);
            if (st != FFT3D_OK) return st;
        }
        for (int st = 0; st < (int)pl.stages.size(); ++st) {
            const fft3d_status r = issue_stage(p, op, pl, st, bufs, user, true);
            if (r != FFT3D_OK) return r;
        }
        return FFT3D_OK;
    }
    // In order on the caller's stream: plans with one stream or one tile per
    // stage, and every call into a stream the caller is capturing (forking
    // onto the plan's streams there would put cross-stream event edges into
    // the caller's graph; the tile order is a topological order of the task
    // graph, so the captured sequence is correct as it stands).
    if (!forks(p) || capturing) {
        for (const Task& t : pl.tasks) {
            const Stage& st = pl.stages[t.stage];
            hipError_t e = launch_task(p, st, make_args(p, st, t.box, bufs), user);
            if (e != hipSuccess) return hip_fail(e, "kernel launch");
        }
        return FFT3D_OK;
    }
    return issue_forked(p, op, pl, bufs, user);
}

fft3d_status run(fft3d_plan_s* p, int op, const void* in, void* out, void* stream)
{
    std::lock_guard<std::mutex> lock(p->mu);
    const Pipeline& pl = get_pipeline(p, op);
    if (pl.stages.empty()) return fail(FFT3D_ERR_WRONG_PLAN, "operation not available for this plan kind");
    hipStream_t user = (hipStream_t)stream;
    void* bufs[3] = {const_cast<void*>(in), out, p->ws};
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (user) {  // the legacy default stream cannot be captured
        e = hipStreamIsCapturing(user, &cap);
        if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
    }
    const bool capturing = cap != hipStreamCaptureStatusNone;
    // the previous call on another stream may still use the workspace
    if (!capturing && p->called && p->last_stream != user) {
        e = hipStreamWaitEvent(user, p->call_done, 0);
        if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent(previous call)");
    }
    if (capturing) p->timed_stages = 0;  // no timing events inside a capture
    fft3d_status st = issue(p, op, pl, bufs, user, capturing);
    if (st != FFT3D_OK || capturing) return st;
    e = hipEventRecord(p->call_done, user);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord(call)");
    p->last_stream = user;
    p->called = true;
    return FFT3D_OK;
}

// Fork onto the plan's streams, one event edge per cross-stream dependency,
// join back onto the caller's stream.
fft3d_status issue_forked(fft3d_plan_s* p, int op, const Pipeline& pl, void* const bufs[3], hipStream_t user)
{
    const std::vector<char>& need = p->needs_event[op];
    hipError_t e = hipEventRecord(p->fork, user);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord(fork)");
    std::vector<char> started(p->nstreams, 0);
    std::vector<int> last(p->nstreams, -1);
    for (size_t i = 0; i < pl.tasks.size(); ++i) {
        const Task& t = pl.tasks[i];
        hipStream_t s = p->streams[t.stream];
        if (!started[t.stream]) {
            e = hipStreamWaitEvent(s, p->fork, 0);
            if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent(fork)");
            started[t.stream] = 1;
        }
        for (int w : t.waits) {
            e = hipStreamWaitEvent(s, p->events[w], 0);
            if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
        }
        const Stage& st = pl.stages[t.stage];
        e = launch_task(p, st, make_args(p, st, t.box, bufs), s);
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
        if (need[i]) {
            e = hipEventRecord(p->events[i], s);
            if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        }
        last[t.stream] = (int)i;
    }
    for (int s = 0; s < p->nstreams; ++s) {
        if (last[s] < 0) continue;
        e = hipStreamWaitEvent(user, p->events[last[s]], 0);
        if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent(join)");
    }
    return FFT3D_OK;
}

void release(fft3d_plan_s* p)
{
    drop_groups(p);  // waits for the last call (work still reading or writing plan memory)
    for (hipStream_t s : p->streams)
        if (s) {
            hipStreamSynchronize(s);
            hipStreamDestroy(s);
        }
    for (hipEvent_t ev : p->events)
        if (ev) hipEventDestroy(ev);
    for (hipEvent_t ev : p->tev)
        if (ev) hipEventDestroy(ev);
    if (p->fork) hipEventDestroy(p->fork);
    if (p->call_done) hipEventDestroy(p->call_done);
    for (void* t : p->tw)
        if (t) hipFree(t);
    for (void* t : p->twp)
        if (t) hipFree(t);
    for (void* t : p->twp_rev)
        if (t) hipFree(t);
    if (p->ws && p->ws_owned) hipFree(p->ws);
    delete p;
}

fft3d_status check_plan_and_ptrs(fft3d_plan_t p, const void* in, const void* out)
{
    if (!p) return fail(FFT3D_ERR_INVALID_ARG, "null plan");
    if (!in || !out) return fail(FFT3D_ERR_INVALID_ARG, "null buffer");
    return FFT3D_OK;
}

}  // namespace

extern "C" {

static fft3d_status make_plan(fft3d_plan_t* plan, const PlanDesc& d)
{
    if (!plan) return fail(FFT3D_ERR_INVALID_ARG, "null plan pointer");
    *plan = nullptr;
    fft3d_status st = validate_desc(d);
    if (st != FFT3D_OK) return st;
    const int64_t nx = d.nx, ny = d.ny, nz = d.nz;
    const int dtype = d.dtype, p1 = d.p1, p2 = d.p2, r2c = d.r2c;

    fft3d_plan_s* p = new fft3d_plan_s();
    p->d = d;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "hipGetDevice");
    }
    // twiddle tables in the plan precision (FP64-generated, rounded for c64)
    const int64_t lens[3] = {nx, ny, nz};
    for (int ax = 0; ax < 3; ++ax) {
        const int64_t n = lens[ax];
        const size_t bytes = (size_t)n * elem_bytes(dtype);
        std::vector<char> host(bytes);
        if (ax == 2 && d.zbc != Z_PERIODIC) {
            // bounded z: the first n roots W_4n^k of the order-4n table
            std::vector<char> t4(4 * bytes);
            if (dtype == DT_F64) twiddles_f64(4 * n, (double*)t4.data());
            else twiddles_f32(4 * n, (float*)t4.data());
            memcpy(host.data(), t4.data(), bytes);
        } else if (dtype == DT_F64) {
            twiddles_f64(n, (double*)host.data());
        } else {
            twiddles_f32(n, (float*)host.data());
        }
        e = hipMalloc(&p->tw[ax], bytes);
        if (e == hipSuccess) e = hipMemcpy(p->tw[ax], host.data(), bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            release(p);
            return hip_fail(e, "twiddle upload");
        }
        // per-pass table of the FFT length the axis kernels run (half of nx for r2c x)
        const int64_t nk = (r2c && ax == 0) ? n / 2 : n;
        const int64_t entries = std::max<int64_t>(1, pass_twiddles_f64(nk, nullptr));
        const size_t pbytes = (size_t)entries * elem_bytes(dtype);
        std::vector<char> phost(pbytes, 0);
        if (dtype == DT_F64) pass_twiddles_f64(nk, (double*)phost.data());
        else pass_twiddles_f32(nk, (float*)phost.data());
        e = hipMalloc(&p->twp[ax], pbytes);
        if (e == hipSuccess) e = hipMemcpy(p->twp[ax], phost.data(), pbytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            release(p);
            return hip_fail(e, "twiddle upload");
        }
        // the reverse radix order's table, for axes whose line kernels are C2C
        if (!(r2c && ax == 0) && radix_order_distinct((int)nk)) {
            const int64_t rentries = pass_twiddles_f64(nk, nullptr, 1);
            const size_t rbytes = (size_t)rentries * elem_bytes(dtype);
            std::vector<char> rhost(rbytes, 0);
            if (dtype == DT_F64) pass_twiddles_f64(nk, (double*)rhost.data(), 1);
            else pass_twiddles_f32(nk, (float*)rhost.data(), 1);
            e = hipMalloc(&p->twp_rev[ax], rbytes);
            if (e == hipSuccess) e = hipMemcpy(p->twp_rev[ax], rhost.data(), rbytes, hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                release(p);
                return hip_fail(e, "twiddle upload");
            }
        }
    }
    if (r2c) {
        p->ws_bytes = (size_t)d.wpitch() * ny * nz * elem_bytes(dtype);
        e = hipMalloc(&p->ws, p->ws_bytes);
        if (e != hipSuccess) {
            p->ws = nullptr;
            release(p);
            return hip_fail(e, "workspace allocation");
        }
        p->ws_owned = true;
        // the forward then runs x into the output, y into the swapped
        // workspace and z back (512^3: 0.79 -> 0.73 ms f32, 1.47 -> 1.41 ms
        // f64); at 1024^3 f32 (4.3 GB) in place is the faster one (forward
        // 6.54 ms against 6.97), so only half spectra below 2 GiB swap
        const size_t half = (size_t)d.nxc() * ny * nz * elem_bytes(dtype);
        if (d.zbc == Z_PERIODIC && ny > 1 && nz > 1 && half >= kSwapStagingMinBytes && half < kR2CSwapMaxBytes)
            p->d.staging = STAGING_SWAP_YZ;
    }
    // large C2C plans stage through a y/z-swapped workspace by default (see
    // fft3d_set_staging); if it cannot be allocated they stage in place
    if (!r2c && ny > 1 && nz > 1 && (size_t)nx * ny * nz * elem_bytes(dtype) >= kSwapStagingMinBytes) {
        const size_t need = (size_t)d.wpitch() * ny * nz * elem_bytes(dtype);
        if (hipMalloc(&p->ws, need) == hipSuccess) {
            p->d.staging = STAGING_SWAP_YZ;
            p->ws_owned = true;
            p->ws_bytes = need;
        } else {
            p->ws = nullptr;
            (void)hipGetLastError();
        }
    }
    // small planes: the fused x-y kernel (two passes instead of three)
    if (!r2c && p->d.staging == STAGING_IN_PLACE && p1 == 1 && ny > 1 &&
        plane_available(nx, ny, elem_bytes(dtype)))
        p->d.staging = STAGING_FUSED_XY;
    p->streams.assign(kMaxStreams, nullptr);
    if (forks(p)) {
        e = ensure_streams(p, p->nstreams);
        if (e != hipSuccess) {
            release(p);
            return hip_fail(e, "hipStreamCreate");
        }
    }
    const size_t max_tasks = 5 * (size_t)p1 * p2;
    p->events.assign(max_tasks, nullptr);
    for (size_t i = 0; i < max_tasks; ++i) {
        e = hipEventCreateWithFlags(&p->events[i], hipEventDisableTiming);
        if (e != hipSuccess) {
            p->events[i] = nullptr;
            release(p);
            return hip_fail(e, "hipEventCreate");
        }
    }
    e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->call_done, hipEventDisableTiming);
    if (e != hipSuccess) {
        release(p);
        return hip_fail(e, "hipEventCreate");
    }
    *plan = p;
    return FFT3D_OK;
}

fft3d_status fft3d_plan(fft3d_plan_t* plan, int64_t nx, int64_t ny, int64_t nz, int dtype, int p1,
                        int p2, int r2c)
{
    PlanDesc d;
    d.nx = nx; d.ny = ny; d.nz = nz; d.dtype = dtype; d.p1 = p1; d.p2 = p2; d.r2c = r2c;
    return make_plan(plan, d);
}

fft3d_status fft3d_plan_ppb(fft3d_plan_t* plan, int64_t nx, int64_t ny, int64_t nz, int dtype, int p1, int p2,
                            int zbc)
{
    PlanDesc d;
    d.nx = nx; d.ny = ny; d.nz = nz; d.dtype = dtype; d.p1 = p1; d.p2 = p2; d.r2c = 1;
    d.zbc = zbc == Z_PERIODIC ? -1 : zbc;  // 0 is not a bounded axis
    return make_plan(plan, d);
}

fft3d_status fft3d_destroy(fft3d_plan_t plan)
{
    if (plan) release(plan);
    return FFT3D_OK;
}

static fft3d_status c2c_or_r2c(fft3d_plan_t p, int op, const void* in, void* out, void* stream)
{
    fft3d_status st = check_plan_and_ptrs(p, in, out);
    if (st != FFT3D_OK) return st;
    const PlanDesc& d = p->d;
    const size_t s = elem_bytes(d.dtype);
    const size_t n = (size_t)d.nx * d.ny * d.nz;
    if (!d.r2c) {
        if (in != out && ranges_overlap(in, n * s, out, n * s))
            return fail(FFT3D_ERR_ALIAS, "in and out partially overlap");
        if (d.staging == STAGING_SWAP_YZ &&
            (ranges_overlap(p->ws, p->ws_bytes, in, n * s) || ranges_overlap(p->ws, p->ws_bytes, out, n * s)))
            return fail(FFT3D_ERR_ALIAS, "workspace overlaps a buffer");
    } else {
        const size_t real_bytes = n * s / 2, half_bytes = (size_t)d.nxc() * d.ny * d.nz * s;
        const size_t in_bytes = op == OP_FORWARD ? real_bytes : half_bytes;
        const size_t out_bytes = op == OP_FORWARD ? half_bytes : real_bytes;
        if (ranges_overlap(in, in_bytes, out, out_bytes))
            return fail(FFT3D_ERR_ALIAS, "real-to-complex transforms cannot run in place");
        if (ranges_overlap(p->ws, p->ws_bytes, in, in_bytes) || ranges_overlap(p->ws, p->ws_bytes, out, out_bytes))
            return fail(FFT3D_ERR_ALIAS, "workspace overlaps a buffer");
    }
    return run(p, op, in, out, stream);
}

fft3d_status fft3d_forward(fft3d_plan_t p, const void* in, void* out, void* stream)
{
    return c2c_or_r2c(p, OP_FORWARD, in, out, stream);
}

fft3d_status fft3d_inverse(fft3d_plan_t p, const void* in, void* out, void* stream)
{
    return c2c_or_r2c(p, OP_INVERSE, in, out, stream);
}

fft3d_status fft3d_backward(fft3d_plan_t p, const void* in, void* out, void* stream)
{
    return c2c_or_r2c(p, OP_BACKWARD, in, out, stream);
}

static_assert(kScratchBytes == FFT3D_SCRATCH_BYTES, "scratch size in the header and the library differ");

fft3d_status fft3d_forward_noalloc(fft3d_plan_t p, const void* in, void* out, void* stream)
{
    fft3d_status st = check_plan_and_ptrs(p, in, out);
    if (st != FFT3D_OK) return st;
    std::lock_guard<std::mutex> lock(p->mu);
    const PlanDesc& d = p->d;
    const size_t s = elem_bytes(d.dtype);
    const size_t n = (size_t)d.nx * d.ny * d.nz;
    const size_t in_bytes = d.r2c ? n * s / 2 : n * s;
    const size_t out_bytes = d.r2c ? (size_t)d.nxc() * d.ny * d.nz * s : n * s;
    if (d.r2c ? ranges_overlap(in, in_bytes, out, out_bytes)
              : (in != out && ranges_overlap(in, in_bytes, out, out_bytes)))
        return fail(FFT3D_ERR_ALIAS, d.r2c ? "real-to-complex transforms cannot run in place"
                                           : "in and out partially overlap");
    // the workspace this plan's forward stages use, taken from the static scratch
    const size_t need = (d.r2c || d.staging == STAGING_SWAP_YZ) ? (size_t)d.wpitch() * d.ny * d.nz * s : 0;
    if (need > kScratchBytes)
        return fail(FFT3D_ERR_WORKSPACE, "workspace of this plan (" + std::to_string(need) +
                                             " bytes) exceeds the static scratch (" +
                                             std::to_string(kScratchBytes) + " bytes)");
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    void* scr = nullptr;
    if (need > 0) {
        e = scratch_address(p->device, &scr);
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (ranges_overlap(scr, need, in, in_bytes) || ranges_overlap(scr, need, out, out_bytes))
            return fail(FFT3D_ERR_ALIAS, "a buffer overlaps the library scratch");
    }
    const Pipeline& pl = get_pipeline(p, OP_FORWARD);
    void* bufs[3] = {const_cast<void*>(in), out, scr};
    // every tile in dependency order on the caller's stream: no internal
    // streams, events or graphs (creating those can allocate)
    hipStream_t user = (hipStream_t)stream;
    for (const Task& t : pl.tasks) {
        const Stage& sg = pl.stages[t.stage];
        e = launch_task(p, sg, make_args(p, sg, t.box, bufs), user);
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
    }
    return FFT3D_OK;
}

static fft3d_status poisson_op(fft3d_plan_t p, int op, const void* f, void* phi, void* stream)
{
    fft3d_status st = check_plan_and_ptrs(p, f, phi);
    if (st != FFT3D_OK) return st;
    if (!p->d.r2c) return fail(FFT3D_ERR_WRONG_PLAN, "the Poisson solve needs a real-to-complex plan");
    const size_t bytes = (size_t)p->d.nx * p->d.ny * p->d.nz * elem_bytes(p->d.dtype) / 2;
    if (f != phi && ranges_overlap(f, bytes, phi, bytes))
        return fail(FFT3D_ERR_ALIAS, "f and phi partially overlap");
    if (ranges_overlap(p->ws, p->ws_bytes, f, bytes) || ranges_overlap(p->ws, p->ws_bytes, phi, bytes))
        return fail(FFT3D_ERR_ALIAS, "workspace overlaps a buffer");
    return run(p, op, f, phi, stream);
}

fft3d_status fft3d_poisson(fft3d_plan_t p, const void* f, void* phi, void* stream)
{
    return poisson_op(p, OP_POISSON, f, phi, stream);
}

fft3d_status fft3d_poisson_backward(fft3d_plan_t p, const void* gphi, void* gf, void* stream)
{
    return poisson_op(p, OP_POISSON_ADJ, gphi, gf, stream);
}

int fft3d_get_staging(fft3d_plan_t p)
{
    if (!p) {
        fail(FFT3D_ERR_INVALID_ARG, "null plan");
        return -1;
    }
    std::lock_guard<std::mutex> lock(p->mu);
    return p->d.staging;
}

size_t fft3d_workspace_bytes(fft3d_plan_t p)
{
    if (!p) return 0;
    if (!p->d.r2c && p->d.staging != STAGING_SWAP_YZ) return 0;
    return (size_t)p->d.wpitch() * p->d.ny * p->d.nz * elem_bytes(p->d.dtype);
}

fft3d_status fft3d_set_workspace(fft3d_plan_t p, void* ws, size_t bytes)
{
    if (!p) return fail(FFT3D_ERR_INVALID_ARG, "null plan");
    std::lock_guard<std::mutex> lock(p->mu);
    if (!p->d.r2c && p->d.staging != STAGING_SWAP_YZ)
        return ws ? fail(FFT3D_ERR_WRONG_PLAN, "in-place C2C staging uses no workspace") : FFT3D_OK;
    const size_t need = fft3d_workspace_bytes(p);
    if (ws && bytes < need) return fail(FFT3D_ERR_WORKSPACE, "workspace smaller than fft3d_workspace_bytes");
    if (ws && ((uintptr_t)ws % 256) != 0) return fail(FFT3D_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    // the old workspace may still be in use by enqueued work
    wait_last_call(p);
    if (ws) {
        if (p->ws_owned) hipFree(p->ws);
        p->ws = ws;
        p->ws_owned = false;
        p->ws_bytes = bytes;
        return FFT3D_OK;
    }
    if (p->ws_owned) return FFT3D_OK;
    void* mine = nullptr;
    hipError_t e = hipMalloc(&mine, need);
    if (e != hipSuccess) return hip_fail(e, "workspace allocation");
    p->ws = mine;
    p->ws_owned = true;
    p->ws_bytes = need;
    return FFT3D_OK;
}

fft3d_status fft3d_set_staging(fft3d_plan_t p, int staging)
{
    if (!p) return fail(FFT3D_ERR_INVALID_ARG, "null plan");
    std::lock_guard<std::mutex> lock(p->mu);
    if (staging != STAGING_IN_PLACE && staging != STAGING_SWAP_YZ && staging != STAGING_FUSED_XY)
        return fail(FFT3D_ERR_INVALID_ARG, "staging must be 0 (in place), 1 (swap y/z) or 2 (fused x-y planes)");
    if (p->d.r2c) {
        // R2C plans always hold the workspace; the staging only changes the forward's stages
        if (staging == STAGING_FUSED_XY) return fail(FFT3D_ERR_WRONG_PLAN, "fused x-y planes are for C2C plans");
        if (p->d.zbc != Z_PERIODIC && staging != STAGING_IN_PLACE)
            return fail(FFT3D_ERR_WRONG_PLAN, "plans with a bounded z axis stage in place");
        if (staging == p->d.staging) return FFT3D_OK;
        drop_groups(p);
        p->d.staging = staging;
        for (int op = 0; op < OP_COUNT; ++op) p->pipe_ok[op] = false;
        return FFT3D_OK;
    }
    if (staging == STAGING_FUSED_XY && (p->d.p1 != 1 || !plane_available(p->d.nx, p->d.ny, elem_bytes(p->d.dtype))))
        return fail(FFT3D_ERR_UNSUPPORTED_SIZE, "no fused x-y kernel for this plane (or p1 > 1)");
    if (staging == p->d.staging) return FFT3D_OK;
    drop_groups(p);  // waits for the last call, which may still use the old workspace
    if (p->ws && p->ws_owned) hipFree(p->ws);
    p->ws = nullptr;
    p->ws_owned = false;
    p->ws_bytes = 0;
    p->d.staging = staging;
    for (int op = 0; op < OP_COUNT; ++op) p->pipe_ok[op] = false;
    if (staging == STAGING_SWAP_YZ) {
        const size_t need = fft3d_workspace_bytes(p);
        hipError_t e = hipMalloc(&p->ws, need);
        if (e != hipSuccess) {
            p->ws = nullptr;
            p->d.staging = STAGING_IN_PLACE;
            return hip_fail(e, "workspace allocation");
        }
        p->ws_owned = true;
        p->ws_bytes = need;
    }
    return FFT3D_OK;
}

fft3d_status fft3d_set_streams(fft3d_plan_t p, int nstreams)
{
    if (!p) return fail(FFT3D_ERR_INVALID_ARG, "null plan");
    std::lock_guard<std::mutex> lock(p->mu);
    if (nstreams < 1 || nstreams > kMaxStreams) return fail(FFT3D_ERR_INVALID_ARG, "nstreams must be 1..16");
    wait_last_call(p);
    p->nstreams = nstreams;
    if (forks(p)) {
        hipError_t e = ensure_streams(p, nstreams);
        if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    }
    return FFT3D_OK;
}

fft3d_status fft3d_set_issue(fft3d_plan_t p, int mode)
{
    if (!p) return fail(FFT3D_ERR_INVALID_ARG, "null plan");
    std::lock_guard<std::mutex> lock(p->mu);
    if (mode != FFT3D_ISSUE_TILES && mode != FFT3D_ISSUE_STAGES)
        return fail(FFT3D_ERR_INVALID_ARG, "issue mode must be 0 (tiles) or 1 (stages)");
    p->issue = mode;
    return FFT3D_OK;
}

int fft3d_get_issue(fft3d_plan_t p)
{
    if (!p) {
        fail(FFT3D_ERR_INVALID_ARG, "null plan");
        return -1;
    }
    std::lock_guard<std::mutex> lock(p->mu);
    return p->issue;
}

fft3d_status fft3d_set_radix_order(fft3d_plan_t p, int axis, int order)
{
    if (!p) return fail(FFT3D_ERR_INVALID_ARG, "null plan");
    std::lock_guard<std::mutex> lock(p->mu);
    if (axis < 0 || axis > 2) return fail(FFT3D_ERR_INVALID_ARG, "axis must be 0..2");
    if (order != 0 && order != 1) return fail(FFT3D_ERR_INVALID_ARG, "order must be 0 or 1");
    if (order == 1) {
        // some C2C line kernel of this axis must have a distinct reverse order
        bool any = false;
        for (int op = 0; op < OP_COUNT; ++op)
            for (const Stage& st : op_stages(p->d, op))
                any = any || (st.axis == axis && st.kind == K_C2C && radix_order_distinct(kernel_length(st)));
        if (!any || !p->twp_rev[axis])
            return fail(FFT3D_ERR_INVALID_ARG, "no line kernel of this axis has another radix order");
    }
    drop_groups(p);
    p->order_override[axis] = order;
    return FFT3D_OK;
}

int fft3d_get_radix_order(fft3d_plan_t p, int axis)
{
    if (!p || axis < 0 || axis > 2) {
        fail(FFT3D_ERR_INVALID_ARG, "null plan or axis out of range");
        return -1;
    }
    std::lock_guard<std::mutex> lock(p->mu);
    return p->order_override[axis];
}

fft3d_status fft3d_set_stage_config(fft3d_plan_t p, int axis, int lw, int tdiv, int split, int pad)
{
    if (!p) return fail(FFT3D_ERR_INVALID_ARG, "null plan");
    std::lock_guard<std::mutex> lock(p->mu);
    if (axis < 0 || axis > 2) return fail(FFT3D_ERR_INVALID_ARG, "axis must be 0..2");
    if (lw == 0) {
        drop_groups(p);
        p->conf_override[axis] = KConf();
        return FFT3D_OK;
    }
    KConf c;
    c.lw = lw;
    c.tdiv = tdiv;
    c.split = split;
    c.pad = pad;
    if (lw < 1 || lw > 1024 || (lw & (lw - 1)) != 0 || tdiv < 1 || split < 0 || split > 1 || pad < 0 || pad > 1)
        return fail(FFT3D_ERR_INVALID_ARG, "lw a power of two <= 1024, tdiv >= 1, split and pad 0 or 1");
    // some stage kernel of this axis must accept the shape (the others keep
    // their default shape)
    bool fits = false, any = false;
    for (int op = 0; op < OP_COUNT; ++op)
        for (const Stage& st : op_stages(p->d, op)) {
            if (st.axis != axis || st.kind == K_C2C_XY) continue;
            any = true;
            fits = fits || conf_fits(st, p->d.dtype, c, axis != 0);
        }
    if (any && !fits)
        return fail(FFT3D_ERR_INVALID_ARG, "shape does not fit a stage kernel of this axis "
                                           "(threads, LDS, or no such kernel variant)");
    drop_groups(p);
    p->conf_override[axis] = c;
    return FFT3D_OK;
}

fft3d_status fft3d_set_timing(fft3d_plan_t p, int enable)
{
    if (!p) return fail(FFT3D_ERR_INVALID_ARG, "null plan");
    std::lock_guard<std::mutex> lock(p->mu);
    if (enable && p->tev.empty()) {
        p->tev.assign(6, nullptr);
        for (auto& ev : p->tev) {
            hipError_t e = hipEventCreate(&ev);
            if (e != hipSuccess) {
                ev = nullptr;
                return hip_fail(e, "hipEventCreate(timing)");
            }
        }
    }
    p->timing = enable != 0;
    p->timed_stages = 0;
    return FFT3D_OK;
}

int fft3d_stage_times(fft3d_plan_t p, float* ms, int cap)
{
    if (!p || !ms) {
        fail(FFT3D_ERR_INVALID_ARG, "null plan or output");
        return -1;
    }
    std::lock_guard<std::mutex> lock(p->mu);
    if (p->timed_stages == 0) {
        fail(FFT3D_ERR_INVALID_ARG, "no timed call recorded");
        return -1;
    }
    if (cap < p->timed_stages) {
        fail(FFT3D_ERR_INVALID_ARG, "cap smaller than the number of stages");
        return -1;
    }
    hipError_t e = hipEventSynchronize(p->tev[p->timed_stages]);
    if (e != hipSuccess) {
        hip_fail(e, "hipEventSynchronize");
        return -1;
    }
    for (int i = 0; i < p->timed_stages; ++i) {
        e = hipEventElapsedTime(&ms[i], p->tev[i], p->tev[i + 1]);
        if (e != hipSuccess) {
            hip_fail(e, "hipEventElapsedTime");
            return -1;
        }
    }
    return p->timed_stages;
}

const char* fft3d_status_string(int status)
{
    switch (status) {
    case FFT3D_OK: return "ok";
    case FFT3D_ERR_INVALID_ARG: return "invalid argument";
    case FFT3D_ERR_UNSUPPORTED_SIZE: return "unsupported size";
    case FFT3D_ERR_ALLOC: return "device allocation failed";
    case FFT3D_ERR_HIP: return "HIP runtime error";
    case FFT3D_ERR_ALIAS: return "buffers overlap";
    case FFT3D_ERR_WORKSPACE: return "workspace too small";
    case FFT3D_ERR_WRONG_PLAN: return "operation not available for this plan kind";
    default: return "unknown status";
    }
}

const char* fft3d_last_error(void) { return g_last_error.c_str(); }

int fft3d_length_supported(int64_t n) { return length_supported(n) ? 1 : 0; }

int fft3d_query_radix_plan(int64_t n, int* out, int cap)
{
    if (!length_supported(n) || !out) return -1;
    const RadixPlan rp = radix_plan((int)n);
    if (cap < rp.np + 2) return -1;
    out[0] = rp.np;
    for (int i = 0; i < rp.np; ++i) out[1 + i] = rp.r[i];
    out[rp.np + 1] = rp.tpl;
    return rp.np + 2;
}

fft3d_status fft3d_query_twiddles(int64_t n, int dtype, void* out)
{
    if (n < 1 || !out) return fail(FFT3D_ERR_INVALID_ARG, "bad length or null output");
    if (dtype == DT_F64) twiddles_f64(n, (double*)out);
    else if (dtype == DT_F32) twiddles_f32(n, (float*)out);
    else return fail(FFT3D_ERR_INVALID_ARG, "bad dtype");
    return FFT3D_OK;
}

int64_t fft3d_query_pipeline(int64_t nx, int64_t ny, int64_t nz, int p1, int p2, int r2c, int staging, int op,
                             int nstreams, int64_t* out, int64_t cap)
{
    PlanDesc d;
    d.nx = nx; d.ny = ny; d.nz = nz; d.dtype = DT_F32; d.p1 = p1; d.p2 = p2; d.r2c = r2c;
    if (validate_desc(d) != FFT3D_OK) return -1;
    if (staging != STAGING_IN_PLACE && staging != STAGING_SWAP_YZ && staging != STAGING_FUSED_XY) return -1;
    if (r2c && staging == STAGING_FUSED_XY) return -1;
    if (staging == STAGING_FUSED_XY && (p1 != 1 || !plane_listed(nx, ny))) return -1;
    d.staging = staging;
    if (op < 0 || op >= OP_COUNT || nstreams < 1 || nstreams > kMaxStreams) return -1;
    const Pipeline pl = build_pipeline(d, op, nstreams);
    std::vector<int64_t> v;
    v.push_back((int64_t)pl.tasks.size());
    v.push_back((int64_t)pl.stages.size());
    for (const Stage& s : pl.stages) {
        int64_t scale_bits;
        memcpy(&scale_bits, &s.scale, sizeof scale_bits);
        int64_t rec[10] = {s.kind, s.axis, s.n, s.conj, s.weight, s.src, s.dst, scale_bits, s.lay_src, s.lay_dst};
        v.insert(v.end(), rec, rec + 10);
    }
    for (const Task& t : pl.tasks) {
        v.push_back(t.stage);
        for (int ax = 0; ax < 3; ++ax) {
            v.push_back(t.box.lo[ax]);
            v.push_back(t.box.hi[ax]);
        }
        v.push_back(t.stream);
        v.push_back((int64_t)t.deps.size());
        v.insert(v.end(), t.deps.begin(), t.deps.end());
        v.push_back((int64_t)t.waits.size());
        v.insert(v.end(), t.waits.begin(), t.waits.end());
    }
    if (out && cap >= (int64_t)v.size()) memcpy(out, v.data(), v.size() * sizeof(int64_t));
    return (int64_t)v.size();
}

int64_t fft3d_query_launches(int64_t nx, int64_t ny, int64_t nz, int dtype, int p1, int p2, int r2c, int staging,
                             int op, int64_t* out, int64_t cap)
{
    PlanDesc d;
    d.nx = nx; d.ny = ny; d.nz = nz; d.dtype = dtype; d.p1 = p1; d.p2 = p2; d.r2c = r2c;
    if (validate_desc(d) != FFT3D_OK) return -1;
    if (staging != STAGING_IN_PLACE && staging != STAGING_SWAP_YZ && staging != STAGING_FUSED_XY) return -1;
    if (r2c && staging == STAGING_FUSED_XY) return -1;
    if (staging == STAGING_FUSED_XY && (p1 != 1 || !plane_listed(nx, ny))) return -1;
    if (op < 0 || op >= OP_COUNT) return -1;
    d.staging = staging;
    // the launch shapes depend only on the plan description (no device state)
    fft3d_plan_s tmp;
    tmp.d = d;
    const Pipeline pl = build_pipeline(d, op, 1);
    void* const bufs[3] = {nullptr, nullptr, nullptr};
    std::vector<int64_t> v;
    v.push_back((int64_t)pl.tasks.size());
    for (const Task& t : pl.tasks) {
        const StageArgs a = make_args(&tmp, pl.stages[t.stage], t.box, bufs);
        const int64_t rec[8] = {a.lw, a.tdiv, a.split, a.pad, a.strided, a.align, a.xcd, a.nt};
        v.insert(v.end(), rec, rec + 8);
    }
    if (out && cap >= (int64_t)v.size()) memcpy(out, v.data(), v.size() * sizeof(int64_t));
    return (int64_t)v.size();
}

}  // extern "C"
