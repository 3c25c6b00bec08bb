// Drives the library's C ABI through every host path the GPU tests take —
// plans of all test shapes and pencil grids, every stream count, every launch
// shape the library accepts, real-to-complex plans with the Poisson
// operations and caller workspaces, timing mode, both issue modes (a launch
// per tile, a grouped launch per stage), and batches with their cached launch
// tables, pointer changes and capture by the caller — against the host-only HIP stand-in, so AddressSanitizer and the
// stand-in's launch checks see all of it.  Prints "hostsim ok" and exits 0
// when nothing was flagged.
//
// Usage: driver [nbatch nx ny nz ...]   (the batch shapes, x fastest)
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <memory>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/fft3d.h"
#include "../../paper_2601_12209_amd/csrc/plane_list.hpp"

extern "C" int hostsim_violations();
extern "C" size_t hostsim_last_capture_members();
extern "C" long hostsim_launches();
extern "C" size_t hostsim_live_allocations();

namespace {

int g_failures = 0;
std::vector<int64_t> g_batch_dims;  // the batch shapes (x fastest)

#define EXPECT(cond)                                                                              \
    do {                                                                                          \
        if (!(cond)) {                                                                            \
            fprintf(stderr, "%s:%d: expectation failed: %s (%s)\n", __FILE__, __LINE__, #cond,    \
                    fft3d_last_error());                                                          \
            ++g_failures;                                                                         \
        }                                                                                         \
    } while (0)

struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
    explicit Buf(size_t b) : bytes(b) { EXPECT(hipMalloc(&p, b) == hipSuccess); }
    ~Buf() { (void)hipFree(p); }
    Buf(const Buf&) = delete;
    Buf& operator=(const Buf&) = delete;
};

size_t es_of(int dtype) { return dtype == FFT3D_C128 ? 16 : 8; }

// Workspace rows are padded to 128 bytes.
size_t padded(int64_t n, int dtype)
{
    const int64_t per = 128 / (int64_t)es_of(dtype);
    return (size_t)((n + per - 1) / per * per);
}

hipStream_t make_stream()
{
    hipStream_t s = nullptr;
    EXPECT(hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess);
    return s;
}

// (nx, ny, nz), p1, p2
struct Case {
    int64_t nx, ny, nz;
    int p1, p2;
};

void c2c_cases(hipStream_t user)
{
    const Case cases[] = {{8, 8, 8, 1, 1},      {32, 32, 32, 2, 2},   {20, 12, 16, 2, 3},    {4, 6, 5, 2, 2},
                          {1, 1, 1, 1, 1},      {8, 4, 1, 1, 1},      {16, 1, 3, 1, 1},      {100, 48, 64, 3, 3},
                          {24, 30, 25, 4, 5},   {100, 120, 128, 4, 4}, {160, 160, 80, 2, 2}, {48, 48, 48, 1, 1},
                          {512, 64, 64, 1, 1},  {16, 8, 512, 1, 1},   {8, 1024, 16, 2, 2},   {2, 2, 4096, 1, 1},
                          {4096, 2, 2, 1, 1},   {32, 32, 32, 1, 1},   {64, 64, 40, 1, 4},    {100, 120, 12, 1, 2},
                          {80, 160, 8, 1, 1},   {128, 128, 16, 1, 1}, {24, 24, 7, 1, 1}};
    for (const Case& c : cases) {
        for (int dtype : {FFT3D_C64, FFT3D_C128}) {
            const size_t bytes = (size_t)c.nx * c.ny * c.nz * es_of(dtype);
            Buf in(bytes), out(bytes);
            fft3d_plan_t p = nullptr;
            EXPECT(fft3d_plan(&p, c.nx, c.ny, c.nz, dtype, c.p1, c.p2, 0) == FFT3D_OK);
            if (!p) continue;
            for (int ns : {1, 2, 4, 16}) {
                EXPECT(fft3d_set_streams(p, ns) == FFT3D_OK);
                EXPECT(fft3d_forward(p, in.p, out.p, user) == FFT3D_OK);
                EXPECT(fft3d_inverse(p, out.p, out.p, user) == FFT3D_OK);
                EXPECT(fft3d_backward(p, out.p, in.p, nullptr) == FFT3D_OK);
            }
            // both issue modes, timed and not
            for (int issue : {FFT3D_ISSUE_TILES, FFT3D_ISSUE_STAGES}) {
                EXPECT(fft3d_set_issue(p, issue) == FFT3D_OK);
                EXPECT(fft3d_get_issue(p) == issue);
                EXPECT(fft3d_set_timing(p, 1) == FFT3D_OK);
                EXPECT(fft3d_forward(p, in.p, out.p, user) == FFT3D_OK);
                EXPECT(fft3d_set_timing(p, 0) == FFT3D_OK);
                EXPECT(fft3d_inverse(p, out.p, out.p, user) == FFT3D_OK);
            }
            EXPECT(fft3d_set_issue(p, 2) == FFT3D_ERR_INVALID_ARG);
            // the reverse radix order on every axis that has one
            for (int ax = 0; ax < 3; ++ax) {
                const int64_t n = ax == 0 ? c.nx : ax == 1 ? c.ny : c.nz;
                // x and y run as fused planes (no line kernel) in that staging
                const bool lines = !(fft3d_get_staging(p) == FFT3D_STAGING_FUSED_XY && ax < 2);
                const fft3d_status r = fft3d_set_radix_order(p, ax, 1);
                EXPECT(r == (lines && fft3d::radix_order_distinct((int)n) ? FFT3D_OK : FFT3D_ERR_INVALID_ARG));
            }
            EXPECT(fft3d_forward(p, in.p, out.p, user) == FFT3D_OK);
            EXPECT(fft3d_inverse(p, out.p, out.p, user) == FFT3D_OK);
            EXPECT(fft3d_set_radix_order(p, 0, 2) == FFT3D_ERR_INVALID_ARG);
            EXPECT(fft3d_set_radix_order(p, 3, 0) == FFT3D_ERR_INVALID_ARG);
            for (int ax = 0; ax < 3; ++ax) EXPECT(fft3d_set_radix_order(p, ax, 0) == FFT3D_OK);
            EXPECT(fft3d_get_radix_order(p, 1) == 0);
            EXPECT(fft3d_get_radix_order(nullptr, 1) == -1);
            EXPECT(fft3d_get_issue(nullptr) == -1);
            // more buffer sets, then a setter
            {
                std::vector<std::unique_ptr<Buf>> extra;
                for (int k = 0; k < 10; ++k) {
                    extra.emplace_back(new Buf(bytes));
                    EXPECT(fft3d_forward(p, in.p, extra.back()->p, user) == FFT3D_OK);
                }
                EXPECT(fft3d_set_streams(p, 3) == FFT3D_OK);
            }
            EXPECT(fft3d_forward(p, in.p, out.p, user) == FFT3D_OK);
            (void)fft3d_set_stage_config(p, 1, 4, 1, 0, 0);  // where the shape fits
            EXPECT(fft3d_forward(p, in.p, out.p, user) == FFT3D_OK);
            EXPECT(fft3d_set_stage_config(p, 1, 0, 1, 0, 0) == FFT3D_OK);
            EXPECT(fft3d_poisson(p, in.p, out.p, user) == FFT3D_ERR_WRONG_PLAN);
            EXPECT(fft3d_get_staging(p) >= 0);
            if (bytes >= 2 * es_of(dtype))  // partial overlap
                EXPECT(fft3d_forward(p, in.p, (char*)in.p + es_of(dtype), user) == FFT3D_ERR_ALIAS);
            // swapped-y/z staging: owned workspace, then a caller one
            EXPECT(fft3d_workspace_bytes(p) == 0);
            EXPECT(fft3d_set_workspace(p, in.p, bytes) == FFT3D_ERR_WRONG_PLAN);
            EXPECT(fft3d_set_staging(p, FFT3D_STAGING_SWAP_YZ) == FFT3D_OK);
            const size_t wsb = padded(c.nx, dtype) * c.ny * c.nz * es_of(dtype);
            EXPECT(fft3d_workspace_bytes(p) == wsb);
            for (int ns : {1, 4}) {
                EXPECT(fft3d_set_streams(p, ns) == FFT3D_OK);
                EXPECT(fft3d_forward(p, in.p, out.p, user) == FFT3D_OK);
                EXPECT(fft3d_inverse(p, out.p, out.p, user) == FFT3D_OK);
                EXPECT(fft3d_backward(p, out.p, in.p, nullptr) == FFT3D_OK);
            }
            {
                Buf ws(wsb);
                EXPECT(fft3d_set_workspace(p, ws.p, wsb - 1) == FFT3D_ERR_WORKSPACE);
                EXPECT(fft3d_set_workspace(p, ws.p, wsb) == FFT3D_OK);
                EXPECT(fft3d_forward(p, in.p, out.p, user) == FFT3D_OK);
                EXPECT(fft3d_forward(p, ws.p, out.p, user) == FFT3D_ERR_ALIAS);
                EXPECT(fft3d_set_staging(p, FFT3D_STAGING_IN_PLACE) == FFT3D_OK);
            }
            EXPECT(fft3d_forward(p, in.p, out.p, user) == FFT3D_OK);
            EXPECT(fft3d_set_staging(p, 3) == FFT3D_ERR_INVALID_ARG);
            // fused x-y planes where a kernel exists (and p1 == 1)
            const bool planes = c.p1 == 1 && c.ny > 1 && fft3d::plane_available(c.nx, c.ny, es_of(dtype));
            EXPECT(fft3d_set_staging(p, FFT3D_STAGING_FUSED_XY) ==
                   (planes ? FFT3D_OK : FFT3D_ERR_UNSUPPORTED_SIZE));
            if (planes) {
                EXPECT(fft3d_workspace_bytes(p) == 0);
                for (int ns : {1, 3}) {
                    EXPECT(fft3d_set_streams(p, ns) == FFT3D_OK);
                    EXPECT(fft3d_forward(p, in.p, out.p, user) == FFT3D_OK);
                    EXPECT(fft3d_inverse(p, out.p, out.p, user) == FFT3D_OK);
                    EXPECT(fft3d_backward(p, out.p, in.p, nullptr) == FFT3D_OK);
                }
            }
            EXPECT(fft3d_destroy(p) == FFT3D_OK);
        }
    }
    {  // large plans default to the swapped staging with an owned workspace
        const size_t bytes = (size_t)512 * 256 * 256 * 16;
        Buf in(bytes), out(bytes);
        fft3d_plan_t p = nullptr;
        EXPECT(fft3d_plan(&p, 512, 256, 256, FFT3D_C128, 2, 2, 0) == FFT3D_OK);
        EXPECT(fft3d_workspace_bytes(p) == bytes);
        EXPECT(fft3d_forward(p, in.p, out.p, user) == FFT3D_OK);
        EXPECT(fft3d_inverse(p, out.p, in.p, user) == FFT3D_OK);
        EXPECT(fft3d_destroy(p) == FFT3D_OK);
        EXPECT(fft3d_plan(&p, 256, 256, 256, FFT3D_C128, 1, 1, 0) == FFT3D_OK);  // 256 MiB: in place
        EXPECT(fft3d_workspace_bytes(p) == 0);
        EXPECT(fft3d_destroy(p) == FFT3D_OK);
    }
    fft3d_plan_t p = nullptr;
    EXPECT(fft3d_plan(&p, 8, 8, 17, FFT3D_C64, 1, 1, 0) == FFT3D_ERR_UNSUPPORTED_SIZE);
    EXPECT(fft3d_plan(&p, 8, 8, 8, FFT3D_C64, 9, 1, 0) == FFT3D_ERR_INVALID_ARG);
    EXPECT(fft3d_plan(&p, 8, 8, 8, 5, 1, 1, 0) == FFT3D_ERR_INVALID_ARG);
}

// Every (axis, lw, tdiv, split, pad) the library accepts, one fresh plan each.
void variant_cases(hipStream_t user)
{
    const Case shapes[] = {{512, 64, 64, 1, 1}, {64, 16, 512, 1, 1}, {32, 512, 16, 1, 1}, {256, 256, 8, 1, 1},
                           {8, 1024, 32, 1, 1}};
    int accepted = 0;
    for (const Case& c : shapes) {
        for (int dtype : {FFT3D_C64, FFT3D_C128}) {
            const size_t bytes = (size_t)c.nx * c.ny * c.nz * es_of(dtype);
            Buf in(bytes), out(bytes);
            for (int axis = 0; axis < 3; ++axis)
                for (int lw = 1; lw <= 64; lw *= 2)
                    for (int tdiv : {1, 2, 4})
                        for (int split = 0; split < 2; ++split)
                            for (int pad = 0; pad < (axis == 0 ? 2 : 1); ++pad) {
                                fft3d_plan_t p = nullptr;
                                EXPECT(fft3d_plan(&p, c.nx, c.ny, c.nz, dtype, 1, 1, 0) == FFT3D_OK);
                                if (!p) continue;
                                if (fft3d_set_stage_config(p, axis, lw, tdiv, split, pad) == FFT3D_OK) {
                                    ++accepted;
                                    EXPECT(fft3d_forward(p, in.p, out.p, user) == FFT3D_OK);
                                    EXPECT(fft3d_inverse(p, out.p, out.p, user) == FFT3D_OK);
                                    EXPECT(fft3d_set_staging(p, FFT3D_STAGING_SWAP_YZ) == FFT3D_OK);
                                    EXPECT(fft3d_forward(p, in.p, out.p, user) == FFT3D_OK);
                                    EXPECT(fft3d_inverse(p, out.p, out.p, user) == FFT3D_OK);
                                }
                                EXPECT(fft3d_destroy(p) == FFT3D_OK);
                            }
        }
    }
    EXPECT(accepted > 100);
}

void r2c_cases(hipStream_t user)
{
    const Case cases[] = {{8, 8, 8, 1, 1},     {10, 6, 8, 2, 2},    {12, 10, 15, 3, 2},  {64, 32, 16, 1, 1},
                          {20, 12, 16, 2, 3},  {40, 24, 32, 2, 2},  {2, 1, 1, 1, 1},     {512, 16, 8, 1, 1},
                          {256, 64, 64, 4, 4}, {100, 30, 24, 2, 5}, {4096, 2, 2, 1, 1}};
    for (const Case& c : cases) {
        for (int dtype : {FFT3D_C64, FFT3D_C128}) {
            const size_t es = es_of(dtype);
            const size_t real_bytes = (size_t)c.nx * c.ny * c.nz * es / 2;
            const size_t half_bytes = (size_t)(c.nx / 2 + 1) * c.ny * c.nz * es;
            Buf r(real_bytes), r2(real_bytes), h(half_bytes);
            fft3d_plan_t p = nullptr;
            EXPECT(fft3d_plan(&p, c.nx, c.ny, c.nz, dtype, c.p1, c.p2, 1) == FFT3D_OK);
            if (!p) continue;
            for (int ns : {1, 3, 4}) {
                EXPECT(fft3d_set_streams(p, ns) == FFT3D_OK);
                EXPECT(fft3d_forward(p, r.p, h.p, user) == FFT3D_OK);
                EXPECT(fft3d_backward(p, h.p, r2.p, user) == FFT3D_OK);
                EXPECT(fft3d_inverse(p, h.p, r2.p, nullptr) == FFT3D_OK);
                EXPECT(fft3d_poisson(p, r.p, r2.p, user) == FFT3D_OK);
                EXPECT(fft3d_poisson(p, r.p, r.p, user) == FFT3D_OK);
                EXPECT(fft3d_poisson_backward(p, r2.p, r.p, user) == FFT3D_OK);
            }
            EXPECT(fft3d_forward(p, r.p, r.p, user) == FFT3D_ERR_ALIAS);
            // radix order: none on the real x kernels; y and z where distinct
            EXPECT(fft3d_set_radix_order(p, 0, 1) == FFT3D_ERR_INVALID_ARG);
            for (int ax : {1, 2}) {
                const int64_t n = ax == 1 ? c.ny : c.nz;
                EXPECT(fft3d_set_radix_order(p, ax, 1) ==
                       (fft3d::radix_order_distinct((int)n) ? FFT3D_OK : FFT3D_ERR_INVALID_ARG));
            }
            EXPECT(fft3d_forward(p, r.p, h.p, user) == FFT3D_OK);
            EXPECT(fft3d_inverse(p, h.p, r2.p, user) == FFT3D_OK);
            EXPECT(fft3d_poisson(p, r.p, r2.p, user) == FFT3D_OK);
            for (int ax : {1, 2}) EXPECT(fft3d_set_radix_order(p, ax, 0) == FFT3D_OK);
            // both forward stagings, then back to in place
            for (int stg : {FFT3D_STAGING_IN_PLACE, FFT3D_STAGING_SWAP_YZ}) {
                EXPECT(fft3d_set_staging(p, stg) == FFT3D_OK);
                EXPECT(fft3d_get_staging(p) == stg);
                EXPECT(fft3d_forward(p, r.p, h.p, user) == FFT3D_OK);
                EXPECT(fft3d_inverse(p, h.p, r2.p, user) == FFT3D_OK);
                EXPECT(fft3d_backward(p, h.p, r2.p, nullptr) == FFT3D_OK);
            }
            EXPECT(fft3d_set_staging(p, FFT3D_STAGING_IN_PLACE) == FFT3D_OK);
            EXPECT(fft3d_set_staging(p, FFT3D_STAGING_FUSED_XY) == FFT3D_ERR_WRONG_PLAN);
            EXPECT(fft3d_set_staging(p, FFT3D_STAGING_SWAP_YZ) == FFT3D_OK);
            for (int ns : {1, 3}) {
                EXPECT(fft3d_set_streams(p, ns) == FFT3D_OK);
                EXPECT(fft3d_forward(p, r.p, h.p, user) == FFT3D_OK);
                EXPECT(fft3d_inverse(p, h.p, r2.p, user) == FFT3D_OK);
                EXPECT(fft3d_poisson(p, r.p, r2.p, user) == FFT3D_OK);
            }
            EXPECT(fft3d_set_staging(p, FFT3D_STAGING_IN_PLACE) == FFT3D_OK);
            // caller workspace, then back to a plan-owned one
            const size_t wsb = fft3d_workspace_bytes(p);
            EXPECT(wsb == padded(c.nx / 2 + 1, dtype) * c.ny * c.nz * es);
            {
                Buf ws(wsb);
                EXPECT(fft3d_set_workspace(p, ws.p, wsb - 1) == FFT3D_ERR_WORKSPACE);
                EXPECT(fft3d_set_workspace(p, ws.p, wsb) == FFT3D_OK);
                EXPECT(fft3d_forward(p, r.p, h.p, user) == FFT3D_OK);
                EXPECT(fft3d_poisson(p, r.p, r2.p, user) == FFT3D_OK);
                EXPECT(fft3d_backward(p, ws.p, r2.p, user) == FFT3D_ERR_ALIAS);
                EXPECT(fft3d_set_workspace(p, nullptr, 0) == FFT3D_OK);
            }
            EXPECT(fft3d_poisson_backward(p, r.p, r2.p, user) == FFT3D_OK);
            // timing mode
            EXPECT(fft3d_set_timing(p, 1) == FFT3D_OK);
            float ms[8];
            EXPECT(fft3d_forward(p, r.p, h.p, user) == FFT3D_OK);
            EXPECT(fft3d_stage_times(p, ms, 8) >= 3);
            EXPECT(fft3d_poisson(p, r.p, r2.p, user) == FFT3D_OK);
            EXPECT(fft3d_stage_times(p, ms, 8) >= 3);
            EXPECT(fft3d_set_timing(p, 0) == FFT3D_OK);
            EXPECT(fft3d_destroy(p) == FFT3D_OK);
        }
    }
    fft3d_plan_t p = nullptr;
    EXPECT(fft3d_plan(&p, 9, 8, 8, FFT3D_C64, 1, 1, 1) == FFT3D_ERR_UNSUPPORTED_SIZE);
}

// Plans with a bounded z axis: every operation, both walls, both precisions,
// tiled and not; the staging they reject; the allocation-free forward.
void ppb_cases(hipStream_t user)
{
    const Case cases[] = {{8, 8, 8, 1, 1}, {20, 12, 16, 2, 3}, {4, 6, 7, 1, 1}, {16, 10, 15, 2, 2}, {8, 4, 1, 1, 1},
                          {100, 48, 64, 3, 3}, {6, 4, 512, 1, 1}};
    for (const Case& c : cases) {
        for (int dtype : {FFT3D_C64, FFT3D_C128}) {
            for (int zbc : {FFT3D_Z_NEUMANN, FFT3D_Z_DIRICHLET}) {
                const size_t es = es_of(dtype);
                const size_t real = (size_t)c.nx * c.ny * c.nz * es / 2;
                const size_t half = (size_t)(c.nx / 2 + 1) * c.ny * c.nz * es;
                Buf r(real), r2(real), h(half);
                fft3d_plan_t p = nullptr;
                EXPECT(fft3d_plan_ppb(&p, c.nx, c.ny, c.nz, dtype, c.p1, c.p2, zbc) == FFT3D_OK);
                if (!p) continue;
                EXPECT(fft3d_get_staging(p) == FFT3D_STAGING_IN_PLACE);
                for (int ns : {1, 3}) {
                    EXPECT(fft3d_set_streams(p, ns) == FFT3D_OK);
                    EXPECT(fft3d_forward(p, r.p, h.p, user) == FFT3D_OK);
                    EXPECT(fft3d_inverse(p, h.p, r2.p, user) == FFT3D_OK);
                    EXPECT(fft3d_backward(p, h.p, r2.p, nullptr) == FFT3D_OK);
                    EXPECT(fft3d_poisson(p, r.p, r2.p, user) == FFT3D_OK);
                    EXPECT(fft3d_poisson(p, r2.p, r2.p, user) == FFT3D_OK);
                    EXPECT(fft3d_poisson_backward(p, r.p, r2.p, user) == FFT3D_OK);
                }
                EXPECT(fft3d_forward_noalloc(p, r.p, h.p, user) == FFT3D_OK);
                EXPECT(fft3d_set_staging(p, FFT3D_STAGING_SWAP_YZ) == FFT3D_ERR_WRONG_PLAN);
                EXPECT(fft3d_set_staging(p, FFT3D_STAGING_IN_PLACE) == FFT3D_OK);
                EXPECT(fft3d_destroy(p) == FFT3D_OK);
            }
        }
    }
    fft3d_plan_t p = nullptr;
    EXPECT(fft3d_plan_ppb(&p, 8, 8, 8, FFT3D_C64, 1, 1, 0) == FFT3D_ERR_INVALID_ARG);
    EXPECT(fft3d_plan_ppb(&p, 8, 8, 8, FFT3D_C64, 1, 1, 3) == FFT3D_ERR_INVALID_ARG);
    EXPECT(fft3d_plan_ppb(&p, 9, 8, 8, FFT3D_C64, 1, 1, FFT3D_Z_NEUMANN) == FFT3D_ERR_UNSUPPORTED_SIZE);
    EXPECT(p == nullptr);
}

// A multi-stream plan launched inside a capture the caller began.
void caller_capture_plan(hipStream_t user)
{
    fft3d_plan_t p = nullptr;
    EXPECT(fft3d_plan(&p, 32, 24, 20, FFT3D_C64, 2, 3, 0) == FFT3D_OK);
    if (!p) return;
    Buf in(32 * 24 * 20 * 8), out(32 * 24 * 20 * 8);
    EXPECT(fft3d_set_streams(p, 4) == FFT3D_OK);
    for (int rep = 0; rep < 2; ++rep) {
        EXPECT(fft3d_forward(p, in.p, out.p, user) == FFT3D_OK);  // an eager call first
        EXPECT(hipStreamBeginCapture(user, hipStreamCaptureModeThreadLocal) == hipSuccess);
        EXPECT(fft3d_forward(p, in.p, out.p, user) == FFT3D_OK);
        EXPECT(fft3d_inverse(p, out.p, out.p, user) == FFT3D_OK);
        hipGraph_t g = nullptr;
        EXPECT(hipStreamEndCapture(user, &g) == hipSuccess);
        // the tiles went in order onto the capturing stream: no internal stream joined
        EXPECT(hostsim_last_capture_members() == 1);
        if (g) (void)hipGraphDestroy(g);
    }
    // a call on another stream after one on `user`, then back
    hipStream_t other = make_stream();
    EXPECT(fft3d_forward(p, in.p, out.p, other) == FFT3D_OK);
    EXPECT(fft3d_inverse(p, out.p, out.p, user) == FFT3D_OK);
    EXPECT(fft3d_destroy(p) == FFT3D_OK);
    (void)hipStreamDestroy(other);
    // the tile cap
    EXPECT(fft3d_plan(&p, 64, 64, 64, FFT3D_C64, 33, 32, 0) == FFT3D_ERR_INVALID_ARG);
    EXPECT(p == nullptr);
}

void batch_cases(const std::vector<int64_t>& dims, hipStream_t user)
{
    const int n = (int)dims.size() / 3;
    for (int dtype : {FFT3D_C64, FFT3D_C128}) {
        std::vector<Buf*> bufs, bufs2;
        std::vector<const void*> in;
        std::vector<void*> out, in2;
        for (int f = 0; f < n; ++f) {
            const size_t b = (size_t)dims[3 * f] * dims[3 * f + 1] * dims[3 * f + 2] * es_of(dtype);
            bufs.push_back(new Buf(b));
            bufs2.push_back(new Buf(b));
            in.push_back(bufs.back()->p);
            out.push_back(bufs2.back()->p);
            in2.push_back(bufs.back()->p);
        }
        fft3d_batch_t b = nullptr;
        EXPECT(fft3d_plan_batch(&b, n, dims.data(), dtype) == FFT3D_OK);
        if (!b) continue;
        for (int rep = 0; rep < 3; ++rep) {
            EXPECT(fft3d_forward_batch(b, in.data(), out.data(), user) == FFT3D_OK);
            EXPECT(fft3d_inverse_batch(b, out.data(), out.data(), user) == FFT3D_OK);
            EXPECT(fft3d_forward_batch(b, in.data(), out.data(), nullptr) == FFT3D_OK);
        }
        // more pointer sets than cached launch tables (one table set each)
        for (int rep = 0; rep < 12; ++rep) {
            std::vector<Buf*> fresh;
            std::vector<void*> o2;
            for (int f = 0; f < n; ++f) {
                fresh.push_back(new Buf(bufs2[f]->bytes));
                o2.push_back(fresh.back()->p);
            }
            EXPECT(fft3d_forward_batch(b, in.data(), o2.data(), user) == FFT3D_OK);
            EXPECT(fft3d_forward_batch(b, in.data(), in2.data(), user) == FFT3D_OK);  // in place
            EXPECT(hipStreamSynchronize(user) == hipSuccess);
            for (Buf* x : fresh) delete x;
        }
        // stage configs of each distinct shape drop the cached launch tables
        for (int f = 0; f < n; ++f) {
            EXPECT(fft3d_batch_set_stage_config(b, dims[3 * f], dims[3 * f + 1], dims[3 * f + 2], 1, 4, 1, 0, 0) ==
                   FFT3D_OK);
        }
        EXPECT(fft3d_forward_batch(b, in.data(), out.data(), user) == FFT3D_OK);
        EXPECT(fft3d_batch_set_stage_config(b, 3, 3, 3, 0, 1, 1, 0, 0) == FFT3D_ERR_INVALID_ARG);
        // staging per shape: in place always, fused planes where a kernel fits
        for (int f = 0; f < n; ++f) {
            const int64_t *d = &dims[3 * f];
            const bool planes = d[1] > 1 && fft3d::plane_available(d[0], d[1], es_of(dtype));
            EXPECT(fft3d_batch_set_staging(b, d[0], d[1], d[2], FFT3D_STAGING_FUSED_XY) ==
                   (planes ? FFT3D_OK : FFT3D_ERR_UNSUPPORTED_SIZE));
            EXPECT(fft3d_forward_batch(b, in.data(), out.data(), user) == FFT3D_OK);
            if (planes) EXPECT(fft3d_batch_get_staging(b, d[0], d[1], d[2]) == FFT3D_STAGING_FUSED_XY);
            EXPECT(fft3d_batch_set_staging(b, d[0], d[1], d[2], FFT3D_STAGING_IN_PLACE) == FFT3D_OK);
            EXPECT(fft3d_batch_set_staging(b, d[0], d[1], d[2], FFT3D_STAGING_SWAP_YZ) == FFT3D_ERR_INVALID_ARG);
        }
        EXPECT(fft3d_inverse_batch(b, out.data(), out.data(), user) == FFT3D_OK);
        EXPECT(fft3d_batch_set_staging(b, 3, 3, 3, FFT3D_STAGING_IN_PLACE) == FFT3D_ERR_INVALID_ARG);
        EXPECT(fft3d_batch_get_staging(b, 3, 3, 3) == -1);
        for (int ns : {1, 2, 16}) {  // shapes on other stream counts
            EXPECT(fft3d_batch_set_streams(b, ns) == FFT3D_OK);
            EXPECT(fft3d_forward_batch(b, in.data(), out.data(), user) == FFT3D_OK);
            EXPECT(fft3d_inverse_batch(b, out.data(), out.data(), nullptr) == FFT3D_OK);
        }
        EXPECT(fft3d_batch_set_streams(b, 0) == FFT3D_ERR_INVALID_ARG);
        EXPECT(fft3d_batch_set_streams(b, 4) == FFT3D_OK);
        EXPECT(fft3d_batch_get_staging(nullptr, 3, 3, 3) == -1);
        // the caller captures the batch into its own graph: twice with a
        // pointer set an earlier call built tables for (grouped launches),
        // then with a fresh set (each plan's direct issue); then a setter
        // retires the captured tables
        for (int rep = 0; rep < 3; ++rep) {
            std::vector<Buf*> fresh;
            std::vector<void*> o2(out.begin(), out.end());
            if (rep == 2)
                for (int f = 0; f < n; ++f) {
                    fresh.push_back(new Buf(bufs2[f]->bytes));
                    o2[f] = fresh.back()->p;
                }
            EXPECT(hipStreamBeginCapture(user, hipStreamCaptureModeThreadLocal) == hipSuccess);
            EXPECT(fft3d_forward_batch(b, in.data(), o2.data(), user) == FFT3D_OK);
            hipGraph_t g = nullptr;
            EXPECT(hipStreamEndCapture(user, &g) == hipSuccess);
            if (g) (void)hipGraphDestroy(g);
            for (Buf* x : fresh) delete x;
        }
        EXPECT(fft3d_batch_set_streams(b, 2) == FFT3D_OK);
        EXPECT(fft3d_forward_batch(b, in.data(), out.data(), user) == FFT3D_OK);
        // a partial overlap of one transform's input and output
        if (bufs[0]->bytes >= 2 * es_of(dtype)) {
            std::vector<void*> shifted(out.begin(), out.end());
            shifted[0] = (char*)in2[0] + es_of(dtype);
            EXPECT(fft3d_forward_batch(b, in.data(), shifted.data(), user) == FFT3D_ERR_ALIAS);
        }
        // overlapping outputs of two transforms
        if (n >= 2) {
            std::vector<void*> bad(out.begin(), out.end());
            bad[1] = bad[0];
            EXPECT(fft3d_forward_batch(b, in.data(), bad.data(), user) == FFT3D_ERR_ALIAS);
        }
        EXPECT(fft3d_batch_destroy(b) == FFT3D_OK);
        for (Buf* x : bufs) delete x;
        for (Buf* x : bufs2) delete x;
    }
    fft3d_batch_t b = nullptr;
    const int64_t bad[3] = {8, 8, 17};
    EXPECT(fft3d_plan_batch(&b, 1, bad, FFT3D_C64) == FFT3D_ERR_UNSUPPORTED_SIZE);
    EXPECT(b == nullptr);
}


// The C-ABI call sequence of bench.py at its full sizes (headline 512^3
// C2C in both precisions, then every extra workload), on the legacy default
// stream and a second stream the way torch hands them over.
void bench_sequence()
{
    hipStream_t side = make_stream();
    float ms[8];
    auto step = [&](const char* what) { printf("bench step: %s\n", what); fflush(stdout); };
    // headline: 512^3 C2C, grid 1x1, one stream, swapped staging
    for (int dtype : {FFT3D_C64, FFT3D_C128}) {
        step(dtype == FFT3D_C64 ? "512^3 c64" : "512^3 c128");
        const size_t b = (size_t)512 * 512 * 512 * es_of(dtype);
        Buf x(b), X(b), Y(b);
        fft3d_plan_t p = nullptr;
        EXPECT(fft3d_plan(&p, 512, 512, 512, dtype, 1, 1, 0) == FFT3D_OK);
        if (!p) continue;
        EXPECT(fft3d_set_streams(p, 1) == FFT3D_OK);
        EXPECT(fft3d_set_staging(p, FFT3D_STAGING_SWAP_YZ) == FFT3D_OK);
        for (int i = 0; i < 23; ++i) {
            EXPECT(fft3d_forward(p, x.p, X.p, side) == FFT3D_OK);
            EXPECT(fft3d_inverse(p, X.p, Y.p, side) == FFT3D_OK);
        }
        EXPECT(fft3d_set_timing(p, 1) == FFT3D_OK);
        for (int i = 0; i < 10; ++i) {
            EXPECT(fft3d_forward(p, x.p, X.p, nullptr) == FFT3D_OK);
            EXPECT(fft3d_stage_times(p, ms, 8) == 3);
            EXPECT(fft3d_inverse(p, X.p, Y.p, nullptr) == FFT3D_OK);
            EXPECT(fft3d_stage_times(p, ms, 8) == 3);
        }
        EXPECT(fft3d_set_timing(p, 0) == FFT3D_OK);
        EXPECT(fft3d_forward(p, x.p, X.p, nullptr) == FFT3D_OK);
        EXPECT(fft3d_inverse(p, X.p, Y.p, nullptr) == FFT3D_OK);
        EXPECT(fft3d_destroy(p) == FFT3D_OK);
    }
    // 512^3 R2C + C2R in both precisions, default stream, with timing
    for (int dtype : {FFT3D_C64, FFT3D_C128}) {
        step(dtype == FFT3D_C64 ? "512^3 r2c f32" : "512^3 r2c f64");
        const size_t es = es_of(dtype);
        Buf x((size_t)512 * 512 * 512 * es / 2), H((size_t)257 * 512 * 512 * es), y((size_t)512 * 512 * 512 * es / 2);
        fft3d_plan_t p = nullptr;
        EXPECT(fft3d_plan(&p, 512, 512, 512, dtype, 1, 1, 1) == FFT3D_OK);
        if (!p) continue;
        for (int i = 0; i < 13; ++i) {
            EXPECT(fft3d_forward(p, x.p, H.p, nullptr) == FFT3D_OK);
            EXPECT(fft3d_inverse(p, H.p, y.p, nullptr) == FFT3D_OK);
        }
        EXPECT(fft3d_set_timing(p, 1) == FFT3D_OK);
        for (int i = 0; i < 10; ++i) {
            EXPECT(fft3d_forward(p, x.p, H.p, nullptr) == FFT3D_OK);
            EXPECT(fft3d_stage_times(p, ms, 8) == 3);
            EXPECT(fft3d_inverse(p, H.p, y.p, nullptr) == FFT3D_OK);
            EXPECT(fft3d_stage_times(p, ms, 8) == 3);
        }
        EXPECT(fft3d_set_timing(p, 0) == FFT3D_OK);
        EXPECT(fft3d_destroy(p) == FFT3D_OK);
    }
    // 256^3 C2C on the 4x4 grid (4 streams, task graph) and 1x1 (1 stream)
    for (int dtype : {FFT3D_C64, FFT3D_C128}) {
        step(dtype == FFT3D_C64 ? "256^3 c64" : "256^3 c128");
        const size_t b = (size_t)256 * 256 * 256 * es_of(dtype);
        Buf x(b), X(b), Y(b);
        for (int g : {4, 1}) {
            fft3d_plan_t p = nullptr;
            EXPECT(fft3d_plan(&p, 256, 256, 256, dtype, g, g, 0) == FFT3D_OK);
            if (!p) continue;
            EXPECT(fft3d_set_streams(p, g == 4 ? 4 : 1) == FFT3D_OK);
            EXPECT(fft3d_forward(p, x.p, X.p, nullptr) == FFT3D_OK);
            for (int i = 0; i < 12; ++i) {
                EXPECT(fft3d_forward(p, x.p, X.p, side) == FFT3D_OK);
                EXPECT(fft3d_inverse(p, X.p, Y.p, side) == FFT3D_OK);
            }
            EXPECT(fft3d_destroy(p) == FFT3D_OK);
        }
    }
    // 1024^3 R2C + C2R f32 on the 8x8 grid and on 1x1
    {
        const size_t real = (size_t)1024 * 1024 * 1024 * 4, half = (size_t)513 * 1024 * 1024 * 8;
        Buf x(real), y(real);
        for (int g : {8, 1}) {
            step(g == 8 ? "1024^3 r2c 8x8" : "1024^3 r2c 1x1");
            Buf H(half);
            fft3d_plan_t p = nullptr;
            EXPECT(fft3d_plan(&p, 1024, 1024, 1024, FFT3D_C64, g, g, 1) == FFT3D_OK);
            if (!p) continue;
            EXPECT(fft3d_forward(p, x.p, H.p, nullptr) == FFT3D_OK);
            for (int i = 0; i < 7; ++i) {
                EXPECT(fft3d_forward(p, x.p, H.p, side) == FFT3D_OK);
                EXPECT(fft3d_inverse(p, H.p, y.p, side) == FFT3D_OK);
            }
            EXPECT(fft3d_destroy(p) == FFT3D_OK);
        }
    }
    // 840^3 C2C complex64, one tile
    {
        step("840^3 c64");
        const size_t b = (size_t)840 * 840 * 840 * 8;
        Buf x(b), X(b), Y(b);
        fft3d_plan_t p = nullptr;
        EXPECT(fft3d_plan(&p, 840, 840, 840, FFT3D_C64, 1, 1, 0) == FFT3D_OK);
        if (p) {
            EXPECT(fft3d_forward(p, x.p, X.p, nullptr) == FFT3D_OK);
            for (int i = 0; i < 7; ++i) {
                EXPECT(fft3d_forward(p, x.p, X.p, side) == FFT3D_OK);
                EXPECT(fft3d_inverse(p, X.p, Y.p, side) == FFT3D_OK);
            }
            EXPECT(fft3d_destroy(p) == FFT3D_OK);
        }
    }
    // 64 uneven transforms: a probe batch for the fused shapes, then a batch
    // whose launch shapes come from the autotuner's search on stand-alone
    // plans (timing mode, every candidate shape), replayed on `side`; the
    // same transforms one by one through plans of their own; a second batch
    {
        step("batch");
        const std::vector<int64_t>& dims = g_batch_dims;
        const int n = (int)dims.size() / 3;
        std::vector<Buf*> bufs;
        std::vector<const void*> in;
        std::vector<void*> out;
        for (int f = 0; f < n; ++f) {
            const size_t b = (size_t)dims[3 * f] * dims[3 * f + 1] * dims[3 * f + 2] * 8;
            bufs.push_back(new Buf(b));
            in.push_back(bufs.back()->p);
            bufs.push_back(new Buf(b));
            out.push_back(bufs.back()->p);
        }
        std::vector<std::vector<int64_t>> shapes;
        for (int f = 0; f < n; ++f) {
            std::vector<int64_t> sh(dims.begin() + 3 * f, dims.begin() + 3 * f + 3);
            if (std::find(shapes.begin(), shapes.end(), sh) == shapes.end()) shapes.push_back(sh);
        }
        fft3d_batch_t probe = nullptr;
        EXPECT(fft3d_plan_batch(&probe, n, dims.data(), FFT3D_C64) == FFT3D_OK);
        for (auto& sh : shapes) (void)fft3d_batch_set_staging(probe, sh[0], sh[1], sh[2], FFT3D_STAGING_FUSED_XY);
        EXPECT(fft3d_batch_destroy(probe) == FFT3D_OK);
        for (int round = 0; round < 2; ++round) {
            fft3d_batch_t bp = nullptr;
            EXPECT(fft3d_plan_batch(&bp, n, dims.data(), FFT3D_C64) == FFT3D_OK);
            if (!bp) break;
            for (auto& sh : shapes) {
                const size_t b = (size_t)sh[0] * sh[1] * sh[2] * 8;
                Buf x(b), o(b);
                fft3d_plan_t p = nullptr;
                EXPECT(fft3d_plan(&p, sh[0], sh[1], sh[2], FFT3D_C64, 1, 1, 0) == FFT3D_OK);
                if (!p) continue;
                EXPECT(fft3d_set_timing(p, 1) == FFT3D_OK);
                EXPECT(fft3d_forward(p, x.p, o.p, nullptr) == FFT3D_OK);
                const int nst = fft3d_stage_times(p, ms, 8);
                EXPECT(nst >= 2);
                EXPECT(fft3d_set_timing(p, 0) == FFT3D_OK);
                std::vector<int> axes = nst == 3 ? std::vector<int>{0, 1, 2} : std::vector<int>{2};
                for (int axis : axes) {
                    int best[4] = {0, 1, 0, 0};
                    EXPECT(fft3d_set_stage_config(p, axis, 0, 1, 0, 0) == FFT3D_OK);
                    for (int lw : {1, 2, 4, 8, 16, 32, 64})
                        for (int td : {1, 2, 4})
                            for (int sp : {0, 1})
                                for (int pd : {0, 1}) {
                                    if (fft3d_set_stage_config(p, axis, lw, td, sp, pd) != FFT3D_OK) continue;
                                    EXPECT(fft3d_set_timing(p, 1) == FFT3D_OK);
                                    for (int r = 0; r < 6; ++r) {
                                        EXPECT(fft3d_forward(p, x.p, o.p, nullptr) == FFT3D_OK);
                                        EXPECT(fft3d_stage_times(p, ms, 8) == nst);
                                    }
                                    EXPECT(fft3d_set_timing(p, 0) == FFT3D_OK);
                                    best[0] = lw; best[1] = td; best[2] = sp; best[3] = pd;
                                }
                    EXPECT(fft3d_set_stage_config(p, axis, best[0], best[1], best[2], best[3]) == FFT3D_OK);
                    EXPECT(fft3d_batch_set_stage_config(bp, sh[0], sh[1], sh[2], axis, best[0], best[1], best[2],
                                                        best[3]) == FFT3D_OK);
                }
                EXPECT(fft3d_destroy(p) == FFT3D_OK);
            }
            for (int r = 0; r < 12; ++r) EXPECT(fft3d_forward_batch(bp, in.data(), out.data(), side) == FFT3D_OK);
            EXPECT(fft3d_batch_destroy(bp) == FFT3D_OK);
            if (round == 0) {
                std::vector<fft3d_plan_t> plans;
                for (auto& sh : shapes) {
                    fft3d_plan_t p = nullptr;
                    EXPECT(fft3d_plan(&p, sh[0], sh[1], sh[2], FFT3D_C64, 1, 1, 0) == FFT3D_OK);
                    if (fft3d_set_staging(p, FFT3D_STAGING_FUSED_XY) != FFT3D_OK)
                        EXPECT(fft3d_set_staging(p, FFT3D_STAGING_IN_PLACE) == FFT3D_OK);
                    plans.push_back(p);
                }
                for (int r = 0; r < 12; ++r)
                    for (int f = 0; f < n; ++f) {
                        std::vector<int64_t> sh(dims.begin() + 3 * f, dims.begin() + 3 * f + 3);
                        const size_t k = std::find(shapes.begin(), shapes.end(), sh) - shapes.begin();
                        EXPECT(fft3d_forward(plans[k], in[f], out[f], side) == FFT3D_OK);
                    }
                for (fft3d_plan_t p : plans) EXPECT(fft3d_destroy(p) == FFT3D_OK);
            }
        }
        for (Buf* x : bufs) delete x;
    }
    // 256^3 Poisson solve + adjoint, float32, default stream
    {
        step("poisson 256^3");
        const size_t real = (size_t)256 * 256 * 256 * 4;
        Buf f(real), w(real), phi(real), g(real);
        fft3d_plan_t p = nullptr;
        EXPECT(fft3d_plan(&p, 256, 256, 256, FFT3D_C64, 1, 1, 1) == FFT3D_OK);
        if (p) {
            for (int r = 0; r < 13; ++r) {
                EXPECT(fft3d_poisson(p, f.p, phi.p, nullptr) == FFT3D_OK);
                EXPECT(fft3d_poisson_backward(p, w.p, g.p, nullptr) == FFT3D_OK);
            }
            EXPECT(fft3d_destroy(p) == FFT3D_OK);
        }
    }
    (void)hipStreamDestroy(side);
}

}  // namespace

int main(int argc, char** argv)
{
    if (argc > 1 && strcmp(argv[1], "bench") == 0) {
        const int nb = argc > 2 ? atoi(argv[2]) : 0;
        for (int i = 0; i < 3 * nb && 3 + i < argc; ++i) g_batch_dims.push_back(atoll(argv[3 + i]));
        if (g_batch_dims.empty()) g_batch_dims = {48, 48, 48, 64, 64, 64, 100, 120, 128, 160, 160, 80};
        const size_t live = hostsim_live_allocations();
        bench_sequence();
        EXPECT(hostsim_live_allocations() == live);
        printf("launches %ld, violations %d, failures %d\n", hostsim_launches(), hostsim_violations(), g_failures);
        if (hostsim_violations() == 0 && g_failures == 0) {
            printf("hostsim ok\n");
            return 0;
        }
        return 1;
    }
    std::vector<int64_t> dims;
    if (argc > 1) {
        const int n = atoi(argv[1]);
        for (int i = 0; i < 3 * n && 2 + i < argc; ++i) dims.push_back(atoll(argv[2 + i]));
    }
    if (dims.empty()) dims = {48, 48, 48, 64, 64, 64, 100, 120, 128, 160, 160, 80};
    hipStream_t user = make_stream();
    const size_t live0 = hostsim_live_allocations();
    c2c_cases(user);
    variant_cases(user);
    r2c_cases(user);
    ppb_cases(user);
    caller_capture_plan(user);
    batch_cases(dims, user);
    (void)hipStreamDestroy(user);
    const size_t leaked = hostsim_live_allocations() - live0;
    EXPECT(leaked == 0);
    printf("launches %ld, violations %d, failures %d, leaked allocations %zu\n", hostsim_launches(),
           hostsim_violations(), g_failures, leaked);
    if (hostsim_violations() == 0 && g_failures == 0) {
        printf("hostsim ok\n");
        return 0;
    }
    return 1;
}
