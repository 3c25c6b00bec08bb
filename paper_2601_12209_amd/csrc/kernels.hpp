// Stage-kernel launchers (one per kernel kind).  Each dispatches on the line
// length to the kernel specialised for it and returns hipErrorInvalidValue for
// a length without a kernel.
#pragma once
#include <hip/hip_runtime.h>

#include <stddef.h>

#include "stage_args.hpp"

namespace fft3d {

// LDS one workgroup may allocate on gfx950 (160 KiB per compute unit).
constexpr size_t kMaxLdsBytes = 160 * 1024;

hipError_t launch_c2c(int n, int dtype, const StageArgs& a, hipStream_t s);
// Whether the C2C kernel of length n has the (tdiv, split) variant.
bool c2c_variant_available(int n, int tdiv, int split);
// Whether the C2C kernel of length n runs the reverse radix order
// (StageArgs::order = 1) in this (tdiv, split) shape.
bool c2c_order_available(int n, int tdiv, int split);
// n is the real line length (even); the complex kernel runs at n/2.
hipError_t launch_r2c_x(int n, int dtype, const StageArgs& a, hipStream_t s);
hipError_t launch_c2r_x(int n, int dtype, const StageArgs& a, hipStream_t s);
hipError_t launch_poisson_z(int n, int dtype, const StageArgs& a, hipStream_t s);
// Bounded z axis: DCT/DST of the z-lines (a.r2r), strided lines as the
// Poisson z stage.
hipError_t launch_r2r_z(int n, int dtype, const StageArgs& a, hipStream_t s);
// Fused x-y planes (plane_list.hpp): a.B planes, rows a.sa / a.sa_o apart,
// planes a.sb / a.sb_o apart.
hipError_t launch_c2c_xy(int nx, int ny, int dtype, const StageArgs& a, hipStream_t s);

// One stage-kernel launch as data: what a hipGraph kernel node needs (every
// stage kernel takes a single StageArgs by value).
struct KernelLaunch {
    const void* func = nullptr;
    dim3 grid;
    dim3 block;
    size_t lds = 0;
    StageArgs args{};
};

// Every launcher above ends in launch_stage_kernel: it launches on `s`, or,
// while a recorder is installed on the calling host thread, writes the launch
// into it (and sets *recorded) instead.  Launchers that have nothing to do
// (an empty grid) return hipSuccess without calling it.
void set_launch_recorder(KernelLaunch* rec, bool* recorded);
hipError_t launch_stage_kernel(const void* func, dim3 grid, dim3 block, const StageArgs& a, size_t lds,
                               hipStream_t s);

// Grouped launches: tile launches of one stage kernel that differ only in
// their tile fields (buffers, origins, line grid, wavenumber origin) become
// one launch whose workgroups look their tile up in a device table
// (StageArgs::tiles, TileEntry).  can_group tells whether the launches
// qualify; make_group fills the table entries (in/out left null when
// own_buffers is false: the tiles of one transform share the launch's
// buffers) and the common launch (grid = tiles x gmax workgroups, args with
// gmax set, and ntiles > 0 interleaving the workgroups of each run of ntiles
// consecutive tiles; the caller sets args.tiles to the device copy of the
// entries).
bool can_group(const KernelLaunch* v, size_t n);
void make_group(const KernelLaunch* v, size_t n, bool own_buffers, int64_t ntiles, TileEntry* entries,
                KernelLaunch* common);

// Size of the library's static device scratch (one per GPU, scratch.hip),
// the workspace of the calls that allocate nothing: 256 MiB holds the R2C
// workspace of every grid up to 256^3 in either precision.
constexpr size_t kScratchBytes = (size_t)256 << 20;
// Device address of that scratch on `device`, which must be the current
// device; looked up once per device (hipGetSymbolAddress) and cached.
hipError_t scratch_address(int device, void** out);

}  // namespace fft3d
