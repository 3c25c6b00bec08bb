// Plane shapes (Nx, Ny) with a fused x-y kernel, and the LDS rule that
// decides whether a precision fits.  Plain C++ (no HIP): the planner and the
// host tests use it too.
#pragma once
#include <stddef.h>

#include "fft_lengths.hpp"

// Small planes: squares up to 128 and the two non-square planes of the
// batched workload (100 x 120 and 80 x 160).
#define FFT3D_FOR_EACH_PLANE(X)                                                                     \
    X(8, 8) X(16, 16) X(24, 24) X(32, 32) X(48, 48) X(64, 64) X(96, 96) X(100, 120) X(80, 160)     \
    X(128, 128)

namespace fft3d {

// Threads of a fused x-y workgroup: enough for every row (then every column)
// of the plane to have its line group at once, so each sweep is one chunk;
// a multiple of the 64-wide wavefront, at most 1024.
constexpr int plane_threads(int nx, int ny)
{
    const int rows = ny * radix_plan(nx).tpl, cols = nx * radix_plan(ny).tpl;
    const int t = ((rows > cols ? rows : cols) + 63) / 64 * 64;
    return t > 1024 ? 1024 : t;
}

constexpr size_t kPlaneMaxLds = 160 * 1024;

// LDS bytes of a fused x-y workgroup with row pitch px: the plane, one
// scratch line for the idle line groups, and the pass tables of both lengths.
constexpr size_t plane_lds_bytes_at(int px, int nx, int ny, size_t elem)
{
    const int scratch = nx > ny ? nx : ny;
    return ((size_t)ny * px + scratch + pass_table_size(radix_plan(nx)) + pass_table_size(radix_plan(ny))) * elem;
}

// Row pitch (elements) of the plane in LDS: odd, so that 32 consecutive rows
// start on 32 different 8-byte bank slots (16 different 16-byte slots).  The
// sweeps give consecutive lanes consecutive lines at the same element, so
// every access of every pass is then free of bank conflicts.
constexpr int plane_pitch(int nx) { return nx % 2 == 0 ? nx + 1 : nx; }

// LDS bytes of the fused x-y workgroup of an (nx, ny) plane.
constexpr size_t plane_lds_bytes(int nx, int ny, size_t elem)
{
    return plane_lds_bytes_at(plane_pitch(nx), nx, ny, elem);
}

inline bool plane_listed(long long nx, long long ny)
{
#define FFT3D_PLANE_CASE(X_, Y_) if (nx == X_ && ny == Y_) return true;
    FFT3D_FOR_EACH_PLANE(FFT3D_PLANE_CASE)
#undef FFT3D_PLANE_CASE
    return false;
}

// Whether the fused x-y kernel exists for this plane and precision.
inline bool plane_available(long long nx, long long ny, size_t elem)
{
    return plane_listed(nx, ny) && plane_lds_bytes((int)nx, (int)ny, elem) <= kPlaneMaxLds;
}

}  // namespace fft3d
