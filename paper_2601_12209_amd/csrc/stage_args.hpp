// Arguments of one stage-kernel launch (one pencil tile of one stage).
// Plain C++: shared by the host planner/executor and the kernels.
#pragma once
#include <stdint.h>

namespace fft3d {

enum KernelKind : int {
    K_C2C = 0,        // batched complex line FFTs, any axis
    K_R2C_X = 1,      // real x-lines -> half-spectrum x-lines
    K_C2R_X = 2,      // half-spectrum x-lines -> real x-lines
    K_POISSON_Z = 3,  // z-lines: forward FFT, spectral multiplier, inverse FFT
    K_C2C_XY = 4,     // whole x-y planes in LDS: x FFTs then y FFTs (small planes)
};

enum DType : int { DT_F32 = 0, DT_F64 = 1 };

// The tile's lines form an A x B grid; line (a, b) starts at element
// off + a*sa + b*sb of the input and its elements are se apart; in the output
// it starts at off_o + a*sa_o + b*sb_o with elements se_o apart.  Elements are
// complex values of the kernel's precision (for R2C input and C2R output, a
// complex value is a pair of consecutive reals).  R2C/C2R lines are contiguous
// (se = se_o = 1).
struct StageArgs {
    const void* in;
    void* out;
    const void* tw;   // forward roots W_n^m = exp(-2 pi i m/n), m < n, n = axis length
    const void* twp;  // per-pass twiddle table of the kernel's FFT length
    const void* twp2; // K_C2C_XY: per-pass table of the y length (twp: the x length)
    int64_t A, B;
    int64_t off, sa, sb, se;
    int64_t off_o, sa_o, sb_o, se_o;
    int strided;  // 1: lanes of a wavefront walk neighbouring lines (requires sa == sa_o == 1)
    int align;    // strided: > 1 shifts each row's line tiles so that output row segments
                  // start on multiples of `align` elements (a cache line); lw % align == 0
    int xcd;      // strided: 1 gives each of the 8 XCDs a contiguous run of tiles
                  // (workgroups go to XCDs round-robin by linear id), so tiles that
                  // share cache lines meet in one L2
    int nt;       // cache policy of the tile's global accesses: 0 plain, 1 non-temporal
                  // stores, 2 non-temporal loads and stores (C2C kernels of the lengths
                  // with launch-shape variants, one thread per butterfly; ignored elsewhere)
    int lw;       // lines per workgroup
    int tdiv;     // threads per line = (default threads per line) / tdiv
    int split;    // 1: exchange real and imaginary parts through LDS separately
    int pad;      // 1: pad contiguous LDS lines by one slot per 8 elements
    int conj;     // 1: conjugate-sign transform, taken as conj(F(conj x))
    int weight;   // R2C: interior bins x2 / C2R: interior bins x1/2 (adjoint paths)
    double scale; // multiplies every output
    // spectral multiplier (K_POISSON_Z): full grid sizes and the global
    // (kx, ky) of line (0, 0)
    int64_t pnx, pny, pnz;
    int64_t kx0, ky0;
};

}  // namespace fft3d
