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
    K_R2R_Z = 5,      // z-lines of a bounded z axis: DCT/DST (StageArgs::r2r)
};

// Real-to-real transform of a K_R2R_Z launch (each applied to the real and
// imaginary parts of the complex z-lines alike), unnormalised:
//   R2R_DCT2  Y_k = 2 sum_j x_j cos(pi (2j+1) k / 2n)          (Neumann walls)
//   R2R_DCT3  x_j = Y_0 + 2 sum_{k>0} Y_k cos(pi k (2j+1) / 2n) (inverse of DCT2 up to 2n)
//   R2R_DST2  Y_k = 2 sum_j x_j sin(pi (2j+1) (k+1) / 2n)      (Dirichlet walls)
//   R2R_DST3  x_j = (-1)^j Y_{n-1} + 2 sum_{k<n-1} Y_k sin(pi (k+1) (2j+1) / 2n)
//   R2R_POISSON_N / _D: DCT2 / DST2, the multiplier -1/|k|^2 (times scale), then
//   DCT3 / DST3, in one kernel.
// With StageArgs::weight, DCT3/DST3 count the first coefficient of the
// (for the DST: reversed) line twice: the transposes of DCT2 and DST2.
enum R2RMode : int {
    R2R_DCT2 = 0,
    R2R_DCT3 = 1,
    R2R_DST2 = 2,
    R2R_DST3 = 3,
    R2R_POISSON_N = 4,
    R2R_POISSON_D = 5,
};

enum DType : int { DT_F32 = 0, DT_F64 = 1 };

// One tile of a grouped launch (one launch covering several tiles, of one
// transform or of several transforms of one shape): the fields of StageArgs
// that differ between those tiles, and the tile's own grid of workgroups.
struct TileEntry {
    const void* in;  // nullptr: the launch's own in/out (tiles of one transform)
    void* out;
    int64_t off, off_o;
    int64_t A, B;
    int64_t kx0, ky0;
    int64_t gx, gy;
};

// The tile's lines form an A x B grid; line (a, b) starts at element
// off + a*sa + b*sb of the input and its elements are se apart; in the output
// it starts at off_o + a*sa_o + b*sb_o with elements se_o apart.  Elements are
// complex values of the kernel's precision (for R2C input and C2R output, a
// complex value is a pair of consecutive reals).  R2C/C2R lines are contiguous
// (se = se_o = 1).
struct StageArgs {
    const void* in;
    void* out;
    const void* tw;   // forward roots W_n^m = exp(-2 pi i m/n), m < n, n = axis length;
                      // K_R2R_Z: W_4n^k, k < n
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
    int weight;   // R2C: interior bins x2 / C2R: interior bins x1/2 (adjoint paths);
                  // K_R2R_Z: the transposed DCT2/DST2 (see R2RMode)
    int r2r;      // K_R2R_Z: R2RMode
    int order;    // K_C2C: 1 runs the radices in the reverse pass order (twp is that
                  // order's per-pass table; one thread per butterfly, no split, plain
                  // accesses)
    double scale; // multiplies every output
    // spectral multiplier (K_POISSON_Z): full grid sizes and the global
    // (kx, ky) of line (0, 0)
    int64_t pnx, pny, pnz;
    int64_t kx0, ky0;
    // grouped launch: tiles[w / gmax] is the tile of workgroup w (nullptr: a
    // launch of this one tile on its own grid); with ntiles > 0 the tiles go in
    // runs of ntiles whose workgroups are interleaved: workgroup w belongs to
    // tile (w / (ntiles gmax)) ntiles + w mod ntiles
    const TileEntry* tiles;
    int64_t gmax;
    int64_t ntiles;
};

}  // namespace fft3d
