// Host-side planning: pencil tiles per stage, the tile dependency graph, the
// placement of tiles on streams, and the twiddle tables.  Plain C++ with no
// HIP dependency, so all of it runs (and is tested) without a GPU.
#pragma once
#include <stdint.h>

#include <vector>

namespace fft3d {

enum Op : int {
    OP_FORWARD = 0,       // C2C: forward; R2C plan: real -> half spectrum
    OP_INVERSE = 1,       // sign +1, scaled 1/N (R2C plan: half spectrum -> real)
    OP_BACKWARD = 2,      // adjoint of OP_FORWARD (unscaled)
    OP_POISSON = 3,       // R2C plan only: phi = irfftn(M .* rfftn(f))
    OP_POISSON_ADJ = 4,   // R2C plan only: adjoint of OP_POISSON
    OP_COUNT = 5,
};

enum Buf : int { BUF_IN = 0, BUF_OUT = 1, BUF_WS = 2 };

// Element order of a buffer between stages.  NATURAL: x fastest, then y,
// then z.  SWAP_YZ: x fastest, then z, then y (z-lines have the row stride
// of y-lines in the natural order).
enum Layout : int { LAY_NATURAL = 0, LAY_SWAP_YZ = 1 };

// How a C2C plan stages its passes.  IN_PLACE: every stage after the first
// works in place on the output (no workspace).  SWAP_YZ: the y stage writes a
// workspace in SWAP_YZ order and the z stage reads it back into the output,
// so no stage reads z-lines at the natural order's plane stride; the inverse
// then also runs x, y, z.  FUSED_XY (small planes, p1 == 1): one kernel does
// the x and y FFTs of whole planes in LDS, then the z stage works in place:
// two passes; the inverse runs z, then the planes.
enum Staging : int { STAGING_IN_PLACE = 0, STAGING_SWAP_YZ = 1, STAGING_FUSED_XY = 2 };

// The z axis of an R2C plan: periodic (DFT), or bounded by walls at both
// ends with the field at cell centres (the (Periodic, Periodic, Bounded)
// topology): homogeneous Neumann walls (cosine modes, DCT-II) or homogeneous
// Dirichlet walls (sine modes, DST-II).
enum ZBound : int { Z_PERIODIC = 0, Z_NEUMANN = 1, Z_DIRICHLET = 2 };

struct PlanDesc {
    int64_t nx, ny, nz;
    int dtype;  // DT_F32 / DT_F64
    int p1, p2;
    int r2c;
    int staging = STAGING_IN_PLACE;  // R2C: IN_PLACE or SWAP_YZ (forward only)
    int zbc = Z_PERIODIC;            // R2C plans: boundary of the z axis (ZBound)
    int64_t nxc() const { return r2c ? nx / 2 + 1 : nx; }  // complex x extent (row pitch of caller buffers)
    // row pitch (complex elements) of the workspace: the complex x extent
    // rounded up to 128 bytes, so workspace rows start on cache-line bounds
    int64_t wpitch() const
    {
        const int64_t per_line = dtype == 1 ? 8 : 16;  // complex values per 128 bytes
        return (nxc() + per_line - 1) / per_line * per_line;
    }
};

// Half-open index box over the complex array (x, y, z).
struct Box {
    int64_t lo[3], hi[3];
    int64_t count() const { return (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]); }
};

bool boxes_overlap(const Box& a, const Box& b);

struct Stage {
    int kind;      // KernelKind
    int axis;      // 0 = x, 1 = y, 2 = z
    int n;         // kernel length (real length for R2C/C2R)
    int conj;      // conjugate-sign transform
    int weight;    // adjoint weighting of interior half-spectrum bins
    double scale;  // output scale
    int src, dst;  // Buf ids
    int lay_src = LAY_NATURAL, lay_dst = LAY_NATURAL;
    int r2r = 0;   // K_R2R_Z: R2RMode
};

struct Task {
    int stage;
    Box box;
    std::vector<int> deps;   // producer tasks (previous stage, overlapping boxes)
    int stream = 0;          // placement
    double cost = 0;         // estimated cost (elements moved)
    std::vector<int> waits;  // producer tasks whose events this task's stream must wait on
};

struct Pipeline {
    std::vector<Stage> stages;
    std::vector<Task> tasks;  // issue order: a topological order (see issue_order)
    int nstreams = 1;
};

// Balanced split of [0, n) into p blocks: block i gets n/p elements plus one
// more while i < n % p.
void split_range(int64_t n, int p, int i, int64_t* lo, int64_t* hi);

// Pencil boxes of one stage, in tile order.  x-pencils split (y, z) over
// p1 x p2, y-pencils split (x, z), z-pencils split (x, y).
std::vector<Box> stage_boxes(const PlanDesc& d, int axis);

// Stages of an operation (empty if the op does not apply to the plan kind).
std::vector<Stage> op_stages(const PlanDesc& d, int op);

// Full task graph of an operation placed on nstreams streams.
Pipeline build_pipeline(const PlanDesc& d, int op, int nstreams);

// Reorder tasks for immediate dispatch: each tile right after its producers,
// deeper stages first (a topological order).
void issue_order(Pipeline& p);

// Locality-aware placement (paper Alg. 3 on one device): each tile goes to
// the least-loaded stream, ties broken by the number of its producers already
// on that stream; then the cross-stream event waits each tile needs.
void place_tasks(Pipeline& p, int nstreams);

// Forward roots W_n^m = exp(-2 pi i m / n), m < n, as interleaved doubles.
void twiddles_f64(int64_t n, double* out);
void twiddles_f32(int64_t n, float* out);  // round-to-nearest-even of the f64 table

// Per-pass table of the length-n Stockham kernel (layout in fft_lengths.hpp),
// built from the same FP64 roots (entries are copies of table values).
// Returns the number of complex entries; writes them if out is non-null.  ord
// 1: the table of the reverse radix order (radix_plan(n, 1)).
int64_t pass_twiddles_f64(int64_t n, double* out, int ord = 0);
int64_t pass_twiddles_f32(int64_t n, float* out, int ord = 0);

// ---------------------------------------------------------------- batches

// Placement of the transforms of a batch on nstreams streams (Alg. 3 with
// estimated costs): transforms in decreasing cost, each on the currently
// least-loaded stream.  Returns, per stream, the transforms in issue order.
std::vector<std::vector<int>> place_batch(const std::vector<double>& cost, int nstreams);

}  // namespace fft3d
