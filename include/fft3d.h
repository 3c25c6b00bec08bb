/*
 * fft3d -- pencil-decomposed 3D FFT for one AMD Instinct MI355X (gfx950).
 *
 * The transform is the 3D DFT of the paper's Sec. III-A,
 *   X[kx,ky,kz] = sum_{x,y,z} A[x,y,z] exp(-2 pi i (kx x/Nx + ky y/Ny + kz z/Nz)),
 * evaluated as three stages of batched 1D FFTs (x, then y, then z; the inverse
 * mirrors the order, Sec. IV-A), each stage cut into P1 x P2 pencil tiles that
 * are issued as tasks on HIP streams with per-tile dependencies (Alg. 1 and
 * the data-dependency scheduler of Sec. IV-D; placement as in Alg. 3).
 *
 * Layout of every array: element (x, y, z) at index x + Nx*(y + Ny*z), x
 * fastest (a C array of shape [Nz][Ny][Nx]).  Complex values are interleaved
 * (re, im) pairs of float (FFT3D_C64) or double (FFT3D_C128).  A real-to-
 * complex plan maps a real Nx x Ny x Nz array to the half spectrum of
 * (Nx/2 + 1) x Ny x Nz complex values (x halved, Sec. V-B's Hermitian
 * symmetry), and back.
 *
 * Pointers named in/out/f/phi are DEVICE pointers owned by the caller.  The
 * `stream` argument is a hipStream_t (NULL: the default stream); all work is
 * enqueued after the work already on that stream and completes before work
 * enqueued on it later.  No call blocks the host on the GPU except
 * fft3d_plan, fft3d_destroy and the setters that free or rebuild plan memory.
 * Calls on one plan are serialised on the host (a per-plan lock), and a call
 * on a different stream than the plan's previous call first waits for that
 * call's completion on the device (the plan's workspace is shared), so one
 * plan may be used from several host threads and streams; its calls then run
 * one after another.  A call into a stream that is being captured records its
 * kernels in order on that stream (no internal streams, no waits on earlier
 * calls): the caller orders replays of the captured graph against other uses
 * of the plan.
 *
 * Errors: every call returns an fft3d_status.  Argument errors are detected
 * before any work is enqueued.  An asynchronous GPU fault surfaces as
 * FFT3D_ERR_HIP from a later call.  fft3d_last_error() gives a text detail for
 * the calling thread's most recent failure.
 */
#ifndef FFT3D_H
#define FFT3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fft3d_plan_s* fft3d_plan_t;

typedef enum {
    FFT3D_C64 = 0,  /* complex64 (real side: float32) */
    FFT3D_C128 = 1  /* complex128 (real side: float64) */
} fft3d_dtype;

typedef enum {
    FFT3D_OK = 0,
    FFT3D_ERR_INVALID_ARG = -1,      /* null pointer, bad dtype, grid, stream count */
    FFT3D_ERR_UNSUPPORTED_SIZE = -2, /* a length without a compiled kernel */
    FFT3D_ERR_ALLOC = -3,            /* device allocation failed */
    FFT3D_ERR_HIP = -4,              /* HIP runtime error (incl. asynchronous faults) */
    FFT3D_ERR_ALIAS = -5,            /* in and out overlap in a way the operation forbids */
    FFT3D_ERR_WORKSPACE = -6,        /* caller workspace too small */
    FFT3D_ERR_WRONG_PLAN = -7        /* operation needs the other plan kind (C2C vs R2C) */
} fft3d_status;

/*
 * Create a plan for an Nx x Ny x Nz transform.
 *   dtype  FFT3D_C64 or FFT3D_C128.
 *   p1,p2  pencil grid: x-pencils are split P1 ways along y and P2 ways along
 *          z, y-pencils P1 along x and P2 along z, z-pencils P1 along x and P2
 *          along y (balanced blocks).  1 <= p1 <= min(Ny, Nxc), 1 <= p2 <=
 *          min(Nz, Ny), Nxc = Nx (C2C) or Nx/2+1 (R2C).
 *   r2c    0: complex-to-complex plan; 1: real-to-complex plan (Nx even).
 * Each of Nx, Ny, Nz must be a supported length (fft3d_length_supported).
 * Allocates the plan's twiddle tables, its streams and events, and a
 * workspace for R2C plans (half spectrum) and for large C2C plans (see
 * fft3d_set_staging); fft3d_set_workspace can replace it.
 */
fft3d_status fft3d_plan(fft3d_plan_t* plan, int64_t nx, int64_t ny, int64_t nz, int dtype,
                        int p1, int p2, int r2c);

/*
 * Create a real-to-complex plan whose z axis is bounded instead of periodic:
 * the (Periodic, Periodic, Bounded) topology of the paper's Poisson solver
 * (Sec. VI-B), with real-to-real transforms along z beside the DFTs along x
 * and y (Sec. V-B's transform types).  The field has Nz cells between two
 * walls, values at the cell centres; zbc selects the walls:
 *   FFT3D_Z_NEUMANN    homogeneous Neumann (cosine modes): DCT-II along z,
 *                      Y_k = 2 sum_j x_j cos(pi (2j+1) k / 2Nz), k = 0..Nz-1
 *   FFT3D_Z_DIRICHLET  homogeneous Dirichlet (sine modes): DST-II along z,
 *                      Y_k = 2 sum_j x_j sin(pi (2j+1) (k+1) / 2Nz)
 * Arguments otherwise as fft3d_plan with r2c = 1 (Nx even; Nx, Nx/2, Ny, Nz
 * supported lengths).  The operations keep their meaning:
 *   fft3d_forward   real Nx*Ny*Nz -> (Nx/2+1)*Ny*Nz complex: DFT along x (half
 *                   spectrum) and y, then the DCT-II / DST-II along z, unscaled;
 *   fft3d_inverse   its inverse: DCT-III / DST-III along z divided by 2 Nz,
 *                   inverse DFT along y (1/Ny) and x (1/Nx, imaginary parts of
 *                   the kx = 0 and Nx/2 bins ignored);
 *   fft3d_backward  the adjoint of fft3d_forward (transposed DCT-II / DST-II,
 *                   unscaled conjugate DFT along y, adjoint of the R2C step);
 *   fft3d_poisson   phi = inverse(M .* forward(f)), M = -1/|k|^2 and 0 for the
 *                   zero wavenumber, on the box (0, 2 pi)^2 x (0, pi): integer
 *                   kx, ky as for periodic plans, kz = k (Neumann) or k + 1
 *                   (Dirichlet, so M is never 0); the z stage runs the DCT
 *                   (DST), the multiplier and the inverse in one kernel;
 *   fft3d_poisson_backward  its adjoint (the solve is self-adjoint).
 * Staging is always FFT3D_STAGING_IN_PLACE (the x and y stages run in the
 * plan workspace).  zbc other than the two values: FFT3D_ERR_INVALID_ARG.
 */
#define FFT3D_Z_NEUMANN 1
#define FFT3D_Z_DIRICHLET 2
fft3d_status fft3d_plan_ppb(fft3d_plan_t* plan, int64_t nx, int64_t ny, int64_t nz, int dtype,
                            int p1, int p2, int zbc);

/* Release everything the plan allocated (not caller buffers), after waiting
 * for the plan's last call to finish on the device.  NULL is accepted. */
fft3d_status fft3d_destroy(fft3d_plan_t plan);

/*
 * Forward transform (Sec. III-A definition: exponent sign -1, unscaled).
 * C2C plan: in, out = Nx*Ny*Nz complex; in == out (in place) is allowed,
 *           partial overlap is FFT3D_ERR_ALIAS.
 * R2C plan: in = Nx*Ny*Nz reals, out = (Nx/2+1)*Ny*Nz complex; no overlap.
 * `in` is never written (except in place).
 */
fft3d_status fft3d_forward(fft3d_plan_t plan, const void* in, void* out, void* stream);

/*
 * Inverse transform: exponent sign +1, scaled by 1/(Nx*Ny*Nz), stages z, y, x
 * (Sec. IV-A; x, y, z with FFT3D_STAGING_SWAP_YZ).  C2C: same buffer rules as
 * forward.  R2C plan: in = half
 * spectrum (left intact; the imaginary parts of its kx = 0 and kx = Nx/2 bins
 * are ignored), out = real array, no overlap; uses the plan workspace.
 */
fft3d_status fft3d_inverse(fft3d_plan_t plan, const void* in, void* out, void* stream);

/*
 * Adjoint of fft3d_forward (the vector-Jacobian product of the forward map).
 * C2C: the unscaled sign +1 transform F^H.  R2C: the adjoint of the real-to-
 * complex map, i.e. the unscaled complex-to-real transform of the half
 * spectrum with its interior bins (0 < kx < Nx/2) halved.  Buffer rules as
 * fft3d_inverse.
 */
fft3d_status fft3d_backward(fft3d_plan_t plan, const void* in, void* out, void* stream);

/*
 * fft3d_forward for callers that cannot allocate device memory or create
 * HIP objects while it runs: code under stream capture into a hipGraph,
 * tight serving or time-stepping loops, and harnesses that forbid
 * allocation.  Same transform, arguments and buffer rules as fft3d_forward
 * (the plan is created beforehand); the result is bitwise that of
 * fft3d_forward (the same kernels on the same tiles).  Differences:
 *   - the workspace (R2C plans; C2C plans staged FFT3D_STAGING_SWAP_YZ) is a
 *     static device array of the library, 256 MiB per GPU (FFT3D_SCRATCH_BYTES),
 *     allocated when the library's code is loaded on that GPU and held until
 *     the process ends; a plan whose workspace is larger (fft3d_workspace_bytes)
 *     gets FFT3D_ERR_WORKSPACE with nothing enqueued.  The plan's own
 *     workspace is not touched.
 *   - every tile is enqueued in dependency order on `stream` itself: no
 *     internal streams, events or graphs, no hipMalloc/hipFree.  The first
 *     call on a GPU looks the scratch address up (hipGetSymbolAddress) and
 *     caches it.
 *   - all calls of this function on one GPU share that GPU's scratch, and it
 *     keeps whatever the last call left there (every call writes the
 *     workspace before reading it, so nothing needs clearing).  Calls whose
 *     execution overlaps on one GPU (different streams or host threads
 *     without ordering between them) race on the scratch and give wrong
 *     results: order them, e.g. on one stream.  Each process has its own
 *     copy of the array.
 */
#define FFT3D_SCRATCH_BYTES ((size_t)256 << 20)
fft3d_status fft3d_forward_noalloc(fft3d_plan_t plan, const void* in, void* out, void* stream);

/*
 * Spectral Poisson solve on a periodic box of side 2 pi (R2C plans only; the
 * paper's Poisson application, Sec. VI-B, (Periodic, Periodic, Periodic)):
 *   phi = irfftn( M .* rfftn(f) ),  M(k) = -1/|k|^2,  M(0) = 0,
 * with integer wavenumbers k_j = j for j <= n/2 and j - n otherwise.  The
 * z stage runs forward FFT, multiplier and inverse FFT in one kernel.  f and
 * phi are real Nx*Ny*Nz arrays; f == phi is allowed, partial overlap is not.
 * Uses the plan workspace.
 */
fft3d_status fft3d_poisson(fft3d_plan_t plan, const void* f, void* phi, void* stream);

/*
 * Backward of fft3d_poisson (its adjoint: the gradient of sum(phi * g) with
 * respect to f, given g = gphi): the adjoint of every stage of the solve,
 * applied in reverse order.  Same buffer rules as fft3d_poisson.
 */
fft3d_status fft3d_poisson_backward(fft3d_plan_t plan, const void* gphi, void* gf, void* stream);

/* Bytes of the plan's workspace: R2C plans (Nx/2+1)*Ny*Nz complex values,
 * C2C plans Nx*Ny*Nz complex values with FFT3D_STAGING_SWAP_YZ, else 0. */
size_t fft3d_workspace_bytes(fft3d_plan_t plan);

/*
 * Replace the plan-owned workspace by a caller buffer of at least
 * fft3d_workspace_bytes(plan) bytes (device memory, 256-byte aligned), which
 * the caller keeps alive while the plan uses it.  NULL restores a plan-owned
 * workspace.  Too small -> FFT3D_ERR_WORKSPACE.
 */
fft3d_status fft3d_set_workspace(fft3d_plan_t plan, void* ws, size_t bytes);

/*
 * How a C2C plan stages its three passes (Sec. III-A's redistributions
 * between the stages, done on one device by where each stage writes).
 *   FFT3D_STAGING_IN_PLACE: the x stage writes `out`, the y and z stages
 *     work in place on it; no workspace.  Inverse stages run z, y, x.
 *   FFT3D_STAGING_SWAP_YZ: the y stage writes a plan workspace of Nx*Ny*Nz
 *     complex values with y and z swapped (x fastest, then z, then y) and the
 *     z stage reads it back into `out`, so z-lines are read with the row
 *     stride of y-lines instead of the plane stride; forward, inverse and
 *     backward all run x, y, z (the same transform up to rounding order).
 *   FFT3D_STAGING_FUSED_XY: one kernel loads each z-plane (Nx x Ny) into LDS
 *     and runs its x and y FFTs there, then the z stage works in place on
 *     `out`: two passes over memory instead of three, no workspace (the slab
 *     form of Sec. III-A: two local transforms, then the third).  Its lines
 *     run the same arithmetic as the x and y stages, so the forward is bitwise
 *     equal to IN_PLACE.  Only for
 *     the planes with a compiled kernel that fit in 160 KiB of LDS (complex64:
 *     squares 8, 16, 24, 32, 48, 64, 96, 128 and 100 x 120, 80 x 160;
 *     complex128: the squares up to 96) and p1 == 1 (else
 *     FFT3D_ERR_UNSUPPORTED_SIZE).  Inverse stages run z, then planes.
 * Default: SWAP_YZ for C2C plans of at least 512 MiB with Ny, Nz > 1 (the
 * workspace is allocated by fft3d_plan; if that fails the plan stages in
 * place), else FUSED_XY where available, else IN_PLACE.  Switching frees or allocates the owned
 * workspace (fft3d_set_workspace can then supply a caller buffer) and waits
 * for the device.  R2C plans always hold their workspace and accept
 * IN_PLACE (the x and y stages of the forward run in the workspace, z writes
 * `out`) and SWAP_YZ (forward only: x writes `out`, y writes the workspace
 * with y and z swapped, z reads it back into `out`; bitwise the same result);
 * their inverse, backward and Poisson stages do not change.  Default for R2C:
 * SWAP_YZ when the half spectrum takes at least 512 MiB and less than 2 GiB
 * (faster at 512^3, slower at 1024^3 on MI355X), else IN_PLACE.
 * FUSED_XY on an R2C plan -> FFT3D_ERR_WRONG_PLAN.
 */
#define FFT3D_STAGING_IN_PLACE 0
#define FFT3D_STAGING_SWAP_YZ 1
#define FFT3D_STAGING_FUSED_XY 2
fft3d_status fft3d_set_staging(fft3d_plan_t plan, int staging);

/* The plan's current staging (one of the FFT3D_STAGING_* values), or -1 for
 * a NULL plan. */
int fft3d_get_staging(fft3d_plan_t plan);

/*
 * Number of internal HIP streams the tiles are placed on (1..16; default 4).
 * The streams are created by the first call that needs them.  With 1 stream,
 * or a 1x1 pencil grid (one tile per stage), every tile is enqueued directly
 * on the caller's stream in dependency order.
 */
fft3d_status fft3d_set_streams(fft3d_plan_t plan, int nstreams);

/*
 * How a plan with more than one tile per stage issues its tiles (the tasks
 * of Alg. 1, Sec. IV-D):
 *   FFT3D_ISSUE_TILES   one kernel launch per tile, placed on the plan's
 *                       streams (Alg. 3 placement) with one event wait per
 *                       producer tile on another stream, forked from and
 *                       joined back to the caller's stream: a tile starts as
 *                       soon as the tiles it reads are done;
 *   FFT3D_ISSUE_STAGES  (default) the tiles of each stage as one launch on the
 *                       caller's stream: every workgroup finds its tile in a
 *                       table the plan keeps on the device, so all tiles of a
 *                       stage are ready together (the task graph with every
 *                       stage's tiles released at once).  Stages whose tiles
 *                       need different kernels or launch shapes fall back to
 *                       one launch per tile, in order.  The first call of an
 *                       operation uploads its tables (a blocking copy).
 * Results are bitwise identical.  A call into a stream the caller is
 * capturing issues its tiles in order on that stream in either mode.
 */
#define FFT3D_ISSUE_TILES 0
#define FFT3D_ISSUE_STAGES 1
fft3d_status fft3d_set_issue(fft3d_plan_t plan, int mode);
/* The plan's issue mode, or -1 for a NULL plan. */
int fft3d_get_issue(fft3d_plan_t plan);

/*
 * Override the launch shape of the stage kernels along one axis (0 = x,
 * 1 = y, 2 = z) of this plan: lw lines per workgroup (a power of two; 0
 * restores the default shape), tdiv divides the threads that cooperate on one
 * line (each then takes tdiv times more butterflies), split = 1 exchanges real
 * and imaginary parts through LDS one after the other (half the LDS), pad = 1
 * pads contiguous LDS lines against bank conflicts.  Stage kernels of that
 * axis that cannot run with the shape (thread or LDS limits, no such kernel
 * variant, e.g. the fused Poisson z stage) keep their default shape;
 * FFT3D_ERR_INVALID_ARG if none of them can.  Used by the autotuner; results
 * do not depend on the shape (the same arithmetic, bitwise).
 */
fft3d_status fft3d_set_stage_config(fft3d_plan_t plan, int axis, int lw, int tdiv, int split, int pad);

/*
 * Radix order of the complex line kernels along one axis (0 = x, 1 = y,
 * 2 = z): 0 the default plan of the length (fft3d_query_radix_plan), 1 the
 * same radices in the reverse pass order.  The reverse-order kernels take
 * one thread per butterfly, the plain exchange and plain accesses, so on an
 * axis in order 1 the launch shape drops its threads-per-line divisor and
 * split exchange (and halves its lines until the threads fit).  The
 * autotuner's third dimension besides the launch shape and the staging.
 * Unlike the launch shape, the order changes the arithmetic: results agree
 * with order 0 to rounding, not bitwise.  FFT3D_ERR_INVALID_ARG for order
 * 1 when no C2C line kernel of that axis has a distinct reverse order (a
 * single pass, a palindrome of radices, or real-to-complex x kernels).
 * fft3d_get_radix_order returns the axis's order, or -1.
 */
fft3d_status fft3d_set_radix_order(fft3d_plan_t plan, int axis, int order);
int fft3d_get_radix_order(fft3d_plan_t plan, int axis);

/*
 * Per-stage timing (tracing).  While enabled, every call on the plan records
 * a timing event on the caller's stream before its first stage and after each
 * stage; the tiles of a stage are forked from and joined back onto the
 * caller's stream, so stages do not overlap while timing is on.
 * fft3d_stage_times waits for the most recent call to finish and writes the
 * elapsed milliseconds of each of its stages to ms[0..k); it returns k, or -1
 * if no timed call was made or cap < k.
 */
fft3d_status fft3d_set_timing(fft3d_plan_t plan, int enable);
int fft3d_stage_times(fft3d_plan_t plan, float* ms, int cap);

/* Text for a status code; and the calling thread's last failure detail. */
const char* fft3d_status_string(int status);
const char* fft3d_last_error(void);

/* --------------------------------------------------------- batches
 * Many independent 3D transforms of (possibly) different sizes (the paper's
 * dynamically scheduled FFT tasks over uneven work, Sec. III-C and IV-D).  A
 * call issues, stage by stage, one grouped launch per distinct shape, largest
 * shape first (the order of Alg. 3's placement): the tiles of that stage of
 * every transform of the shape in one kernel launch, each workgroup finding
 * its transform's buffers and tile in a device table.  Each shape's chain of
 * stage launches runs on one of the batch's own streams (4 by default,
 * fft3d_batch_set_streams), shapes placed by Alg. 3's rule on their total
 * cost, forked from and joined back to the caller's stream, so transforms of
 * different shapes overlap.  The tables of a pointer set are built on its
 * first call (a blocking upload) and cached (at most 8 sets).  A call into a
 * stream the caller is capturing issues, in order on that stream, the grouped
 * launches of a pointer set that an earlier call has built (their tables are
 * then kept until the batch is destroyed, since the caller's graph refers to
 * them), and otherwise the transforms one after another. */
typedef struct fft3d_batch_s* fft3d_batch_t;

/* dims holds count triples (nx, ny, nz), each a shape fft3d_plan accepts;
 * dtype FFT3D_C64 or FFT3D_C128.  Creates one plan per distinct shape. */
fft3d_status fft3d_plan_batch(fft3d_batch_t* plan, int count, const int64_t* dims, int dtype);

/* Forward (sign -1, unscaled) / inverse (sign +1, 1/N per transform) of every
 * transform: in[f], out[f] are device pointers to Nx*Ny*Nz complex values (x
 * fastest); in[f] == out[f] is allowed, a partial overlap is FFT3D_ERR_ALIAS,
 * and so is any overlap between buffers of different transforms. */
fft3d_status fft3d_forward_batch(fft3d_batch_t plan, const void* const* in, void* const* out, void* stream);
fft3d_status fft3d_inverse_batch(fft3d_batch_t plan, const void* const* in, void* const* out, void* stream);

/* Launch shape of one stage of the transforms of one shape (arguments as
 * fft3d_set_stage_config); waits for the last call and drops the cached
 * launch tables.  Used by the autotuner; results do not depend on it. */
fft3d_status fft3d_batch_set_stage_config(fft3d_batch_t plan, int64_t nx, int64_t ny, int64_t nz, int axis,
                                          int lw, int tdiv, int split, int pad);

/* Radix order of one axis of the transforms of one shape (arguments as
 * fft3d_set_radix_order); waits for the last call and drops the cached
 * launch tables. */
fft3d_status fft3d_batch_set_radix_order(fft3d_batch_t plan, int64_t nx, int64_t ny, int64_t nz, int axis,
                                         int order);

/* Staging of the transforms of one shape: FFT3D_STAGING_IN_PLACE or
 * FFT3D_STAGING_FUSED_XY (the default where a fused kernel fits the plane;
 * UNSUPPORTED_SIZE where none does); a workspace staging is
 * FFT3D_ERR_INVALID_ARG, since transforms of one shape share their plan.
 * Waits for the last call and drops the cached launch tables; results are
 * bitwise the same in both stagings. */
fft3d_status fft3d_batch_set_staging(fft3d_batch_t plan, int64_t nx, int64_t ny, int64_t nz, int staging);
/* Streams the batch's shapes run on concurrently (1..16, default 4; 1 runs
 * every shape's launches in order on the caller's stream).  Waits for the last
 * call and drops the cached launch tables; results are bitwise the same. */
fft3d_status fft3d_batch_set_streams(fft3d_batch_t plan, int nstreams);

/* Staging of the transforms of one shape, or -1 (NULL plan, or no transform
 * of that shape). */
int fft3d_batch_get_staging(fft3d_batch_t plan, int64_t nx, int64_t ny, int64_t nz);

fft3d_status fft3d_batch_destroy(fft3d_batch_t plan);

/* Host-only: Alg. 3's placement of a batch on nstreams streams (the batch's
 * issue order is the placement on one stream) as int64 records
 * [nstreams] then per stream [n, transform indices in issue order...].
 * Returns the number of values needed; writes them if cap is large enough;
 * -1 on invalid arguments. */
int64_t fft3d_query_batch_placement(int count, const int64_t* dims, int nstreams, int64_t* out, int64_t cap);

/* ----------------------------------------------------- host-side queries
 * These run on the host only and need no GPU; tests use them to check the
 * planner. */

/* 1 if n has a compiled kernel, else 0. */
int fft3d_length_supported(int64_t n);

/* Radix plan of length n: out[0] = number of passes np, out[1..np] the
 * radices, out[np+1] threads per line.  Returns the count written, or -1 for
 * an unsupported length or cap too small. */
int fft3d_query_radix_plan(int64_t n, int* out, int cap);

/* Forward twiddle table W_n^m = exp(-2 pi i m/n), m < n, interleaved (re, im)
 * in the plan precision (float for FFT3D_C64, double for FFT3D_C128).
 * out holds 2n values of that type. */
fft3d_status fft3d_query_twiddles(int64_t n, int dtype, void* out);

/*
 * Task graph of an operation (0 forward, 1 inverse, 2 backward, 3 Poisson,
 * 4 Poisson adjoint) for the given plan parameters (staging as in
 * fft3d_set_staging) and stream count, written
 * as int64 records:
 *   header: [ntasks, nstages]
 *   per stage: [kind, axis, n, conj, weight, src, dst, scale, lay_src, lay_dst]
 *     kind 0 C2C, 1 R2C along x, 2 C2R along x, 3 fused Poisson z stage;
 *     axis 0..2; n the line length; conj 1 for the sign +1 transform; weight 1
 *     for the adjoint bin weighting; src/dst 0 = in, 1 = out, 2 = workspace;
 *     scale the output factor as the bit pattern of an IEEE double; lay_src,
 *     lay_dst the element order read / written (0 natural, 1 y and z swapped);
 *     kind 4 is the fused x-y plane stage (x and y FFTs of whole planes)
 *   per task:  [stage, x0, x1, y0, y1, z0, z1, stream, ndeps, deps..., nwaits, waits...]
 * Boxes are half-open ranges over the complex array.  Returns the number of
 * int64 values needed; writes them only if cap is large enough.  Negative on
 * invalid arguments.
 */
int64_t fft3d_query_pipeline(int64_t nx, int64_t ny, int64_t nz, int p1, int p2, int r2c, int staging, int op,
                             int nstreams, int64_t* out, int64_t cap);

/*
 * Default launch configuration of every task of the same task graph (plan
 * precision dtype, one stream, no stage overrides), in task order, as int64
 * records after a header [ntasks]:
 *   [lw, tdiv, split, pad, strided, align, xcd, nt]
 * lw lines per workgroup; tdiv threads-per-line divisor; split re/im LDS
 * exchange; pad padded contiguous LDS lines; strided 1 when the lanes of a
 * wavefront walk neighbouring lines; align > 1: row tiles shifted so stored
 * segments start on multiples of align elements; xcd 1: XCD-grouped tile
 * order; nt cache policy (0 plain, 1 non-temporal stores, 2 non-temporal
 * loads and stores).  Host-side only (no device work).  Returns the number of
 * int64 values needed, writes them only if cap is large enough, negative on
 * invalid arguments.
 */
int64_t fft3d_query_launches(int64_t nx, int64_t ny, int64_t nz, int dtype, int p1, int p2, int r2c, int staging,
                             int op, int64_t* out, int64_t cap);

#ifdef __cplusplus
}
#endif

#endif /* FFT3D_H */
