// Work-queue description of a batch of independent 3D FFTs run by one
// persistent kernel.  Plain C++: shared by the host planner and the kernel.
#pragma once
#include <stdint.h>

namespace fft3d {

// One (FFT, stage) segment of the queue: `items` consecutive queue entries,
// each a batch of lw lines of one stage of one FFT.  Line geometry as in
// StageArgs (line (a, b) starts at off + a*sa + b*sb, elements se apart).
struct BatchSeg {
    const void* in;
    void* out;
    const void* twp;  // per-pass twiddle table of length n
    int64_t first;    // queue index of the segment's first item
    int64_t items;
    int64_t A, B, off, sa, sb, se;
    int64_t blocks_a;  // strided: ceil(A / lw) item columns per b
    int n, strided, lw, conj;
    int dep;            // completion counter this segment waits on (-1: none)
    int done_idx;       // completion counter its items increment
    int64_t dep_count;  // value of counter `dep` that releases this segment
    float scale;
    int pad_;
};

// Control block: queue head, per-segment completion counters and an error
// flag live in device memory (zeroed before every launch by a fill kernel).
struct BatchCtl {
    int* head;
    int* done;
    int* error;  // set to 1 if a wait exceeds spin_limit; every workgroup then exits
    const BatchSeg* segs;
    int nsegs;
    int spin_limit;
    int64_t item_base;  // first queue index this launch processes
    int64_t total;      // one past the last queue index this launch processes
    int ignore_deps;    // 1: the caller orders the stages (one launch per stage)
    int pad_;
};

}  // namespace fft3d
