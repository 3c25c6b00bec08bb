// Persistent kernel for a batch of independent, unevenly sized 3D FFTs.
//
// The paper schedules each FFT stage as tasks that run as soon as their
// inputs are ready, with no global barrier between stages (Sec. III-C,
// Sec. IV-D).  Here the tasks of many FFTs share one launch: every workgroup
// repeatedly takes the next item of a device-side queue (one item = a batch of
// lines of one stage of one FFT), waits until the previous stage of that FFT
// is complete, transforms its lines and counts the item as done.  The queue
// lists all first-stage items before any second-stage item (and so on), so an
// item only ever waits on items taken earlier by workgroups that are running:
// the kernel cannot deadlock, whatever the grid size.
//
// Stages of one FFT can be processed on different XCDs, whose L2 caches are
// separate, so completion is published with an agent-scope release and
// observed with an agent-scope acquire.  A wait that exceeds the spin limit
// sets the error flag; every workgroup then leaves the loop.
#include "batch_args.hpp"
#include "device_fft.hpp"
#include "kernels.hpp"

namespace fft3d {

constexpr int kBatchThreads = kBatchThreadsPerBlock;

template <int N>
__device__ void batch_item(const BatchSeg& s, int64_t local, unsigned char* smem)
{
    using T = float;
    constexpr int TPL = radix_plan(N).tpl;
    const int t = threadIdx.x;
    const int lw = s.lw;
    const bool active = t < lw * TPL;
    int line, tj;
    if (s.strided) {
        line = t % lw;
        tj = t / lw;
    } else {
        tj = t % TPL;
        line = t / TPL;
    }
    if (!active) {  // idle threads work on a scratch line slot; their results are dropped
        line = lw;
        tj = t % TPL;
    }
    int64_t base;
    bool ok;
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem);
    LdsView<cpx<T>> L;
    if (s.strided) {
        const int64_t ablk = local % s.blocks_a, b = local / s.blocks_a;
        const int64_t aa = ablk * lw + line;
        ok = active && aa < s.A;
        base = s.off + aa + b * s.sb;
        L = LdsView<cpx<T>>{lds + line, lw + 1, 0};
    } else {
        const int64_t l = local * lw + line;
        ok = active && l < s.A * s.B;
        const int64_t aa = ok ? l % s.A : 0, bb = ok ? l / s.A : 0;
        base = s.off + aa * s.sa + bb * s.sb;
        L = LdsView<cpx<T>>{lds + line * N, 1, 0};
    }
    LdsView<T> Ls{nullptr, 0, 0};
    cpx<T>* twl = reinterpret_cast<cpx<T>*>(smem + align16((size_t)(lw + 1) * N * sizeof(cpx<T>)));
    stage_pass_twiddles<T, N>(twl, reinterpret_cast<const cpx<T>*>(s.twp), t, kBatchThreads);
    const cpx<T>* __restrict__ in = reinterpret_cast<const cpx<T>*>(s.in) + base;
    cpx<T>* __restrict__ out = reinterpret_cast<cpx<T>*>(s.out) + base;
    const int64_t se = s.se;
    const bool cj = s.conj != 0;
    const T scale = s.scale;
    auto load = [&](int e) -> cpx<T> {
        cpx<T> v = ok ? in[e * se] : cpx<T>{0.f, 0.f};
        return cj ? conj(v) : v;
    };
    auto store = [&](int e, cpx<T> v) {
        if (cj) v = conj(v);
        if (ok) out[e * se] = v * scale;
    };
    // the first twiddle use comes after the first exchange barrier; with a
    // single pass there are no twiddles
    fft_line<T, N, TPL>(L, Ls, tj, twl, load, store);
}

__device__ int find_segment(const BatchCtl& c, int64_t item)
{
    int lo = 0, hi = c.nsegs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (c.segs[mid].first <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kBatchThreads) void k_batch(BatchCtl c)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int s_item;
    __shared__ int s_stop;
    for (;;) {
        if (threadIdx.x == 0) {
            s_item = __hip_atomic_fetch_add(c.head, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_stop = __hip_atomic_load(c.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        const int64_t item = c.item_base + s_item;
        if (item >= c.total || s_stop) break;
        const int si = find_segment(c, item);
        const BatchSeg& s = c.segs[si];
        if (s.dep >= 0 && !c.ignore_deps) {
            if (threadIdx.x == 0) {
                int spins = 0;
                while (__hip_atomic_load(&c.done[s.dep], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) <
                       s.dep_count) {
                    if (++spins > c.spin_limit ||
                        __hip_atomic_load(c.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        __hip_atomic_store(c.error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        s_stop = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
            __syncthreads();
            if (s_stop) break;
            // every wave observes the producers' writes
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        const int64_t local = item - s.first;
        switch (s.n) {
#define FFT3D_BATCH_CASE(L) \
    case L:                 \
        batch_item<L>(s, local, smem_raw); \
        break;
            FFT3D_FOR_EACH_BATCH_LENGTH(FFT3D_BATCH_CASE)
#undef FFT3D_BATCH_CASE
        default:
            break;
        }
        // publish: every thread's stores, then one count per item
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(&c.done[s.done_idx], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Zero the queue head, the counters and the error flag (a plain kernel, so a
// captured graph holds no memset node).
__global__ void k_batch_reset(int* head, int* done, int ndone, int* error)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        *head = 0;
        *error = 0;
    }
    if (i < ndone) done[i] = 0;
}

hipError_t launch_batch(const BatchCtl& c, int ndone, int grid, size_t lds, hipStream_t s)
{
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       (int)kMaxLdsBytes);
    (void)attr;
    const int rb = (ndone + 255) / 256;
    hipLaunchKernelGGL(k_batch_reset, dim3(rb < 1 ? 1 : rb), dim3(256), 0, s, c.head, c.done, ndone,
                       c.error);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (grid < 1 || c.total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch, dim3(grid), dim3(kBatchThreads), lds, s, c);
    return hipGetLastError();
}

int batch_max_blocks_per_cu(size_t lds)
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void*>(&k_batch),
                                                     kBatchThreads, lds) != hipSuccess)
        return 1;
    return blocks < 1 ? 1 : blocks;
}

}  // namespace fft3d
