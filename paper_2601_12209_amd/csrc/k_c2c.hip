// Batched complex line FFTs for one pencil tile of one stage (x, y or z).
//
// Each stage of the pencil pipeline (paper Sec. III-A, Alg. 1) applies 1D FFTs
// along one axis to every line of a pencil tile.  On one GPU the paper's
// redistribution between stages becomes the access pattern of the next stage:
// a workgroup of the y or z stage reads lw neighbouring lines at once, so each
// wavefront load covers lw consecutive complex values of the x-fastest array,
// and the reorientation happens in registers and LDS (the LDS tile holds the
// lines element-major, line index fastest).  x-stage lines are contiguous, so
// there the lanes walk along one line instead.  Every stage reads and writes
// each element of the tile once.
#include "device_fft.hpp"
#include "kernels.hpp"
#include "stage_args.hpp"

namespace fft3d {

template <typename T, int N>
__global__ __launch_bounds__(1024) void k_c2c(StageArgs a)
{
    constexpr int TPL = radix_plan(N).tpl;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    const int t = threadIdx.x;
    int lw, tj;
    int64_t base;
    bool ok;
    LdsLine<T> L;
    if (a.strided) {
        lw = t % a.lw;
        tj = t / a.lw;
        const int64_t aa = (int64_t)blockIdx.x * a.lw + lw;
        ok = aa < a.A;
        base = a.off + aa + (int64_t)blockIdx.y * a.sb;
        L = LdsLine<T>{lds + lw, a.lw};
    } else {
        tj = t % TPL;
        lw = t / TPL;
        const int64_t l = (int64_t)blockIdx.x * a.lw + lw;
        ok = l < a.A * a.B;
        const int64_t aa = ok ? l % a.A : 0, bb = ok ? l / a.A : 0;
        base = a.off + aa * a.sa + bb * a.sb;
        L = LdsLine<T>{lds + lw * N, 1};
    }
    const cpx<T>* __restrict__ in = reinterpret_cast<const cpx<T>*>(a.in) + base;
    cpx<T>* __restrict__ out = reinterpret_cast<cpx<T>*>(a.out) + base;
    const cpx<T>* __restrict__ tw = reinterpret_cast<const cpx<T>*>(a.tw);
    const int64_t se = a.se;
    const bool cj = a.conj != 0;
    const T scale = (T)a.scale;
    auto load = [&](int e) -> cpx<T> {
        cpx<T> v = ok ? in[e * se] : cpx<T>{(T)0, (T)0};
        return cj ? conj(v) : v;
    };
    auto store = [&](int e, cpx<T> v) {
        if (cj) v = conj(v);
        if (ok) out[e * se] = v * scale;
    };
    fft_line<T, N>(L, tj, tw, load, store);
}

template <typename T, int N>
static hipError_t launch_c2c_n(const StageArgs& a, hipStream_t s)
{
    constexpr int TPL = radix_plan(N).tpl;
    const int threads = a.lw * TPL;
    const size_t lds = (size_t)a.lw * N * sizeof(cpx<T>);
    dim3 grid;
    if (a.strided) grid = dim3((unsigned)((a.A + a.lw - 1) / a.lw), (unsigned)a.B, 1);
    else grid = dim3((unsigned)((a.A * a.B + a.lw - 1) / a.lw), 1, 1);
    if (grid.x == 0 || grid.y == 0) return hipSuccess;
    static const hipError_t attr = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&k_c2c<T, N>), hipFuncAttributeMaxDynamicSharedMemorySize,
        (int)kMaxLdsBytes);
    (void)attr;
    hipLaunchKernelGGL((k_c2c<T, N>), grid, dim3(threads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_c2c(int n, int dtype, const StageArgs& a, hipStream_t s)
{
#define FFT3D_C2C_CASE(L)                                                               \
    case L:                                                                             \
        return dtype == DT_F64 ? launch_c2c_n<double, L>(a, s) : launch_c2c_n<float, L>(a, s);
    switch (n) {
        FFT3D_FOR_EACH_LENGTH(FFT3D_C2C_CASE)
    default:
        return hipErrorInvalidValue;
    }
#undef FFT3D_C2C_CASE
}

}  // namespace fft3d
