// Real-to-complex and complex-to-real x-stage kernels.
//
// R2C exploits Hermitian symmetry (paper Sec. V-B): a real line x of even
// length n is read as the complex line z[m] = x[2m] + i x[2m+1] of length
// h = n/2, transformed with the length-h kernel, and split in LDS:
//   E[k] = (Z[k] + conj Z[h-k]) / 2        (DFT of the even samples)
//   O[k] = (Z[k] - conj Z[h-k]) / (2i)     (DFT of the odd samples)
//   X[k] = E[k] + W_n^k O[k],  k = 0..h    (indices of Z taken mod h)
// C2R runs the same algebra backwards: from the half spectrum X[0..h],
//   Z'[k] = (X[k] + conj X[h-k]) + i W_n^-k (X[k] - conj X[h-k]),  k < h,
// whose length-h conjugate-sign DFT is the unscaled real line, interleaved
// (even samples in the real parts, odd in the imaginary parts).  The
// imaginary parts of X[0] and X[h] are dropped first, which is what a real
// result requires of a consistent half spectrum.
#include "device_fft.hpp"
#include "kernels.hpp"
#include "stage_args.hpp"

namespace fft3d {

// LDS slots of one line: H + 1 values, plus one slot per eight with `pad`
// (element e at e + (e / 8) * pad; without it the first pass's outputs, R
// consecutive values per thread, put the lanes of a line R slots apart, all
// on the same banks for R = 16).
template <int N>
__host__ __device__ constexpr int real_line_slots(int pad)
{
    return N / 2 + 1 + (pad ? N / 16 : 0);
}

// LDS bytes of a real-kernel launch: lw lines and the pass table of the
// length-H FFT.
template <typename T, int N>
constexpr size_t real_lds_bytes(int lw, int pad)
{
    constexpr int H = N / 2;
    return align16((size_t)lw * real_line_slots<N>(pad) * sizeof(cpx<T>)) + pass_table_bytes<T, H>();
}

template <typename T, int N>
__global__ __launch_bounds__(1024) void k_r2c_x(StageArgs a)
{
    constexpr int H = N / 2;
    constexpr int TPL = radix_plan(H).tpl;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    const int t = threadIdx.x;
    const int tj = t % TPL, lw = t / TPL;
    TileCoord tc;
    if (!tile_coord(a, tc)) return;
    const int64_t l0 = tc.bx * a.lw + lw;
    const bool ok = l0 < a.A * a.B;
    const int64_t l = ok ? l0 : a.A * a.B - 1;  // past the end: load the last line, store nothing
    const int64_t aa = l % a.A, bb = l / a.A;
    const cpx<T>* __restrict__ in =
        reinterpret_cast<const cpx<T>*>(a.in) + a.off + aa * a.sa + bb * a.sb;
    cpx<T>* __restrict__ out = reinterpret_cast<cpx<T>*>(a.out) + a.off_o + aa * a.sa_o + bb * a.sb_o;
    // W_N^k for the split step: a few KiB read by every workgroup, served by the caches
    const cpx<T>* __restrict__ tw = reinterpret_cast<const cpx<T>*>(a.tw);
    const int slots = real_line_slots<N>(a.pad);
    LdsView<cpx<T>> L{lds + lw * slots, 1, a.pad};
    LdsView<T> Ls{nullptr, 0, 0};
    cpx<T>* twl = reinterpret_cast<cpx<T>*>(smem_raw + align16((size_t)a.lw * slots * sizeof(cpx<T>)));
    stage_pass_twiddles<T, H>(twl, reinterpret_cast<const cpx<T>*>(a.twp), t, blockDim.x);
    auto load = [&](int e) -> cpx<T> { return in[e]; };
    auto store_lds = [&](int e, cpx<T> v) { L[e] = v; };
    fft_line<T, H, TPL, false, false, true>(L, Ls, tj, twl, load, store_lds);
    __syncthreads();
    const T half = (T)0.5;
    const T wgt = a.weight ? (T)2 : (T)1;
    const T scale = (T)a.scale;
    // bins k = tj + i*TPL (i < H/TPL) on every thread, bin H on thread 0
    auto bin = [&](int k) {
        const cpx<T> zk = L[k == H ? 0 : k];
        const cpx<T> zr = conj(L[k == 0 ? 0 : H - k]);
        const cpx<T> e = (zk + zr) * half;
        const cpx<T> o = mul_negi(zk - zr) * half;
        cpx<T> x = e + cmul(tw[k], o);
        if (k > 0 && k < H) x = x * wgt;
        if (ok) out[k] = x * scale;
    };
#pragma unroll
    for (int i = 0; i < H / TPL; ++i) bin(tj + i * TPL);
    if (tj == 0) bin(H);
}

template <typename T, int N>
__global__ __launch_bounds__(1024) void k_c2r_x(StageArgs a)
{
    constexpr int H = N / 2;
    constexpr int TPL = radix_plan(H).tpl;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    const int t = threadIdx.x;
    const int tj = t % TPL, lw = t / TPL;
    TileCoord tc;
    if (!tile_coord(a, tc)) return;
    const int64_t l0 = tc.bx * a.lw + lw;
    const bool ok = l0 < a.A * a.B;
    const int64_t l = ok ? l0 : a.A * a.B - 1;  // past the end: load the last line, store nothing
    const int64_t aa = l % a.A, bb = l / a.A;
    const cpx<T>* __restrict__ in =
        reinterpret_cast<const cpx<T>*>(a.in) + a.off + aa * a.sa + bb * a.sb;
    cpx<T>* __restrict__ out = reinterpret_cast<cpx<T>*>(a.out) + a.off_o + aa * a.sa_o + bb * a.sb_o;
    // W_N^k for the merge step: a few KiB read by every workgroup, served by the caches
    const cpx<T>* __restrict__ tw = reinterpret_cast<const cpx<T>*>(a.tw);
    const int slots = real_line_slots<N>(a.pad);
    LdsView<cpx<T>> L{lds + lw * slots, 1, a.pad};
    LdsView<T> Ls{nullptr, 0, 0};
    cpx<T>* twl = reinterpret_cast<cpx<T>*>(smem_raw + align16((size_t)a.lw * slots * sizeof(cpx<T>)));
    stage_pass_twiddles<T, H>(twl, reinterpret_cast<const cpx<T>*>(a.twp), t, blockDim.x);
    const T wgt = a.weight ? (T)0.5 : (T)1;
    // every load first (bins tj + i*TPL, and bin H on thread 0), then the LDS writes
    cpx<T> pre[H / TPL];
#pragma unroll
    for (int i = 0; i < H / TPL; ++i) pre[i] = in[tj + i * TPL];
    cpx<T> top = in[H];
#pragma unroll
    for (int i = 0; i < H / TPL; ++i) {
        const int k = tj + i * TPL;
        cpx<T> v = pre[i];
        if (k == 0) v.im = (T)0;
        else v = v * wgt;
        L[k] = v;
    }
    if (tj == 0) {
        top.im = (T)0;
        L[H] = top;
    }
    __syncthreads();
    // conjugate-sign DFT as conj(F(conj Z'))
    auto load = [&](int e) -> cpx<T> {
        const cpx<T> xe = L[e], xr = conj(L[H - e]);
        const cpx<T> s = xe + xr, d = xe - xr;
        const cpx<T> z = s + mul_i(cmul(conj(tw[e]), d));
        return conj(z);
    };
    const T scale = (T)a.scale;
    auto store = [&](int e, cpx<T> v) {
        if (ok) {
            if constexpr (sizeof(T) == 8) {  // FP64: a.nt asks for non-temporal stores
                if (a.nt) store_nt(&out[e], conj(v) * scale);
                else out[e] = conj(v) * scale;
            } else {
                out[e] = conj(v) * scale;
            }
        }
    };
    fft_line<T, H, TPL, false, true, false>(L, Ls, tj, twl, load, store);
}

template <typename T, int N>
static hipError_t launch_real_n(bool r2c, const StageArgs& a, hipStream_t s)
{
    if constexpr (N % 2 != 0) {
        return hipErrorInvalidValue;
    } else {
        constexpr int H = N / 2;
        constexpr int TPL = radix_plan(H).tpl;
        const int threads = a.lw * TPL;
        const size_t lds = real_lds_bytes<T, N>(a.lw, a.pad);
        const dim3 grid((unsigned)((a.A * a.B + a.lw - 1) / a.lw), 1, 1);
        if (grid.x == 0) return hipSuccess;
        if (threads > 1024 || lds > kMaxLdsBytes) return hipErrorInvalidConfiguration;
        const void* f = r2c ? reinterpret_cast<const void*>(&k_r2c_x<T, N>)
                            : reinterpret_cast<const void*>(&k_c2r_x<T, N>);
        return launch_stage_kernel(f, grid, dim3(threads), a, lds, s);
    }
}

static hipError_t launch_real(bool r2c, int n, int dtype, const StageArgs& a, hipStream_t s)
{
    // the half length must have a kernel of its own
#define FFT3D_REAL_CASE(L)                                                                \
    case 2 * L:                                                                           \
        return dtype == DT_F64 ? launch_real_n<double, 2 * L>(r2c, a, s)                  \
                               : launch_real_n<float, 2 * L>(r2c, a, s);
    switch (n) {
        FFT3D_FOR_EACH_LENGTH(FFT3D_REAL_CASE)
    default:
        return hipErrorInvalidValue;
    }
#undef FFT3D_REAL_CASE
}

hipError_t launch_r2c_x(int n, int dtype, const StageArgs& a, hipStream_t s)
{
    return launch_real(true, n, dtype, a, s);
}

hipError_t launch_c2r_x(int n, int dtype, const StageArgs& a, hipStream_t s)
{
    return launch_real(false, n, dtype, a, s);
}

}  // namespace fft3d
