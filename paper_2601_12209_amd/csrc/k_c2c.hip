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
//
// Variants: TDIV divides the threads per line (more butterflies per thread, so
// more lines per workgroup and longer row segments); SPLIT halves the LDS tile
// by exchanging real and imaginary parts one after the other; NT marks the
// global stores (NT >= 1) and loads (NT == 2) non-temporal, so the streamed
// tile does not displace reusable lines from the caches (every element is read
// and written once per stage).
#include "device_fft.hpp"
#include "kernels.hpp"
#include "stage_args.hpp"

namespace fft3d {

template <typename T, int N, int TDIV, bool SPLIT, int NT, int ORD>
__global__ __launch_bounds__(1024) void k_c2c(StageArgs a)
{
    constexpr int TPL = radix_plan(N).tpl / TDIV;
    TileCoord tc;
    if (!tile_coord(a, tc)) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    T* ldsr = reinterpret_cast<T*>(smem_raw);
    const int t = threadIdx.x;
    int tj;
    int64_t base, base_o;
    bool ok;
    LdsView<cpx<T>> L;
    LdsView<T> Ls;
    // Lanes past the last line load a valid line (the last one) and never
    // store: the loads then need no branch, so all of them are in flight at once.
    if (a.strided) {
        const int lw = t % a.lw;
        tj = t / a.lw;
        int64_t bx = tc.bx, by = tc.by;
        if (a.xcd) {  // host guarantees the tile's gx * gy % 8 == 0
            const int64_t lin = bx + by * tc.gx, per = tc.gx * tc.gy / 8;
            const int64_t tile = (lin % 8) * per + lin / 8;
            bx = tile % tc.gx;
            by = tile / tc.gx;
        }
        // with a.align, the tiles of this row start `shift` lines early so that
        // every output segment covers whole cache lines
        const int64_t shift = a.align > 1 ? (a.off_o + by * a.sb_o) % a.align : 0;
        const int64_t aa0 = bx * a.lw + lw - shift;
        ok = aa0 >= 0 && aa0 < a.A;
        const int64_t aa = aa0 < 0 ? 0 : (aa0 < a.A ? aa0 : a.A - 1);
        base = a.off + aa + by * a.sb;
        base_o = a.off_o + aa + by * a.sb_o;
        L = LdsView<cpx<T>>{lds + lw, a.lw, 0};
        Ls = LdsView<T>{ldsr + lw, a.lw, 0};
    } else {
        tj = t % TPL;
        const int lw = t / TPL;
        const int64_t l0 = tc.bx * a.lw + lw;
        ok = l0 < a.A * a.B;
        const int64_t l = ok ? l0 : a.A * a.B - 1;
        const int64_t aa = l % a.A, bb = l / a.A;
        base = a.off + aa * a.sa + bb * a.sb;
        base_o = a.off_o + aa * a.sa_o + bb * a.sb_o;
        const int stride = N + a.pad * (N / 8);
        L = LdsView<cpx<T>>{lds + lw * stride, 1, a.pad};
        Ls = LdsView<T>{ldsr + lw * stride, 1, a.pad};
    }
    const size_t line = a.strided ? (size_t)N : (size_t)(N + a.pad * (N / 8));
    cpx<T>* twl = reinterpret_cast<cpx<T>*>(smem_raw + align16((size_t)a.lw * line * (SPLIT ? sizeof(T) : sizeof(cpx<T>))));
    stage_pass_twiddles<T, N, ORD>(twl, reinterpret_cast<const cpx<T>*>(a.twp), t, blockDim.x);
    const int64_t se = a.se, se_o = a.se_o;
    // element e of this thread's line sits (e - tj) * se past the thread base;
    // e - tj is a compile-time constant at every call site
    const cpx<T>* __restrict__ in = reinterpret_cast<const cpx<T>*>(a.in) + base + tj * se;
    cpx<T>* __restrict__ out = reinterpret_cast<cpx<T>*>(a.out) + base_o + tj * se_o;
    const bool cj = a.conj != 0;
    const T scale = (T)a.scale;
    auto load = [&](int e) -> cpx<T> {
        cpx<T> v;
        if constexpr (NT == 2) v = load_nt(&in[(e - tj) * se]);
        else v = in[(e - tj) * se];
        return cj ? conj(v) : v;
    };
    auto store = [&](int e, cpx<T> v) {
        if (cj) v = conj(v);
        if (ok) {
            if constexpr (NT >= 1) store_nt(&out[(e - tj) * se_o], v * scale);
            else out[(e - tj) * se_o] = v * scale;
        }
    };
    fft_line<T, N, TPL, SPLIT, false, false, ORD>(L, Ls, tj, twl, load, store);
}

template <typename T, int N, int TDIV, bool SPLIT, int NT = 0, int ORD = 0>
static hipError_t launch_c2c_v(const StageArgs& a, hipStream_t s)
{
    constexpr int TPL = radix_plan(N).tpl / TDIV;
    const int threads = a.lw * TPL;
    const size_t elem = SPLIT ? sizeof(T) : sizeof(cpx<T>);
    const size_t line = a.strided ? (size_t)N : (size_t)(N + a.pad * (N / 8));
    const size_t lds = align16((size_t)a.lw * line * elem) + pass_table_bytes<T, N, ORD>();
    dim3 grid;
    if (a.strided) grid = dim3((unsigned)((a.A + (a.align > 1 ? a.align - 1 : 0) + a.lw - 1) / a.lw), (unsigned)a.B, 1);
    else grid = dim3((unsigned)((a.A * a.B + a.lw - 1) / a.lw), 1, 1);
    if (grid.x == 0 || grid.y == 0) return hipSuccess;
    if (threads > 1024 || lds > kMaxLdsBytes) return hipErrorInvalidConfiguration;
    StageArgs arg = a;
    // the XCD-grouped tile order needs whole groups of 8 workgroups
    if (!a.strided || ((uint64_t)grid.x * grid.y) % 8 != 0) arg.xcd = 0;
    return launch_stage_kernel(reinterpret_cast<const void*>(&k_c2c<T, N, TDIV, SPLIT, NT, ORD>), grid,
                               dim3(threads), arg, lds, s);
}

// Lengths that also get the TDIV = 2, 4 and SPLIT variants: the powers of
// two, and 840 (the paper's largest GPU grid), whose radix-15 plan has 56
// threads per line.  (With the earlier 105 threads per line a TDIV 3 variant
// for 840 spilled and ran slower than 8-line tiles, as did the split
// exchange.)
template <int N>
constexpr bool has_variants()
{
    return N == 64 || N == 128 || N == 256 || N == 512 || N == 1024 || N == 2048 || N == 4096 || N == 840;
}

template <typename T, int N>
static hipError_t launch_c2c_n(const StageArgs& a, hipStream_t s)
{
    const int tdiv = a.tdiv < 1 ? 1 : a.tdiv;
    if (a.order == 1) {  // the reverse radix order: one thread per butterfly, plain exchange and accesses
        if constexpr (radix_order_distinct(N)) {
            if (tdiv == 1 && !a.split && a.nt == 0) return launch_c2c_v<T, N, 1, false, 0, 1>(a, s);
        }
        return hipErrorInvalidValue;
    }
    if constexpr (has_variants<N>()) {
        // non-temporal variants: one thread per butterfly only
        if (tdiv == 1 && a.nt == 1)
            return a.split ? launch_c2c_v<T, N, 1, true, 1>(a, s) : launch_c2c_v<T, N, 1, false, 1>(a, s);
        if (tdiv == 1 && a.nt == 2)
            return a.split ? launch_c2c_v<T, N, 1, true, 2>(a, s) : launch_c2c_v<T, N, 1, false, 2>(a, s);
    }
    if (tdiv == 1 && !a.split) return launch_c2c_v<T, N, 1, false>(a, s);
    if constexpr (has_variants<N>()) {
        constexpr int tpl = radix_plan(N).tpl;
        if (tdiv == 1) return launch_c2c_v<T, N, 1, true>(a, s);
        if constexpr (tpl % 2 == 0) {
            if (tdiv == 2) return a.split ? launch_c2c_v<T, N, 2, true>(a, s) : launch_c2c_v<T, N, 2, false>(a, s);
        }
        if constexpr (tpl % 4 == 0) {
            if (tdiv == 4) return a.split ? launch_c2c_v<T, N, 4, true>(a, s) : launch_c2c_v<T, N, 4, false>(a, s);
        }
    }
    return hipErrorInvalidValue;
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

bool c2c_order_available(int n, int tdiv, int split)
{
    return length_supported(n) && radix_order_distinct(n) && tdiv == 1 && !split;
}

bool c2c_variant_available(int n, int tdiv, int split)
{
    const bool var = n == 64 || n == 128 || n == 256 || n == 512 || n == 1024 || n == 2048 || n == 4096 || n == 840;
    if (tdiv == 1 && !split) return length_supported(n);
    if (!var) return false;
    const int tpl = radix_plan(n).tpl;
    return tdiv == 1 || (tdiv == 2 && tpl % 2 == 0) || (tdiv == 4 && tpl % 4 == 0);
}

}  // namespace fft3d
