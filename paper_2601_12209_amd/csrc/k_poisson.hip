// Fused z-stage of the spectral Poisson solve: for each z-line of the half
// spectrum, forward FFT along z, multiply by the spectral multiplier, inverse
// FFT along z, all without leaving the workgroup.  This folds the z-stage of
// the forward transform, the pointwise solve and the z-stage of the inverse
// transform into one read and one write of the field (the paper's Poisson
// application, Sec. VI-B, uses the forward and inverse 3D FFT around a
// pointwise division by -|k|^2).
//
// Multiplier, for a periodic box of side 2 pi with integer wavenumbers
// k_j = j (j <= n/2) or j - n (j > n/2):  M(k) = -1/|k|^2, M(0) = 0, times the
// scale in the arguments (1/N for the whole solve).  M is real, so the same
// kernel is its own adjoint.
#include "device_fft.hpp"
#include "kernels.hpp"
#include "stage_args.hpp"

namespace fft3d {

template <typename T>
FD T wavenumber(int64_t j, int64_t n)
{
    return (T)(2 * j <= n ? j : j - n);
}

template <typename T, int N>
__global__ __launch_bounds__(1024) void k_poisson_z(StageArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    const int t = threadIdx.x;
    const int lw = t % a.lw, tj = t / a.lw;
    TileCoord tc;
    if (!tile_coord(a, tc)) return;
    const int64_t aa = tc.bx * a.lw + lw;
    const bool ok = aa < a.A;
    const int64_t ac = ok ? aa : a.A - 1;  // see k_c2c
    const int64_t base = a.off + ac + tc.by * a.sb;
    const int64_t base_o = a.off_o + ac + tc.by * a.sb_o;
    const int64_t se = a.se, se_o = a.se_o;
    const cpx<T>* __restrict__ in = reinterpret_cast<const cpx<T>*>(a.in) + base + tj * se;
    cpx<T>* __restrict__ out = reinterpret_cast<cpx<T>*>(a.out) + base_o + tj * se_o;
    LdsView<cpx<T>> L{lds + lw, a.lw, 0};
    LdsView<T> Ls{nullptr, 0, 0};
    constexpr int TPL = radix_plan(N).tpl;
    cpx<T>* twl = reinterpret_cast<cpx<T>*>(smem_raw + align16((size_t)a.lw * N * sizeof(cpx<T>)));
    stage_pass_twiddles<T, N>(twl, reinterpret_cast<const cpx<T>*>(a.twp), t, blockDim.x);

    // wavenumbers of this line: kx from the half-spectrum column, ky from the row
    const T kx = (T)(a.kx0 + aa);
    const T ky = wavenumber<T>(a.ky0 + tc.by, a.pny);
    const T kxy2 = kx * kx + ky * ky;
    const T scale = (T)a.scale;

    auto load = [&](int e) -> cpx<T> { return in[(e - tj) * se]; };
    auto store_lds = [&](int e, cpx<T> v) { L[e] = v; };
    fft_line<T, N, TPL, false, false, true>(L, Ls, tj, twl, load, store_lds);
    __syncthreads();
    // inverse transform of M .* Xhat as conj(F(conj(M .* Xhat))), M real
    auto load_mul = [&](int e) -> cpx<T> {
        const T kz = wavenumber<T>(e, N);
        const T k2 = kxy2 + kz * kz;
        const T m = k2 == (T)0 ? (T)0 : -scale / k2;
        return conj(L[e] * m);
    };
    auto store = [&](int e, cpx<T> v) {
        if (ok) out[(e - tj) * se_o] = conj(v);
    };
    fft_line<T, N, TPL, false, true, false>(L, Ls, tj, twl, load_mul, store);
}

template <typename T, int N>
static hipError_t launch_poisson_n(const StageArgs& a, hipStream_t s)
{
    constexpr int TPL = radix_plan(N).tpl;
    const int threads = a.lw * TPL;
    const size_t lds = align16((size_t)a.lw * N * sizeof(cpx<T>)) + pass_table_bytes<T, N>();
    const dim3 grid((unsigned)((a.A + a.lw - 1) / a.lw), (unsigned)a.B, 1);
    if (grid.x == 0 || grid.y == 0) return hipSuccess;
    return launch_stage_kernel(reinterpret_cast<const void*>(&k_poisson_z<T, N>), grid, dim3(threads), a, lds,
                               s);
}

hipError_t launch_poisson_z(int n, int dtype, const StageArgs& a, hipStream_t s)
{
#define FFT3D_POISSON_CASE(L)                                                             \
    case L:                                                                               \
        return dtype == DT_F64 ? launch_poisson_n<double, L>(a, s)                        \
                               : launch_poisson_n<float, L>(a, s);
    switch (n) {
        FFT3D_FOR_EACH_LENGTH(FFT3D_POISSON_CASE)
    default:
        return hipErrorInvalidValue;
    }
#undef FFT3D_POISSON_CASE
}

}  // namespace fft3d
