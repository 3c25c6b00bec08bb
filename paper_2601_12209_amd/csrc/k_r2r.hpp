// Real-to-real transforms along the bounded z axis of the (Periodic,
// Periodic, Bounded) topology, the paper's second Poisson-solver case
// (Sec. VI-B; DCT/DST plans beside C2C and R2C, Sec. V-B).
//
// Each z-line of the half spectrum holds complex values whose real and
// imaginary parts are two independent real sequences; a real-to-real
// transform applied to both is complex-linear, so it is computed on the
// complex line with one length-N complex FFT (Makhoul's reordering):
//
//   DCT-II   Y_k = 2 sum_j x_j cos(pi (2j+1) k / 2N):
//            v_e = x_{2e} (e < ceil(N/2)), v_e = x_{2(N-1-e)+1} (else),
//            V = DFT_N(v),  Y_k = w_k V_k + conj(w_k) V_{(N-k) mod N},
//            w_k = exp(-i pi k / 2N)
//   DCT-III  x_j = Y_0 + 2 sum_{k>0} Y_k cos(pi k (2j+1) / 2N)  (inverse of
//            DCT-II up to 2N):  U_k = conj(w_k) (Y_k - i Y_{N-k}), Y_N = 0,
//            u = sum_k U_k exp(+2 pi i k e / N), x_{2e} / x_{2(N-1-e)+1} = u_e
//   DST-II   = DCT-II of (-1)^j x_j, output index reversed
//   DST-III  = (-1)^j DCT-III of the reversed input
//
// The lanes of a wavefront walk neighbouring lines (consecutive kx), so
// every load and store is a row segment, as in the strided C2C stages.  The
// Poisson mode runs DCT-II (DST-II), the multiplier -1/|k|^2 and DCT-III
// (DST-III) without leaving the workgroup: the (k, N-k) pairs that both the
// post-processing of the forward and the pre-processing of the inverse need
// are combined in one step in LDS.
#pragma once
#include "device_fft.hpp"
#include "kernels.hpp"
#include "stage_args.hpp"

namespace fft3d {

template <typename T>
FD T wavenumber_r2r(int64_t j, int64_t n)
{
    return (T)(2 * j <= n ? j : j - n);
}

template <typename T, int N, int MODE>
__global__ __launch_bounds__(1024) void k_r2r_z(StageArgs a)
{
    constexpr bool DST = MODE == R2R_DST2 || MODE == R2R_DST3 || MODE == R2R_POISSON_D;
    constexpr bool FWD = MODE == R2R_DCT2 || MODE == R2R_DST2;
    constexpr bool INV = MODE == R2R_DCT3 || MODE == R2R_DST3;
    constexpr int TPL = radix_plan(N).tpl;
    constexpr int H = (N + 1) / 2;  // even-indexed inputs go first in Makhoul's order
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    const int t = threadIdx.x;
    const int lw = t % a.lw, tj = t / a.lw;
    TileCoord tc;
    if (!tile_coord(a, tc)) return;
    const int64_t aa = tc.bx * a.lw + lw;
    const bool ok = aa < a.A;
    const int64_t ac = ok ? aa : a.A - 1;  // lanes past the last line load a valid one, store nothing
    const int64_t se = a.se, se_o = a.se_o;
    const cpx<T>* __restrict__ in = reinterpret_cast<const cpx<T>*>(a.in) + a.off + ac + tc.by * a.sb;
    cpx<T>* __restrict__ out = reinterpret_cast<cpx<T>*>(a.out) + a.off_o + ac + tc.by * a.sb_o;
    LdsView<cpx<T>> L{lds + lw, a.lw, 0};
    LdsView<T> Ls{nullptr, 0, 0};
    cpx<T>* twl = reinterpret_cast<cpx<T>*>(smem_raw + align16((size_t)a.lw * N * sizeof(cpx<T>)));
    stage_pass_twiddles<T, N>(twl, reinterpret_cast<const cpx<T>*>(a.twp), t, blockDim.x);
    cpx<T>* w4 = twl + pass_table_size(radix_plan(N));  // w_k = W_4N^k, k < N
    for (int i = t; i < N; i += blockDim.x) w4[i] = reinterpret_cast<const cpx<T>*>(a.tw)[i];
    const T scale = (T)a.scale;

    // position of Makhoul element e in the real sequence, and (-1)^j there
    auto src_index = [](int e) { return e < H ? 2 * e : 2 * (N - 1 - e) + 1; };

    if constexpr (FWD || MODE == R2R_POISSON_N || MODE == R2R_POISSON_D) {
        auto load = [&](int e) -> cpx<T> {
            cpx<T> v = in[(int64_t)src_index(e) * se];
            if (DST && e >= H) v = cpx<T>{-v.re, -v.im};
            return v;
        };
        auto store_lds = [&](int e, cpx<T> v) { L[e] = v; };
        fft_line<T, N, TPL, false, false, true>(L, Ls, tj, twl, load, store_lds);
        __syncthreads();  // V complete in LDS; w4 visible
        if constexpr (FWD) {
            for (int k = tj; k < N; k += TPL) {
                const cpx<T> w = w4[k];
                const cpx<T> y = cmul(L[k], w) + cmul(L[k == 0 ? 0 : N - k], conj(w));
                if (ok) out[(int64_t)(DST ? N - 1 - k : k) * se_o] = y * scale;
            }
            return;
        } else {
            // wavenumbers of this line: kx from the half-spectrum column, ky
            // from the row; along z the DCT index k (Neumann) or, for the
            // DST, index N-1-k with wavenumber N-k (Dirichlet)
            const T kx = (T)(a.kx0 + aa);
            const T ky = wavenumber_r2r<T>(a.ky0 + tc.by, a.pny);
            const T kxy2 = kx * kx + ky * ky;
            auto mult = [&](int k) -> T {
                const T kz = DST ? (T)(N - k) : (T)k;
                const T k2 = kxy2 + kz * kz;
                return k2 == (T)0 ? (T)0 : -scale / k2;
            };
            for (int k = tj; 2 * k <= N; k += TPL) {
                const int kp = k == 0 ? 0 : N - k;
                const cpx<T> vk = L[k], vp = L[kp];
                const cpx<T> wk = w4[k], wp = w4[kp];
                // forward post-processing of the pair, then the multiplier
                const cpx<T> zk = (cmul(vk, wk) + cmul(vp, conj(wk))) * mult(k);
                const cpx<T> zp = (cmul(vp, wp) + cmul(vk, conj(wp))) * mult(kp);
                // inverse pre-processing; stored conjugated for the sign +1 FFT
                if (k == 0) {
                    L[0] = conj(zk);
                } else if (kp == k) {
                    L[k] = conj(cmul(zk + mul_negi(zk), conj(wk)));
                } else {
                    L[k] = conj(cmul(zk + mul_negi(zp), conj(wk)));
                    L[kp] = conj(cmul(zp + mul_negi(zk), conj(wp)));
                }
            }
            __syncthreads();
            auto load2 = [&](int e) -> cpx<T> { return L[e]; };
            auto store = [&](int e, cpx<T> v) {
                v = conj(v);
                if (DST && e >= H) v = cpx<T>{-v.re, -v.im};
                if (ok) out[(int64_t)src_index(e) * se_o] = v;
            };
            fft_line<T, N, TPL, false, true, false>(L, Ls, tj, twl, load2, store);
        }
    } else {
        static_assert(INV, "unknown mode");
        // the line into LDS (DST: reversed); the adjoint of the forward counts
        // the first coefficient (of the reversed line for the DST) twice
        for (int e = tj; e < N; e += TPL) {
            cpx<T> v = in[(int64_t)e * se];
            const int d = DST ? N - 1 - e : e;
            if (a.weight && d == 0) v = v * (T)2;
            L[d] = v;
        }
        __syncthreads();
        auto load = [&](int k) -> cpx<T> {
            const cpx<T> yk = L[k];
            const cpx<T> ym = k == 0 ? cpx<T>{(T)0, (T)0} : L[N - k];
            return conj(cmul(yk + mul_negi(ym), conj(w4[k])));
        };
        auto store = [&](int e, cpx<T> v) {
            v = conj(v) * scale;
            if (DST && e >= H) v = cpx<T>{-v.re, -v.im};
            if (ok) out[(int64_t)src_index(e) * se_o] = v;
        };
        fft_line<T, N, TPL, false, true, false>(L, Ls, tj, twl, load, store);
    }
}

template <typename T, int N, int MODE>
hipError_t launch_r2r_m(const StageArgs& a, hipStream_t s)
{
    constexpr int TPL = radix_plan(N).tpl;
    const int threads = a.lw * TPL;
    const size_t lds = align16((size_t)a.lw * N * sizeof(cpx<T>)) + pass_table_bytes<T, N>() + N * sizeof(cpx<T>);
    const dim3 grid((unsigned)((a.A + a.lw - 1) / a.lw), (unsigned)a.B, 1);
    if (grid.x == 0 || grid.y == 0) return hipSuccess;
    if (threads > 1024 || lds > kMaxLdsBytes) return hipErrorInvalidConfiguration;
    return launch_stage_kernel(reinterpret_cast<const void*>(&k_r2r_z<T, N, MODE>), grid, dim3(threads), a, lds,
                               s);
}

template <typename T, int N>
hipError_t launch_r2r_n(const StageArgs& a, hipStream_t s)
{
    switch (a.r2r) {
    case R2R_DCT2: return launch_r2r_m<T, N, R2R_DCT2>(a, s);
    case R2R_DCT3: return launch_r2r_m<T, N, R2R_DCT3>(a, s);
    case R2R_DST2: return launch_r2r_m<T, N, R2R_DST2>(a, s);
    case R2R_DST3: return launch_r2r_m<T, N, R2R_DST3>(a, s);
    case R2R_POISSON_N: return launch_r2r_m<T, N, R2R_POISSON_N>(a, s);
    case R2R_POISSON_D: return launch_r2r_m<T, N, R2R_POISSON_D>(a, s);
    default: return hipErrorInvalidValue;
    }
}

// One translation unit per precision (k_r2r_f32.hip, k_r2r_f64.hip) keeps
// the build parallel.
hipError_t launch_r2r_z_f32(int n, const StageArgs& a, hipStream_t s);
hipError_t launch_r2r_z_f64(int n, const StageArgs& a, hipStream_t s);

}  // namespace fft3d
