// Fused x-y stage for small planes: one workgroup loads a whole z-plane of
// the tile into LDS, runs the 1D FFTs along x on its rows and then along y on
// its columns in place in LDS, and writes the plane back.  The 3D transform
// then takes two passes over HBM (this one and the z stage) instead of three.
// This is the slab form of the decomposition (the first two transforms local
// to a slab, then one reorientation for the last, Sec. III-A; the 2D-FFT task
// of Table I's slab stage), used where a plane fits in LDS.
//
// Line groups: a line of length n is handled by TPL(n) threads; the NT
// threads of the workgroup take LPC = floor(NT / TPL) lines at a time and walk
// the rows (then the columns) in chunks.  NT is sized so that a sweep is one
// chunk wherever 1024 threads allow it.  Consecutive threads take consecutive
// lines (thread t: line t % LPC, part t / LPC of it), so the lanes of a wave
// touch one element of many lines: with an odd row pitch no two of 32 lanes
// share a bank slot, whatever the pass's element pattern.  Threads without a
// line in a chunk (a short last chunk, or the NT - LPC * TPL left over) run
// the same code on one shared scratch line, so every thread reaches every
// barrier; their results are garbage and never stored.
#include "device_fft.hpp"
#include "kernels.hpp"
#include "plane_list.hpp"
#include "stage_args.hpp"

namespace fft3d {

// One sweep of length-N line FFTs over `count` lines of the plane, in place:
// line k starts at base + k * line_step, its elements es apart.
template <typename T, int N, int NT>
FD void plane_sweep(cpx<T>* base, int count, int line_step, int es, cpx<T>* scratch, const cpx<T>* twl, int t)
{
    constexpr int TPL = radix_plan(N).tpl;
    constexpr int LPC = NT / TPL;  // lines per chunk
    const int g = t % LPC, part = t / LPC, tj = part % TPL;
    LdsView<T> Ls{nullptr, 0, 0};
    for (int c0 = 0; c0 < count; c0 += LPC) {
        const int k = c0 + g;
        const bool real = part < TPL && k < count;
        LdsView<cpx<T>> L = real ? LdsView<cpx<T>>{base + k * line_step, es, 0} : LdsView<cpx<T>>{scratch, 1, 0};
        auto load = [&](int e) -> cpx<T> { return L[e]; };
        auto store = [&](int e, cpx<T> v) { L[e] = v; };
        fft_line<T, N, TPL, false, true, true>(L, Ls, tj, twl, load, store);
        __syncthreads();  // the next chunk's lines may share the scratch line
    }
}

template <typename T, int NX, int NY, int NT>
__global__ __launch_bounds__(NT) void k_c2c_xy(StageArgs a)
{
    constexpr int PX = plane_pitch(NX);
    constexpr int SX = pass_table_size(radix_plan(NX));
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* plane = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* scratch = plane + NY * PX;
    cpx<T>* twx = scratch + (NX > NY ? NX : NY);
    cpx<T>* twy = twx + SX;
    const int t = threadIdx.x;
    TileCoord tc;
    if (!tile_coord(a, tc)) return;
    stage_pass_twiddles<T, NX>(twx, reinterpret_cast<const cpx<T>*>(a.twp), t, NT);
    stage_pass_twiddles<T, NY>(twy, reinterpret_cast<const cpx<T>*>(a.twp2), t, NT);
    // plane b of the tile: rows of NX values a.sa apart, planes a.sb apart
    const cpx<T>* __restrict__ in = reinterpret_cast<const cpx<T>*>(a.in) + a.off + tc.bx * a.sb;
    cpx<T>* __restrict__ out = reinterpret_cast<cpx<T>*>(a.out) + a.off_o + tc.bx * a.sb_o;
    const bool cj = a.conj != 0;
    // every load of the thread in flight at once, then into LDS
    constexpr int E = (NX * NY + NT - 1) / NT;
    cpx<T> v[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int i = t + j * NT, y = i / NX, x = i - y * NX;
        if (i < NX * NY) v[j] = in[(int64_t)y * a.sa + x];
    }
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int i = t + j * NT, y = i / NX, x = i - y * NX;
        if (i < NX * NY) plane[y * PX + x] = cj ? conj(v[j]) : v[j];
    }
    __syncthreads();
    plane_sweep<T, NX, NT>(plane, NY, PX, 1, scratch, twx, t);   // rows: the x FFTs
    plane_sweep<T, NY, NT>(plane, NX, 1, PX, scratch, twy, t);   // columns: the y FFTs
    const T scale = (T)a.scale;
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int i = t + j * NT, y = i / NX, x = i - y * NX;
        if (i < NX * NY) {
            cpx<T> w = plane[y * PX + x];
            if (cj) w = conj(w);
            out[(int64_t)y * a.sa_o + x] = w * scale;
        }
    }
}

template <typename T, int NX, int NY>
static hipError_t launch_plane(const StageArgs& a, hipStream_t s)
{
    constexpr size_t lds = plane_lds_bytes(NX, NY, sizeof(cpx<T>));  // folded here, not per launch
    if constexpr (lds > kPlaneMaxLds) {
        return hipErrorInvalidValue;
    } else {
        if (a.B == 0) return hipSuccess;
        constexpr int NT = plane_threads(NX, NY);
        return launch_stage_kernel(reinterpret_cast<const void*>(&k_c2c_xy<T, NX, NY, NT>), dim3((unsigned)a.B),
                                   dim3(NT), a, lds, s);
    }
}

hipError_t launch_c2c_xy(int nx, int ny, int dtype, const StageArgs& a, hipStream_t s)
{
#define FFT3D_PLANE_LAUNCH(X_, Y_)                                                                   \
    if (nx == X_ && ny == Y_)                                                                      \
        return dtype == DT_F64 ? launch_plane<double, X_, Y_>(a, s) : launch_plane<float, X_, Y_>(a, s);
    FFT3D_FOR_EACH_PLANE(FFT3D_PLANE_LAUNCH)
#undef FFT3D_PLANE_LAUNCH
    return hipErrorInvalidValue;
}

}  // namespace fft3d
