// Bounded-z real-to-real stage kernels in double precision (see k_r2r.hpp).
#include "k_r2r.hpp"

namespace fft3d {

hipError_t launch_r2r_z_f64(int n, const StageArgs& a, hipStream_t s)
{
#define FFT3D_R2R_CASE(L) \
    case L:               \
        return launch_r2r_n<double, L>(a, s);
    switch (n) {
        FFT3D_FOR_EACH_LENGTH(FFT3D_R2R_CASE)
    default:
        return hipErrorInvalidValue;
    }
#undef FFT3D_R2R_CASE
}

}  // namespace fft3d
