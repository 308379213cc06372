// Wavefront stencil kernels of one mode (MODE_RESID), FP32 and FP64.
#include "wave_impl.h"

namespace h27 {

template <typename R, int MODE>
int launch_wave_m(const WaveArgs<R>& a, bool shifted, int ry, hipStream_t s) {
    return shifted ? launch_wave_mode<R, MODE, true>(a, ry, s) : launch_wave_mode<R, MODE, false>(a, ry, s);
}
template int launch_wave_m<float, MODE_RESID>(const WaveArgs<float>&, bool, int, hipStream_t);
template int launch_wave_m<double, MODE_RESID>(const WaveArgs<double>&, bool, int, hipStream_t);

}  // namespace h27
