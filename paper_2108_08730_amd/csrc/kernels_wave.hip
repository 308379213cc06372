// Mode dispatch of the wavefront-per-tile stencil kernels (the kernels and
// their launchers are in wave_impl.h; each mode is compiled in its own
// translation unit, kernels_wave_<mode>.hip).
#include "wave_impl.h"

namespace h27 {

template <typename R>
int launch_wave(const WaveArgs<R>& a, int mode, bool shifted, int ry, int rq, hipStream_t s) {
    (void)rq;
    if (a.n_items <= 0) return HELM27_OK;
    switch (mode) {
        case MODE_APPLY: return launch_wave_m<R, MODE_APPLY>(a, shifted, ry, s);
        case MODE_RESID: return launch_wave_m<R, MODE_RESID>(a, shifted, ry, s);
        case MODE_JACOBI: return launch_wave_m<R, MODE_JACOBI>(a, shifted, ry, s);
        case MODE_JACOBI0: return launch_wave_m<R, MODE_JACOBI0>(a, shifted, ry, s);
        default: return HELM27_EINVAL;
    }
}
template int launch_wave<float>(const WaveArgs<float>&, int, bool, int, int, hipStream_t);
template int launch_wave<double>(const WaveArgs<double>&, int, bool, int, int, hipStream_t);

template <typename R>
int frame_rows() { return FrameRows<R>::value; }
template int frame_rows<float>();
template int frame_rows<double>();

// byte offset of the LDS row ring (after the table slice and the z nodes, 16-byte aligned)
size_t wave_ring_offset(int n_tab, int nz, bool fp64) {
    return (wave_lds_bytes(n_tab, nz, fp64) + 15) & ~static_cast<size_t>(15);
}

size_t wave_ring_bytes(int ry, int nb, bool fp64, bool mass_a) {
    const size_t bw = static_cast<size_t>(blk_waves(fp64));
    const size_t rows = nb > 1 ? static_cast<size_t>(nb) * (bw + 2) : bw * static_cast<size_t>(ry) + 2;
    return 2 * rows * 64 * (fp64 ? 16 : 8) * (mass_a ? 2 : 1);
}

size_t wave_lds_bytes(int n_tab, int nz, bool fp64) {
    return fp64 ? static_cast<size_t>(n_tab) * sizeof(TabEntry<double>) + static_cast<size_t>(nz) * sizeof(AxisNode<double>)
                : static_cast<size_t>(n_tab) * sizeof(TabEntry<float>) + static_cast<size_t>(nz) * sizeof(AxisNode<float>);
}

}  // namespace h27
