// Fused apply of several grids (batches of small grids): one launch of the
// wavefront kernel covers up to kWaveBatch grids, each with its own table
// slice, PML profiles, right-hand sides and output.
#include <algorithm>
#include <climits>

#include "wave_impl.h"

namespace h27 {

static_assert(sizeof(WaveBatch<double>) <= 4096, "batched kernel arguments must fit the 4 KiB argument segment");

template <typename R, bool SH, bool ROWC, bool MA>
static int batch_launch(const WaveArgs<R>* const* w, int n, hipStream_t s) {
    constexpr int RY = (sizeof(R) == 4 && !MA) ? 2 : 1;
    constexpr int RQ = FrameRows<R>::value;
    constexpr int waves = kBlock / 64;
    for (int i0 = 0; i0 < n; i0 += kWaveBatch) {
        const int m = std::min(kWaveBatch, n - i0);
        WaveBatch<R> B{};
        B.n = m;
        int64_t blocks = 0;
        size_t lds = 0;
        for (int j = 0; j < m; ++j) {
            const WaveArgs<R>& a = *w[i0 + j];
            B.a[j] = a;
            B.bstart[j] = static_cast<int>(blocks);
            blocks += (a.n_items + waves - 1) / waves;   // one work item per wavefront
            if (blocks > INT_MAX) return HELM27_EINVAL;
            lds = std::max(lds, wave_ring_offset(ROWC ? 0 : a.n_tab, z_lds_nodes(a.g.nz, a.g.zlo, a.g.zhi),
                                                 sizeof(R) == 8));
        }
        for (int j = m; j <= kWaveBatch; ++j) B.bstart[j] = static_cast<int>(blocks);
        if (blocks == 0) continue;
        H27_CHECK_HIP(launch(wave27_batch_kernel<R, MODE_APPLY, SH, RY, RQ, ROWC, MA>, dim3(static_cast<unsigned>(blocks)),
                             dim3(kBlock), lds, s, B));
    }
    return HELM27_OK;
}

template <typename R>
int launch_wave_batch(const WaveArgs<R>* const* w, int n, bool shifted, bool rowc, bool mass_a, hipStream_t s) {
    const int k = (shifted ? 1 : 0) | (rowc ? 2 : 0) | (mass_a ? 4 : 0);
    switch (k) {
        case 0: return batch_launch<R, false, false, false>(w, n, s);
        case 1: return batch_launch<R, true, false, false>(w, n, s);
        case 2: return batch_launch<R, false, true, false>(w, n, s);
        case 3: return batch_launch<R, true, true, false>(w, n, s);
        case 4: return batch_launch<R, false, false, true>(w, n, s);
        case 5: return batch_launch<R, true, false, true>(w, n, s);
        case 6: return batch_launch<R, false, true, true>(w, n, s);
        default: return batch_launch<R, true, true, true>(w, n, s);
    }
}
template int launch_wave_batch<float>(const WaveArgs<float>* const*, int, bool, bool, bool, hipStream_t);
template int launch_wave_batch<double>(const WaveArgs<double>* const*, int, bool, bool, bool, hipStream_t);

}  // namespace h27
