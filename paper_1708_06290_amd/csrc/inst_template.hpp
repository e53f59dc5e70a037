// Instantiates the sweep and Q* kernels for precision REAL_T and the m values
// M_FIRST..M_LAST, with launcher names suffixed SUFFIX.
#include <algorithm>

#include "kernels.hpp"

namespace shs {

template <int MM>
struct Inst {
    static void geometry(bool dense, SweepGeometry *g)
    {
        if (dense) {
            g->rows_per_lane = rows_per_lane<REAL_T, MM, true>();
            g->slot = slot_elems(MM, true);
        } else {
            g->rows_per_lane = rows_per_lane<REAL_T, MM, false>();
            g->slot = slot_elems(MM, false);
        }
        g->tile_rows = kWave * g->rows_per_lane;
        g->tile_stride = refl_tile_stride<REAL_T>(g->tile_rows, g->slot);
    }
    static void sweep(bool dense, const SweepArgs<REAL_T> &a, hipStream_t st)
    {
        if (dense)
            hipLaunchKernelGGL((sweep_kernel<REAL_T, MM, true>), dim3(a.count), dim3(kWave), 0, st, a);
        else
            hipLaunchKernelGGL((sweep_kernel<REAL_T, MM, false>), dim3(a.count), dim3(kWave), 0, st, a);
    }
    static bool qstar(bool dense_in, const QstarArgs<REAL_T> &a, hipStream_t st)
    {
        if (dense_in) {
            if (a.count <= 0) return true;
            // the wave kernel: its chunk must hold a whole phase group plus
            // the next slot, and a tile at least one phase group
            const int spw = qstar_dense_spw(a.count, MM);
            constexpr int S = slot_elems(MM, true);
            const int cs = (MM + 1) * (std::min((kQstarLds / spw - 1) / S - 1, a.tile_rows) / (MM + 1));
            if (a.slot == S && a.tile_rows >= MM + 1 && cs >= MM + 1) {
                hipLaunchKernelGGL((qstar_wave_dense_kernel<REAL_T, MM>), dim3((a.count + spw - 1) / spw),
                                   dim3(kWave), 0, st, a, spw);
            } else {
                constexpr int spl = kWave / MM;
                hipLaunchKernelGGL((qstar_kernel<REAL_T, MM, true>), dim3((a.count + spl - 1) / spl), dim3(kWave), 0,
                                   st, a);
            }
        } else if (a.count > 0) {
            // the kernel reads the structured store's slots (and needs a tile
            // of at least one phase group)
            if (a.slot != slot_elems(MM, false) || a.tile_rows < MM + 1 || a.accumulate) return false;
            const int spw = qstar_spw(a.count, MM);
            hipLaunchKernelGGL((qstar_wave_kernel<REAL_T, MM>), dim3((a.count + spw - 1) / spw), dim3(kWave), 0, st,
                               a, spw);
        }
        return true;
    }
};

#define SHS_CAT3_(a, b, c) a##b##c
#define SHS_CAT3(a, b, c) SHS_CAT3_(a, b, c)

bool SHS_CAT3(sweep_geometry_, SUFFIX, PART)(int m, bool dense, SweepGeometry *g)
{
    bool ok = false;
    SHS_DISPATCH_M(m, if constexpr (MM >= M_FIRST && MM <= M_LAST) { Inst<MM>::geometry(dense, g); ok = true; });
    return ok;
}

bool SHS_CAT3(launch_sweep_, SUFFIX, PART)(int m, bool dense, const SweepArgs<REAL_T> &a, hipStream_t st)
{
    bool ok = false;
    SHS_DISPATCH_M(m, if constexpr (MM >= M_FIRST && MM <= M_LAST) { Inst<MM>::sweep(dense, a, st); ok = true; });
    return ok;
}

bool SHS_CAT3(launch_qstar_, SUFFIX, PART)(int m, bool dense_in, const QstarArgs<REAL_T> &a, hipStream_t st)
{
    bool ok = false;
    SHS_DISPATCH_M(m, if constexpr (MM >= M_FIRST && MM <= M_LAST) { ok = Inst<MM>::qstar(dense_in, a, st); });
    return ok;
}

}  // namespace shs
