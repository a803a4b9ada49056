// The log-domain row sweep compiled for batches of short rows (every n <=
// kShortRowN): the same kernel as the long-row sweep, for two workgroups per
// CU. It is instantiated here, in a translation unit of its own, so that its
// tighter register budget leaves the long-row kernel's code unchanged.
#include "sk_rowsweep.h"

namespace sk {

hipError_t launch_row_sweep_short(const Inst *d_insts, const RowUnit *d_units, int nunits,
                                  const int32_t *bounds, int grid, size_t lds_bytes, int nt_loads,
                                  hipStream_t st, hipEvent_t stop) {
    if (nt_loads)
        launch_stamped(k_row_sweep<true, 8>, dim3(grid), dim3(kRowWaves * kWave), lds_bytes, st, stop,
                       d_insts, d_units, nunits, bounds);
    else
        launch_stamped(k_row_sweep<false, 8>, dim3(grid), dim3(kRowWaves * kWave), lds_bytes, st, stop,
                       d_insts, d_units, nunits, bounds);
    return hipGetLastError();
}

hipError_t set_row_sweep_short_attributes() {
    const int lds = (int)(kShortRowN * sizeof(ColPot));
    for (const void *f : {(const void *)k_row_sweep<true, 8>, (const void *)k_row_sweep<false, 8>}) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace sk
