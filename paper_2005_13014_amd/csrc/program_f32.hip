// Batched timestep kernels instantiated for float storage.
#include "launch.hpp"
#include "program_kernels.hpp"

namespace stl {

template <int VD, int TJ, int PF, bool PIPE>
static hipError_t by_levels(const ColumnBatch &b, int kh, int ntiles, hipStream_t st) {
    switch (kh) {
    case 16: return launch_column_batch_t<float, VD, TJ, PF, 16, 2, PIPE>(b, ntiles, st);
    case 32: return launch_column_batch_t<float, VD, TJ, PF, 32, 2, PIPE>(b, ntiles, st);
    case 40: return launch_column_batch_t<float, VD, TJ, PF, 40, 2, PIPE>(b, ntiles, st);
    case 45: return launch_column_batch_t<float, VD, TJ, PF, 45, 2, PIPE>(b, ntiles, st);
    case 48: return launch_column_batch_t<float, VD, TJ, PF, 48, 1, PIPE>(b, ntiles, st);
    }
    return hipErrorInvalidValue;
}

template <int TJ, int PF, bool PIPE>
static hipError_t by_vd(const ColumnBatch &b, int vd, int kh, int ntiles, hipStream_t st) {
    return vd == 2   ? by_levels<2, TJ, PF, PIPE>(b, kh, ntiles, st)
           : vd == 1 ? by_levels<1, TJ, PF, PIPE>(b, kh, ntiles, st)
                     : by_levels<0, TJ, PF, PIPE>(b, kh, ntiles, st);
}

// Compiled variants (tile_j, prefetch, schedule, fields per workgroup):
// staged (1) and pipelined (2), tile_j 2 or 4, one field per workgroup.
bool batch_variant_f32(int tile_j, int prefetch, int sched, int fpw) {
    return prefetch == 4 && fpw == 1 && (tile_j == 2 || tile_j == 4) && (sched == 1 || sched == 2);
}

hipError_t launch_column_batch_f32(const ColumnBatch &b, int vd, int kh, int tile_j, int prefetch, int sched,
                                   int fpw, int ntiles, hipStream_t st) {
    if (!batch_variant_f32(tile_j, prefetch, sched, fpw)) return hipErrorInvalidValue;
    if (sched == 2)
        return tile_j == 2 ? by_vd<2, 4, true>(b, vd, kh, ntiles, st) : by_vd<4, 4, true>(b, vd, kh, ntiles, st);
    return tile_j == 2 ? by_vd<2, 4, false>(b, vd, kh, ntiles, st) : by_vd<4, 4, false>(b, vd, kh, ntiles, st);
}

hipError_t launch_hgrad_batch_f32(const HgradBatch &b, int ntiles, hipStream_t st) {
    return launch_hgrad_batch_t<float>(b, ntiles, st);
}

}  // namespace stl
