// Batched timestep kernels instantiated for double storage.
#include "launch.hpp"
#include "program_kernels.hpp"

namespace stl {

template <int VD, int TJ, int PF>
static hipError_t by_levels(const ColumnBatch &b, int kh, int ntiles, hipStream_t st) {
    switch (kh) {
    case 16: return launch_column_batch_t<double, VD, TJ, PF, 16, 2>(b, ntiles, st);
    case 32: return launch_column_batch_t<double, VD, TJ, PF, 32, 1>(b, ntiles, st);
    case 40: return launch_column_batch_t<double, VD, TJ, PF, 40, 1>(b, ntiles, st);
    case 45: return launch_column_batch_t<double, VD, TJ, PF, 45, 1>(b, ntiles, st);
    case 48: return launch_column_batch_t<double, VD, TJ, PF, 48, 1>(b, ntiles, st);
    }
    return hipErrorInvalidValue;
}

bool batch_variant_f64(int tile_j, int prefetch, int sched, int fpw) {
    if (sched != 1 || fpw != 1) return false;  // staged, one field per workgroup
    if (tile_j == 2 && prefetch == 2) return true;
    return false;
}

hipError_t launch_column_batch_f64(const ColumnBatch &b, int vd, int kh, int tile_j,
                                   int prefetch, int sched, int fpw, int ntiles, hipStream_t st) {
    if (sched != 1 || fpw != 1) return hipErrorInvalidValue;
    if (tile_j == 2 && prefetch == 2)
        return vd == 2   ? by_levels<2, 2, 2>(b, kh, ntiles, st)
               : vd == 1 ? by_levels<1, 2, 2>(b, kh, ntiles, st)
                         : by_levels<0, 2, 2>(b, kh, ntiles, st);
    return hipErrorInvalidValue;
}

hipError_t launch_hgrad_batch_f64(const HgradBatch &b, int ntiles, hipStream_t st) {
    return launch_hgrad_batch_t<double>(b, ntiles, st);
}

}  // namespace stl
