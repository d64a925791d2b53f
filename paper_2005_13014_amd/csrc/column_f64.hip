// Column kernels instantiated for double storage.
#include "column.hpp"
#include "launch.hpp"

namespace stl {

template <int TJ, int PF>
static hipError_t fused_k(const VadvArgs &a, hipStream_t st) {
    if (a.K <= 32) return launch_fused_t<double, TJ, PF, 32>(a, st);
    if (a.K <= 64) return launch_fused_t<double, TJ, PF, 64>(a, st);
    return launch_fused_t<double, TJ, PF, 80>(a, st);
}

hipError_t launch_fused_f64(const VadvArgs &a, int tile_j, int prefetch, hipStream_t st) {
    if (tile_j == 4 && prefetch == 2) return fused_k<4, 2>(a, st);
    return hipErrorInvalidValue;
}

hipError_t launch_vadv_f64(const VadvArgs &a, hipStream_t st) {
    if (a.K <= 32) return launch_vadv_t<double, 4, 2, 32>(a, st);
    if (a.K <= 64) return launch_vadv_t<double, 4, 2, 64>(a, st);
    return launch_vadv_t<double, 4, 2, 80>(a, st);
}

}  // namespace stl
