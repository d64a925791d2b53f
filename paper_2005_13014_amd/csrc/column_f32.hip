// Column kernels instantiated for float storage.
#include "column.hpp"
#include "launch.hpp"

namespace stl {

template <int TJ, int PF>
static hipError_t fused_k(const VadvArgs &a, hipStream_t st) {
    if (a.K <= 32) return launch_fused_t<float, TJ, PF, 32>(a, st);
    if (a.K <= 64) return launch_fused_t<float, TJ, PF, 64>(a, st);
    if (a.K <= 80) return launch_fused_t<float, TJ, PF, 80>(a, st);
    return launch_fused_t<float, TJ, PF, 96>(a, st);
}

hipError_t launch_fused_f32(const VadvArgs &a, int tile_j, int prefetch, hipStream_t st) {
    if (tile_j == 4 && prefetch == 4) return fused_k<4, 4>(a, st);
    if (tile_j == 4 && prefetch == 2) return fused_k<4, 2>(a, st);
    if (tile_j == 4 && prefetch == 8) return fused_k<4, 8>(a, st);
    if (tile_j == 2 && prefetch == 4) return fused_k<2, 4>(a, st);
    if (tile_j == 1 && prefetch == 8) return fused_k<1, 8>(a, st);
    return hipErrorInvalidValue;
}

hipError_t launch_vadv_f32(const VadvArgs &a, hipStream_t st) {
    if (a.K <= 32) return launch_vadv_t<float, 4, 4, 32>(a, st);
    if (a.K <= 64) return launch_vadv_t<float, 4, 4, 64>(a, st);
    if (a.K <= 80) return launch_vadv_t<float, 4, 4, 80>(a, st);
    return launch_vadv_t<float, 4, 4, 96>(a, st);
}

}  // namespace stl
