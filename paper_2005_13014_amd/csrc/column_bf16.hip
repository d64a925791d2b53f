// Column kernels instantiated for bfloat16 storage.
#include "column.hpp"
#include "launch.hpp"

namespace stl {

template <int TJ, int PF>
static hipError_t fused_k(const VadvArgs &a, hipStream_t st) {
    if (a.K <= 32) return launch_fused_t<uint16_t, TJ, PF, 32>(a, st);
    if (a.K <= 64) return launch_fused_t<uint16_t, TJ, PF, 64>(a, st);
    if (a.K <= 80) return launch_fused_t<uint16_t, TJ, PF, 80>(a, st);
    return launch_fused_t<uint16_t, TJ, PF, 96>(a, st);
}

hipError_t launch_fused_bf16(const VadvArgs &a, int tile_j, int prefetch, hipStream_t st) {
    if (tile_j == 4 && prefetch == 4) return fused_k<4, 4>(a, st);
    return hipErrorInvalidValue;
}

hipError_t launch_vadv_bf16(const VadvArgs &a, hipStream_t st) {
    if (a.K <= 32) return launch_vadv_t<uint16_t, 4, 4, 32>(a, st);
    if (a.K <= 64) return launch_vadv_t<uint16_t, 4, 4, 64>(a, st);
    if (a.K <= 80) return launch_vadv_t<uint16_t, 4, 4, 80>(a, st);
    return launch_vadv_t<uint16_t, 4, 4, 96>(a, st);
}

}  // namespace stl
