// Column kernels (column.hpp) instantiated for float storage.
#include "column.hpp"
#include "launch.hpp"

namespace stl {

// Register-resident half columns of KH levels serve nk <= 2 KH.
template <bool FUSED, int TJ, int PF, bool NT = false>
static hipError_t by_levels(const ColumnArgs &a, hipStream_t st) {
    const int m = (a.K + 1) / 2;
    if (m <= 16) return launch_column_t<float, FUSED, TJ, PF, 16, 2, NT>(a, st);
    if (m <= 32) return launch_column_t<float, FUSED, TJ, PF, 32, 2, NT>(a, st);
    if (m <= 40) return launch_column_t<float, FUSED, TJ, PF, 40, 2, NT>(a, st);
    return launch_column_t<float, FUSED, TJ, PF, 48, 1, NT>(a, st);
}

bool column_variant_f32(int tile_j, int prefetch, bool nt) {
    if (!nt && tile_j == 2 && prefetch == 4) return true;
    if (!nt && tile_j == 4 && prefetch == 4) return true;
    if (!nt && tile_j == 2 && prefetch == 2) return true;
    if (!nt && tile_j == 2 && prefetch == 8) return true;
    if (!nt && tile_j == 1 && prefetch == 4) return true;
    if (nt && tile_j == 2 && prefetch == 4) return true;
    if (nt && tile_j == 4 && prefetch == 4) return true;
    if (nt && tile_j == 2 && prefetch == 8) return true;
    if (nt && tile_j == 2 && prefetch == 2) return true;
    return false;
}

hipError_t launch_column_f32(bool fused, const ColumnArgs &a, int tile_j, int prefetch, bool nt,
                             hipStream_t st) {
    if (!fused) return by_levels<false, 2, 4>(a, st);
    if (!nt && tile_j == 2 && prefetch == 4) return by_levels<true, 2, 4>(a, st);
    if (!nt && tile_j == 4 && prefetch == 4) return by_levels<true, 4, 4>(a, st);
    if (!nt && tile_j == 2 && prefetch == 2) return by_levels<true, 2, 2>(a, st);
    if (!nt && tile_j == 2 && prefetch == 8) return by_levels<true, 2, 8>(a, st);
    if (!nt && tile_j == 1 && prefetch == 4) return by_levels<true, 1, 4>(a, st);
    if (nt && tile_j == 2 && prefetch == 4) return by_levels<true, 2, 4, true>(a, st);
    if (nt && tile_j == 4 && prefetch == 4) return by_levels<true, 4, 4, true>(a, st);
    if (nt && tile_j == 2 && prefetch == 8) return by_levels<true, 2, 8, true>(a, st);
    if (nt && tile_j == 2 && prefetch == 2) return by_levels<true, 2, 2, true>(a, st);
    return hipErrorInvalidValue;
}

}  // namespace stl
