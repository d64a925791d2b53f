// Column kernels (column.hpp, column4.hpp) instantiated for double storage.
#include "column.hpp"
#include "column4.hpp"
#include "launch.hpp"

namespace stl {

// Register-resident half columns of KH levels serve nk <= 2 KH; a depth
// that fills its bucket exactly (nk = 2 KH) takes the kernel without
// padding steps.
template <bool FUSED, int TJ, int PF, bool NT>
static hipError_t staged(const ColumnArgs &a, hipStream_t st) {
    const int m = (a.K + 1) / 2;
    constexpr bool X = FUSED;
    if (m <= 16) return X && a.K == 32 ? launch_column_t<double, FUSED, TJ, PF, 16, 2, NT, X>(a, st)
                                       : launch_column_t<double, FUSED, TJ, PF, 16, 2, NT>(a, st);
    if (m <= 32) return X && a.K == 64 ? launch_column_t<double, FUSED, TJ, PF, 32, 1, NT, X>(a, st)
                                       : launch_column_t<double, FUSED, TJ, PF, 32, 1, NT>(a, st);
    if (m <= 40) return X && a.K == 80 ? launch_column_t<double, FUSED, TJ, PF, 40, 1, NT, X>(a, st)
                                       : launch_column_t<double, FUSED, TJ, PF, 40, 1, NT>(a, st);
    return X && a.K == 96 ? launch_column_t<double, FUSED, TJ, PF, 48, 1, NT, X>(a, st)
                          : launch_column_t<double, FUSED, TJ, PF, 48, 1, NT>(a, st);
}

template <int TJ, int PF, bool NT, bool CHAIN>
static hipError_t pipelined(const ColumnArgs &a, hipStream_t st) {
    const int m = (a.K + 1) / 2;
    if (m <= 16) return a.K == 32 ? launch_column_pipe_t<double, TJ, PF, 16, 2, NT, true, CHAIN>(a, st)
                                  : launch_column_pipe_t<double, TJ, PF, 16, 2, NT, false, CHAIN>(a, st);
    if (m <= 32) return a.K == 64 ? launch_column_pipe_t<double, TJ, PF, 32, 1, NT, true, CHAIN>(a, st)
                                  : launch_column_pipe_t<double, TJ, PF, 32, 1, NT, false, CHAIN>(a, st);
    if (m <= 40) return a.K == 80 ? launch_column_pipe_t<double, TJ, PF, 40, 1, NT, true, CHAIN>(a, st)
                                  : launch_column_pipe_t<double, TJ, PF, 40, 1, NT, false, CHAIN>(a, st);
    // 48 levels: 64 x 4 tiles would spill registers to scratch; 64 x 2 (same bits).
    constexpr int TJ48 = TJ > 2 ? 2 : TJ;
    return a.K == 96 ? launch_column_pipe_t<double, TJ48, PF, 48, 1, NT, true, CHAIN>(a, st)
                     : launch_column_pipe_t<double, TJ48, PF, 48, 1, NT, false, CHAIN>(a, st);
}

// Four lanes per column: segments of ceil(nk / 4) <= KH levels, nk >= 8,
// 2 levels prefetched.
static hipError_t four_lanes(const ColumnArgs &a, hipStream_t st) {
    const int m = (a.K + 3) / 4;
    if (m <= 8) return launch_column4_t<double, 2, 8, true>(a, st);
    if (m <= 12) return launch_column4_t<double, 2, 12, true>(a, st);
    if (m <= 16) return launch_column4_t<double, 2, 16, true>(a, st);
    if (m <= 20) return launch_column4_t<double, 2, 20, true>(a, st);
    return launch_column4_t<double, 2, 24, true>(a, st);
}

static const ColumnEntry kFused[] = {
    {2, 2, false, 1, staged<true, 2, 2, false>},
    {2, 4, false, 1, staged<true, 2, 4, false>},
    {2, 2, true, 1, staged<true, 2, 2, true>},
    {2, 2, true, 2, pipelined<2, 2, true, false>},
    {4, 2, true, 2, pipelined<4, 2, true, false>},
};

bool column_variant_f64(const ColumnVariant &v) {
    if (v.sched == SCHED_FOUR) return v.tile_j == 1 && v.prefetch == 2 && v.nt;
    return find_column_entry(kFused, v) != nullptr;
}

hipError_t launch_column_f64(bool fused, const ColumnArgs &a, const ColumnVariant &v, hipStream_t st) {
    if (!fused) return staged<false, 2, 2, false>(a, st);
    if (v.sched == SCHED_FOUR) return four_lanes(a, st);
    const ColumnEntry *e = find_column_entry(kFused, v);
    return e ? e->launch(a, st) : hipErrorInvalidValue;
}

}  // namespace stl
