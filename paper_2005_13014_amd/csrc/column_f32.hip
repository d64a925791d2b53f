// Column kernels (column.hpp, column4.hpp) instantiated for float storage.
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
    constexpr bool X = FUSED && NT;
    if (m <= 16) return X && a.K == 32 ? launch_column_t<float, FUSED, TJ, PF, 16, 2, NT, X>(a, st)
                                       : launch_column_t<float, FUSED, TJ, PF, 16, 2, NT>(a, st);
    if (m <= 32) return X && a.K == 64 ? launch_column_t<float, FUSED, TJ, PF, 32, 2, NT, X>(a, st)
                                       : launch_column_t<float, FUSED, TJ, PF, 32, 2, NT>(a, st);
    if (m <= 40) return X && a.K == 80 ? launch_column_t<float, FUSED, TJ, PF, 40, 2, NT, X>(a, st)
                                       : launch_column_t<float, FUSED, TJ, PF, 40, 2, NT>(a, st);
    return X && a.K == 96 ? launch_column_t<float, FUSED, TJ, PF, 48, 1, NT, X>(a, st)
                          : launch_column_t<float, FUSED, TJ, PF, 48, 1, NT>(a, st);
}

template <int TJ, int PF, bool NT, bool CHAIN, int TI = 64>
static hipError_t pipelined(const ColumnArgs &a, hipStream_t st) {
    const int m = (a.K + 1) / 2;
    if (m <= 16) return a.K == 32 ? launch_column_pipe_t<float, TJ, PF, 16, 2, NT, true, CHAIN, TI>(a, st)
                                  : launch_column_pipe_t<float, TJ, PF, 16, 2, NT, false, CHAIN, TI>(a, st);
    if (m <= 32) return a.K == 64 ? launch_column_pipe_t<float, TJ, PF, 32, 2, NT, true, CHAIN, TI>(a, st)
                                  : launch_column_pipe_t<float, TJ, PF, 32, 2, NT, false, CHAIN, TI>(a, st);
    if (m <= 40) return a.K == 80 ? launch_column_pipe_t<float, TJ, PF, 40, 2, NT, true, CHAIN, TI>(a, st)
                                  : launch_column_pipe_t<float, TJ, PF, 40, 2, NT, false, CHAIN, TI>(a, st);
    return a.K == 96 ? launch_column_pipe_t<float, TJ, PF, 48, 1, NT, true, CHAIN, TI>(a, st)
                     : launch_column_pipe_t<float, TJ, PF, 48, 1, NT, false, CHAIN, TI>(a, st);
}

// Four lanes per column: segments of ceil(nk / 4) <= KH levels, nk >= 8,
// 4 levels prefetched.
static hipError_t four_lanes(const ColumnArgs &a, hipStream_t st) {
    const int m = (a.K + 3) / 4;
    if (m <= 8) return launch_column4_t<float, 4, 8, true>(a, st);
    if (m <= 12) return launch_column4_t<float, 4, 12, true>(a, st);
    if (m <= 16) return launch_column4_t<float, 4, 16, true>(a, st);
    if (m <= 20) return launch_column4_t<float, 4, 20, true>(a, st);
    return launch_column4_t<float, 4, 24, true>(a, st);
}

static const ColumnEntry kFused[] = {
    {2, 4, false, 1, staged<true, 2, 4, false>},
    {4, 4, false, 1, staged<true, 4, 4, false>},
    {2, 2, false, 1, staged<true, 2, 2, false>},
    {2, 8, false, 1, staged<true, 2, 8, false>},
    {1, 4, false, 1, staged<true, 1, 4, false>},
    {2, 4, true, 1, staged<true, 2, 4, true>},
    {4, 4, true, 1, staged<true, 4, 4, true>},
    {2, 8, true, 1, staged<true, 2, 8, true>},
    {2, 2, true, 1, staged<true, 2, 2, true>},
    {2, 4, true, 2, pipelined<2, 4, true, false>},
    {2, 8, true, 2, pipelined<2, 8, true, false>},
    {2, 4, true, 3, pipelined<2, 4, true, true>},
    {4, 4, true, 2, pipelined<4, 4, true, false>},
    {4, 2, true, 2, pipelined<4, 2, true, false>},
    {1, 4, true, 2, pipelined<1, 4, true, false>},
    {2, 2, true, 2, pipelined<2, 2, true, false>},
    // wider tiles: longer contiguous row segments per field and level
    {1, 4, true, 2, pipelined<1, 4, true, false, 128>, 128},
    {2, 4, true, 2, pipelined<2, 4, true, false, 128>, 128},
    {1, 4, true, 2, pipelined<1, 4, true, false, 256>, 256},
};

bool column_variant_f32(const ColumnVariant &v) {
    if (v.sched == SCHED_FOUR) return v.tile_j == 1 && v.prefetch == 4 && v.nt;
    return find_column_entry(kFused, v) != nullptr;
}

hipError_t launch_column_f32(bool fused, const ColumnArgs &a, const ColumnVariant &v, hipStream_t st) {
    if (!fused) return staged<false, 2, 4, false>(a, st);
    if (v.sched == SCHED_FOUR) return four_lanes(a, st);
    const ColumnEntry *e = find_column_entry(kFused, v);
    return e ? e->launch(a, st) : hipErrorInvalidValue;
}

}  // namespace stl
