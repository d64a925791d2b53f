// Column kernels (column.hpp) instantiated for bfloat16 storage.
#include "column.hpp"

#include "launch.hpp"

namespace stl {

// Register-resident half columns of KH levels serve nk <= 2 KH; a depth
// that fills its bucket exactly (nk = 2 KH) takes the kernel without
// padding steps.
template <bool FUSED, int TJ, int PF, bool NT>
static hipError_t staged(const ColumnArgs &a, hipStream_t st) {
    const int m = (a.K + 1) / 2;
    constexpr bool X = FUSED;
    if (m <= 16) return X && a.K == 32 ? launch_column_t<uint16_t, FUSED, TJ, PF, 16, 2, NT, X>(a, st)
                                       : launch_column_t<uint16_t, FUSED, TJ, PF, 16, 2, NT>(a, st);
    if (m <= 32) return X && a.K == 64 ? launch_column_t<uint16_t, FUSED, TJ, PF, 32, 2, NT, X>(a, st)
                                       : launch_column_t<uint16_t, FUSED, TJ, PF, 32, 2, NT>(a, st);
    if (m <= 40) return X && a.K == 80 ? launch_column_t<uint16_t, FUSED, TJ, PF, 40, 2, NT, X>(a, st)
                                       : launch_column_t<uint16_t, FUSED, TJ, PF, 40, 2, NT>(a, st);
    return X && a.K == 96 ? launch_column_t<uint16_t, FUSED, TJ, PF, 48, 1, NT, X>(a, st)
                          : launch_column_t<uint16_t, FUSED, TJ, PF, 48, 1, NT>(a, st);
}

template <int TJ, int PF, bool NT, bool CHAIN>
static hipError_t pipelined(const ColumnArgs &a, hipStream_t st) {
    const int m = (a.K + 1) / 2;
    if (m <= 16) return a.K == 32 ? launch_column_pipe_t<uint16_t, TJ, PF, 16, 2, NT, true, CHAIN>(a, st)
                                  : launch_column_pipe_t<uint16_t, TJ, PF, 16, 2, NT, false, CHAIN>(a, st);
    if (m <= 32) return a.K == 64 ? launch_column_pipe_t<uint16_t, TJ, PF, 32, 2, NT, true, CHAIN>(a, st)
                                  : launch_column_pipe_t<uint16_t, TJ, PF, 32, 2, NT, false, CHAIN>(a, st);
    if (m <= 40) return a.K == 80 ? launch_column_pipe_t<uint16_t, TJ, PF, 40, 2, NT, true, CHAIN>(a, st)
                                  : launch_column_pipe_t<uint16_t, TJ, PF, 40, 2, NT, false, CHAIN>(a, st);
    return a.K == 96 ? launch_column_pipe_t<uint16_t, TJ, PF, 48, 1, NT, true, CHAIN>(a, st)
                     : launch_column_pipe_t<uint16_t, TJ, PF, 48, 1, NT, false, CHAIN>(a, st);
}

static const ColumnEntry kFused[] = {
    {2, 4, false, 1, staged<true, 2, 4, false>},
    {4, 4, false, 1, staged<true, 4, 4, false>},
    {2, 4, true, 1, staged<true, 2, 4, true>},
    {2, 4, true, 2, pipelined<2, 4, true, false>},
    {2, 8, true, 2, pipelined<2, 8, true, false>},
    {4, 4, true, 2, pipelined<4, 4, true, false>},
};

bool column_variant_bf16(const ColumnVariant &v) {
    if (v.sched == SCHED_FOUR) return false;
    return find_column_entry(kFused, v) != nullptr;
}

hipError_t launch_column_bf16(bool fused, const ColumnArgs &a, const ColumnVariant &v, hipStream_t st) {
    if (!fused) return staged<false, 2, 4, false>(a, st);
    const ColumnEntry *e = find_column_entry(kFused, v);
    return e ? e->launch(a, st) : hipErrorInvalidValue;
}

}  // namespace stl
