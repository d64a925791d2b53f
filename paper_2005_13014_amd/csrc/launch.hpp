// Host-side declarations of the kernel launchers (one set per kernel family
// and storage type).  Launchers enqueue on `st` and return the launch status.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace stl {

enum { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2 };

// Largest vertical extent of the register-resident column kernels, per dtype.
constexpr int KMAX_COLUMN_F64 = 80;
constexpr int KMAX_COLUMN_F32 = 96;

// (tile_j, prefetch) variants of the fused kernel compiled per dtype
// (column_<dtype>.hip).
inline bool fused_variant_compiled(int dtype, int tj, int pf) {
    if (dtype == DT_F64) return tj == 4 && pf == 2;
    if (dtype == DT_BF16) return tj == 4 && pf == 4;
    return (tj == 4 && (pf == 2 || pf == 4 || pf == 8)) || (tj == 2 && pf == 4) ||
           (tj == 1 && pf == 8);
}

// Fused hdiff + vadv (column.hpp); (tile_j, prefetch) picks a compiled variant.
hipError_t launch_fused_f64(const VadvArgs &a, int tile_j, int prefetch, hipStream_t st);
hipError_t launch_fused_f32(const VadvArgs &a, int tile_j, int prefetch, hipStream_t st);
hipError_t launch_fused_bf16(const VadvArgs &a, int tile_j, int prefetch, hipStream_t st);
// vadv alone (column.hpp).
hipError_t launch_vadv_f64(const VadvArgs &a, hipStream_t st);
hipError_t launch_vadv_f32(const VadvArgs &a, hipStream_t st);
hipError_t launch_vadv_bf16(const VadvArgs &a, hipStream_t st);

// Horizontal diffusion alone, inlined, with j-unroll 1, 2 or 4 (hdiff.hip).
hipError_t launch_hdiff(int dtype, const HdiffArgs &a, int unroll, hipStream_t st);

// The "original" level: one kernel per operator through device scratch
// (plain.hip).  u == nullptr runs vadv alone on h; vadv == false runs hdiff
// alone into x.
struct PlainArgs {
    const void *u, *coeff, *h, *wcon, *a, *b, *c;
    void *x;
    void *scratch;  // plain_scratch_bytes() bytes, 256-byte aligned
    int I, J, K, sj, sk;
    double dt;
    bool vadv;
};
size_t plain_scratch_bytes(int dtype, int I, int J, int K, bool vadv);
hipError_t launch_plain(int dtype, const PlainArgs &a, hipStream_t st);

// Streaming copy used as the bandwidth probe (probe.hip).
hipError_t launch_probe_copy(const void *src, void *dst, long long nbytes, hipStream_t st);

}  // namespace stl
