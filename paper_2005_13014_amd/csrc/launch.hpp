// Host-side declarations of the kernel launchers (one set per kernel family
// and storage type).  Launchers enqueue on `st` and return the launch status.
#pragma once

#include <algorithm>

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace stl {

enum { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2 };

// Column kernels (column.hpp): register-resident half columns serve
// nk <= KMAX_COLUMN.  A fused variant is chosen by rows per workgroup,
// levels prefetched, non-temporal streams and the level-loop schedule
// (staged; pipelined, so hdiff of one level overlaps the elimination of an
// earlier one; pipelined on a persistent grid that chains tiles; or four
// lanes per column, partitioned, for small grids); only the compiled
// combinations are accepted.
constexpr int KMAX_COLUMN = 96;
enum { SCHED_STAGED = 1, SCHED_PIPELINED = 2, SCHED_PERSISTENT = 3, SCHED_FOUR = 4 };
struct ColumnVariant {
    int tile_j, prefetch;
    bool nt;
    int sched;        // SCHED_*
    int tile_i = 64;  // columns per tile row (pipelined kernels)
};
bool column_variant_f64(const ColumnVariant &v);
bool column_variant_f32(const ColumnVariant &v);
bool column_variant_bf16(const ColumnVariant &v);
hipError_t launch_column_f64(bool fused, const ColumnArgs &a, const ColumnVariant &v, hipStream_t st);
hipError_t launch_column_f32(bool fused, const ColumnArgs &a, const ColumnVariant &v, hipStream_t st);
hipError_t launch_column_bf16(bool fused, const ColumnArgs &a, const ColumnVariant &v, hipStream_t st);

// Horizontal diffusion alone, inlined, with j-unroll 1, 2 or 4 (hdiff.hip).
hipError_t launch_hdiff(int dtype, const HdiffArgs &a, int unroll, hipStream_t st);
// Same operator, result kept in the compute type (double for F64, else float).
hipError_t launch_hdiff_compute(int dtype, const HdiffArgs &a, hipStream_t st);

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

// Reverse mode of the fused program (adjoint.hip).  All fields share strides;
// gu has a halo of at least 2.  scratch: adjoint_scratch_bytes() bytes.
struct AdjointArgs {
    const void *u, *coeff, *wcon, *a, *b, *c, *w;
    void *gu, *gcoeff, *gwcon;
    const void *x;         // forward result; read only when ga, gb or gc is set
    void *ga, *gb, *gc;    // optional matrix gradients (nullptr skips)
    int I, J, K, sj, sk;
    double dt;
    int hdiff_schedule;    // hdiff adjoint: 1 the LDS-staged tile, else register strips
    int hdiff_tile_j;      // register strips: rows per strip (4 or 8; FP64 4), 0 default
    int hdiff_prefetch;    // register strips: levels in flight (1 or 2), 0 default
};
constexpr int KMAX_ADJOINT = 96;
size_t adjoint_scratch_bytes(int dtype, int sk, int K);

// Levels per workgroup for a kernel that splits each tile's k range into runs:
// the multiple of `step` (at least min_len, at most K rounded up) that
// minimises rounds x (run length + lead), where a round is one wave of
// `slots` resident workgroups over tiles x ceil(K / run) of them and `lead`
// prices a run's prefetch prologue in levels; ties go to the longer run.
inline int level_run(long long tiles, long long slots, int K, int step, int min_len, int lead) {
    if (slots <= 0) slots = 2048;
    const int top = (K + step - 1) / step * step;
    int best_kc = top;
    long long best = -1;
    for (int kc = std::min(top, (min_len + step - 1) / step * step); kc <= top; kc += step) {
        const long long wgs = tiles * ((K + kc - 1) / kc);
        const long long cost = (wgs + slots - 1) / slots * (kc + lead);
        if (best < 0 || cost <= best) {
            best = cost;
            best_kc = kc;
        }
    }
    return best_kc;
}

// Forward mode (tangent) of the fused program.  u and du at interior
// origins with a halo of at least 2; every other field at its interior
// origin; all share (sj, sk).  Tangent pointers may be NULL (zero); x (the
// forward solution) is read only when da, db or dc is given.  nk <= KMAX_JVP.
struct JvpArgs {
    const void *u, *coeff, *wcon, *a, *b, *c, *x;
    const void *du, *dcoeff, *dwcon, *da, *db, *dc;
    void *dx;
    int I, J, K, sj, sk;
    double dt;
};
constexpr int KMAX_JVP = 96;
hipError_t launch_jvp(int dtype, const JvpArgs &a, hipStream_t st);
hipError_t launch_adjoint(int dtype, const AdjointArgs &a, void *scratch, hipStream_t st);
// The fixed scratch of the reverse pass that allocates nothing: a device
// array of ADJOINT_FIXED_SCRATCH_BYTES in the code object; *out receives the
// current device's address of it (looked up once per device).
constexpr size_t ADJOINT_FIXED_SCRATCH_BYTES = size_t(128) << 20;
hipError_t adjoint_fixed_scratch(void **out);

// Halo exchange between the shares of a horizontally decomposed grid and its
// transpose (halo.hip).  Share (p, q) is s[p + px q]; its interior is ni[p] x
// nj[q] x K; w is the halo width exchanged (every share's halo holds at
// least w cells and every interior at least w).
constexpr int HALO_MAX_SHARES = 64;
struct HaloShare {
    void *origin;
    long long sj, sk;
};
struct HaloArgs {
    HaloShare s[HALO_MAX_SHARES];
    int ni[HALO_MAX_SHARES], nj[HALO_MAX_SHARES];
    int px, py, w, K;
};
hipError_t launch_halo(int dtype, const HaloArgs &a, bool accumulate, hipStream_t st);

// Streaming copy used as the bandwidth probe (probe.hip).
hipError_t launch_probe_copy(const void *src, void *dst, long long nbytes, hipStream_t st);
hipError_t launch_probe_read(const void *src, long long nbytes, unsigned key, void *sink, hipStream_t st);
hipError_t launch_probe_streams(const void *const *src, int nsrc, void *dst, long long nbytes, hipStream_t st);

}  // namespace stl
