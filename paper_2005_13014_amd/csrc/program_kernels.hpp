// Batched timestep kernels: the fused hdiff + vadv (+ vdiff) column kernel
// over a table of subdomains and fields (column.hpp), and the 7-point
// horizontal-gradient update over the same kind of table.
#pragma once

#include "column.hpp"
#include "common.hpp"

namespace stl {

// z = y - beta_h ((y(i+1) - y(i-1))/2 + (y(j+1) - y(j-1))/2) - beta_v Dk y,
// Dk y = (y(k+1) - y(k-1))/2 inside the column, y(1) - y(0) at the bottom and
// y(K-1) - y(K-2) at the top (0 for a single level).  y carries a 1-cell halo.
// Register buckets of the batched column kernels: a half column of up to KH
// levels is held in registers, and a shorter one pays KH - levels padding
// steps (at the same cost as real ones).  Every bucket is a launch of its own
// with its own ramp-up and tail (≈25 us for a few thousand workgroups), so
// finer buckets pay only where they keep subdomains together: KH = 45 serves
// nk 81..90 (84 and 90 levels in one launch, 3 and 0 padding steps).
constexpr int PROGRAM_BUCKETS[] = {16, 32, 40, 45, 48};

constexpr int HGRAD_ROWS = 8;  // rows of an hgrad strip (16 measured slower)
// Levels per wave: a run of consecutive levels (runs of 4, 6, 8, 16, 32 and 96
// levels took 319, 309, 302, 308, 328 and 363 us for the 6 x 8 FP32 step:
// short runs give more waves to hide latency, each run rereads two levels).
constexpr int HGRAD_RUN = 8;

struct HgradSub {
    const void *y[BATCH_FIELDS];  // interior origins
    void *z[BATCH_FIELDS];
    int I, J, K, sj, sk;
    int nbi, nbj, ngroups, nruns, tile0, nfields;
    uint32_t y_bytes, z_bytes;  // addressable bytes from y's cell (-1, -1, 0) and from z's origin
};

struct HgradBatch {
    HgradSub sub[BATCH_SUBS];
    int nsub, kc;
    double beta_h, beta_v;
};

// Register strips: one wave per strip of 64 columns x TJ rows of one field,
// marching a run of kc levels; four independent waves per workgroup (no LDS,
// no barrier).  Workgroups are numbered per subdomain field-major, then run,
// then strip group, so that neighbouring strips share an XCD's L2.  At each
// level a lane holds its column's y on the strip's rows j0 - 1 .. j0 + TJ;
// y(i +- 1) comes from the neighbouring lanes, and for the strip's end lanes
// from one more load per row (lanes 0..31 load y(i0 - 1), lanes 32..63
// y(i0 + 64), the value the end lane is given by the shift; one load per row
// and level measured faster than one per level read out lane by lane);
// y(j +- 1) is the row above or below and y(k +- 1) the previous or next
// level's row.  The next PF levels are requested before a level is computed.
// Cells are clamped into [-1, I] x [-1, J] x [0, K), which only values that
// are never used can reach.
template <class T, int TJ, int PF>
__global__ __launch_bounds__(256) void k_hgrad_strip(HgradBatch b) {
#pragma clang fp contract(off)
    using S = Storage<T>;
    using C = typename S::C;
    using IO = BufIO<T>;
    using R = typename IO::R;
    constexpr int NR = TJ + 2;
    constexpr uint32_t ES = sizeof(T);
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    int s = 0;
    while (s + 1 < b.nsub && b.sub[s + 1].tile0 <= t) ++s;
    const HgradSub &sb = b.sub[s];
    const int local = t - sb.tile0;
    const int group = local % sb.ngroups, rest = local / sb.ngroups;
    const int run = rest % sb.nruns, f = rest / sb.nruns;
    const int strip = group * 4 + __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    if (strip >= sb.nbi * sb.nbj) return;
    const int I = sb.I, J = sb.J, K = sb.K;
    const uint32_t sj = static_cast<uint32_t>(sb.sj), skb = static_cast<uint32_t>(sb.sk) * ES;
    const int k0 = run * b.kc, k1 = min(K, k0 + b.kc);
    const int i0 = (strip % sb.nbi) * 64, j0 = (strip / sb.nbi) * TJ;
    const int lane = threadIdx.x & 63, gi = i0 + lane;
    const bool active_i = gi < I;
    // y from its cell (-1, -1, 0): a lane's own column and its end value.
    const auto ry = make_rsrc(static_cast<const char *>(sb.y[f]) - (1 + sb.sj) * static_cast<int>(ES), sb.y_bytes);
    const auto rz = make_rsrc(sb.z[f], sb.z_bytes);
    const uint32_t v_own = static_cast<uint32_t>(min(gi, I) + 1) * ES;
    const uint32_t v_end = static_cast<uint32_t>(min(lane < 32 ? i0 - 1 : i0 + 64, I) + 1) * ES;
    const uint32_t v_z = static_cast<uint32_t>(min(gi, I - 1)) * ES;
    auto row = [&](int r) {  // byte offset of y row j0 - 1 + r (uniform)
        return static_cast<uint32_t>(min(j0 - 1 + r, J) + 1) * sj * ES;
    };
    auto lev = [&](int k) { return static_cast<uint32_t>(min(max(k, 0), K - 1)) * skb; };

    // Ring of the next PF levels (raw stored bits): slot q holds level
    // k0 + 1 + q + m PF.
    R ring[PF][NR], rend[PF][TJ];
    auto load = [&](int q, int k) {
        const uint32_t so = lev(k);
#pragma unroll
        for (int r = 0; r < NR; ++r) ring[q][r] = IO::load_raw(ry, v_own, row(r) + so);
#pragma unroll
        for (int r = 0; r < TJ; ++r) rend[q][r] = IO::load_raw(ry, v_end, row(r + 1) + so);
    };
    C dn[TJ], cur[NR], end[TJ];
    {
        R d0[TJ], c0[NR], e0[TJ];
#pragma unroll
        for (int r = 0; r < TJ; ++r) d0[r] = IO::load_raw(ry, v_own, row(r + 1) + lev(k0 - 1));
#pragma unroll
        for (int r = 0; r < NR; ++r) c0[r] = IO::load_raw(ry, v_own, row(r) + lev(k0));
#pragma unroll
        for (int r = 0; r < TJ; ++r) e0[r] = IO::load_raw(ry, v_end, row(r + 1) + lev(k0));
#pragma unroll
        for (int q = 0; q < PF; ++q) load(q, k0 + 1 + q);
#pragma unroll
        for (int r = 0; r < TJ; ++r) {
            dn[r] = IO::cvt(d0[r]);
            end[r] = IO::cvt(e0[r]);
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) cur[r] = IO::cvt(c0[r]);
    }

    const C bh = static_cast<C>(b.beta_h), bv = static_cast<C>(b.beta_v), half = C(0.5);
    for (int kk = k0; kk < k1; kk += PF) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int k = kk + q;
            if (k >= k1) break;
            C up[TJ];
#pragma unroll
            for (int r = 0; r < TJ; ++r) up[r] = IO::cvt(ring[q][r + 1]);
            const uint32_t so = static_cast<uint32_t>(k) * skb;
#pragma unroll
            for (int r = 0; r < TJ; ++r) {
                const C yc = cur[r + 1];
                const C ye = lane_next(yc, end[r]), yw = lane_prev(yc, end[r]);
                const C gi_ = half * (ye - yw);
                const C gj_ = half * (cur[r + 2] - cur[r]);
                C gk;
                if (K == 1)
                    gk = C(0);
                else if (k == 0)
                    gk = up[r] - yc;
                else if (k == K - 1)
                    gk = yc - dn[r];
                else
                    gk = half * (up[r] - dn[r]);
                const C z = yc - bh * (gi_ + gj_) - bv * gk;
                const int j = j0 + r;
                if (active_i && j < J)
                    IO::template store_d<2>(rz, v_z, static_cast<uint32_t>(j) * sj * ES + so, static_cast<double>(z));
            }
#pragma unroll
            for (int r = 0; r < TJ; ++r) {
                dn[r] = cur[r + 1];
                end[r] = IO::cvt(rend[q][r]);
            }
#pragma unroll
            for (int r = 0; r < NR; ++r) cur[r] = IO::cvt(ring[q][r]);
            if (k + 1 + PF <= k1) load(q, k + 1 + PF);
        }
    }
}

// PIPE: the software-pipelined tile, else the staged one.
template <class T, int VD, int TJ, int PF, int KH, int WPE, bool PIPE = false>
static hipError_t launch_column_batch_t(const ColumnBatch &b, int ntiles, hipStream_t st) {
    if constexpr (PIPE)
        hipLaunchKernelGGL((k_column_batch_pipe<T, VD, TJ, PF, KH, WPE>), dim3(ntiles), dim3(128 * TJ), 0, st,
                           b);
    else
        hipLaunchKernelGGL((k_column_batch<T, VD, TJ, PF, KH, WPE>), dim3(ntiles), dim3(128 * TJ), 0, st,
                           b);
    return hipGetLastError();
}

template <class T>
static hipError_t launch_hgrad_batch_t(const HgradBatch &b, int ntiles, hipStream_t st) {
    // 4 levels in flight (with runs of 8 levels 2, 3 and 4 measured within 1%); FP64 2, for its registers.
    hipLaunchKernelGGL((k_hgrad_strip<T, HGRAD_ROWS, sizeof(T) == 8 ? 2 : 4>), dim3(ntiles), dim3(256), 0, st, b);
    return hipGetLastError();
}

}  // namespace stl
