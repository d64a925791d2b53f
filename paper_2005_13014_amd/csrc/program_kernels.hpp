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
constexpr int HGRAD_ROWS = 4;  // rows of an hgrad tile, one wave each (8 measured no faster)

struct HgradSub {
    const void *y[BATCH_FIELDS];  // interior origins
    void *z[BATCH_FIELDS];
    int I, J, K, sj, sk;
    int nbi, nbj, tile0, nfields;
    uint32_t y_bytes, z_bytes;  // addressable bytes from y's cell (-1, -1, 0) and from z's origin
};

struct HgradBatch {
    HgradSub sub[BATCH_SUBS];
    int nsub;
    double beta_h, beta_v;
};

// One 64 x TR tile of one field per workgroup (one wave per row), marching k.
// Per level the tile's y rows j0 - 1 .. j0 + TR and its side columns i0 - 1, i0 + 64 are
// staged in LDS (each wave loads its own row, which holds its centre values;
// waves 0 and 1 also load the rows above and below the tile, wave 2 the side
// columns), the horizontal neighbours are read from the tile and the vertical
// ones are kept in registers.  Loads run PF levels ahead.
template <class T, int TR = HGRAD_ROWS, int PF = 8>
__global__ __launch_bounds__(64 * TR) void k_hgrad_batch(HgradBatch b) {
    static_assert(PF % 2 == 0, "the LDS tile alternates with the ring slot");
    static_assert(TR >= 3 && 2 * (TR + 2) <= 64, "wave 2 stages both side columns of every tile row");
    using S = Storage<T>;
    using C = typename S::C;
    using IO = BufIO<T>;
    constexpr int PI = 68, ROWS = TR + 2, TILE = ROWS * PI;
    constexpr uint32_t ES = sizeof(T);
    __shared__ C tile[2 * TILE];
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    int s = 0;
    while (s + 1 < b.nsub && b.sub[s + 1].tile0 <= t) ++s;
    const HgradSub &sb = b.sub[s];
    const int local = t - sb.tile0;
    const int f = local % sb.nfields, tl = local / sb.nfields;
    const int bi = tl % sb.nbi, bj = tl / sb.nbi;
    const int tid = threadIdx.x, ti = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int I = sb.I, J = sb.J, sj = sb.sj, K = sb.K;
    const int i0 = bi * 64, j0 = bj * TR;
    const int gi = i0 + ti, gj = j0 + w;
    const bool active = gi < I && gj < J;
    // y is addressed from its cell (-1, -1, 0); cells are clamped into
    // [-1, I] x [-1, J], which only lanes that store nothing can reach.
    const auto ry = make_rsrc(static_cast<const char *>(sb.y[f]) - (1 + sj) * static_cast<int>(ES), sb.y_bytes);
    const auto rz = make_rsrc(sb.z[f], sb.z_bytes);
    auto voff = [&](int i, int j) {
        return static_cast<uint32_t>(min(max(i, -1), I) + 1 + (min(max(j, -1), J) + 1) * sj) * ES;
    };
    const uint32_t v_own = voff(gi, gj);
    // Second row: wave 0 the row above the tile (tile row 0), wave 1 the row
    // below it (tile row TR + 1), wave 2 the side columns (lanes 0 .. 2 ROWS - 1),
    // the other waves none.
    const int sr = ti >> 1, scol = (ti & 1) ? 65 : 0;  // side: tile row, tile column
    const uint32_t v_two = w == 0 ? voff(gi, j0 - 1) : w == 1 ? voff(gi, j0 + TR) : voff(i0 - 1 + scol, j0 - 1 + min(sr, ROWS - 1));
    const bool two = w < 2 || (w == 2 && ti < 2 * ROWS);
    const int l_own = (w + 1) * PI + ti + 1;
    const int l_two = w == 0 ? ti + 1 : w == 1 ? (TR + 1) * PI + ti + 1 : min(sr, ROWS - 1) * PI + scol;
    const uint32_t vz = static_cast<uint32_t>(min(gi, I - 1) + min(gj, J - 1) * sj) * ES;
    const uint32_t skb = static_cast<uint32_t>(sb.sk) * ES;

    // Register ring of the next PF levels (raw stored bits, widened where
    // used): slot q holds level k with k % PF == q.
    using R = typename IO::R;
    R own[PF], tw[PF];
    // Levels past the top are clamped to it (their values are never used),
    // so no load sits behind a branch whose join would wait for it.
    auto load = [&](int q, int k) {
        const uint32_t so = static_cast<uint32_t>(min(k, K - 1)) * skb;
        own[q] = IO::load_raw(ry, v_own, so);
        tw[q] = IO::load_raw(ry, v_two, so);
    };
#pragma unroll
    for (int q = 0; q < PF; ++q) load(q, q);

    const C bh = static_cast<C>(b.beta_h), bv = static_cast<C>(b.beta_v), half = C(0.5);
    C y_dn = C(0), y_c = IO::cvt(own[0]);
    for (int k0 = 0; k0 < K; k0 += PF) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int k = k0 + q;
            if (k >= K) break;
            C *tb = &tile[(q & 1) * TILE];  // PF is even: q & 1 == k & 1
            tb[l_own] = IO::cvt(own[q]);
            if (two) tb[l_two] = IO::cvt(tw[q]);
            const C y_up = k + 1 < K ? IO::cvt(own[(q + 1) % PF]) : C(0);
            load(q, k + PF);
            __syncthreads();
            const C *c = &tb[(w + 1) * PI + ti + 1];
            const C gi_ = half * (c[1] - c[-1]);
            const C gj_ = half * (c[PI] - c[-PI]);
            C gk;
            if (K == 1)
                gk = C(0);
            else if (k == 0)
                gk = y_up - y_c;
            else if (k == K - 1)
                gk = y_c - y_dn;
            else
                gk = half * (y_up - y_dn);
            const C z = y_c - bh * (gi_ + gj_) - bv * gk;
            if (active) IO::template store_d<2>(rz, vz, static_cast<uint32_t>(k) * skb, static_cast<double>(z));
            y_dn = y_c;
            y_c = y_up;
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
    hipLaunchKernelGGL((k_hgrad_batch<T>), dim3(ntiles), dim3(64 * HGRAD_ROWS), 0, st, b);
    return hipGetLastError();
}

}  // namespace stl
