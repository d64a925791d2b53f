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

template <class T>
__global__ __launch_bounds__(256) void k_hgrad_batch(HgradBatch b) {
    using S = Storage<T>;
    using C = typename S::C;
    using IO = BufIO<T>;
    constexpr uint32_t ES = sizeof(T);
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    int s = 0;
    while (s + 1 < b.nsub && b.sub[s + 1].tile0 <= t) ++s;
    const HgradSub &sb = b.sub[s];
    const int local = t - sb.tile0;
    const int f = local % sb.nfields, tile = local / sb.nfields;
    const int bi = tile % sb.nbi, bj = tile / sb.nbi;
    const int gi = bi * 64 + (threadIdx.x & 63), gj = bj * 4 + (threadIdx.x >> 6);
    if (gi >= sb.I || gj >= sb.J) return;
    const int sj = sb.sj, K = sb.K;
    // y is addressed from its cell (-1, -1, 0).
    const auto ry = make_rsrc(static_cast<const char *>(sb.y[f]) - (1 + sj) * static_cast<int>(ES),
                              sb.y_bytes);
    const auto rz = make_rsrc(sb.z[f], sb.z_bytes);
    const uint32_t vc = static_cast<uint32_t>(gi + 1 + (gj + 1) * sj) * ES;
    const uint32_t ve = vc + ES, vw = vc - ES, vn = vc + sj * ES, vs = vc - sj * ES;
    const uint32_t vz = static_cast<uint32_t>(gi + gj * sj) * ES;
    const uint32_t skb = static_cast<uint32_t>(sb.sk) * ES;
    const C bh = static_cast<C>(b.beta_h), bv = static_cast<C>(b.beta_v), half = C(0.5);
    C y_dn = C(0), y_c = IO::load(ry, vc, 0);
    for (int k = 0; k < K; ++k) {
        const uint32_t so = k * skb;
        const C y_up = k + 1 < K ? IO::load(ry, vc, so + skb) : C(0);
        const C gi_ = half * (IO::load(ry, ve, so) - IO::load(ry, vw, so));
        const C gj_ = half * (IO::load(ry, vn, so) - IO::load(ry, vs, so));
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
        IO::store_d(rz, vz, so, static_cast<double>(z));
        y_dn = y_c;
        y_c = y_up;
    }
}

template <class T, bool VDIFF, int TJ, int PF, int KH, int WPE>
static hipError_t launch_column_batch_t(const ColumnBatch &b, int ntiles, hipStream_t st) {
    hipLaunchKernelGGL((k_column_batch<T, VDIFF, TJ, PF, KH, WPE>), dim3(ntiles), dim3(128 * TJ), 0, st,
                       b);
    return hipGetLastError();
}

template <class T>
static hipError_t launch_hgrad_batch_t(const HgradBatch &b, int ntiles, hipStream_t st) {
    hipLaunchKernelGGL((k_hgrad_batch<T>), dim3(ntiles), dim3(256), 0, st, b);
    return hipGetLastError();
}

}  // namespace stl
