// Horizontal diffusion alone: inlined (one kernel, temporaries on chip) with
// stencil unrolling along j (Sec. V-A).
//
// A workgroup owns a 64 x (TJ*UJ) tile of columns and marches up the k levels.
// Per level, u on the tile plus its 2-cell halo is staged in LDS (double
// buffered, one barrier per level); lane (ti, tj) then evaluates UJ points
// stacked in j.  Unrolling lets neighbouring points share work the way common
// subexpression elimination does in the paper: the Laplacian at the lane's
// own column is computed once for the UJ + 2 rows it touches, and each
// j-flux is computed once and used by the two points on either side of it.
// The inputs of the next PF levels are prefetched into registers (raw stored
// bits, widened where used).  The k range is split into runs of kc levels,
// one per workgroup, so that small grids still give the chip enough
// workgroups.
#include <algorithm>
#include <type_traits>

#include "column.hpp"
#include "common.hpp"
#include "launch.hpp"

namespace stl {

template <class C, int P>
__device__ __forceinline__ C lap_at(const C *t) {
    return C(4) * t[0] - t[1] - t[-1] - t[P] - t[-P];
}

template <class C>
__device__ __forceinline__ C limit(C f, C du) {
    return (f * du > C(0)) ? C(0) : f;
}

// TO = T writes the storage dtype; TO = C keeps the compute type (scratch).
// Fields are addressed through raw buffers (column.hpp): u from its cell
// (-2, -2, 0), coeff and out from their origins; the level offset is scalar.
// (With TO = T = C, as for FP64 and FP32 storage, the buffer store is taken.)
template <class T, class TO, int TJ, int UJ, int PF>
__global__ __launch_bounds__(64 * TJ) void k_hdiff(HdiffArgs p) {
    using S = Storage<T>;
    using C = typename S::C;
    using IO = BufIO<T>;
    constexpr int TI = 64, RJ = TJ * UJ, PI = TI + 4, PJ = RJ + 4;
    constexpr int MR = (PJ + TJ - 1) / TJ;
    constexpr uint32_t ES = sizeof(T);
    __shared__ C tile[2][PJ * PI + 64];

    const int tid = threadIdx.x, ti = tid & 63;
    const int tj = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int pos = xcd_tile(blockIdx.x, gridDim.x), ntiles = p.nbi * p.nbj;
    const int t = pos % ntiles, run = pos / ntiles;
    const int bi = t % p.nbi, bj = t / p.nbi;
    const int i0 = bi * TI, j0 = bj * RJ;
    const int gi = i0 + ti;
    const int jr = tj * UJ;  // first tile row (interior numbering) of this lane
    const int I = p.I, J = p.J, sj = p.sj;
    const uint32_t skb = static_cast<uint32_t>(p.sk) * ES;

    const auto ru = make_rsrc(static_cast<const char *>(p.u) - (2 + 2 * sj) * static_cast<int>(ES),
                              p.u_bytes);
    const auto rcf = make_rsrc(p.coeff, p.col_bytes);
    const auto rout = make_rsrc(p.out, p.col_bytes);

    // Tile element (r, c) holds u(i0 - 2 + c, j0 - 2 + r); loads past the
    // addressable ring are clamped onto valid cells (never read by an active lane).
    uint32_t vmain[MR];
    int lmain[MR];
    bool mrow[MR];
#pragma unroll
    for (int m = 0; m < MR; ++m) {
        const int r = tj + m * TJ;
        mrow[m] = r < PJ;
        const int gx = min(gi, I + 1), gy = min(j0 - 2 + r, J + 1);
        vmain[m] = static_cast<uint32_t>(gx + 2 + (gy + 2) * sj) * ES;
        lmain[m] = r * PI + ti + 2;
    }
    // The 4 PJ side cells are staged by lanes 0 .. 4 PJ - 1 of the workgroup,
    // i.e. by its first (4 PJ + 63) / 64 waves; their remaining lanes write a
    // dummy slot.
    const bool side_wave = tj < (4 * PJ + 63) / 64;
    const int sr = min(tid >> 2, PJ - 1), sq = tid & 3;
    const int sc = sq < 2 ? sq : sq + 64;
    const uint32_t vside =
        static_cast<uint32_t>(min(i0 - 2 + sc, I + 1) + 2 + (min(j0 - 2 + sr, J + 1) + 2) * sj) * ES;
    const int lside = tid < 4 * PJ ? sr * PI + sc : PJ * PI + ti;

    uint32_t vcol[UJ];
    bool cact[UJ];
#pragma unroll
    for (int v = 0; v < UJ; ++v) {
        const int gj = j0 + jr + v;
        cact[v] = gi < I && gj < J;
        vcol[v] = static_cast<uint32_t>(min(gi, I - 1) + min(gj, J - 1) * sj) * ES;
    }

    using R = typename IO::R;
    R rum[PF][MR], rus[PF], rcf_[PF][UJ];
    auto load = [&](int q, int k) {
        const uint32_t so = static_cast<uint32_t>(k) * skb;
#pragma unroll
        for (int m = 0; m < MR; ++m)
            if (mrow[m]) rum[q][m] = IO::load_raw(ru, vmain[m], so);
        if (side_wave) rus[q] = IO::load_raw(ru, vside, so);
#pragma unroll
        for (int v = 0; v < UJ; ++v) rcf_[q][v] = IO::load_raw(rcf, vcol[v], so);
    };

    const int kb = run * p.kc, K = min(p.K, kb + p.kc);
#pragma unroll
    for (int q = 0; q < PF; ++q)
        if (kb + q < K) load(q, kb + q);

    for (int k0 = kb; k0 < K; k0 += PF) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int k = k0 + q;
            if (k < K) {
                C *tb = tile[q & 1];  // PF is even, so q & 1 == (k - kb) & 1
#pragma unroll
                for (int m = 0; m < MR; ++m)
                    if (mrow[m]) tb[lmain[m]] = IO::cvt(rum[q][m]);
                if (side_wave) tb[lside] = IO::cvt(rus[q]);
                C cf[UJ];
#pragma unroll
                for (int v = 0; v < UJ; ++v) cf[v] = IO::cvt(rcf_[q][v]);
                if (k + PF < K) load(q, k + PF);
                __syncthreads();

                // Centre column, rows jr - 1 .. jr + UJ (tile rows offset by 2).
                const C *c0 = tb + (jr + 2) * PI + ti + 2;
                C lc[UJ + 2], uc[UJ + 2];
#pragma unroll
                for (int v = -1; v <= UJ; ++v) {
                    lc[v + 1] = lap_at<C, PI>(c0 + v * PI);
                    uc[v + 1] = c0[v * PI];
                }
                // j-fluxes between consecutive rows: fly at row jr + v, v = -1 .. UJ-1.
                C fy[UJ + 1];
#pragma unroll
                for (int v = 0; v <= UJ; ++v) fy[v] = limit(lc[v + 1] - lc[v], uc[v + 1] - uc[v]);
#pragma unroll
                for (int v = 0; v < UJ; ++v) {
                    const C *cv = c0 + v * PI;
                    const C le = lap_at<C, PI>(cv + 1), lw = lap_at<C, PI>(cv - 1);
                    const C fe = limit(le - lc[v + 1], cv[1] - uc[v + 1]);
                    const C fw = limit(lc[v + 1] - lw, uc[v + 1] - cv[-1]);
                    const C h = uc[v + 1] - cf[v] * (fe - fw + fy[v + 1] - fy[v]);
                    if (cact[v]) {
                        if constexpr (std::is_same<TO, T>::value) {
                            // Storage output: a non-temporal buffer store (no output
                            // line displaces the inputs' halo rows in the caches).
                            IO::template store_d<2>(rout, vcol[v], static_cast<uint32_t>(k) * skb,
                                                    static_cast<double>(h));
                        } else {
                            const uint32_t o = vcol[v] / ES + static_cast<uint32_t>(k) * p.sk;
                            static_cast<TO *>(p.out)[o] = h;
                        }
                    }
                }
            }
        }
    }
}

template <class T, int TJ, int UJ, int PF, class TO = T>
static hipError_t launch_hdiff_t(HdiffArgs a, hipStream_t st) {
    if (a.I <= 0 || a.J <= 0 || a.K <= 0) return hipSuccess;
    a.nbi = (a.I + 63) / 64;
    a.nbj = (a.J + TJ * UJ - 1) / (TJ * UJ);
    const long long es = sizeof(T);
    a.u_bytes = static_cast<uint32_t>(((a.I + 3) + static_cast<long long>(a.J + 3) * a.sj +
                                       static_cast<long long>(a.K - 1) * a.sk + 1) * es);
    a.col_bytes = static_cast<uint32_t>(((a.I - 1) + static_cast<long long>(a.J - 1) * a.sj +
                                         static_cast<long long>(a.K - 1) * a.sk + 1) * es);
    // Runs of levels sized against the resident workgroups, each a multiple
    // of PF and at least 2 PF levels long.
    const long long tiles = static_cast<long long>(a.nbi) * a.nbj;
    auto kern = k_hdiff<T, TO, TJ, UJ, PF>;
    const long long slots = resident_workgroups(reinterpret_cast<const void *>(kern), 64 * TJ);
    a.kc = level_run(tiles, slots, a.K, PF, 2 * PF, PF);
    const long long blocks = tiles * ((a.K + a.kc - 1) / a.kc);
    if (blocks > 2147483647LL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(blocks)), dim3(64 * TJ), 0, st, a);
    return hipGetLastError();
}

template <class T>
static hipError_t hdiff_unroll(const HdiffArgs &a, int unroll, hipStream_t st) {
    switch (unroll) {
    case 1: return launch_hdiff_t<T, 16, 1, 4>(a, st);
    case 2: return launch_hdiff_t<T, 8, 2, 4>(a, st);
    case 4: return launch_hdiff_t<T, 8, 4, 4>(a, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_hdiff_compute(int dtype, const HdiffArgs &a, hipStream_t st) {
    switch (dtype) {
    case DT_F64: return launch_hdiff_t<double, 4, 1, 4, double>(a, st);
    case DT_F32: return launch_hdiff_t<float, 4, 1, 4, float>(a, st);
    case DT_BF16: return launch_hdiff_t<uint16_t, 4, 1, 4, float>(a, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_hdiff(int dtype, const HdiffArgs &a, int unroll, hipStream_t st) {
    switch (dtype) {
    case DT_F64: return hdiff_unroll<double>(a, unroll, st);
    case DT_F32: return hdiff_unroll<float>(a, unroll, st);
    case DT_BF16: return hdiff_unroll<uint16_t>(a, unroll, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace stl
