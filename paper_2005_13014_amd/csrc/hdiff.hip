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
// The inputs of the next PF levels are prefetched into registers.
#include <type_traits>

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
template <class T, class TO, int TJ, int UJ, int PF>
__global__ __launch_bounds__(64 * TJ) void k_hdiff(HdiffArgs p) {
    using S = Storage<T>;
    using C = typename S::C;
    constexpr int TI = 64, RJ = TJ * UJ, PI = TI + 4, PJ = RJ + 4;
    constexpr int MR = (PJ + TJ - 1) / TJ;
    __shared__ C tile[2][PJ * PI];

    const T *__restrict__ u = static_cast<const T *>(p.u);
    const T *__restrict__ coeff = static_cast<const T *>(p.coeff);
    TO *__restrict__ out = static_cast<TO *>(p.out);

    const int tid = threadIdx.x, ti = tid & 63, tj = tid >> 6;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int bi = t % p.nbi, bj = t / p.nbi;
    const int i0 = bi * TI, j0 = bj * RJ;
    const int gi = i0 + ti;
    const int jr = tj * UJ;  // first tile row (interior numbering) of this lane

    int moff[MR], mlds[MR];
    bool mrow[MR], mok[MR];
#pragma unroll
    for (int m = 0; m < MR; ++m) {
        const int r = tj + m * TJ, gy = j0 - 2 + r;
        mrow[m] = r < PJ;
        mok[m] = mrow[m] && gi < p.I + 2 && gy < p.J + 2;
        moff[m] = gi + gy * p.sj;
        mlds[m] = r * PI + ti + 2;
    }
    const int sr = tid >> 2, sq = tid & 3;
    const int sc = sq < 2 ? sq : sq + 64;
    const int sgx = i0 - 2 + sc, sgy = j0 - 2 + sr;
    const bool srow = tid < 4 * PJ;
    const bool sok = srow && sgx < p.I + 2 && sgy < p.J + 2;
    const int soff = sgx + sgy * p.sj;
    const int slds = sr * PI + sc;

    int coff[UJ];
    bool cact[UJ];
#pragma unroll
    for (int v = 0; v < UJ; ++v) {
        const int gj = j0 + jr + v;
        cact[v] = gi < p.I && gj < p.J;
        coff[v] = min(gi, p.I - 1) + min(gj, p.J - 1) * p.sj;
    }

    C rum[PF][MR], rus[PF], rcf[PF][UJ];
    auto load = [&](int q, int k) {
        const int ko = k * p.sk;
#pragma unroll
        for (int m = 0; m < MR; ++m) rum[q][m] = mok[m] ? S::load(u + moff[m] + ko) : C(0);
        rus[q] = sok ? S::load(u + soff + ko) : C(0);
#pragma unroll
        for (int v = 0; v < UJ; ++v) rcf[q][v] = S::load(coeff + coff[v] + ko);
    };

    const int K = p.K;
#pragma unroll
    for (int q = 0; q < PF; ++q)
        if (q < K) load(q, q);

    for (int k0 = 0; k0 < K; k0 += PF) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int k = k0 + q;
            if (k < K) {
                C *tb = tile[q & 1];  // PF is even, so q & 1 == k & 1
#pragma unroll
                for (int m = 0; m < MR; ++m)
                    if (mrow[m]) tb[mlds[m]] = rum[q][m];
                if (srow) tb[slds] = rus[q];
                C cf[UJ];
#pragma unroll
                for (int v = 0; v < UJ; ++v) cf[v] = rcf[q][v];
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
                        if constexpr (std::is_same<TO, C>::value)
                            out[coff[v] + k * p.sk] = h;
                        else
                            S::store(out + coff[v] + k * p.sk, h);
                    }
                }
            }
        }
    }
}

template <class T, int TJ, int UJ, int PF, class TO = T>
static hipError_t launch_hdiff_t(HdiffArgs a, hipStream_t st) {
    a.nbi = (a.I + 63) / 64;
    a.nbj = (a.J + TJ * UJ - 1) / (TJ * UJ);
    hipLaunchKernelGGL((k_hdiff<T, TO, TJ, UJ, PF>), dim3(a.nbi * a.nbj), dim3(64 * TJ), 0, st, a);
    return hipGetLastError();
}

template <class T>
static hipError_t hdiff_unroll(const HdiffArgs &a, int unroll, hipStream_t st) {
    switch (unroll) {
    case 1: return launch_hdiff_t<T, 4, 1, 4>(a, st);
    case 2: return launch_hdiff_t<T, 4, 2, 4>(a, st);
    case 4: return launch_hdiff_t<T, 4, 4, 4>(a, st);
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
