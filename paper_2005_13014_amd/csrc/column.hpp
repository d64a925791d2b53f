// Column kernels: the fused hdiff + vadv program and vadv alone.
//
// One lane owns one (i, j) column and marches up the k levels.  Per level it
// (1) stages the u tile with its 2-cell halo into LDS (fused kernel only),
// (2) evaluates the horizontal-diffusion operator from the tile, (3) forms the
// flux-form right-hand side of the level below, whose upper face needs h one
// level ahead, and (4) takes one Thomas forward-elimination step in double
// precision.  The eliminated coefficients c'(k), d'(k) of the whole column
// stay in registers (the level loop is fully unrolled over a compile-time
// bound KMAX >= K, so the arrays are only indexed with constants), and the
// back-substitution then writes x from the top level down.  Every input is
// read from device memory once and x written once: the temporaries lap, flx,
// fly, h, d, c', d' never leave the chip (stencil inlining, Sec. V-A).  Inputs
// of the next PF levels are loaded ahead into a register ring so that many
// loads stay in flight while a level is being computed.
//
// Thomas forward elimination (double precision):
//   k = 0: c'(0) = c(0)/b(0),  d'(0) = d(0)/b(0)
//   k > 0: m = b(k) - a(k) c'(k-1),  c'(k) = c(k)/m,  d'(k) = (d(k) - a(k) d'(k-1))/m
// computed with one reciprocal of m per level.  Back-substitution:
//   x(K-1) = d'(K-1),  x(k) = d'(k) - c'(k) x(k+1), rounded once to storage.
#pragma once

#include "common.hpp"

namespace stl {

// ---------------------------------------------------------------------------
// Fused hdiff + vadv.  Workgroup = 64 x TJ lanes = a 64 x TJ tile of columns.
// ---------------------------------------------------------------------------
template <class T, int TJ, int PF, int KMAX>
__global__ __launch_bounds__(64 * TJ) void k_hdiff_vadv(VadvArgs p) {
    using S = Storage<T>;
    using C = typename S::C;
    constexpr int TI = 64, PI = TI + 4, PJ = TJ + 4;
    constexpr int MR = (PJ + TJ - 1) / TJ;  // tile rows loaded per lane (main block)
    __shared__ C tile[2][PJ * PI];

    const T *__restrict__ u = static_cast<const T *>(p.u);
    const T *__restrict__ coeff = static_cast<const T *>(p.coeff);
    const T *__restrict__ wcon = static_cast<const T *>(p.wcon);
    const T *__restrict__ fa = static_cast<const T *>(p.a);
    const T *__restrict__ fb = static_cast<const T *>(p.b);
    const T *__restrict__ fc = static_cast<const T *>(p.c);
    T *__restrict__ x = static_cast<T *>(p.x);

    const int tid = threadIdx.x, ti = tid & 63, tj = tid >> 6;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int bi = t % p.nbi, bj = t / p.nbi;
    const int i0 = bi * TI, j0 = bj * TJ;
    const int gi = i0 + ti, gj = j0 + tj;
    const bool active = gi < p.I && gj < p.J;
    // Lanes past a ragged edge read a valid column and store nothing.
    const int col = min(gi, p.I - 1) + min(gj, p.J - 1) * p.sj;

    // Tile element (r, c) holds u(i0 - 2 + c, j0 - 2 + r).  Main block
    // c in [2, 66): lane (ti, tj) loads rows tj, tj + TJ, ...; the four side
    // columns c in {0, 1, 66, 67} are loaded by lanes 0 .. 4 PJ - 1.  Cells
    // outside [-2, I+2) x [-2, J+2) are never read by an active lane; they get 0.
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

    // Prefetch ring: slot q holds the inputs of every level s with s % PF == q.
    C rum[PF][MR], rus[PF], rcf[PF], rw[PF], ra[PF], rb[PF], rc[PF];
    auto load = [&](int q, int k) {
        const int ko = k * p.sk;
#pragma unroll
        for (int m = 0; m < MR; ++m) rum[q][m] = mok[m] ? S::load(u + moff[m] + ko) : C(0);
        rus[q] = sok ? S::load(u + soff + ko) : C(0);
        rcf[q] = S::load(coeff + col + ko);
        rw[q] = S::load(wcon + col + ko);
        ra[q] = S::load(fa + col + ko);
        rb[q] = S::load(fb + col + ko);
        rc[q] = S::load(fc + col + ko);
    };

    const int K = p.K;
#pragma unroll
    for (int q = 0; q < PF; ++q)
        if (q < K) load(q, q);

    const C dt = static_cast<C>(p.dt);
    C h_prev = C(0), w_prev = C(0), f_prev = C(0);
    double a_prev = 0.0, b_prev = 1.0, c_prev = 0.0;
    double cp[KMAX], dp[KMAX];

#pragma unroll
    for (int s = 0; s < KMAX; ++s) {
        if (s < K) {
            const int q = s % PF;
            C *tb = tile[s & 1];
#pragma unroll
            for (int m = 0; m < MR; ++m)
                if (mrow[m]) tb[mlds[m]] = rum[q][m];
            if (srow) tb[slds] = rus[q];
            const C cf = rcf[q], wv = rw[q];
            const double av = static_cast<double>(ra[q]), bv = static_cast<double>(rb[q]),
                         cv = static_cast<double>(rc[q]);
            if (s + PF < K) load(q, s + PF);
            __syncthreads();
            const C h = hdiff_point<C, PI>(tb + (tj + 2) * PI + ti + 2, cf);
            if (s > 0) {
                // F(s - 1/2), then the right-hand side and elimination of level s - 1.
                const int l = s > 0 ? s - 1 : 0;
                const C f = (C(0.5) * (w_prev + wv)) * (C(0.5) * (h_prev + h));
                const double d = static_cast<double>(h_prev - dt * (f - f_prev));
                if (l == 0) {
                    const double r = 1.0 / b_prev;
                    cp[0] = c_prev * r;
                    dp[0] = d * r;
                } else {
                    const int lm = l > 0 ? l - 1 : 0;
                    const double r = 1.0 / (b_prev - a_prev * cp[lm]);
                    cp[l] = c_prev * r;
                    dp[l] = (d - a_prev * dp[lm]) * r;
                }
                f_prev = f;
            }
            if (s == K - 1) {
                // Top level: no flux through the upper face.
                const double d = static_cast<double>(h - dt * (C(0) - f_prev));
                if (s == 0) {
                    dp[0] = d / bv;
                } else {
                    const int lm = s > 0 ? s - 1 : 0;
                    dp[s] = (d - av * dp[lm]) / (bv - av * cp[lm]);
                }
            }
            h_prev = h;
            w_prev = wv;
            a_prev = av;
            b_prev = bv;
            c_prev = cv;
        }
    }

    double xn = 0.0;
#pragma unroll
    for (int s = KMAX - 1; s >= 0; --s) {
        if (s < K) {
            xn = (s == K - 1) ? dp[s] : dp[s] - cp[s] * xn;
            if (active) S::store_d(x + col + s * p.sk, xn);
        }
    }
}

// ---------------------------------------------------------------------------
// vadv alone: h is read from memory.  Workgroup = 64 x TJ columns.
// ---------------------------------------------------------------------------
template <class T, int TJ, int PF, int KMAX>
__global__ __launch_bounds__(64 * TJ) void k_vadv(VadvArgs p) {
    using S = Storage<T>;
    using C = typename S::C;
    const T *__restrict__ hin = static_cast<const T *>(p.u);
    const T *__restrict__ wcon = static_cast<const T *>(p.wcon);
    const T *__restrict__ fa = static_cast<const T *>(p.a);
    const T *__restrict__ fb = static_cast<const T *>(p.b);
    const T *__restrict__ fc = static_cast<const T *>(p.c);
    T *__restrict__ x = static_cast<T *>(p.x);

    const int tid = threadIdx.x, ti = tid & 63, tj = tid >> 6;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int bi = t % p.nbi, bj = t / p.nbi;
    const int gi = bi * 64 + ti, gj = bj * TJ + tj;
    const bool active = gi < p.I && gj < p.J;
    const int col = min(gi, p.I - 1) + min(gj, p.J - 1) * p.sj;

    C rh[PF], rw[PF], ra[PF], rb[PF], rc[PF];
    auto load = [&](int q, int k) {
        const int o = col + k * p.sk;
        rh[q] = S::load(hin + o);
        rw[q] = S::load(wcon + o);
        ra[q] = S::load(fa + o);
        rb[q] = S::load(fb + o);
        rc[q] = S::load(fc + o);
    };
    const int K = p.K;
#pragma unroll
    for (int q = 0; q < PF; ++q)
        if (q < K) load(q, q);

    const C dt = static_cast<C>(p.dt);
    C h_prev = C(0), w_prev = C(0), f_prev = C(0);
    double a_prev = 0.0, b_prev = 1.0, c_prev = 0.0;
    double cp[KMAX], dp[KMAX];

#pragma unroll
    for (int s = 0; s < KMAX; ++s) {
        if (s < K) {
            const int q = s % PF;
            const C h = rh[q], wv = rw[q];
            const double av = static_cast<double>(ra[q]), bv = static_cast<double>(rb[q]),
                         cv = static_cast<double>(rc[q]);
            if (s + PF < K) load(q, s + PF);
            if (s > 0) {
                const int l = s > 0 ? s - 1 : 0;
                const C f = (C(0.5) * (w_prev + wv)) * (C(0.5) * (h_prev + h));
                const double d = static_cast<double>(h_prev - dt * (f - f_prev));
                if (l == 0) {
                    const double r = 1.0 / b_prev;
                    cp[0] = c_prev * r;
                    dp[0] = d * r;
                } else {
                    const int lm = l > 0 ? l - 1 : 0;
                    const double r = 1.0 / (b_prev - a_prev * cp[lm]);
                    cp[l] = c_prev * r;
                    dp[l] = (d - a_prev * dp[lm]) * r;
                }
                f_prev = f;
            }
            if (s == K - 1) {
                const double d = static_cast<double>(h - dt * (C(0) - f_prev));
                if (s == 0) {
                    dp[0] = d / bv;
                } else {
                    const int lm = s > 0 ? s - 1 : 0;
                    dp[s] = (d - av * dp[lm]) / (bv - av * cp[lm]);
                }
            }
            h_prev = h;
            w_prev = wv;
            a_prev = av;
            b_prev = bv;
            c_prev = cv;
        }
    }

    double xn = 0.0;
#pragma unroll
    for (int s = KMAX - 1; s >= 0; --s) {
        if (s < K) {
            xn = (s == K - 1) ? dp[s] : dp[s] - cp[s] * xn;
            if (active) S::store_d(x + col + s * p.sk, xn);
        }
    }
}

// ---------------------------------------------------------------------------
// Host launchers, instantiated per storage type in column_<dtype>.hip.
// ---------------------------------------------------------------------------
template <class T, int TJ, int PF, int KMAX>
static hipError_t launch_fused_t(VadvArgs a, hipStream_t st) {
    a.nbi = (a.I + 63) / 64;
    a.nbj = (a.J + TJ - 1) / TJ;
    hipLaunchKernelGGL((k_hdiff_vadv<T, TJ, PF, KMAX>), dim3(a.nbi * a.nbj), dim3(64 * TJ), 0, st,
                       a);
    return hipGetLastError();
}

template <class T, int TJ, int PF, int KMAX>
static hipError_t launch_vadv_t(VadvArgs a, hipStream_t st) {
    a.nbi = (a.I + 63) / 64;
    a.nbj = (a.J + TJ - 1) / TJ;
    hipLaunchKernelGGL((k_vadv<T, TJ, PF, KMAX>), dim3(a.nbi * a.nbj), dim3(64 * TJ), 0, st, a);
    return hipGetLastError();
}

// Register-resident columns are compiled for these vertical extents.
#define STL_FOR_KMAX(K, F) \
    ((K) <= 32 ? F(32) : (K) <= 64 ? F(64) : (K) <= 80 ? F(80) : F(96))

}  // namespace stl
