// Fused hdiff + vadv with four lanes per column, for grids too small to fill
// the chip at two lanes per column.  The column is cut into four segments
// [s_j, s_{j+1}), s_j = j K / 4, one wave per segment, and solved by the
// partition method:
//   1. each segment eliminates its rows upward, carrying a spike column V for
//      the unknown below it, x(s - 1): row k becomes
//      x(k) + P(k) x(k+1) + V(k) x(s-1) = D(k);
//   2. a backward sweep rewrites every row in terms of the two unknowns just
//      outside the segment: x(k) = D'(k) - W(k) x(e+1) - V'(k) x(s-1);
//   3. the first and last rows of the four segments give a 6-unknown system
//      over the three interfaces, block tridiagonal in 2 x 2 blocks (x(e_i),
//      x(s_{i+1})), which every lane solves for its own column;
//   4. each lane recovers its rows from the two outside values.
// Every wave stages its own 5-row u tile, so the level loop has no workgroup
// barrier.  The right-hand side needs h one level beyond each end of the
// segment, so a segment marches levels s - 1 .. e + 1.  Segments shorter than
// the register bucket KH start with identity padding rows whose spike is -1,
// which makes the first real row start its spike at a(s) / b(s).
#pragma once

#include "column.hpp"

namespace stl {

constexpr int NSEG = 4;

template <class T, int PF, int KH, bool NT>
__device__ __forceinline__ void column4_tile(const ColumnArgs &p, int bi, int bj) {
#pragma clang fp contract(off)
    using S = Storage<T>;
    using C = typename S::C;
    using IO = BufIO<T>;
    constexpr int CP = NT ? 2 : 0;
    constexpr int TI = 64, PI = TI + 4, PJ = 5;
    constexpr int TILE = PJ * PI + 64;
    constexpr uint32_t ES = sizeof(T);
    constexpr int NST = KH + 2;  // steps: levels s - 1 .. e + 1 of the padded segment
    __shared__ C tile[NSEG * 2 * TILE];
    __shared__ double xch[NSEG * 6 * 64];

    const int tid = threadIdx.x;
    const int seg = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int ti = tid & 63;
    const int i0 = bi * TI, gi = i0 + ti, gj = bj;
    const int I = p.I, J = p.J, K = p.K, sj = p.sj;
    const bool active = gi < I && gj < J;
    const uint32_t vcol = static_cast<uint32_t>(min(gi, I - 1) + min(gj, J - 1) * sj) * ES;
    const uint32_t sk_bytes = static_cast<uint32_t>(p.sk) * ES;

    const auto ru = make_rsrc(p.u, p.u_bytes);
    const auto rcf = make_rsrc(p.coeff, p.col_bytes);
    const auto rw = make_rsrc(p.wcon, p.col_bytes);
    const auto ra = make_rsrc(p.a, p.col_bytes);
    const auto rb = make_rsrc(p.b, p.col_bytes);
    const auto rc = make_rsrc(p.c, p.col_bytes);
    const auto rx = make_rsrc(p.x, p.col_bytes);

    // u tile rows j - 2 .. j + 2 of this wave's 64 columns plus the four side
    // columns {0, 1, 66, 67} of each row (20 values, lanes 0 .. 19).
    uint32_t vmain[PJ];
#pragma unroll
    for (int m = 0; m < PJ; ++m) {
        const int gx = min(gi, I + 1), gy = min(gj - 2 + m, J + 1);
        vmain[m] = static_cast<uint32_t>(gx + 2 + (gy + 2) * sj) * ES;
    }
    const int sr = min(ti >> 2, PJ - 1), sq = ti & 3;
    const int sc = sq < 2 ? sq : sq + 64;
    const uint32_t vside =
        static_cast<uint32_t>(min(i0 - 2 + sc, I + 1) + 2 + (min(gj - 2 + sr, J + 1) + 2) * sj) * ES;
    const int lside = ti < 4 * PJ ? sr * PI + sc : PJ * PI + ti;

    const int s0 = (seg * K) / NSEG, n = ((seg + 1) * K) / NSEG - s0;
    const int shift = KH - n;
    // Level of step st (padding steps map below s - 1; their loads are clamped).
    auto lev = [&](int st) { return s0 - 1 + st - shift; };
    auto clampk = [&](int k) { return static_cast<uint32_t>(min(max(k, 0), K - 1)); };

    C rum[PF][PJ], rus[PF], rcfv[PF], rwv[PF], rav[PF], rbv[PF], rcv[PF];
    auto load = [&](int q, int st) {
        const uint32_t so = clampk(lev(st)) * sk_bytes;
#pragma unroll
        for (int m = 0; m < PJ; ++m) rum[q][m] = IO::load(ru, vmain[m], so);
        rus[q] = IO::load(ru, vside, so);
        rcfv[q] = IO::template load<CP>(rcf, vcol, so);
        rwv[q] = IO::template load<CP>(rw, vcol, so);
        rav[q] = IO::template load<CP>(ra, vcol, so);
        rbv[q] = IO::template load<CP>(rb, vcol, so);
        rcv[q] = IO::template load<CP>(rc, vcol, so);
    };
#pragma unroll
    for (int q = 0; q < PF && q < NST; ++q) load(q, q);

    const C dt = static_cast<C>(p.dt);
    C h_prev = C(0), w_prev = C(0), f_prev = C(0);
    double a_prev = 0.0, b_prev = 1.0, c_prev = 0.0;
    double P[KH], V[KH], D[KH];
#pragma unroll
    for (int st = 0; st < NST; ++st) {
        const int q = st % PF;
        C *tb = &tile[(seg * 2 + (st & 1)) * TILE];
#pragma unroll
        for (int m = 0; m < PJ; ++m) tb[m * PI + ti + 2] = rum[q][m];
        tb[lside] = rus[q];
        const C cf = rcfv[q], wv = rwv[q];
        const double av = rav[q], bv = rbv[q], cv = rcv[q];
        if (st + PF < NST) load(q, st + PF);
        __builtin_amdgcn_wave_barrier();
        const int k = lev(st);
        const C h = hdiff_point<C, PI>(tb + 2 * PI + ti + 2, cf);
        // Face between levels k - 1 and k (zero outside the column).
        C f = (C(0.5) * (w_prev + wv)) * (C(0.5) * (h_prev + h));
        if (k - 1 < 0 || k >= K) f = C(0);
        if (st >= 2) {
            // Row of level k - 1 (padded index r = st - 2).
            const int r = st >= 2 ? st - 2 : 0;
            const int kr = k - 1;
            double d = static_cast<double>(fmadd(-dt, f - f_prev, h_prev));
            double ar = kr == 0 ? 0.0 : a_prev, br = b_prev, cr = kr == K - 1 ? 0.0 : c_prev;
            if (r < shift) {  // identity padding row, spike seed -1
                d = 0.0;
                ar = 0.0;
                br = 1.0;
                cr = 0.0;
            }
            const double Pp = r > 0 ? P[r > 0 ? r - 1 : 0] : 0.0;
            const double Dp = r > 0 ? D[r > 0 ? r - 1 : 0] : 0.0;
            const double Vp = r > 0 ? V[r > 0 ? r - 1 : 0] : -1.0;
            const double rm = recip(fmadd(-ar, Pp, br));
            P[r] = cr * rm;
            V[r] = -ar * Vp * rm;
            D[r] = fmadd(-ar, Dp, d) * rm;
            if (r < shift) V[r] = -1.0;
            pin(P[r]);
            pin(V[r]);
            pin(D[r]);
        }
        h_prev = h;
        w_prev = wv;
        f_prev = f;
        a_prev = av;
        b_prev = bv;
        c_prev = cv;
        __builtin_amdgcn_wave_barrier();
    }

    // Backward sweep: x(k) = D'(k) - W(k) x(e+1) - V'(k) x(s-1), W kept in P.
    // Padding rows (below the first real row) are swept too; nothing reads them.
    double Db = D[KH - 1], Wb = P[KH - 1], Vb = V[KH - 1];  // first real row (n = 1 case)
#pragma unroll
    for (int r = KH - 2; r >= 0; --r) {
        D[r] = fmadd(-P[r], D[r + 1], D[r]);
        V[r] = fmadd(-P[r], V[r + 1], V[r]);
        P[r] = -P[r] * P[r + 1];
        if (r == shift) {
            Db = D[r];
            Wb = P[r];
            Vb = V[r];
        }
    }
    double *xs = &xch[seg * 6 * 64];
    xs[0 * 64 + ti] = Db;
    xs[1 * 64 + ti] = Wb;
    xs[2 * 64 + ti] = Vb;
    xs[3 * 64 + ti] = D[KH - 1];
    xs[4 * 64 + ti] = P[KH - 1];
    xs[5 * 64 + ti] = V[KH - 1];
    __syncthreads();
    // Interfaces i = 0 .. 2: u_i = (x(e_i), x(s_{i+1})) with
    //   x(e_i) + We_i x(s_{i+1}) + Ve_i x(e_{i-1}) = De_i
    //   x(s_{i+1}) + Ws_{i+1} x(s_{i+2}) + Vs_{i+1} x(e_i) = Ds_{i+1}
    // Block elimination forward (2 x 2 blocks), then back-substitution.
    auto get = [&](int sgm, int f) { return xch[sgm * 6 * 64 + f * 64 + ti]; };
    double Ainv[3][4], rr[3][2];
#pragma unroll
    for (int i = 0; i < NSEG - 1; ++i) {
        // A_i = [[1, We_i], [Vs_{i+1}, 1]], r_i = (De_i, Ds_{i+1});
        // B_i u_{i-1} = (Ve_i x(e_{i-1}), 0); C_{i-1} u_i = (0, Ws_i x(s_{i+1})).
        double a00 = 1.0, a01 = get(i, 4), a10 = get(i + 1, 2), a11 = 1.0;
        double r0 = get(i, 3), r1 = get(i + 1, 0);
        if (i > 0) {
            // Eliminate x(e_{i-1}) = row 0 of A'_{i-1}^-1 (r'_{i-1} - C_{i-1} u_i),
            // where C_{i-1} u_i = (0, Ws_i x(s_{i+1})).
            const double Ve = get(i, 5), Ws = get(i, 1);
            const double *iv = Ainv[i - 1];
            // x(e_{i-1}) = iv00 r'0 + iv01 (r'1 - Ws x(s_{i+1})): substituted into row e_i.
            r0 -= Ve * (iv[0] * rr[i - 1][0] + iv[1] * rr[i - 1][1]);
            a01 -= Ve * iv[1] * Ws;
        }
        const double det = a00 * a11 - a01 * a10;
        Ainv[i][0] = a11 / det;
        Ainv[i][1] = -a01 / det;
        Ainv[i][2] = -a10 / det;
        Ainv[i][3] = a00 / det;
        rr[i][0] = r0;
        rr[i][1] = r1;
    }
    double ue[3], us[3];  // x(e_i), x(s_{i+1})
#pragma unroll
    for (int i = NSEG - 2; i >= 0; --i) {
        double r0 = rr[i][0], r1 = rr[i][1];
        if (i < NSEG - 2) r1 -= get(i + 1, 1) * us[i + 1];  // Ws_{i+1} x(s_{i+2})
        ue[i] = Ainv[i][0] * r0 + Ainv[i][1] * r1;
        us[i] = Ainv[i][2] * r0 + Ainv[i][3] * r1;
    }
    const double xL = seg > 0 ? ue[seg > 0 ? seg - 1 : 0] : 0.0;
    const double xR = seg < NSEG - 1 ? us[seg < NSEG - 1 ? seg : 0] : 0.0;
#pragma unroll
    for (int r = 0; r < KH; ++r) {
        if (r >= shift) {
            const double x = fmadd(-V[r], xL, fmadd(-P[r], xR, D[r]));
            if (active)
                IO::template store_d<CP>(rx, vcol, static_cast<uint32_t>(s0 + r - shift) * sk_bytes, x);
        }
    }
}

template <class T, int PF, int KH, bool NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_column4(ColumnArgs p) {
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    column4_tile<T, PF, KH, NT>(p, t % p.nbi, t / p.nbi);
}

// nk >= 8 (every segment has at least two rows) and ceil(nk / 4) <= KH.
template <class T, int PF, int KH, bool NT>
static hipError_t launch_column4_t(ColumnArgs a, hipStream_t st) {
    if (a.K < 8 || (a.K + NSEG - 1) / NSEG > KH) return hipErrorInvalidValue;
    a.nbi = (a.I + 63) / 64;
    a.nbj = a.J;
    hipLaunchKernelGGL((k_column4<T, PF, KH, NT>), dim3(a.nbi * a.nbj), dim3(64 * NSEG), 0, st, a);
    return hipGetLastError();
}

}  // namespace stl
