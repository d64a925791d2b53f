// Forward mode of the fused program: the tangent dx = J v of
// x = vadv(hdiff(u, coeff), wcon, a, b, c) in a direction
// v = (du, dcoeff, dwcon, da, db, dc), in one k-march per column.
//
// Each stage is differentiated where it is evaluated (inlining applies to the
// tangent as to the forward pass, Sec. V-A): per level the tiles of u and du
// are staged in LDS, hdiff and its tangent are evaluated together under the
// forward limiter decisions, the right-hand side's tangent is formed from
// both, and T dx = dd - dT x is solved with the same two-way split and FP64
// elimination as the forward kernel.  x (the forward solution) is an input,
// read one level ahead for dT x.  A NULL tangent is a zero one, read through
// a zero-size buffer descriptor (range-checked loads return 0).
#include <type_traits>

#include "column.hpp"
#include "launch.hpp"

namespace stl {

struct JvpK {
    const void *u, *du;  // both at interior cell (-2, -2, 0)
    const void *coeff, *wcon, *a, *b, *c, *x;
    const void *dcoeff, *dwcon, *da, *db, *dc;
    void *dx;
    uint32_t u_bytes, col_bytes;
    int I, J, K, sj, sk, nbi;
    double dt;
};

// hdiff and its tangent at one point from staged tiles of u (t) and du (s);
// h is bitwise the forward operator's value.  The flux kept / zeroed
// decisions are the forward ones; a zeroed flux has a zero tangent.
template <class C, int PITCH, bool DU>
__device__ __forceinline__ void hdiff_tangent_point(const C *t, const C *s, C cf, C dcf, C &h, C &dh) {
#pragma clang fp contract(off)
    const C four = C(4);
    const C uc = t[0], ue = t[1], uw = t[-1], un = t[PITCH], us = t[-PITCH];
    const C uee = t[2], uww = t[-2], unn = t[2 * PITCH], uss = t[-2 * PITCH];
    const C une = t[PITCH + 1], unw = t[PITCH - 1], use = t[-PITCH + 1], usw = t[-PITCH - 1];
    const C lc = fmadd(four, uc, -ue) - uw - un - us;
    const C le = fmadd(four, ue, -uee) - uc - une - use;
    const C lw = fmadd(four, uw, -uc) - uww - unw - usw;
    const C ln = fmadd(four, un, -une) - unw - unn - uc;
    const C ls = fmadd(four, us, -use) - usw - uc - uss;
    const C fe0 = le - lc, fw0 = lc - lw, fn0 = ln - lc, fs0 = lc - ls;
    const bool ke = !(fe0 * (ue - uc) > C(0)), kw = !(fw0 * (uc - uw) > C(0));
    const bool kn = !(fn0 * (un - uc) > C(0)), ks = !(fs0 * (uc - us) > C(0));
    const C fe = ke ? fe0 : C(0), fw = kw ? fw0 : C(0), fn = kn ? fn0 : C(0), fs = ks ? fs0 : C(0);
    const C div = fe - fw + fn - fs;
    h = fmadd(-cf, div, uc);
    C ddiv = C(0), vc = C(0);
    if constexpr (DU) {
        vc = s[0];
        const C ve = s[1], vw = s[-1], vn = s[PITCH], vs = s[-PITCH];
        const C vee = s[2], vww = s[-2], vnn = s[2 * PITCH], vss = s[-2 * PITCH];
        const C vne = s[PITCH + 1], vnw = s[PITCH - 1], vse = s[-PITCH + 1], vsw = s[-PITCH - 1];
        const C mc = fmadd(four, vc, -ve) - vw - vn - vs;
        const C me = fmadd(four, ve, -vee) - vc - vne - vse;
        const C mw = fmadd(four, vw, -vc) - vww - vnw - vsw;
        const C mn = fmadd(four, vn, -vne) - vnw - vnn - vc;
        const C ms = fmadd(four, vs, -vse) - vsw - vc - vss;
        const C ge = ke ? me - mc : C(0), gw = kw ? mc - mw : C(0);
        const C gn = kn ? mn - mc : C(0), gs = ks ? mc - ms : C(0);
        ddiv = ge - gw + gn - gs;
    }
    dh = fmadd(-cf, ddiv, fmadd(-dcf, div, vc));
}

// One 64 x TJ tile; workgroup = 2 halves x (64 x TJ lanes) as in the forward
// kernel.  Padding steps (nsteps < KH) are identity rows with a zero
// right-hand side and no flux through their faces.
template <class T, int TJ, int PF, int KH, bool DU>
__device__ __forceinline__ void jvp_tile(const JvpK &p, int bi, int bj) {
#pragma clang fp contract(off)
    using C = typename Storage<T>::C;
    using IO = BufIO<T>;
    using R = typename IO::R;
    constexpr int TI = 64, PI = TI + 4, PJ = TJ + 4, MR = PJ / TJ, NH = 64 * TJ;
    static_assert(PJ % TJ == 0, "tile rows must split evenly over the lanes");
    constexpr int TILE = PJ * PI + 64;
    constexpr uint32_t ES = sizeof(T);
    constexpr int CPX = 2;  // the output streams
    __shared__ C tile[2 * 2 * TILE];
    __shared__ C dtile[DU ? 2 * 2 * TILE : 1];
    __shared__ double2 xch[2 * NH];
    __shared__ double xch1[2 * NH];

    const int tid = threadIdx.x;
    const int half = __builtin_amdgcn_readfirstlane(tid >= NH ? 1 : 0);
    const int l = tid - half * NH, ti = l & 63;
    const int tj = __builtin_amdgcn_readfirstlane(l >> 6);
    const int xo = half ? l : NH + l;  // the other half's lane of this column
    const int i0 = bi * TI, j0 = bj * TJ;
    const int gi = i0 + ti, gj = j0 + tj;
    const bool active = gi < p.I && gj < p.J;
    const int I = p.I, J = p.J, K = p.K, sj = p.sj;
    const uint32_t vcol = static_cast<uint32_t>(min(gi, I - 1) + min(gj, J - 1) * sj) * ES;
    const uint32_t sk_bytes = static_cast<uint32_t>(p.sk) * ES;

    const bool has_dcf = p.dcoeff, has_dw = p.dwcon, has_dlo = half ? p.dc : p.da, has_db = p.db;
    const bool has_dup = half ? p.da : p.dc;
    const bool has_dm = has_dlo || has_db || has_dup;
    const auto ru = make_rsrc(p.u, p.u_bytes);
    const auto rdu = make_rsrc(p.du, DU ? p.u_bytes : 0);
    const auto rcf = make_rsrc(p.coeff, p.col_bytes);
    const auto rw = make_rsrc(p.wcon, p.col_bytes);
    const auto rlo = make_rsrc(half ? p.c : p.a, p.col_bytes);
    const auto rb = make_rsrc(p.b, p.col_bytes);
    const auto rup = make_rsrc(half ? p.a : p.c, p.col_bytes);
    const auto rx = make_rsrc(p.x, has_dm ? p.col_bytes : 0);
    const auto rdcf = make_rsrc(p.dcoeff, has_dcf ? p.col_bytes : 0);
    const auto rdw = make_rsrc(p.dwcon, has_dw ? p.col_bytes : 0);
    const auto rdlo = make_rsrc(half ? p.dc : p.da, has_dlo ? p.col_bytes : 0);
    const auto rdb = make_rsrc(p.db, has_db ? p.col_bytes : 0);
    const auto rdup = make_rsrc(half ? p.da : p.dc, has_dup ? p.col_bytes : 0);
    const auto rdx = make_rsrc(p.dx, p.col_bytes);

    // u and du tiles: the forward kernel's layout (main block by rows, the four
    // side columns by the first lanes of the half's first wave; loads clamped
    // onto valid cells).
    uint32_t vmain[MR];
    int lmain[MR];
#pragma unroll
    for (int m = 0; m < MR; ++m) {
        const int r = tj + m * TJ;
        const int gx = min(gi, I + 1), gy = min(j0 - 2 + r, J + 1);
        vmain[m] = static_cast<uint32_t>(gx + 2 + (gy + 2) * sj) * ES;
        lmain[m] = r * PI + ti + 2;
    }
    const bool side_wave = tj == 0;
    const int sr = min(l >> 2, PJ - 1), sq = l & 3;
    const int sc = sq < 2 ? sq : sq + 64;
    const uint32_t vside =
        static_cast<uint32_t>(min(i0 - 2 + sc, I + 1) + 2 + (min(j0 - 2 + sr, J + 1) + 2) * sj) * ES;
    const int lside = l < 4 * PJ ? sr * PI + sc : PJ * PI + ti;

    const int M = (K + 1) >> 1;
    const int nsteps = half ? K - M : M;
    const int shift = KH - nsteps;
    auto level = [&](int t) { return half ? K - 1 - t : t; };

    // Raw rings (widened where used); tangents absent from the call read 0.
    R rum[PF][MR], rus[PF], rvm[PF][MR], rvs[PF];
    R rcfv[PF], rwv[PF], rlov[PF], rbv[PF], rupv[PF], rxv[PF];
    R rdcfv[PF], rdwv[PF], rdlov[PF], rdbv[PF], rdupv[PF];
    auto load = [&](int q, int s) {  // inputs of step s (padding steps re-read level 0)
        const uint32_t so = static_cast<uint32_t>(level(max(s - shift, 0))) * sk_bytes;
#pragma unroll
        for (int m = 0; m < MR; ++m) rum[q][m] = IO::load_raw(ru, vmain[m], so);
        if (side_wave) rus[q] = IO::load_raw(ru, vside, so);
        if constexpr (DU) {
#pragma unroll
            for (int m = 0; m < MR; ++m) rvm[q][m] = IO::load_raw(rdu, vmain[m], so);
            if (side_wave) rvs[q] = IO::load_raw(rdu, vside, so);
        }
        rcfv[q] = IO::template load_raw<2>(rcf, vcol, so);
        rwv[q] = IO::template load_raw<2>(rw, vcol, so);
        rlov[q] = IO::template load_raw<2>(rlo, vcol, so);
        rbv[q] = IO::template load_raw<2>(rb, vcol, so);
        rupv[q] = IO::template load_raw<2>(rup, vcol, so);
        // An absent tangent has a zero-size descriptor: its loads return 0
        // without a memory access (no branch, so no wait at a join).
        rxv[q] = IO::template load_raw<2>(rx, vcol, so);
        rdcfv[q] = IO::template load_raw<2>(rdcf, vcol, so);
        rdwv[q] = IO::template load_raw<2>(rdw, vcol, so);
        rdlov[q] = IO::template load_raw<2>(rdlo, vcol, so);
        rdbv[q] = IO::template load_raw<2>(rdb, vcol, so);
        rdupv[q] = IO::template load_raw<2>(rdup, vcol, so);
    };
#pragma unroll
    for (int q = 0; q < PF && q < KH; ++q) load(q, q);

    // Walk order: half 0 upward, half 1 downward; dts = +dt / -dt turns the
    // face difference into d = h - dt (F above - F below) for both.
    const C dts = half ? -static_cast<C>(p.dt) : static_cast<C>(p.dt);
    C h_prev = C(0), dh_prev = C(0), w_prev = C(0), dw_prev = C(0), df_old = C(0);
    double lo_prev = 0.0, b_prev = 1.0, up_prev = 0.0, dlo_prev = 0.0, db_prev = 0.0, dup_prev = 0.0;
    double x_pp = 0.0, x_p = 0.0;  // x two steps and one step back
    double P[KH], D[KH];

    // Row tt (local level tt - shift) of T dx = dd - dT x, its neighbour away
    // from the interface being x_lo_n, its own x_c, toward the interface x_up_n.
    auto rhs_row = [&](C df_new, double x_lo_n, double x_c, double x_up_n, bool first) {
        double r = static_cast<double>(fmadd(-dts, df_new - df_old, dh_prev));
        r = fmadd(-db_prev, x_c, r);
        r = fmadd(-dup_prev, x_up_n, r);
        if (!first) r = fmadd(-dlo_prev, x_lo_n, r);
        return r;
    };
    auto eliminate = [&](int tt, double r, double bt, double upt) {
        if (tt == 0) {
            const double q = recip(bt);
            P[0] = upt * q;
            D[0] = r * q;
        } else {
            const int tm = tt > 0 ? tt - 1 : 0;
            const double q = recip(fmadd(-lo_prev, P[tm], bt));
            P[tt] = upt * q;
            D[tt] = fmadd(-lo_prev, D[tm], r) * q;
        }
        pin(P[tt]);
        pin(D[tt]);
    };

#pragma unroll
    for (int s = 0; s < KH; ++s) {
        const int q = s % PF;
        C *tb = &tile[(half * 2 + (s & 1)) * TILE];
        C *vb = DU ? &dtile[(half * 2 + (s & 1)) * TILE] : tb;  // (unread without du)
#pragma unroll
        for (int m = 0; m < MR; ++m) tb[lmain[m]] = IO::cvt(rum[q][m]);
        if (side_wave) tb[lside] = IO::cvt(rus[q]);
        if constexpr (DU) {
#pragma unroll
            for (int m = 0; m < MR; ++m) vb[lmain[m]] = IO::cvt(rvm[q][m]);
            if (side_wave) vb[lside] = IO::cvt(rvs[q]);
        }
        const C cf = IO::cvt(rcfv[q]), dcf = IO::cvt(rdcfv[q]);
        const C wv = IO::cvt(rwv[q]), dwv = IO::cvt(rdwv[q]);
        const double lov = static_cast<double>(IO::cvt(rlov[q])), bv = static_cast<double>(IO::cvt(rbv[q])),
                     upv = static_cast<double>(IO::cvt(rupv[q]));
        const double dlov = static_cast<double>(IO::cvt(rdlov[q])),
                     dbv = static_cast<double>(IO::cvt(rdbv[q])), dupv = static_cast<double>(IO::cvt(rdupv[q]));
        const double xv = static_cast<double>(IO::cvt(rxv[q]));
        if (s + PF < KH) load(q, s + PF);
        __syncthreads();
        C h, dh;
        hdiff_tangent_point<C, PI, DU>(tb + (tj + 2) * PI + ti + 2, vb + (tj + 2) * PI + ti + 2, cf, dcf, h, dh);
        if (s > 0) {
            // Face between the previous step's level and this one; row of the previous level.
            const int tt = s - 1;
            const bool pad = tt < shift;
            const C wf = C(0.5) * (w_prev + wv), hf = C(0.5) * (h_prev + h);
            C df_new = (C(0.5) * (dw_prev + dwv)) * hf + wf * (C(0.5) * (dh_prev + dh));
            if (pad) df_new = C(0);
            double r = rhs_row(df_new, x_pp, x_p, xv, tt == shift);
            double bt = b_prev, upt = up_prev;
            if (pad) {
                r = 0.0;
                bt = 1.0;
                upt = 0.0;
            }
            eliminate(tt, r, bt, upt);
            df_old = df_new;
        }
        h_prev = h;
        dh_prev = dh;
        w_prev = wv;
        dw_prev = dwv;
        lo_prev = lov;
        b_prev = bv;
        up_prev = upv;
        dlo_prev = dlov;
        db_prev = dbv;
        dup_prev = dupv;
        x_pp = x_p;
        x_p = xv;
    }
    const double P_last = KH > 1 ? P[KH > 1 ? KH - 2 : 0] : 0.0;
    const double D_last = KH > 1 ? D[KH > 1 ? KH - 2 : 0] : 0.0;

    // Interface: the face between levels M-1 and M, and the x across it.
    xch[tid] = make_double2(static_cast<double>(h_prev), static_cast<double>(w_prev));
    xch1[tid] = x_p;
    __syncthreads();
    const double2 o1 = xch[xo];
    const double x_across = xch1[xo];
    __syncthreads();
    xch[tid] = make_double2(static_cast<double>(dh_prev), static_cast<double>(dw_prev));
    __syncthreads();
    const double2 o1d = xch[xo];
    C df_mid = C(0);
    if (K - M > 0) {
        const C wf = C(0.5) * (w_prev + static_cast<C>(o1.y)), hf = C(0.5) * (h_prev + static_cast<C>(o1.x));
        df_mid = (C(0.5) * (dw_prev + static_cast<C>(o1d.y))) * hf + wf * (C(0.5) * (dh_prev + static_cast<C>(o1d.x)));
    }
    double Pm = 0.0, Dm = 0.0;  // this half's eliminated interface row
    if (nsteps > 0) {
        const double r = rhs_row(df_mid, x_pp, x_p, K - M > 0 ? x_across : 0.0, nsteps == 1);
        const double m = nsteps > 1 ? fmadd(-lo_prev, P_last, b_prev) : b_prev;
        const double q = recip(m);
        Pm = up_prev * q;
        Dm = (nsteps > 1 ? fmadd(-lo_prev, D_last, r) : r) * q;
    }
    __syncthreads();
    xch[tid] = make_double2(Pm, Dm);
    __syncthreads();
    const double2 o2 = xch[xo];
    const double P0 = half ? o2.x : Pm, D0 = half ? o2.y : Dm;
    const double P1 = half ? Pm : o2.x, D1 = half ? Dm : o2.y;
    const double x_lo = fmadd(-P0, D1, D0) / fmadd(-P0, P1, 1.0);  // dx(M-1)
    const double x_hi = fmadd(-P1, x_lo, D1);                      // dx(M)
    column_backsub<T, 0, KH, CPX>(rdx, vcol, sk_bytes, active, half, K, M, nsteps, shift, level, P, D, x_lo,
                                  x_hi, 0.0, xch, tid, xo);
}

template <class T, int TJ, int PF, int KH, int WPE, bool DU>
__global__ __launch_bounds__(128 * TJ) __attribute__((amdgpu_waves_per_eu(WPE, 8))) void k_jvp(JvpK p) {
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    jvp_tile<T, TJ, PF, KH, DU>(p, t % p.nbi, t / p.nbi);
}

// Waves per SIMD asked of the compiler per level bucket: two where the
// registers fit without spilling, else one.
template <class T, int TJ, int PF, bool DU>
static hipError_t launch_jvp_kh(JvpK p, hipStream_t st) {
    constexpr bool wide = sizeof(T) == 8;
    constexpr int W32 = wide ? 1 : 2, W40 = wide || DU ? 1 : 2;
    const int m = (p.K + 1) / 2;
    p.nbi = (p.I + 63) / 64;
    const int nbj = (p.J + TJ - 1) / TJ;
    const dim3 grid(p.nbi * nbj), block(128 * TJ);
    if (m <= 16) hipLaunchKernelGGL((k_jvp<T, TJ, PF, 16, 2, DU>), grid, block, 0, st, p);
    else if (m <= 32) hipLaunchKernelGGL((k_jvp<T, TJ, PF, 32, W32, DU>), grid, block, 0, st, p);
    else if (m <= 40) hipLaunchKernelGGL((k_jvp<T, TJ, PF, 40, W40, DU>), grid, block, 0, st, p);
    else if (m <= 48) hipLaunchKernelGGL((k_jvp<T, TJ, PF, 48, 1, DU>), grid, block, 0, st, p);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

template <class T, int PF>
static hipError_t launch_jvp_t(const JvpArgs &a, hipStream_t st) {
    JvpK p{};
    const long long es = sizeof(T);
    // u and du are addressed from their cell (-2, -2, 0).
    p.u = static_cast<const char *>(a.u) - (2 + 2 * static_cast<long long>(a.sj)) * es;
    p.du = a.du ? static_cast<const char *>(a.du) - (2 + 2 * static_cast<long long>(a.sj)) * es : nullptr;
    p.coeff = a.coeff; p.wcon = a.wcon; p.a = a.a; p.b = a.b; p.c = a.c; p.x = a.x;
    p.dcoeff = a.dcoeff; p.dwcon = a.dwcon; p.da = a.da; p.db = a.db; p.dc = a.dc;
    p.dx = a.dx;
    p.I = a.I; p.J = a.J; p.K = a.K; p.sj = a.sj; p.sk = a.sk;
    p.u_bytes = static_cast<uint32_t>(((a.I + 3) + (a.J + 3) * static_cast<long long>(a.sj) +
                                       (a.K - 1) * static_cast<long long>(a.sk) + 1) * es);
    p.col_bytes = static_cast<uint32_t>(((a.I - 1) + (a.J - 1) * static_cast<long long>(a.sj) +
                                         (a.K - 1) * static_cast<long long>(a.sk) + 1) * es);
    p.dt = a.dt;
    // FP32: 64 x 4 tiles (two u and du rows loaded per lane and level instead
    // of three; 256 x 256 x 80: 0.048 ms against 0.056 with 64 x 2); FP64 64 x 2
    // (64 x 4 spills registers: 0.114 against 0.098 ms); bf16 64 x 2.
    constexpr int TJ = std::is_same<T, float>::value ? 4 : 2;
    return p.du ? launch_jvp_kh<T, TJ, PF, true>(p, st) : launch_jvp_kh<T, TJ, PF, false>(p, st);
}

hipError_t launch_jvp(int dtype, const JvpArgs &a, hipStream_t st) {
    switch (dtype) {
    case DT_F64: return launch_jvp_t<double, 2>(a, st);
    case DT_F32: return launch_jvp_t<float, 2>(a, st);
    case DT_BF16: return launch_jvp_t<uint16_t, 2>(a, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace stl
