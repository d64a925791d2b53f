// Column kernels: the fused hdiff + vadv program, and vadv alone.
//
// Each (i, j) column is solved by two lanes of one workgroup that meet in the
// middle (a "burn at both ends" Thomas solve).  With M = ceil(K / 2), the
// lanes of half 0 march up through levels 0 .. M-1 eliminating top-down, the
// lanes of half 1 march down through levels K-1 .. M eliminating bottom-up.
// Per level a lane
//   (1) stages u of its level, with a 2-cell halo, into LDS (fused kernel),
//   (2) evaluates horizontal diffusion from the tile (stencil inlining: the
//       Laplacian and both limited fluxes are recomputed, never stored),
//   (3) forms the flux-form right-hand side of the level before (whose outer
//       face needs h one level ahead), and
//   (4) takes one elimination step in double precision.
// The interface levels M-1 and M exchange h and w, finish their elimination,
// then exchange the two eliminated rows
//     x(M-1) + P0 x(M) = D0,      x(M) + P1 x(M-1) = D1,
// and solve that 2 x 2 system; each half then back-substitutes outward.
//
// Splitting the column halves the double-precision coefficients each lane
// keeps in registers (the level loop is fully unrolled over a compile-time
// bound KH >= M so the arrays are only indexed with constants), which lets two
// waves share each SIMD, and halves the length of each sequential chain.
// Every input is read from device memory once and x written once (stencil
// inlining, Sec. V-A).  Inputs of the next PF levels are prefetched into a
// register ring through buffer loads whose per-level offset is a scalar.
//
// Elimination (half 0: lower = a, upper = c; half 1: lower = c, upper = a):
//   t = 0: P(0) = upper / b,  D(0) = d / b
//   t > 0: m = b - lower P(t-1),  P(t) = upper / m,  D(t) = (d - lower D(t-1)) / m
// with 1/m from the hardware reciprocal refined by two Newton steps (error
// within an ulp).  Back-substitution: x = D(t) - P(t) x(next), rounded once to
// the storage dtype.
#pragma once

#include "common.hpp"

namespace stl {

// ---------------------------------------------------------------------------
// Raw buffer access (gfx9 family descriptor).  Byte offsets: `vo` per lane,
// `so` uniform (held in an SGPR, so advancing a level costs no vector work).
// ---------------------------------------------------------------------------
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), static_cast<short>(0),
                                             static_cast<int>(nbytes), 0x00020000);
}

template <class T> struct BufIO;

// Cache policy operand of the buffer intrinsics: 0 = default, 2 = non-temporal.
// load_raw returns the stored bits in a register of type R and cvt widens
// them to the compute type; a prefetch ring holds raw values, so a load issued
// in a conditional block needs no conversion (and no wait for its data) there.
template <> struct BufIO<float> {
    using R = float;
    template <int CP = 0>
    static __device__ __forceinline__ float load_raw(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, vo, so, CP));
    }
    static __device__ __forceinline__ float cvt(float v) { return v; }
    template <int CP = 0>
    static __device__ __forceinline__ float load(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
        return load_raw<CP>(r, vo, so);
    }
    template <int CP = 0>
    static __device__ __forceinline__ void store_d(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so,
                                                   double v) {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(static_cast<float>(v)), r, vo, so, CP);
    }
};

template <> struct BufIO<double> {
    using R = double;
    template <int CP = 0>
    static __device__ __forceinline__ double load_raw(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, CP));
    }
    static __device__ __forceinline__ double cvt(double v) { return v; }
    template <int CP = 0>
    static __device__ __forceinline__ double load(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
        return load_raw<CP>(r, vo, so);
    }
    template <int CP = 0>
    static __device__ __forceinline__ void store_d(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so,
                                                   double v) {
        using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, vo, so, CP);
    }
};

template <> struct BufIO<uint16_t> {
    using R = uint32_t;  // the 16 stored bits, zero-extended
    template <int CP = 0>
    static __device__ __forceinline__ uint32_t load_raw(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
        return __builtin_amdgcn_raw_buffer_load_b16(r, vo, so, CP);
    }
    static __device__ __forceinline__ float cvt(uint32_t b) { return __uint_as_float(b << 16); }
    template <int CP = 0>
    static __device__ __forceinline__ float load(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
        return cvt(load_raw<CP>(r, vo, so));
    }
    template <int CP = 0>
    static __device__ __forceinline__ void store_d(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so,
                                                   double v) {
        __builtin_amdgcn_raw_buffer_store_b16(Storage<uint16_t>::round_d(v), r, vo, so, CP);
    }
};

// 1/m: hardware reciprocal plus two Newton-Raphson steps.
__device__ __forceinline__ double recip(double m) {
    double r = __builtin_amdgcn_rcp(m);
    double e = __builtin_fma(-m, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-m, r, 1.0);
    return __builtin_fma(r, e, r);
}

// Marks a value as produced here: the compiler may not defer its arithmetic
// past this point (left alone, it sinks a straight-line level loop's whole
// elimination below the last barrier and spills the loaded operands).
__device__ __forceinline__ void pin(double &v) { asm volatile("" : "+v"(v)); }


// Back-substitution of one column half, outward from the interface values
// x_lo = x(M-1) and x_hi = x(M), and the vertical-diffusion epilogue VD: 0
// stores x; 1 the explicit y = x + kappa (x(k+1) - 2 x(k) + x(k-1)); 2 the
// implicit y - kappa (y(k+1) - 2 y(k) + y(k-1)) = x; both with zero flux
// through the bottom and top faces.  Row tt of the elimination (P, D) is
// local level tt - shift; level(t) maps a local level to k.  With VD = 2 every
// thread of the workgroup must call it (it exchanges the interface rows of
// the second solve through xch, partner slot xo).
template <class T, int VD, int KH, int CPX, class Level>
__device__ __forceinline__ void column_backsub(__amdgpu_buffer_rsrc_t rx, uint32_t vcol, uint32_t sk_bytes,
                                               bool active, int half, int K, int M, int nsteps, int shift,
                                               const Level &level, double (&P)[KH], double (&D)[KH],
                                               double x_lo, double x_hi, double kappa, double2 *xch, int tid,
                                               int xo) {
#pragma clang fp contract(off)
    using IO = BufIO<T>;
    double xn = half ? x_hi : x_lo;
    if constexpr (VD == 0) {
        if (active && nsteps > 0)
            IO::template store_d<CPX>(rx, vcol, static_cast<uint32_t>(level(nsteps - 1)) * sk_bytes, xn);
#pragma unroll
        for (int tt = KH - 2; tt >= 0; --tt) {
            if (tt >= shift) {
                xn = fmadd(-P[tt], xn, D[tt]);
                if (active)
                    IO::template store_d<CPX>(rx, vcol, static_cast<uint32_t>(level(tt - shift)) * sk_bytes, xn);
            }
        }
    } else if constexpr (VD == 1) {
        // y at local level t + 1 is finished once x(t) is known: its neighbour
        // toward the interface is x(t + 2) (the other half's interface value
        // for t + 1 = nsteps - 1), away from it x(t).  Half 0 walks down
        // (toward = up), half 1 walks up (toward = down).
        const bool has_other = K > 1;
        double x_in = half ? x_lo : x_hi;  // toward-interface neighbour of the current level
        double x_cur = xn;
        auto finish = [&](int t_loc, double toward, bool has_toward, double away, bool has_away) {
            const double up = half ? away : toward, dn = half ? toward : away;
            const bool has_up = half ? has_away : has_toward, has_dn = half ? has_toward : has_away;
            const double g_up = has_up ? up - x_cur : 0.0;
            const double g_dn = has_dn ? x_cur - dn : 0.0;
            const double y = fmadd(kappa, g_up - g_dn, x_cur);
            if (active) IO::template store_d<CPX>(rx, vcol, static_cast<uint32_t>(level(t_loc)) * sk_bytes, y);
        };
#pragma unroll
        for (int tt = KH - 2; tt >= 0; --tt) {
            if (tt >= shift) {
                const int t = tt - shift;
                const double xt = fmadd(-P[tt], x_cur, D[tt]);
                finish(t + 1, x_in, t + 1 < nsteps - 1 || has_other, xt, true);
                x_in = x_cur;
                x_cur = xt;
            }
        }
        if (nsteps > 0) finish(0, x_in, nsteps > 1 || has_other, 0.0, false);
    } else {
        // Implicit vertical diffusion, y - kappa (G(k+1/2) - G(k-1/2)) = x with
        // zero-flux end faces: a second, constant-coefficient tridiagonal
        // solve over the same two-way split.  x(t) replaces D(t) as the walk
        // produces it, then each half eliminates from its far end again
        // (lower = the neighbour toward the far end, upper = toward the
        // interface, both -kappa where they exist), the interface rows are
        // solved as before and y is stored during the second walk outward.
        D[KH - 1] = xn;
#pragma unroll
        for (int tt = KH - 2; tt >= 0; --tt)
            if (tt >= shift) D[tt] = fmadd(-P[tt], D[tt + 1], D[tt]);
        const bool toward_last = K - M > 0;  // the interface row has a neighbour across
#pragma unroll
        for (int st = 0; st < KH; ++st) {
            const int t = st - shift;
            const bool has_lo = t > 0, has_up = t < nsteps - 1 || toward_last;
            double lo = has_lo ? -kappa : 0.0, up = has_up ? -kappa : 0.0;
            double bd = 1.0 + (has_lo ? kappa : 0.0) + (has_up ? kappa : 0.0);
            double xt = D[st];
            if (t < 0) {  // padding row: identity with zero right-hand side
                lo = 0.0;
                up = 0.0;
                bd = 1.0;
                xt = 0.0;
            }
            if (st == 0) {
                const double r = recip(bd);
                P[0] = up * r;
                D[0] = xt * r;
            } else {
                const int sm = st > 0 ? st - 1 : 0;
                const double r = recip(fmadd(-lo, P[sm], bd));
                P[st] = up * r;
                D[st] = fmadd(-lo, D[sm], xt) * r;
            }
        }
        const double Qm = nsteps > 0 ? P[KH - 1] : 0.0, Em = nsteps > 0 ? D[KH - 1] : 0.0;
        __syncthreads();
        xch[tid] = make_double2(Qm, Em);
        __syncthreads();
        const double2 o3 = xch[xo];
        const double Q0 = half ? o3.x : Qm, E0 = half ? o3.y : Em;
        const double Q1 = half ? Qm : o3.x, E1 = half ? Em : o3.y;
        const double y_lo = fmadd(-Q0, E1, E0) / fmadd(-Q0, Q1, 1.0);  // y(M-1)
        const double y_hi = fmadd(-Q1, y_lo, E1);                      // y(M)
        double yn = half ? y_hi : y_lo;
        if (active && nsteps > 0)
            IO::template store_d<CPX>(rx, vcol, static_cast<uint32_t>(level(nsteps - 1)) * sk_bytes, yn);
#pragma unroll
        for (int tt = KH - 2; tt >= 0; --tt) {
            if (tt >= shift) {
                yn = fmadd(-P[tt], yn, D[tt]);
                if (active)
                    IO::template store_d<CPX>(rx, vcol, static_cast<uint32_t>(level(tt - shift)) * sk_bytes, yn);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Workgroup = 2 halves x (64 x TJ lanes); the tile is 64 x TJ columns.
// ---------------------------------------------------------------------------
// One 64 x TJ tile of columns.  VD = 1 replaces x by y = x + kappa (x(k+1) -
// 2 x(k) + x(k-1)) (zero flux through the bottom and top faces), finished
// level by level during the back-substitution; VD = 2 by the implicit
// counterpart, y - kappa (y(k+1) - 2 y(k) + y(k-1)) = x (same end faces).
// NT: the read-once column inputs and the output use non-temporal accesses
// (u is re-read by neighbouring tiles through L2 and keeps the default).
// NTX: only the output is non-temporal (for column inputs that other
// workgroups re-read, such as coefficients shared by several fields).
// EXACT: nk == 2 KH, so both halves take exactly KH levels; every level
// guard is then a compile-time constant and each barrier interval of the
// level loop is one straight-line scheduling region.
template <class T, bool FUSED, int VD, int TJ, int PF, int KH, bool NT = false, bool EXACT = false,
          bool NTX = NT>
__device__ __forceinline__ void column_tile(const ColumnArgs &p, int bi, int bj, double kappa) {
#pragma clang fp contract(off)
    using S = Storage<T>;
    using C = typename S::C;
    using IO = BufIO<T>;
    constexpr int CP = NT ? 2 : 0;    // column inputs
    constexpr int CPX = NTX ? 2 : 0;  // output
    constexpr int TI = 64, PI = TI + 4, PJ = TJ + 4, MR = PJ / TJ, NH = 64 * TJ;
    static_assert(PJ % TJ == 0, "tile rows must split evenly over the lanes");
    constexpr int TILE = PJ * PI + 64;  // + one dummy slot per lane of the side-loading wave
    constexpr uint32_t ES = sizeof(T);
    __shared__ C tile[FUSED ? 2 * 2 * TILE : 1];
    __shared__ double2 xch[2 * NH];

    const int tid = threadIdx.x;
    // Each half is a whole number of waves, so half and the wave's tile row
    // are wave-uniform; readfirstlane lets the compiler keep them (and every
    // per-level buffer offset derived from them) in scalar registers.
    const int half = __builtin_amdgcn_readfirstlane(tid >= NH ? 1 : 0);
    const int l = tid - half * NH, ti = l & 63;
    const int tj = __builtin_amdgcn_readfirstlane(l >> 6);
    const int i0 = p.i_lo + bi * TI, j0 = bj * TJ;
    const int gi = i0 + ti, gj = j0 + tj;
    const bool active = gi >= 0 && gi < p.I && gj < p.J;
    const int I = p.I, J = p.J, K = p.K, sj = p.sj;
    // Lanes past a ragged edge read a valid column and store nothing.
    const uint32_t vcol = static_cast<uint32_t>(min(max(gi, 0), I - 1) + min(gj, J - 1) * sj) * ES;
    const uint32_t sk_bytes = static_cast<uint32_t>(p.sk) * ES;

    const auto ru = make_rsrc(p.u, FUSED ? p.u_bytes : p.col_bytes);
    const auto rcf = make_rsrc(p.coeff, p.col_bytes);
    const auto rw = make_rsrc(p.wcon, p.col_bytes);
    // "lower" multiplies the neighbour already eliminated, "upper" the next:
    // a and c for half 0, c and a for half 1 (swapped once here, not per level).
    const auto rlo = make_rsrc(half ? p.c : p.a, p.col_bytes);
    const auto rb = make_rsrc(p.b, p.col_bytes);
    const auto rup = make_rsrc(half ? p.a : p.c, p.col_bytes);
    const auto rx = make_rsrc(p.x, p.col_bytes);

    // u tile (fused): element (r, c) holds u(i0 - 2 + c, j0 - 2 + r).  Main block
    // c in [2, 66): lane (ti, tj) stages rows tj, tj + TJ, ...; the four side
    // columns c in {0, 1, 66, 67} are staged by the first 4 PJ lanes of the
    // half's first wave (its other lanes write a dummy slot).  Cells past
    // [-2, I+2) x [-2, J+2) are never read by an active lane: their loads are
    // clamped onto valid cells instead of being predicated.
    uint32_t vmain[MR];
    int lmain[MR];
#pragma unroll
    for (int m = 0; m < MR; ++m) {
        const int r = tj + m * TJ;
        const int gx = min(max(gi, -2), I + 1), gy = min(j0 - 2 + r, J + 1);
        vmain[m] = static_cast<uint32_t>(gx + 2 + (gy + 2) * sj) * ES;
        lmain[m] = r * PI + ti + 2;
    }
    const bool side_wave = tj == 0;
    const int sr = min(l >> 2, PJ - 1), sq = l & 3;
    const int sc = sq < 2 ? sq : sq + 64;
    const uint32_t vside =
        static_cast<uint32_t>(min(max(i0 - 2 + sc, -2), I + 1) + 2 + (min(j0 - 2 + sr, J + 1) + 2) * sj) * ES;
    const int lside = l < 4 * PJ ? sr * PI + sc : PJ * PI + ti;

    // Both halves run KH steps.  A half with nsteps < KH levels starts with
    // shift = KH - nsteps padding steps: identity rows (b = 1, upper = 0,
    // zero right-hand side, no flux through their faces) that leave the
    // elimination of the real rows unchanged; step s holds local level
    // s - shift.  The loop has no run-time guards (EXACT: shift = 0).
    const int M = (K + 1) >> 1;
    const int nsteps = EXACT ? KH : half ? K - M : M;
    const int shift = EXACT ? 0 : KH - nsteps;
    auto level = [&](int t) { return half ? (EXACT ? 2 * KH : K) - 1 - t : t; };

    using R = typename IO::R;
    R rum[PF][FUSED ? MR : 1], rus[PF], rcfv[PF], rwv[PF], rlov[PF], rbv[PF], rupv[PF];
    auto load = [&](int q, int s) {  // inputs of step s (padding steps re-read level 0)
        const uint32_t so = static_cast<uint32_t>(level(max(s - shift, 0))) * sk_bytes;
        if constexpr (FUSED) {
#pragma unroll
            for (int m = 0; m < MR; ++m) rum[q][m] = IO::load_raw(ru, vmain[m], so);
            if (side_wave) rus[q] = IO::load_raw(ru, vside, so);
            rcfv[q] = IO::template load_raw<CP>(rcf, vcol, so);
        } else {
            rum[q][0] = IO::template load_raw<CP>(ru, vcol, so);
        }
        rwv[q] = IO::template load_raw<CP>(rw, vcol, so);
        rlov[q] = IO::template load_raw<CP>(rlo, vcol, so);
        rbv[q] = IO::template load_raw<CP>(rb, vcol, so);
        rupv[q] = IO::template load_raw<CP>(rup, vcol, so);
    };
#pragma unroll
    for (int q = 0; q < PF && q < KH; ++q) load(q, q);

    // d(prev) = h(prev) - dt (F above - F below).  Half 0 walks up (the new
    // face is above the previous level), half 1 walks down (it is below), so
    // d = h - dts (f_new - f_old) with dts = +dt or -dt (negation is exact).
    const C dts = half ? -static_cast<C>(p.dt) : static_cast<C>(p.dt);
    C h_prev = C(0), w_prev = C(0), f_old = C(0);
    double lo_prev = 0.0, b_prev = 1.0, up_prev = 0.0;
    double P[KH], D[KH];

#pragma unroll
    for (int s = 0; s < KH; ++s) {
        const int q = s % PF;
        C *tb = &tile[(half * 2 + (s & 1)) * TILE];
        if constexpr (FUSED) {
#pragma unroll
            for (int m = 0; m < MR; ++m) tb[lmain[m]] = IO::cvt(rum[q][m]);
            if (side_wave) tb[lside] = IO::cvt(rus[q]);
        }
        const C hv = FUSED ? C(0) : IO::cvt(rum[q][0]);
        const C cf = FUSED ? IO::cvt(rcfv[q]) : C(0);
        const C wv = IO::cvt(rwv[q]);
        const double lov = static_cast<double>(IO::cvt(rlov[q])), bv = static_cast<double>(IO::cvt(rbv[q])),
                     upv = static_cast<double>(IO::cvt(rupv[q]));
        if (s + PF < KH) load(q, s + PF);
        if constexpr (FUSED) __syncthreads();
        const C h = FUSED ? hdiff_point<C, PI>(tb + (tj + 2) * PI + ti + 2, cf) : hv;
        if (s > 0) {
            // Face between the previous and this step's level; right-hand
            // side and elimination of the previous level (row tt).
            const int tt = s > 0 ? s - 1 : 0;
            const bool pad = tt < shift;
            C f_new = (C(0.5) * (w_prev + wv)) * (C(0.5) * (h_prev + h));
            if (pad) f_new = C(0);
            double d = static_cast<double>(fmadd(-dts, f_new - f_old, h_prev));
            double bt = b_prev, upt = up_prev;
            if (pad) {
                d = 0.0;
                bt = 1.0;
                upt = 0.0;
            }
            if (tt == 0) {
                const double r = recip(bt);
                P[0] = upt * r;
                D[0] = d * r;
            } else {
                const int tm = tt > 0 ? tt - 1 : 0;
                const double r = recip(fmadd(-lo_prev, P[tm], bt));
                P[tt] = upt * r;
                D[tt] = fmadd(-lo_prev, D[tm], d) * r;
            }
            pin(P[tt]);
            pin(D[tt]);
            f_old = f_new;
        }
        h_prev = h;
        w_prev = wv;
        lo_prev = lov;
        up_prev = upv;
        b_prev = bv;
    }
    const double P_last = KH > 1 ? P[KH > 1 ? KH - 2 : 0] : 0.0;
    const double D_last = KH > 1 ? D[KH > 1 ? KH - 2 : 0] : 0.0;

    // Interface, part 1: the face between levels M-1 and M.
    xch[tid] = make_double2(static_cast<double>(h_prev), static_cast<double>(w_prev));
    __syncthreads();
    const double2 o1 = xch[half ? l : NH + l];
    C f_mid = C(0);
    if (K - M > 0)
        f_mid = (C(0.5) * (w_prev + static_cast<C>(o1.y))) * (C(0.5) * (h_prev + static_cast<C>(o1.x)));
    double Pm = 0.0, Dm = 0.0;  // this half's eliminated interface row
    if (nsteps > 0) {
        const double d = static_cast<double>(fmadd(-dts, f_mid - f_old, h_prev));
        const double m = nsteps > 1 ? fmadd(-lo_prev, P_last, b_prev) : b_prev;
        const double r = recip(m);
        Pm = up_prev * r;
        Dm = (nsteps > 1 ? fmadd(-lo_prev, D_last, d) : d) * r;
    }
    __syncthreads();
    // Interface, part 2: x(M-1) + P0 x(M) = D0 and x(M) + P1 x(M-1) = D1.
    xch[tid] = make_double2(Pm, Dm);
    __syncthreads();
    const double2 o2 = xch[half ? l : NH + l];
    const double P0 = half ? o2.x : Pm, D0 = half ? o2.y : Dm;
    const double P1 = half ? Pm : o2.x, D1 = half ? Dm : o2.y;
    const double x_lo = fmadd(-P0, D1, D0) / fmadd(-P0, P1, 1.0);  // x(M-1)
    const double x_hi = fmadd(-P1, x_lo, D1);                      // x(M)

    // Back-substitution outward from the interface (local level nsteps - 1)
    // down to local level 0.
    column_backsub<T, VD, KH, CPX>(rx, vcol, sk_bytes, active, half, K, M, nsteps, shift, level, P, D, x_lo,
                                   x_hi, kappa, xch, tid, half ? l : NH + l);
}

// Software-pipelined form of the fused tile (same arithmetic, same results).
// Step s of a half: stage the tile of level s+1 into a triple-buffered LDS
// ring and refill the register ring; evaluate hdiff at level s from the tile
// staged one step earlier; form d(s-1); eliminate level s-2, whose inputs were
// ready a step ago, so its double-precision chain is independent of this
// step's hdiff and the two interleave; one barrier closes the step.
//
// A workgroup walks the tiles first, first + stride, ... below ntiles.  With
// a persistent grid (stride = resident workgroups) the first PF levels of the
// next tile are requested before the current tile's back-substitution, so
// their latency hides behind the output stores instead of opening each tile
// with an idle wait.  A one-shot grid passes stride = ntiles.
//
// VD selects the vertical-diffusion epilogue of column_backsub (0: x is the
// output); NTX makes the output non-temporal on its own (for the batched
// timestep, whose coefficient fields are shared by several fields and keep
// the default policy).
template <class T, int TJ, int PF, int KH, bool NT, bool EXACT, bool CHAIN, int TI = 64, int VD = 0,
          bool NTX = NT>
__device__ __forceinline__ void column_tile_pipe(const ColumnArgs &p, int first, int stride, int ntiles,
                                                 double kappa = 0.0) {
#pragma clang fp contract(off)
    using S = Storage<T>;
    using C = typename S::C;
    using IO = BufIO<T>;
    constexpr int CP = NT ? 2 : 0;
    constexpr int CPX = NTX ? 2 : 0;
    constexpr int PI = TI + 4, PJ = TJ + 4, MR = PJ / TJ, NH = TI * TJ;
    static_assert(PJ % TJ == 0, "tile rows must split evenly over the lanes");
    static_assert(TI % 64 == 0 && 4 * PJ <= 64, "whole waves per tile row; one wave stages the side columns");
    constexpr int TILE = PJ * PI + 64;
    constexpr uint32_t ES = sizeof(T);
    __shared__ C tile[2 * 3 * TILE];
    __shared__ double2 xch[2 * NH];

    const int tid = threadIdx.x;
    const int half = __builtin_amdgcn_readfirstlane(tid >= NH ? 1 : 0);
    const int l = tid - half * NH, ti = l % TI;
    const int tj = __builtin_amdgcn_readfirstlane(l / TI);
    const int I = p.I, J = p.J, K = p.K, sj = p.sj;
    const uint32_t sk_bytes = static_cast<uint32_t>(p.sk) * ES;

    const auto ru = make_rsrc(p.u, p.u_bytes);
    const auto rcf = make_rsrc(p.coeff, p.col_bytes);
    const auto rw = make_rsrc(p.wcon, p.col_bytes);
    const auto rlo = make_rsrc(half ? p.c : p.a, p.col_bytes);
    const auto rb = make_rsrc(p.b, p.col_bytes);
    const auto rup = make_rsrc(half ? p.a : p.c, p.col_bytes);
    const auto rx = make_rsrc(p.x, p.col_bytes);

    int lmain[MR];
#pragma unroll
    for (int m = 0; m < MR; ++m) lmain[m] = (tj + m * TJ) * PI + ti + 2;
    // The side columns c in {0, 1, TI + 2, TI + 3} are staged by the first
    // 4 PJ lanes of the half's first wave (its other lanes write a dummy slot).
    const bool side_wave = __builtin_amdgcn_readfirstlane(l >> 6) == 0;
    const int sr = min(l >> 2, PJ - 1), sq = l & 3;
    const int sc = sq < 2 ? sq : sq + TI;
    const int lside = l < 4 * PJ ? sr * PI + sc : PJ * PI + (l & 63);

    // Per-tile lane offsets (bytes from each field's interior origin).
    uint32_t vmain[MR], vside = 0, vcol = 0;
    bool active = false;
    auto locate = [&](int t) {
        const int i0 = p.i_lo + (t % p.nbi) * TI, j0 = (t / p.nbi) * TJ;
        const int gi = i0 + ti, gj = j0 + tj;
        active = gi >= 0 && gi < I && gj < J;
        vcol = static_cast<uint32_t>(min(max(gi, 0), I - 1) + min(gj, J - 1) * sj) * ES;
#pragma unroll
        for (int m = 0; m < MR; ++m) {
            const int gx = min(max(gi, -2), I + 1), gy = min(j0 - 2 + tj + m * TJ, J + 1);
            vmain[m] = static_cast<uint32_t>(gx + 2 + (gy + 2) * sj) * ES;
        }
        vside = static_cast<uint32_t>(min(max(i0 - 2 + sc, -2), I + 1) + 2 + (min(j0 - 2 + sr, J + 1) + 2) * sj) *
                ES;
    };

    const int M = (K + 1) >> 1;
    const int nsteps = EXACT ? KH : half ? K - M : M;
    const int shift = EXACT ? 0 : KH - nsteps;  // leading identity rows, as in column_tile
    auto level = [&](int t) { return half ? (EXACT ? 2 * KH : K) - 1 - t : t; };

    using R = typename IO::R;  // raw ring values, widened where used
    R rum[PF][MR], rus[PF], rcfv[PF], rwv[PF], rlov[PF], rbv[PF], rupv[PF];
    auto load = [&](int q, int s) {
        const uint32_t so = static_cast<uint32_t>(level(max(s - shift, 0))) * sk_bytes;
#pragma unroll
        for (int m = 0; m < MR; ++m) rum[q][m] = IO::load_raw(ru, vmain[m], so);
        if (side_wave) rus[q] = IO::load_raw(ru, vside, so);
        rcfv[q] = IO::template load_raw<CP>(rcf, vcol, so);
        rwv[q] = IO::template load_raw<CP>(rw, vcol, so);
        rlov[q] = IO::template load_raw<CP>(rlo, vcol, so);
        rbv[q] = IO::template load_raw<CP>(rb, vcol, so);
        rupv[q] = IO::template load_raw<CP>(rup, vcol, so);
    };
    // Column values of the step whose hdiff comes next ("cur").
    C cf_c = C(0), w_c = C(0);
    double lo_c = 0.0, b_c = 1.0, up_c = 0.0;
    auto stage = [&](int s) {  // tile and column values of step s from the ring
        const int q = s % PF;
        C *tb = &tile[(half * 3 + s % 3) * TILE];
#pragma unroll
        for (int m = 0; m < MR; ++m) tb[lmain[m]] = IO::cvt(rum[q][m]);
        if (side_wave) tb[lside] = IO::cvt(rus[q]);
        cf_c = IO::cvt(rcfv[q]);
        w_c = IO::cvt(rwv[q]);
        lo_c = static_cast<double>(IO::cvt(rlov[q]));
        b_c = static_cast<double>(IO::cvt(rbv[q]));
        up_c = static_cast<double>(IO::cvt(rupv[q]));
        if (s + PF < KH) load(q, s + PF);
    };

    const C dts = half ? -static_cast<C>(p.dt) : static_cast<C>(p.dt);
    double P[KH], D[KH];
    double d_pend = 0.0, lo_pend = 0.0, b_pend = 1.0, up_pend = 0.0;  // row s-2
    auto eliminate = [&](int t) {  // row t from the pending values
        if (t == 0) {
            const double r = recip(b_pend);
            P[0] = up_pend * r;
            D[0] = d_pend * r;
        } else {
            const int tm = t > 0 ? t - 1 : 0;
            const double r = recip(fmadd(-lo_pend, P[tm], b_pend));
            P[t] = up_pend * r;
            D[t] = fmadd(-lo_pend, D[tm], d_pend) * r;
        }
        pin(P[t]);
        pin(D[t]);
    };

    int t = first;
    if (t >= ntiles) return;
    locate(t);
#pragma unroll
    for (int q = 0; q < PF && q < KH; ++q) load(q, q);

    for (;;) {
        stage(0);
        __syncthreads();
        C h_prev = C(0), w_prev = C(0), f_old = C(0);
        double lo_prev = 0.0, b_prev = 1.0, up_prev = 0.0;  // step s-1
#pragma unroll
        for (int s = 0; s < KH; ++s) {
            // Values of step s (staged one step ago) before the next stage overwrites them.
            const C cf = cf_c, wv = w_c;
            const double lov = lo_c, bv = b_c, upv = up_c;
            if (s + 1 < KH) stage(s + 1);
            const C *tb = &tile[(half * 3 + s % 3) * TILE];
            const C h = hdiff_point<C, PI>(tb + (tj + 2) * PI + ti + 2, cf);
            if (s >= 2) eliminate(s >= 2 ? s - 2 : 0);
            if (s >= 1) {
                const bool pad = s - 1 < shift;
                C f_new = (C(0.5) * (w_prev + wv)) * (C(0.5) * (h_prev + h));
                if (pad) f_new = C(0);
                d_pend = static_cast<double>(fmadd(-dts, f_new - f_old, h_prev));
                f_old = f_new;
                lo_pend = lo_prev;
                b_pend = b_prev;
                up_pend = up_prev;
                if (pad) {
                    d_pend = 0.0;
                    b_pend = 1.0;
                    up_pend = 0.0;
                }
            }
            h_prev = h;
            w_prev = wv;
            lo_prev = lov;
            b_prev = bv;
            up_prev = upv;
            __syncthreads();
        }
        // The last step left row KH - 2 pending.
        if (KH >= 2) eliminate(KH >= 2 ? KH - 2 : 0);
        const double P_last = KH > 1 ? P[KH > 1 ? KH - 2 : 0] : 0.0;
        const double D_last = KH > 1 ? D[KH > 1 ? KH - 2 : 0] : 0.0;

        // Interface, part 1: the face between levels M-1 and M.
        xch[tid] = make_double2(static_cast<double>(h_prev), static_cast<double>(w_prev));
        __syncthreads();
        const double2 o1 = xch[half ? l : NH + l];
        C f_mid = C(0);
        if (K - M > 0)
            f_mid = (C(0.5) * (w_prev + static_cast<C>(o1.y))) * (C(0.5) * (h_prev + static_cast<C>(o1.x)));
        double Pm = 0.0, Dm = 0.0;
        if (nsteps > 0) {
            const double d = static_cast<double>(fmadd(-dts, f_mid - f_old, h_prev));
            const double m = nsteps > 1 ? fmadd(-lo_prev, P_last, b_prev) : b_prev;
            const double r = recip(m);
            Pm = up_prev * r;
            Dm = (nsteps > 1 ? fmadd(-lo_prev, D_last, d) : d) * r;
        }
        __syncthreads();
        xch[tid] = make_double2(Pm, Dm);
        __syncthreads();
        const double2 o2 = xch[half ? l : NH + l];
        const double P0 = half ? o2.x : Pm, D0 = half ? o2.y : Dm;
        const double P1 = half ? Pm : o2.x, D1 = half ? Dm : o2.y;
        const double x_lo = fmadd(-P0, D1, D0) / fmadd(-P0, P1, 1.0);
        const double x_hi = fmadd(-P1, x_lo, D1);

        // Request the next tile's first levels, then store this one.
        const uint32_t vx = vcol;
        const bool store = active;
        const int tn = t + stride;
        const bool more = CHAIN && tn < ntiles;
        if (more) {
            locate(tn);
#pragma unroll
            for (int q = 0; q < PF && q < KH; ++q) load(q, q);
        }
        column_backsub<T, VD, KH, CPX>(rx, vx, sk_bytes, store, half, K, M, nsteps, shift, level, P, D, x_lo,
                                       x_hi, kappa, xch, tid, half ? l : NH + l);
        if (!more) break;
        t = tn;
    }
}

template <class T, int TJ, int PF, int KH, int WPE, bool NT, bool EXACT, bool CHAIN, int TI>
__global__ __launch_bounds__(2 * TI * TJ) __attribute__((amdgpu_waves_per_eu(WPE, 8))) void
k_column_pipe(ColumnArgs p, int ntiles) {
    // Consecutive tile positions share an XCD (and its L2) in every round.
    column_tile_pipe<T, TJ, PF, KH, NT, EXACT, CHAIN, TI>(p, xcd_tile(blockIdx.x, gridDim.x), gridDim.x,
                                                          ntiles);
}

// CHAIN: a persistent grid of resident workgroups walks the tiles; otherwise
// one workgroup per tile.  Tiles are TI x TJ columns.
template <class T, int TJ, int PF, int KH, int WPE, bool NT, bool EXACT = false, bool CHAIN = false, int TI = 64>
static hipError_t launch_column_pipe_t(ColumnArgs a, hipStream_t st) {
    if ((EXACT && a.K != 2 * KH) || (a.K + 1) / 2 > KH) return hipErrorInvalidValue;
    a.nbi = (a.I + TI - 1) / TI;
    a.nbj = (a.J + TJ - 1) / TJ;
    const int ntiles = a.nbi * a.nbj;
    auto kern = k_column_pipe<T, TJ, PF, KH, WPE, NT, EXACT, CHAIN, TI>;
    int grid = ntiles;
    if (CHAIN) {
        const int res = resident_workgroups(reinterpret_cast<const void *>(kern), 2 * TI * TJ);
        if (res > 0 && res < grid) grid = res;
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(2 * TI * TJ), 0, st, a, ntiles);
    return hipGetLastError();
}

template <class T, bool FUSED, int TJ, int PF, int KH, int WPE, bool NT, bool EXACT>
__global__ __launch_bounds__(128 * TJ) __attribute__((amdgpu_waves_per_eu(WPE, 8))) void
k_column(ColumnArgs p) {
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    column_tile<T, FUSED, 0, TJ, PF, KH, NT, EXACT>(p, t % p.nbi, t / p.nbi, 0.0);
}

// ---------------------------------------------------------------------------
// Batched form: many (subdomain, field) problems in one launch.  The tiles of
// all problems are numbered consecutively, subdomain by subdomain, with the
// field index fastest, so the workgroups of the fields that share a
// subdomain's coefficient fields run next to each other on one XCD (the
// tile map keeps consecutive tiles on the same XCD) and share those loads in
// its L2.  The table travels in the kernel arguments.
// ---------------------------------------------------------------------------
constexpr int BATCH_SUBS = 8;
constexpr int BATCH_FIELDS = 8;

struct ColumnBatchSub {
    ColumnArgs a;                        // shared coefficients; u, x unused
    const void *u[BATCH_FIELDS];
    void *x[BATCH_FIELDS];
    int tile0;                           // first batch tile of this subdomain
    int nfields;
};

struct ColumnBatch {
    ColumnBatchSub sub[BATCH_SUBS];
    int nsub;
    double kappa;
};

template <class T, int VD, int TJ, int PF, int KH, int WPE>
__global__ __launch_bounds__(128 * TJ) __attribute__((amdgpu_waves_per_eu(WPE, 8))) void
k_column_batch(ColumnBatch b) {
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    int s = 0;
    while (s + 1 < b.nsub && b.sub[s + 1].tile0 <= t) ++s;
    const ColumnBatchSub &sb = b.sub[s];
    const int local = t - sb.tile0;
    const int f = local % sb.nfields, tile = local / sb.nfields;
    ColumnArgs a = sb.a;
    a.u = sb.u[f];
    a.x = sb.x[f];
    // Coefficients are shared by the fields of a subdomain (re-read through
    // L2): default policy; the output streams.  (The software-pipelined tile
    // measured no faster here: the coefficient re-reads hit L2.)
    column_tile<T, true, VD, TJ, PF, KH, false, false, true>(a, tile % a.nbi, tile / a.nbi, b.kappa);
}

// The same table over the software-pipelined tile (one barrier per level,
// the FP64 elimination of level s - 2 interleaved with hdiff of level s).
template <class T, int VD, int TJ, int PF, int KH, int WPE>
__global__ __launch_bounds__(128 * TJ) __attribute__((amdgpu_waves_per_eu(WPE, 8))) void
k_column_batch_pipe(ColumnBatch b) {
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    int s = 0;
    while (s + 1 < b.nsub && b.sub[s + 1].tile0 <= t) ++s;
    const ColumnBatchSub &sb = b.sub[s];
    const int local = t - sb.tile0;
    const int f = local % sb.nfields, tile = local / sb.nfields;
    ColumnArgs a = sb.a;
    a.u = sb.u[f];
    a.x = sb.x[f];
    column_tile_pipe<T, TJ, PF, KH, false, false, false, 64, VD, true>(a, tile, a.nbi * a.nbj, a.nbi * a.nbj,
                                                                      b.kappa);
}

// ---------------------------------------------------------------------------
// Host launchers, instantiated per storage type in column_<dtype>.hip.
// ---------------------------------------------------------------------------
template <class T, bool FUSED, int TJ, int PF, int KH, int WPE, bool NT = false, bool EXACT = false>
static hipError_t launch_column_t(ColumnArgs a, hipStream_t st) {
    if ((EXACT && a.K != 2 * KH) || (a.K + 1) / 2 > KH) return hipErrorInvalidValue;
    a.nbi = (a.I + 63) / 64;
    a.nbj = (a.J + TJ - 1) / TJ;
    hipLaunchKernelGGL((k_column<T, FUSED, TJ, PF, KH, WPE, NT, EXACT>), dim3(a.nbi * a.nbj),
                       dim3(128 * TJ), 0, st, a);
    return hipGetLastError();
}

// A compiled fused variant: its knobs and the launcher of its KH buckets.
struct ColumnEntry {
    int tile_j, prefetch;
    bool nt;
    int sched;
    hipError_t (*launch)(const ColumnArgs &, hipStream_t);
    int tile_i = 64;
};

template <int N, class Variant>
static const ColumnEntry *find_column_entry(const ColumnEntry (&tab)[N], const Variant &v) {
    for (int q = 0; q < N; ++q)
        if (tab[q].tile_j == v.tile_j && tab[q].prefetch == v.prefetch && tab[q].nt == v.nt &&
            tab[q].sched == v.sched && tab[q].tile_i == v.tile_i)
            return &tab[q];
    return nullptr;
}

}  // namespace stl
