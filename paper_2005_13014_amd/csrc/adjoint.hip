// Reverse mode of x = vadv(hdiff(u, coeff), wcon, a, b, c, dt) for the loss
// L = sum over the interior of w * x, with the limiter decisions of the
// forward pass frozen (their derivative is taken as zero).
//
// Three launches on one stream (two with FP32 or bfloat16 storage, where the
// column kernel evaluates h itself from an LDS tile of u during its
// elimination sweep and keeps it in LDS):
//   1. hdiff recomputes h (compute type) into scratch (FP64 storage);
//   2. k_vadv_adjoint, one lane per column: the transposed Thomas solve
//      lam = T^-T w (double precision), then, walking down the column, the
//      adjoint of the flux-form right-hand side
//        Fhat(k+1/2) = -dt (lam(k) - lam(k+1))
//        gh(k)  = lam(k) + Fhat(k-1/2) wbar(k-1/2)/2 + Fhat(k+1/2) wbar(k+1/2)/2
//        gwcon(k) =        Fhat(k-1/2) hbar(k-1/2)/2 + Fhat(k+1/2) hbar(k+1/2)/2
//      (wbar, hbar: face means of wcon and h); gh goes to scratch;
//   3. k_hdiff_adjoint, one workgroup per (tile, run of levels): with g = -coeff gh,
//      the transposed update, limited flux and Laplacian stencils, staged
//      through LDS, give gu on the interior and its 2-cell ring and
//      gcoeff = -gh (flx - flx(i-1) + fly - fly(j-1)) on the interior.
#include <algorithm>
#include <cstdint>
#include <map>
#include <mutex>
#include <type_traits>

#include "column.hpp"
#include "common.hpp"
#include "launch.hpp"

namespace stl {

struct AdjArgs {
    const void *u, *coeff, *wcon, *a, *b, *c, *w;  // interior origins
    void *gu, *gcoeff, *gwcon;                      // interior origins (gu has a 2-cell halo)
    const void *x;                                  // forward result (MATRIX only)
    void *ga, *gb, *gc;                             // matrix gradients, each optional
    void *h, *gh;                                   // scratch, compute type, same strides
    int I, J, K, sj, sk;
    double dt;
};

// ---------------------------------------------------------------------------
// Transposed Thomas solve and right-hand-side adjoint.  T^T has, in row k,
// c(k-1) below the diagonal, b(k) on it and a(k+1) above it.  Like the
// forward column kernel, two lanes share a column: half 0 eliminates rows
// [0, M) upward and half 1 rows [M, K) downward (M = ceil(K/2)), the two
// interface rows are solved as a 2 x 2 system, and each half walks back
// outward from the interface.  During that walk a level is finished as soon
// as lam is known on both of its sides:
//   Fhat(k+1/2) = -dt (lam(k) - lam(k+1))
//   gh(k)    = lam(k) + sum over its faces f of Fhat(f) wbar(f) / 2
//   gwcon(k) = sum over its faces f of Fhat(f) hbar(f) / 2
// and with MATRIX also ga(k) = -lam(k) x(k-1), gb(k) = -lam(k) x(k),
// gc(k) = -lam(k) x(k+1).  A half with fewer than KH levels starts with
// identity padding rows so the elimination loop has no run-time guards.
// ---------------------------------------------------------------------------
// FUSEH: h = hdiff(u, coeff) is evaluated here during the elimination sweep
// (which visits the levels in the forward kernel's order) from a u tile
// staged in LDS per level, and kept in LDS for the outward walk, instead of
// being read from a separately computed scratch field.
template <class T, int TJ, int PF, int KH, bool MATRIX, bool FUSEH, int WR>
__global__ __launch_bounds__(128 * TJ) __attribute__((amdgpu_waves_per_eu(2, 8))) void
k_vadv_adjoint(AdjArgs p, int nbi) {
#pragma clang fp contract(off)
    using S = Storage<T>;
    using C = typename S::C;
    using IO = BufIO<T>;
    using IOC = BufIO<C>;
    using R = typename IO::R;
    constexpr int NH = 64 * TJ;
    constexpr uint32_t ES = sizeof(T), EC = sizeof(C);
    constexpr int PI = 68, PJ = TJ + 4, MR = PJ / TJ, TILE = PJ * PI + 64;
    static_assert(PJ % TJ == 0, "tile rows must split evenly over the lanes");
    __shared__ double2 xch[2 * NH];
    __shared__ C utile[FUSEH ? 2 * 2 * TILE : 1];
    __shared__ C hs[FUSEH ? KH * 2 * NH : 1];  // h of step s (local level s - shift), per lane

    const int tid = threadIdx.x;
    const int half = __builtin_amdgcn_readfirstlane(tid >= NH ? 1 : 0);
    const int l = tid - half * NH, ti = l & 63;
    const int tj = __builtin_amdgcn_readfirstlane(l >> 6);
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int gi = (tile % nbi) * 64 + ti, gj = (tile / nbi) * TJ + tj;
    const int I = p.I, J = p.J, K = p.K;
    const bool active = gi < I && gj < J;
    // Lanes past a ragged edge work on a valid column and store nothing.
    const uint32_t col = static_cast<uint32_t>(min(gi, I - 1) + min(gj, J - 1) * p.sj);
    const uint32_t vt = col * ES, vc = col * EC;
    const uint32_t skt = static_cast<uint32_t>(p.sk) * ES, skc = static_cast<uint32_t>(p.sk) * EC;
    // Addressable bytes from an interior origin (the host checks < 2^31).
    const uint32_t tbytes = static_cast<uint32_t>((static_cast<size_t>(I - 1) +
                                                   static_cast<size_t>(J - 1) * p.sj +
                                                   static_cast<size_t>(K - 1) * p.sk + 1) * ES);
    const uint32_t cbytes = tbytes / ES * EC;
    // The neighbour toward the far end multiplies "lower", the one toward the
    // interface "upper": c(k-1) and a(k+1) in half 0, a(k+1) and c(k-1) in half 1.
    const auto rlo = make_rsrc(half ? p.a : p.c, tbytes);
    const auto rup = make_rsrc(half ? p.c : p.a, tbytes);
    const auto rb = make_rsrc(p.b, tbytes);
    const auto rw = make_rsrc(p.w, tbytes);
    const auto rwc = make_rsrc(p.wcon, tbytes);
    const auto rh = make_rsrc(p.h, cbytes);
    const auto rgh = make_rsrc(p.gh, cbytes);
    const auto rgw = make_rsrc(p.gwcon, tbytes);

    const int M = (K + 1) >> 1;
    const int nsteps = half ? K - M : M;
    const int shift = KH - nsteps;
    auto level = [&](int t) { return half ? K - 1 - t : t; };
    // Level of local index t clamped into the column (for loads whose value
    // is unused outside it).
    auto clampk = [&](int t) {
        const int k = level(t);
        return static_cast<uint32_t>(min(max(k, 0), K - 1));
    };

    // FUSEH: u tile of the forward kernel's layout, element (r, c) holding
    // u(i0 - 2 + c, j0 - 2 + r), u addressed from its cell (-2, -2, 0); loads
    // past the ring are clamped onto valid cells (never read by an active lane).
    const int i0 = (tile % nbi) * 64, j0 = (tile / nbi) * TJ;
    const auto ru = make_rsrc(FUSEH ? static_cast<const T *>(p.u) - 2 - 2 * p.sj : nullptr,
                              FUSEH ? static_cast<uint32_t>(((I + 3) + static_cast<size_t>(J + 3) * p.sj +
                                                             static_cast<size_t>(K - 1) * p.sk + 1) * ES)
                                    : 0u);
    const auto rcf = make_rsrc(p.coeff, FUSEH ? tbytes : 0u);
    uint32_t vmain[MR];
    int lmain[MR];
#pragma unroll
    for (int m = 0; m < MR; ++m) {
        const int r = tj + m * TJ;
        vmain[m] = static_cast<uint32_t>(min(gi, I + 1) + 2 + (min(j0 - 2 + r, J + 1) + 2) * p.sj) * ES;
        lmain[m] = r * PI + ti + 2;
    }
    const bool side_wave = tj == 0;
    const int sr = min(l >> 2, PJ - 1), sq = l & 3;
    const int sc = sq < 2 ? sq : sq + 64;
    const uint32_t vside =
        static_cast<uint32_t>(min(i0 - 2 + sc, I + 1) + 2 + (min(j0 - 2 + sr, J + 1) + 2) * p.sj) * ES;
    const int lside = l < 4 * PJ ? sr * PI + sc : PJ * PI + ti;

    // Elimination: ring of the next PF steps' b, w, lower (of level t, used at
    // step t + 1) and upper (of level t + 1); with FUSEH also the u tile and
    // coeff of level t (raw stored bits).
    double rbv[PF], rwv[PF], rlov[PF], rupv[PF];
    R rum[PF][FUSEH ? MR : 1], rus[PF], rcv[PF];
    auto load = [&](int q, int s) {
        const int t = max(s - shift, 0);
        const uint32_t o = clampk(t) * skt, o1 = clampk(t + 1) * skt;
        rbv[q] = IO::template load<2>(rb, vt, o);
        rwv[q] = IO::template load<2>(rw, vt, o);
        rlov[q] = IO::template load<2>(rlo, vt, o);
        rupv[q] = IO::template load<2>(rup, vt, o1);
        if constexpr (FUSEH) {
#pragma unroll
            for (int m = 0; m < MR; ++m) rum[q][m] = IO::load_raw(ru, vmain[m], o);
            if (side_wave) rus[q] = IO::load_raw(ru, vside, o);
            rcv[q] = IO::template load_raw<2>(rcf, vt, o);
        }
    };
#pragma unroll
    for (int q = 0; q < PF && q < KH; ++q) load(q, q);

    double P[KH], D[KH];
    double lo_carry = 0.0;  // lower of this step's row: the far-side neighbour's coefficient
#pragma unroll
    for (int s = 0; s < KH; ++s) {
        const int q = s % PF;
        const bool pad = s < shift, first = s == shift;
        double bt = rbv[q], wt = rwv[q], upt = rupv[q];
        const double lot = first ? 0.0 : lo_carry;  // the far-end row has no lower neighbour
        lo_carry = rlov[q];
        C cf = C(0);
        C *tb = &utile[FUSEH ? (half * 2 + (s & 1)) * TILE : 0];
        if constexpr (FUSEH) {
#pragma unroll
            for (int m = 0; m < MR; ++m) tb[lmain[m]] = IO::cvt(rum[q][m]);
            if (side_wave) tb[lside] = IO::cvt(rus[q]);
            cf = IO::cvt(rcv[q]);
        }
        if (s + PF < KH) load(q, s + PF);
        if constexpr (FUSEH) {
            __syncthreads();
            hs[s * 2 * NH + tid] = hdiff_point<C, PI>(tb + (tj + 2) * PI + ti + 2, cf);
        }
        // The interface row's upper belongs to the other half's first level;
        // with an empty other half (K = 1) it is never used.
        if (pad) {
            bt = 1.0;
            wt = 0.0;
            upt = 0.0;
        }
        if (s == 0) {
            const double r = recip(bt);
            P[0] = upt * r;
            D[0] = wt * r;
        } else {
            const int sm = s > 0 ? s - 1 : 0;
            const double r = recip(fmadd(-lot, P[sm], bt));
            P[s] = upt * r;
            D[s] = fmadd(-lot, D[sm], wt) * r;
        }
        pin(P[s]);
        pin(D[s]);
    }

    // Interface: x(M-1) + P0 x(M) = D0 and x(M) + P1 x(M-1) = D1 (lam here).
    const double Pm = nsteps > 0 ? P[KH - 1] : 0.0, Dm = nsteps > 0 ? D[KH - 1] : 0.0;
    xch[tid] = make_double2(Pm, Dm);
    __syncthreads();
    const double2 o2 = xch[half ? l : NH + l];
    const double P0 = half ? o2.x : Pm, D0 = half ? o2.y : Dm;
    const double P1 = half ? Pm : o2.x, D1 = half ? Dm : o2.y;
    const double x_lo = fmadd(-P0, D1, D0) / fmadd(-P0, P1, 1.0);
    const double x_hi = fmadd(-P1, x_lo, D1);
    if (nsteps == 0) return;  // after the only barrier

    // Outward walk.  "in" is the side toward the interface (local t + 1),
    // "out" the side toward the far end.  dts orients the face flux: in half 0
    // local t + 1 is the level above, in half 1 the level below.
    const double dt = p.dt, dts = half ? -dt : dt;
    const bool other = K - M > 0;  // the interface level has a neighbour across it
    const auto rx = make_rsrc(MATRIX ? p.x : p.w, tbytes);
    // wcon, h (and x) of local level t: a ring of the next WR levels out.
    double rwc_[WR], rh_[WR], rx_[WR];
    auto wload = [&](int q, int t) {
        const uint32_t k = clampk(t);
        rwc_[q] = IO::template load<2>(rwc, vt, k * skt);
        rh_[q] = FUSEH ? 0.0 : static_cast<double>(IOC::load(rh, vc, k * skc));
        rx_[q] = MATRIX ? static_cast<double>(IO::template load<2>(rx, vt, k * skt)) : 0.0;
    };
    // h of step index st (FUSEH: from LDS; the other half's via its lane xo).
    const int xo = half ? l : NH + l;
    // Slot q holds local level (step index q) - shift, step index = static.
    // Walk order: the interface level (step KH - 1), then steps KH - 2, ...
#pragma unroll
    for (int q = 0; q < WR; ++q) wload(q, KH - 1 - q - shift);
    // The level across the interface.
    double lam_in = half ? x_lo : x_hi;
    double wc_in = 0.0, h_in = 0.0, x_in = 0.0;
    if (other) {
        const uint32_t k = clampk(nsteps);
        wc_in = IO::template load<2>(rwc, vt, k * skt);
        h_in = FUSEH ? static_cast<double>(hs[(KH - 1) * 2 * NH + xo]) : static_cast<double>(IOC::load(rh, vc, k * skc));
        if constexpr (MATRIX) x_in = IO::template load<2>(rx, vt, k * skt);
    }
    bool has_in = other;
    double lam = half ? x_hi : x_lo;  // lam of the current level
    double wc_t = rwc_[0], h_t = FUSEH ? static_cast<double>(hs[(KH - 1) * 2 * NH + tid]) : rh_[0], x_t = rx_[0];
    if (KH - 1 - WR >= 0) wload(0, KH - 1 - WR - shift);
    double fh_in = 0.0, wb_in = 0.0, hb_in = 0.0;  // face between the current level and "in"
    if (has_in) {
        fh_in = -dts * (lam - lam_in);
        wb_in = 0.5 * (wc_t + wc_in);
        hb_in = 0.5 * (h_t + h_in);
    }
#pragma unroll
    for (int st = KH - 1; st >= 0; --st) {
        // Step index st is the current level (local st - shift); st - 1 the next one out.
        if (st >= shift) {
            const int t = st - shift;
            const bool has_out = t > 0;
            const int so = st > 0 ? st - 1 : 0;
            const int q = (KH - 1 - so) % WR;
            const double lam_o = has_out ? fmadd(-P[so], lam, D[so]) : 0.0;
            const double wc_o = rwc_[q], x_o = rx_[q];
            const double h_o = FUSEH ? static_cast<double>(hs[so * 2 * NH + tid]) : rh_[q];
            double g = lam, gw = 0.0, fh_o = 0.0, wb_o = 0.0, hb_o = 0.0;
            if (has_in) {
                g = fmadd(0.5 * fh_in, wb_in, g);
                gw = fmadd(0.5 * fh_in, hb_in, gw);
            }
            if (has_out) {
                fh_o = -dts * (lam_o - lam);
                wb_o = 0.5 * (wc_t + wc_o);
                hb_o = 0.5 * (h_t + h_o);
                g = fmadd(0.5 * fh_o, wb_o, g);
                gw = fmadd(0.5 * fh_o, hb_o, gw);
            }
            if (active) {
                const uint32_t k = static_cast<uint32_t>(level(t));
                IOC::store_d(rgh, vc, k * skc, g);
                IO::template store_d<2>(rgw, vt, k * skt, gw);
                if constexpr (MATRIX) {
                    // x(k-1) and x(k+1): the far-end and interface sides, swapped in half 1.
                    const double x_dn = half ? x_in : x_o, x_upv = half ? x_o : x_in;
                    const bool has_dn = half ? has_in : has_out, has_up = half ? has_out : has_in;
                    if (p.ga)
                        IO::template store_d<2>(make_rsrc(p.ga, tbytes), vt, k * skt, has_dn ? -lam * x_dn : 0.0);
                    if (p.gb) IO::template store_d<2>(make_rsrc(p.gb, tbytes), vt, k * skt, -lam * x_t);
                    if (p.gc)
                        IO::template store_d<2>(make_rsrc(p.gc, tbytes), vt, k * skt, has_up ? -lam * x_upv : 0.0);
                }
            }
            // Step out: the face just used becomes the next level's "in" face.
            fh_in = fh_o;
            wb_in = wb_o;
            hb_in = hb_o;
            has_in = true;
            lam_in = lam;
            x_in = x_t;
            lam = lam_o;
            wc_t = wc_o;
            h_t = h_o;
            x_t = x_o;
        }
        // Refill the slot just consumed with the level WR steps further out.
        const int so = st > 0 ? st - 1 : 0;
        if (st > 0 && so - WR >= 0) wload((KH - 1 - so) % WR, so - WR - shift);
    }
}

// ---------------------------------------------------------------------------
// hdiff adjoint.  Tile of 64 x TJ output points of the extended domain
// [-2, I+2) x [-2, J+2), local coordinates (lx, ly) = (i - x0, j - y0); a
// workgroup marches over kc consecutive levels of its tile.  Per level
// (each stage ends with a barrier):
//   U  u on lx in [-3, 67), ly in [-3, TJ+3) (0 outside u's 2-cell halo)
//   G  g = -coeff gh on lx in [-2, 66), ly in [-2, TJ+2) (0 outside the interior)
//   L  lap on lx in [-2, 66), ly in [-2, TJ+2)
//   X  x-faces lx in [-2, 65), ly in [-1, TJ+1): gfx = kx (g(i) - g(i+1)), flx = kx (lap(i+1) - lap(i))
//   Y  y-faces lx in [-1, 65), ly in [-2, TJ+1): likewise in j
//   H  glap = gfx(i-1) - gfx(i) + gfy(j-1) - gfy(j) on lx in [-1, 65), ly in [-1, TJ+1)
// then gu = gh (interior) - glap(j-1) - glap(i-1) + 4 glap - glap(i+1) - glap(j+1)
// and gcoeff = -gh (flx - flx(i-1) + fly - fly(j-1)).
// The global values of U and G (and gh at the outputs) for the next PF
// levels are requested into a register ring before a level's stages run, so
// their latency overlaps that level's LDS work.  Loads address clamped,
// valid cells; a select applies the zero outside the domain.
// ---------------------------------------------------------------------------
template <class T, int TJ, int PF>
__global__ __launch_bounds__(256) void k_hdiff_adjoint(AdjArgs p, int nbi, int ntiles, int kc) {
#pragma clang fp contract(off)
    using S = Storage<T>;
    using C = typename S::C;
    using IO = BufIO<T>;
    using IOC = BufIO<C>;
    using R = typename IO::R;
    using RC = typename IOC::R;
    constexpr int TI = 64;
    constexpr int UX = TI + 6, UY = TJ + 6;     // offset 3
    constexpr int GX = TI + 4, GY = TJ + 4;     // offset 2 (g and lap)
    constexpr int XX = TI + 3, XY = TJ + 2;     // x-faces: lx + 2, ly + 1
    constexpr int YX = TI + 2, YY = TJ + 3;     // y-faces: lx + 1, ly + 2
    constexpr int HX = TI + 2, HY = TJ + 2;     // glap: lx + 1, ly + 1
    constexpr int NU = (UY * UX + 255) / 256, NG = (GY * GX + 255) / 256, NO = (TJ + 3) / 4;
    constexpr uint32_t ES = sizeof(T), ESC = sizeof(C);
    __shared__ C su[UY * UX], sg[GY * GX], sl[GY * GX];
    __shared__ C sgx[XY * XX], sfx[XY * XX], sgy[YY * YX], sfy[YY * YX], sh[HY * HX];

    T *__restrict__ gu = static_cast<T *>(p.gu);
    T *__restrict__ gcoeff = static_cast<T *>(p.gcoeff);
    const int I = p.I, J = p.J, K = p.K, sj = p.sj;
    // Workgroups numbered chunk-major: consecutive positions are neighbouring
    // tiles of one level range, kept on one XCD so their shared halo rows
    // meet in its L2.
    const int pos = xcd_tile(blockIdx.x, gridDim.x);
    const int tile = pos % ntiles, chunk = pos / ntiles;
    const int k0 = chunk * kc, k1 = min(K, k0 + kc);
    const int bi = tile % nbi, bj = tile / nbi;
    const int x0 = -2 + bi * TI, y0 = -2 + bj * TJ;
    const int tid = threadIdx.x;

    // u from its cell (-2, -2, 0); coeff and gh from the interior origin.
    const long long cells = static_cast<long long>(K - 1) * p.sk;
    const auto ru = make_rsrc(static_cast<const T *>(p.u) - 2 - 2 * sj,
                              static_cast<uint32_t>(((I + 3) + (J + 3) * static_cast<long long>(sj) + cells + 1) * ES));
    const uint32_t col = static_cast<uint32_t>((I - 1) + (J - 1) * static_cast<long long>(sj) + cells + 1);
    const auto rcf = make_rsrc(p.coeff, col * ES);
    const auto rgh = make_rsrc(p.gh, col * ESC);
    uint32_t vu[NU], vg[NG], vo[NO];
    bool okv[NU], okg[NG], inner[NO];
#pragma unroll
    for (int n = 0; n < NU; ++n) {
        const int e = min(tid + 256 * n, UY * UX - 1);
        const int i = x0 - 3 + e % UX, j = y0 - 3 + e / UX;
        okv[n] = i >= -2 && i < I + 2 && j >= -2 && j < J + 2;
        vu[n] = static_cast<uint32_t>(min(max(i, -2), I + 1) + 2 + (min(max(j, -2), J + 1) + 2) * sj);
    }
#pragma unroll
    for (int n = 0; n < NG; ++n) {
        const int e = min(tid + 256 * n, GY * GX - 1);
        const int i = x0 - 2 + e % GX, j = y0 - 2 + e / GX;
        okg[n] = i >= 0 && i < I && j >= 0 && j < J;
        vg[n] = static_cast<uint32_t>(min(max(i, 0), I - 1) + min(max(j, 0), J - 1) * sj);
    }
#pragma unroll
    for (int n = 0; n < NO; ++n) {
        const int i = x0 + (tid & 63), j = y0 + (tid >> 6) + 4 * n;
        inner[n] = i >= 0 && i < I && j >= 0 && j < J;
        vo[n] = static_cast<uint32_t>(min(max(i, 0), I - 1) + min(max(j, 0), J - 1) * sj);
    }

    R rum[PF][NU], rcv[PF][NG];
    RC rgv[PF][NG], rov[PF][NO];
    auto load = [&](int q, int k) {
        const uint32_t ko = static_cast<uint32_t>(k) * static_cast<uint32_t>(p.sk);
#pragma unroll
        for (int n = 0; n < NU; ++n) rum[q][n] = IO::load_raw(ru, (vu[n] + ko) * ES, 0);
#pragma unroll
        for (int n = 0; n < NG; ++n) {
            rcv[q][n] = IO::load_raw(rcf, (vg[n] + ko) * ES, 0);
            rgv[q][n] = IOC::load_raw(rgh, (vg[n] + ko) * ESC, 0);
        }
#pragma unroll
        for (int n = 0; n < NO; ++n) rov[q][n] = IOC::load_raw(rgh, (vo[n] + ko) * ESC, 0);
    };
#pragma unroll
    for (int q = 0; q < PF; ++q)
        if (k0 + q < k1) load(q, k0 + q);

    for (int kk = k0; kk < k1; kk += PF) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int k = kk + q;
            if (k >= k1) break;
#pragma unroll
            for (int n = 0; n < NU; ++n)
                if (tid + 256 * n < UY * UX) su[tid + 256 * n] = okv[n] ? IO::cvt(rum[q][n]) : C(0);
#pragma unroll
            for (int n = 0; n < NG; ++n)
                if (tid + 256 * n < GY * GX)
                    sg[tid + 256 * n] = okg[n] ? -IO::cvt(rcv[q][n]) * IOC::cvt(rgv[q][n]) : C(0);
            C gho[NO];
#pragma unroll
            for (int n = 0; n < NO; ++n) gho[n] = inner[n] ? IOC::cvt(rov[q][n]) : C(0);
            if (k + PF < k1) load(q, k + PF);
            __syncthreads();
            for (int e = tid; e < GY * GX; e += 256) {
                const C *c = &su[(e / GX + 1) * UX + e % GX + 1];
                sl[e] = C(4) * c[0] - c[1] - c[-1] - c[UX] - c[-UX];
            }
            __syncthreads();
            for (int e = tid; e < XY * XX; e += 256) {
                const int lx = e % XX - 2, ly = e / XX - 1;
                const int gl = (ly + 2) * GX + lx + 2, ul = (ly + 3) * UX + lx + 3;
                const C f = sl[gl + 1] - sl[gl];
                const C du = su[ul + 1] - su[ul];
                const bool kept = !(f * du > C(0));
                sfx[e] = kept ? f : C(0);
                sgx[e] = kept ? sg[gl] - sg[gl + 1] : C(0);
            }
            for (int e = tid; e < YY * YX; e += 256) {
                const int lx = e % YX - 1, ly = e / YX - 2;
                const int gl = (ly + 2) * GX + lx + 2, ul = (ly + 3) * UX + lx + 3;
                const C f = sl[gl + GX] - sl[gl];
                const C du = su[ul + UX] - su[ul];
                const bool kept = !(f * du > C(0));
                sfy[e] = kept ? f : C(0);
                sgy[e] = kept ? sg[gl] - sg[gl + GX] : C(0);
            }
            __syncthreads();
            for (int e = tid; e < HY * HX; e += 256) {
                const int lx = e % HX - 1, ly = e / HX - 1;
                const int xi = (ly + 1) * XX + lx + 2, yi = (ly + 2) * YX + lx + 1;
                sh[e] = sgx[xi - 1] - sgx[xi] + sgy[yi - YX] - sgy[yi];
            }
            __syncthreads();
            const long long ko = static_cast<long long>(k) * p.sk;
#pragma unroll
            for (int n = 0; n < NO; ++n) {
                const int lx = tid & 63, ly = (tid >> 6) + 4 * n;
                const int i = x0 + lx, j = y0 + ly;
                if (ly < TJ && i < I + 2 && j < J + 2) {
                    const int hc = (ly + 1) * HX + lx + 1;
                    const long long o = i + static_cast<long long>(j) * sj + ko;
                    const C ghv = gho[n];
                    const C g = ghv - sh[hc - HX] - sh[hc - 1] + C(4) * sh[hc] - sh[hc + 1] - sh[hc + HX];
                    S::store(gu + o, g);
                    if (inner[n]) {
                        const int xi = (ly + 1) * XX + lx + 2, yi = (ly + 2) * YX + lx + 1;
                        const C div = sfx[xi] - sfx[xi - 1] + sfy[yi] - sfy[yi - YX];
                        S::store(gcoeff + o, -ghv * div);
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// hdiff adjoint without LDS: one wave per strip of 64 columns x TJ rows.
// Lane l holds column x0 + l; the strip's rows live in the lane's registers,
// so neighbours in j are other registers and neighbours in i are the next or
// previous lane, fetched with a whole-wave DPP shift.  Each shift leaves the
// wave's edge lane without a neighbour, and gu at column i depends on columns
// i - 3 .. i + 3, so a strip writes its middle 58 columns (lanes 3 .. 60) and
// strips step by 58 columns.  Rows (relative to the strip's first output row
// y0): u on [-3, TJ+3), g = -coeff gh and lap on [-2, TJ+2), y-faces between
// rows t and t+1 for t in [-2, TJ+1), x-faces and glap on [-1, TJ+1),
// outputs on [0, TJ).  The arithmetic is that of the LDS formulation above,
// operation for operation.  No barriers: the four waves of a workgroup are
// four neighbouring strips.  Row offsets are wave-uniform (scalar operands of
// the buffer loads); columns outside a field are clamped onto valid cells
// and a select applies the zero.
// ---------------------------------------------------------------------------
constexpr int ADJ_STRIP = 58;  // output columns per 64-lane strip

// Value of lane l + 1 (from_right) or l - 1 (from_left) of the wave, 0 past
// the wave's ends (lane shifts of common.hpp: uniform control flow only).
template <class V> __device__ __forceinline__ V from_right(V v) { return lane_next(v, V(0)); }
template <class V> __device__ __forceinline__ V from_left(V v) { return lane_prev(v, V(0)); }

template <class T, int TJ, int PF>
__global__ __launch_bounds__(256) void k_hdiff_adjoint_dpp(AdjArgs p, int nbi, int nstrips, int kc) {
#pragma clang fp contract(off)
    using S = Storage<T>;
    using C = typename S::C;
    using IO = BufIO<T>;
    using IOC = BufIO<C>;
    using R = typename IO::R;
    using RC = typename IOC::R;
    constexpr int NU = TJ + 6, NG = TJ + 4;
    constexpr uint32_t ES = sizeof(T), ESC = sizeof(C);
    T *__restrict__ gu = static_cast<T *>(p.gu);
    T *__restrict__ gcoeff = static_cast<T *>(p.gcoeff);
    const int I = p.I, J = p.J, K = p.K, sj = p.sj;
    // Workgroups numbered chunk-major (a chunk is a run of kc levels);
    // consecutive positions hold neighbouring strips and stay on one XCD.
    const int ngroups = (nstrips + 3) / 4;
    const int pos = xcd_tile(blockIdx.x, gridDim.x);
    const int group = pos % ngroups, chunk = pos / ngroups;
    const int strip = group * 4 + __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    if (strip >= nstrips) return;
    const int k0 = chunk * kc, k1 = min(K, k0 + kc);
    const int bi = strip % nbi, bj = strip / nbi;
    const int x0 = -5 + ADJ_STRIP * bi, y0 = -2 + TJ * bj;
    const int lane = threadIdx.x & 63, i = x0 + lane;
    const bool okcu = i >= -2 && i < I + 2, okcg = i >= 0 && i < I;
    const bool out_col = lane >= 3 && lane < 3 + ADJ_STRIP && i < I + 2;

    // u from its cell (-2, -2, 0); coeff and gh from the interior origin.
    const long long cells = static_cast<long long>(K - 1) * p.sk;
    const auto ru = make_rsrc(static_cast<const T *>(p.u) - 2 - 2 * sj,
                              static_cast<uint32_t>(((I + 3) + (J + 3) * static_cast<long long>(sj) + cells + 1) * ES));
    const uint32_t col = static_cast<uint32_t>((I - 1) + (J - 1) * static_cast<long long>(sj) + cells + 1);
    const auto rcf = make_rsrc(p.coeff, col * ES);
    const auto rgh = make_rsrc(p.gh, col * ESC);
    const uint32_t vu = static_cast<uint32_t>(min(max(i, -2), I + 1) + 2);
    const uint32_t vg = static_cast<uint32_t>(min(max(i, 0), I - 1));
    auto urow = [&](int t) {  // u row y0 - 3 + t, in elements from u's cell (-2, -2)
        return static_cast<uint32_t>((min(max(y0 - 3 + t, -2), J + 1) + 2) * sj);
    };
    auto grow = [&](int t) {  // g row y0 - 2 + t, from the interior origin
        return static_cast<uint32_t>(min(max(y0 - 2 + t, 0), J - 1) * sj);
    };

    R rum[PF][NU], rcv[PF][NG];
    RC rgv[PF][NG];
    auto load = [&](int q, int k) {
        const uint32_t ko = static_cast<uint32_t>(k) * static_cast<uint32_t>(p.sk);
#pragma unroll
        for (int t = 0; t < NU; ++t) rum[q][t] = IO::load_raw(ru, vu * ES, (urow(t) + ko) * ES);
#pragma unroll
        for (int t = 0; t < NG; ++t) {
            rcv[q][t] = IO::load_raw(rcf, vg * ES, (grow(t) + ko) * ES);
            rgv[q][t] = IOC::load_raw(rgh, vg * ESC, (grow(t) + ko) * ESC);
        }
    };
#pragma unroll
    for (int q = 0; q < PF; ++q)
        if (k0 + q < k1) load(q, k0 + q);

    for (int kk = k0; kk < k1; kk += PF) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int k = kk + q;
            if (k >= k1) break;
            C u[NU], g[NG], gho[TJ];
#pragma unroll
            for (int t = 0; t < NU; ++t) {
                const int j = y0 - 3 + t;
                u[t] = okcu && j >= -2 && j < J + 2 ? IO::cvt(rum[q][t]) : C(0);
            }
#pragma unroll
            for (int t = 0; t < NG; ++t) {
                const int j = y0 - 2 + t;
                const bool ok = okcg && j >= 0 && j < J;
                const C ghx = IOC::cvt(rgv[q][t]);
                g[t] = ok ? -IO::cvt(rcv[q][t]) * ghx : C(0);
                if (t >= 2 && t < TJ + 2) gho[t - 2] = ok ? ghx : C(0);
            }
            if (k + PF < k1) load(q, k + PF);
            // One pass down the strip's rows: at g row t the Laplacian of row
            // t, the y-face between rows t - 1 and t, the x-face and glap of
            // row t - 1 and the outputs of row t - 2, so that every value
            // dies a few rows after it is made.
            C lap[NG], ue[NG], fy[NG - 1], gfy[NG - 1], fx[NG], glap[NG];
            const long long ko = static_cast<long long>(k) * p.sk;
#pragma unroll
            for (int t = 0; t < NG + 1; ++t) {
                if (t < NG) {  // Laplacian on g row t (u row t + 1), and u of the next column
                    const C uc = u[t + 1];
                    ue[t] = from_right(uc);
                    const C uw = from_left(uc);
                    lap[t] = C(4) * uc - ue[t] - uw - u[t + 2] - u[t];
                }
                if (t >= 1 && t < NG) {  // y-face between g rows t - 1 and t
                    const C f = lap[t] - lap[t - 1];
                    const C du = u[t + 1] - u[t];
                    const bool kept = !(f * du > C(0));
                    fy[t - 1] = kept ? f : C(0);
                    gfy[t - 1] = kept ? g[t - 1] - g[t] : C(0);
                }
                const int r = t - 1;  // x-face (between this column and the next) and glap of row r
                if (r >= 1 && r < NG - 1) {
                    // (every shift outside the selects: an operand of ?: is evaluated conditionally)
                    const C lap_e = from_right(lap[r]), g_e = from_right(g[r]);
                    const C f = lap_e - lap[r];
                    const C du = ue[r] - u[r + 1];
                    const bool kept = !(f * du > C(0));
                    fx[r] = kept ? f : C(0);
                    const C gfx = kept ? g[r] - g_e : C(0);
                    glap[r] = from_left(gfx) - gfx + gfy[r - 1] - gfy[r];
                }
                const int o = t - 2;  // outputs of row o
                if (o >= 2 && o < TJ + 2) {
                    const int j = y0 + o - 2;
                    const C sv = glap[o];
                    const C ghv = gho[o - 2];
                    const C gv = ghv - glap[o - 1] - from_left(sv) + C(4) * sv - from_right(sv) - glap[o + 1];
                    const C div = fx[o] - from_left(fx[o]) + fy[o] - fy[o - 1];
                    if (out_col && j < J + 2) {
                        const long long off = i + static_cast<long long>(j) * sj + ko;
                        S::store(gu + off, gv);
                        if (okcg && j >= 0 && j < J) S::store(gcoeff + off, -ghv * div);
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------

// Scratch: gh, and for FP64 storage also h (FP32 and bfloat16 storage
// evaluate h inside the column kernel); each plane in the compute type with
// the fields' strides, 256-byte aligned.
size_t adjoint_scratch_bytes(int dtype, int sk, int K) {
    const size_t cs = dtype == DT_F64 ? 8 : 4;
    const size_t plane = (static_cast<size_t>(sk) * K * cs + 255) / 256 * 256;
    return dtype == DT_F64 ? 2 * plane : plane;
}

template <class T, int KH, bool FUSEH>
static void launch_vadv_adjoint_t(const AdjArgs &a, hipStream_t st) {
    // 64 x 2 tiles (64 x 4 and 64 x 1 measured no faster).  The elimination
    // prefetches PF levels (2 while it also stages the u tile: 4 and 8 were
    // slower), the outward walk WR levels: at 256 x 256 x 80 FP32 a grid of
    // one round runs every workgroup's walk at once, and the walk took 17.7 us
    // of the kernel's 40.9 with WR = 4, 13.2 with 8, 11.3 with 16 (12 and 24
    // slower than 16).  FP64 keeps 4: its ring also holds h, and with the
    // matrix gradients x, two registers each a slot (8 spills at KH = 48;
    // without them, 8 measured 1% slower).
    constexpr int TJ = 2, PF = FUSEH ? 2 : 4, WR = FUSEH ? 16 : 4;
    const int nbi = (a.I + 63) / 64, nbj = (a.J + TJ - 1) / TJ;
    if (a.ga || a.gb || a.gc)
        hipLaunchKernelGGL((k_vadv_adjoint<T, TJ, PF, KH, true, FUSEH, WR>), dim3(nbi * nbj), dim3(128 * TJ), 0,
                           st, a, nbi);
    else
        hipLaunchKernelGGL((k_vadv_adjoint<T, TJ, PF, KH, false, FUSEH, WR>), dim3(nbi * nbj), dim3(128 * TJ), 0,
                           st, a, nbi);
}

template <class T, int TJ, int PF>
static hipError_t launch_hdiff_adjoint_dpp(const AdjArgs &a, hipStream_t st) {
    const int nbi = (a.I + 4 + ADJ_STRIP - 1) / ADJ_STRIP, nbj = (a.J + 4 + TJ - 1) / TJ;
    const long long nstrips = static_cast<long long>(nbi) * nbj, groups = (nstrips + 3) / 4;
    auto kern = k_hdiff_adjoint_dpp<T, TJ, PF>;
    const long long slots = resident_workgroups(reinterpret_cast<const void *>(kern), 256);
    const int kc = level_run(groups, slots, a.K, 1, 1, PF);
    const long long blocks = groups * ((a.K + kc - 1) / kc);
    if (blocks > 2147483647LL || nstrips > 2147483647LL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, a, nbi,
                       static_cast<int>(nstrips), kc);
    return hipGetLastError();
}

template <class T>
static hipError_t adjoint_run(AdjArgs a, void *scratch, bool staged_hdiff, int strip_rows, int strip_prefetch,
                              hipStream_t st) {
    using C = typename Storage<T>::C;
    const size_t plane = (static_cast<size_t>(a.sk) * a.K * sizeof(C) + 255) / 256 * 256;
    // FP32 and bfloat16 storage evaluate h inside the column kernel (FUSEH,
    // h held in LDS) and need only the gh plane; FP64's h would take twice
    // the LDS, so it is computed by the hdiff kernel into a second plane first.
    constexpr bool FUSEH = !std::is_same<T, double>::value;
    a.gh = scratch;
    a.h = FUSEH ? scratch : static_cast<char *>(scratch) + plane;  // (never read with FUSEH)
    hipError_t e = hipSuccess;
    if constexpr (!FUSEH) {
        HdiffArgs hd{};
        hd.u = a.u;
        hd.coeff = a.coeff;
        hd.out = a.h;
        hd.I = a.I; hd.J = a.J; hd.K = a.K; hd.sj = a.sj; hd.sk = a.sk;
        e = launch_hdiff_compute(DT_F64, hd, st);
        if (e != hipSuccess) return e;
    }
    const int m = (a.K + 1) / 2;  // levels of the longer half
    if (m <= 16) launch_vadv_adjoint_t<T, 16, FUSEH>(a, st);
    else if (m <= 32) launch_vadv_adjoint_t<T, 32, FUSEH>(a, st);
    else if (m <= 40) launch_vadv_adjoint_t<T, 40, FUSEH>(a, st);
    else launch_vadv_adjoint_t<T, 48, FUSEH>(a, st);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (!staged_hdiff) {
        // Register strips, DPP neighbours: rows per strip and levels in flight
        // from the caller's knobs, else 12 rows and one level (measured at
        // 256 x 256 x 80 FP32: reverse pass 0.0704 ms against 0.0722 for 8
        // rows and two levels, 0.0747 for 8 and one, 0.0754 for 16 and one);
        // FP64 4 rows and one level (its values take twice the registers).
        constexpr bool f64 = std::is_same<T, double>::value;
        const int tj = strip_rows ? strip_rows : f64 ? 4 : 12, pf = strip_prefetch ? strip_prefetch : 1;
        if (tj == 4 && pf == 1) return launch_hdiff_adjoint_dpp<T, 4, 1>(a, st);
        if (tj == 4 && pf == 2) return launch_hdiff_adjoint_dpp<T, 4, 2>(a, st);
        if constexpr (!f64) {
            if (tj == 8 && pf == 1) return launch_hdiff_adjoint_dpp<T, 8, 1>(a, st);
            if (tj == 8 && pf == 2) return launch_hdiff_adjoint_dpp<T, 8, 2>(a, st);
            if (tj == 12 && pf == 1) return launch_hdiff_adjoint_dpp<T, 12, 1>(a, st);
        }
        return hipErrorInvalidValue;
    }
    // The LDS formulation: rows per tile 8 (two per thread) where the staged
    // tile fits often enough in LDS; FP64's twice larger tile keeps 4.  Each
    // workgroup marches over kc levels with HPF levels in flight; kc is chosen
    // against the resident workgroup count (a mostly empty last round of
    // workgroups costs nearly as much as a full one).
    constexpr int HTJ = std::is_same<T, double>::value ? 4 : 8, HPF = 2;
    const int nbi = (a.I + 4 + 63) / 64, nbj = (a.J + 4 + HTJ - 1) / HTJ;
    const long long tiles = static_cast<long long>(nbi) * nbj;
    auto kern = k_hdiff_adjoint<T, HTJ, HPF>;
    const long long slots = resident_workgroups(reinterpret_cast<const void *>(kern), 256);
    const int kc = level_run(tiles, slots, a.K, 1, 1, HPF);
    const long long blocks = tiles * ((a.K + kc - 1) / kc);
    if (blocks > 2147483647LL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, a, nbi,
                       static_cast<int>(tiles), kc);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed scratch for the reverse pass that allocates nothing
// (stencil_hdiff_vadv_adjoint_noalloc).  The array is part of the code
// object: every device the library runs on holds its own copy, at its own
// address, until the process ends.  Host code never passes the array's name
// to a kernel (on the host it is only a stand-in for the symbol); it looks up
// each device's address once, with that device current, and uses that.
// Nothing in it needs to start at zero: the column kernel writes gh (and the
// FP64 hdiff kernel h) on the whole interior before any kernel reads it, and
// the hdiff adjoint masks what it reads outside the interior.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char adjoint_scratch[ADJOINT_FIXED_SCRATCH_BYTES];

namespace {
std::mutex g_fixed_mu;
std::map<int, void *> g_fixed_ptr;  // device -> address of its adjoint_scratch
}  // namespace

hipError_t adjoint_fixed_scratch(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(g_fixed_mu);
    auto it = g_fixed_ptr.find(dev);
    if (it == g_fixed_ptr.end()) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(adjoint_scratch));
        if (e != hipSuccess) return e;
        if (p == nullptr || reinterpret_cast<uintptr_t>(p) % 256 != 0) return hipErrorInvalidSymbol;
        it = g_fixed_ptr.emplace(dev, p).first;
    }
    *out = it->second;
    return hipSuccess;
}

hipError_t launch_adjoint(int dtype, const AdjointArgs &x, void *scratch, hipStream_t st) {
    const bool staged = x.hdiff_schedule == 1;
    const int rows = x.hdiff_tile_j, pf = x.hdiff_prefetch;
    AdjArgs a{};
    a.u = x.u; a.coeff = x.coeff; a.wcon = x.wcon; a.a = x.a; a.b = x.b; a.c = x.c; a.w = x.w;
    a.gu = x.gu; a.gcoeff = x.gcoeff; a.gwcon = x.gwcon;
    a.x = x.x; a.ga = x.ga; a.gb = x.gb; a.gc = x.gc;
    a.I = x.I; a.J = x.J; a.K = x.K; a.sj = x.sj; a.sk = x.sk;
    a.dt = x.dt;
    switch (dtype) {
    case DT_F64: return adjoint_run<double>(a, scratch, staged, rows, pf, st);
    case DT_F32: return adjoint_run<float>(a, scratch, staged, rows, pf, st);
    case DT_BF16: return adjoint_run<uint16_t>(a, scratch, staged, rows, pf, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace stl
