// Reverse mode of x = vadv(hdiff(u, coeff), wcon, a, b, c, dt) for the loss
// L = sum over the interior of w * x, with the limiter decisions of the
// forward pass frozen (their derivative is taken as zero).
//
// Three launches on one stream:
//   1. hdiff recomputes h (compute type) into scratch;
//   2. k_vadv_adjoint, one lane per column: the transposed Thomas solve
//      lam = T^-T w (double precision), then, walking down the column, the
//      adjoint of the flux-form right-hand side
//        Fhat(k+1/2) = -dt (lam(k) - lam(k+1))
//        gh(k)  = lam(k) + Fhat(k-1/2) wbar(k-1/2)/2 + Fhat(k+1/2) wbar(k+1/2)/2
//        gwcon(k) =        Fhat(k-1/2) hbar(k-1/2)/2 + Fhat(k+1/2) hbar(k+1/2)/2
//      (wbar, hbar: face means of wcon and h); gh goes to scratch;
//   3. k_hdiff_adjoint, one workgroup per (tile, level): with g = -coeff gh,
//      the transposed update, limited flux and Laplacian stencils, staged
//      through LDS, give gu on the interior and its 2-cell ring and
//      gcoeff = -gh (flx - flx(i-1) + fly - fly(j-1)) on the interior.
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
// Transposed Thomas solve and right-hand-side adjoint, one lane per column.
// T^T has sub-diagonal c(k-1), diagonal b(k), super-diagonal a(k+1).
// ---------------------------------------------------------------------------
// MATRIX: also ga(k) = -lam(k) x(k-1), gb(k) = -lam(k) x(k), gc(k) = -lam(k) x(k+1)
// from the forward result x, for whichever of ga, gb, gc is set.
template <class T, int KMAX, bool MATRIX>
__global__ __launch_bounds__(256) void k_vadv_adjoint(AdjArgs p) {
    using S = Storage<T>;
    using C = typename S::C;
    const T *__restrict__ fa = static_cast<const T *>(p.a);
    const T *__restrict__ fb = static_cast<const T *>(p.b);
    const T *__restrict__ fc = static_cast<const T *>(p.c);
    const T *__restrict__ fw = static_cast<const T *>(p.w);
    const T *__restrict__ wcon = static_cast<const T *>(p.wcon);
    const C *__restrict__ hs = static_cast<const C *>(p.h);
    C *__restrict__ ghs = static_cast<C *>(p.gh);
    T *__restrict__ gwc = static_cast<T *>(p.gwcon);

    const int gi = blockIdx.x * 64 + (threadIdx.x & 63);
    const int gj = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (gi >= p.I || gj >= p.J) return;
    const int col = gi + gj * p.sj, sk = p.sk, K = p.K;
    const double dt = p.dt;

    // Forward elimination of T^T lam = w.  Row t is eliminated at step t + 1,
    // once its super-diagonal a(t + 1) has been read.
    double P[KMAX], D[KMAX];
    double b_t = 0.0, w_t = 0.0, c_tm1 = 0.0, c_t = 0.0;
#pragma unroll
    for (int s = 0; s < KMAX; ++s) {
        if (s < K) {
            const int o = col + s * sk;
            const double as = S::load(fa + o), bs = S::load(fb + o), cs = S::load(fc + o),
                         ws = S::load(fw + o);
            if (s > 0) {
                const int t = s - 1;
                if (t == 0) {
                    const double r = recip(b_t);
                    P[0] = as * r;
                    D[0] = w_t * r;
                } else {
                    const int tm = t > 0 ? t - 1 : 0;
                    const double r = recip(b_t - c_tm1 * P[tm]);
                    P[t] = as * r;
                    D[t] = (w_t - c_tm1 * D[tm]) * r;
                }
            }
            c_tm1 = c_t;
            c_t = cs;
            b_t = bs;
            w_t = ws;
            if (s == K - 1) {
                // Last row: no super-diagonal.
                if (s == 0) {
                    D[0] = w_t / b_t;
                } else {
                    const int tm = s > 0 ? s - 1 : 0;
                    D[s] = (w_t - c_tm1 * D[tm]) / (b_t - c_tm1 * P[tm]);
                }
            }
        }
    }

    // Back-substitution lam(k) = D(k) - P(k) lam(k+1), walking down; level
    // k + 1 is finished once lam(k) gives the face below it.
    double lam_up = 0.0, fh_up = 0.0;   // lam(k+1), Fhat(k+3/2)
    double h_up = 0.0, wc_up = 0.0;     // h(k+1), wcon(k+1)
    double h_up2 = 0.0, wc_up2 = 0.0;   // h(k+2), wcon(k+2)
#pragma unroll
    for (int s = KMAX - 1; s >= 0; --s) {
        if (s < K) {
            const int o = col + s * sk;
            const double lam = (s == K - 1) ? D[s] : D[s] - P[s] * lam_up;
            if constexpr (MATRIX) {
                const T *__restrict__ fx = static_cast<const T *>(p.x);
                const double xk = S::load(fx + o);
                if (p.ga) S::store_d(static_cast<T *>(p.ga) + o, s > 0 ? -lam * S::load(fx + o - sk) : 0.0);
                if (p.gb) S::store_d(static_cast<T *>(p.gb) + o, -lam * xk);
                if (p.gc) S::store_d(static_cast<T *>(p.gc) + o, s < K - 1 ? -lam * S::load(fx + o + sk) : 0.0);
            }
            const double hk = static_cast<double>(hs[o]), wk = static_cast<double>(S::load(wcon + o));
            if (s < K - 1) {
                // Face s + 1/2, then level s + 1 is complete.
                const double fh = -dt * (lam - lam_up);
                const double wbar = 0.5 * (wk + wc_up), hbar = 0.5 * (hk + h_up);
                double g = lam_up, gw = 0.0;
                g += 0.5 * fh * wbar;
                gw += 0.5 * fh * hbar;
                if (s + 1 < K - 1) {
                    const double wbar2 = 0.5 * (wc_up + wc_up2), hbar2 = 0.5 * (h_up + h_up2);
                    g += 0.5 * fh_up * wbar2;
                    gw += 0.5 * fh_up * hbar2;
                }
                const int o1 = o + sk;
                ghs[o1] = static_cast<C>(g);
                S::store_d(gwc + o1, gw);
                fh_up = fh;
            }
            h_up2 = h_up;
            wc_up2 = wc_up;
            h_up = hk;
            wc_up = wk;
            lam_up = lam;
        }
    }
    // Level 0: only the face above it.
    {
        double g = lam_up, gw = 0.0;
        if (K > 1) {
            const double wbar = 0.5 * (wc_up + wc_up2), hbar = 0.5 * (h_up + h_up2);
            g += 0.5 * fh_up * wbar;
            gw += 0.5 * fh_up * hbar;
        }
        ghs[col] = static_cast<C>(g);
        S::store_d(gwc + col, gw);
    }
}

// ---------------------------------------------------------------------------
// hdiff adjoint.  Tile of 64 x 4 output points of the extended domain
// [-2, I+2) x [-2, J+2) at one level, local coordinates (lx, ly) = (i - x0,
// j - y0).  Stages (each ends with a barrier):
//   U  u on lx in [-3, 67), ly in [-3, 7) (0 outside u's 2-cell halo)
//   G  g = -coeff gh on lx in [-2, 66), ly in [-2, 6) (0 outside the interior)
//   L  lap on lx in [-2, 66), ly in [-2, 6)
//   X  x-faces lx in [-2, 65), ly in [-1, 5): gfx = kx (g(i) - g(i+1)), flx = kx (lap(i+1) - lap(i))
//   Y  y-faces lx in [-1, 65), ly in [-2, 5): likewise in j
//   H  glap = gfx(i-1) - gfx(i) + gfy(j-1) - gfy(j) on lx in [-1, 65), ly in [-1, 5)
// then gu = gh (interior) - glap(j-1) - glap(i-1) + 4 glap - glap(i+1) - glap(j+1)
// and gcoeff = -gh (flx - flx(i-1) + fly - fly(j-1)).
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void k_hdiff_adjoint(AdjArgs p, int nbi) {
    using S = Storage<T>;
    using C = typename S::C;
    constexpr int TI = 64, TJ = 4;
    constexpr int UX = TI + 6, UY = TJ + 6;     // offset 3
    constexpr int GX = TI + 4, GY = TJ + 4;     // offset 2 (g and lap)
    constexpr int XX = TI + 3, XY = TJ + 2;     // x-faces: lx + 2, ly + 1
    constexpr int YX = TI + 2, YY = TJ + 3;     // y-faces: lx + 1, ly + 2
    constexpr int HX = TI + 2, HY = TJ + 2;     // glap: lx + 1, ly + 1
    __shared__ C su[UY * UX], sg[GY * GX], sl[GY * GX];
    __shared__ C sgx[XY * XX], sfx[XY * XX], sgy[YY * YX], sfy[YY * YX], sh[HY * HX];

    const T *__restrict__ u = static_cast<const T *>(p.u);
    const T *__restrict__ coeff = static_cast<const T *>(p.coeff);
    const C *__restrict__ gh = static_cast<const C *>(p.gh);
    T *__restrict__ gu = static_cast<T *>(p.gu);
    T *__restrict__ gcoeff = static_cast<T *>(p.gcoeff);
    const int I = p.I, J = p.J, sj = p.sj;
    const int bi = blockIdx.x % nbi, bj = blockIdx.x / nbi, k = blockIdx.y;
    const int x0 = -2 + bi * TI, y0 = -2 + bj * TJ;
    const int ko = k * p.sk;
    const int tid = threadIdx.x;

    for (int e = tid; e < UY * UX; e += 256) {
        const int i = x0 - 3 + e % UX, j = y0 - 3 + e / UX;
        su[e] = (i >= -2 && i < I + 2 && j >= -2 && j < J + 2) ? S::load(u + i + j * sj + ko) : C(0);
    }
    for (int e = tid; e < GY * GX; e += 256) {
        const int i = x0 - 2 + e % GX, j = y0 - 2 + e / GX;
        C g = C(0);
        if (i >= 0 && i < I && j >= 0 && j < J) {
            const int o = i + j * sj + ko;
            g = -S::load(coeff + o) * gh[o];
        }
        sg[e] = g;
    }
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
    {
        const int lx = tid & 63, ly = tid >> 6;
        const int i = x0 + lx, j = y0 + ly;
        if (i < I + 2 && j < J + 2) {
            const int hc = (ly + 1) * HX + lx + 1;
            const bool inner = i >= 0 && i < I && j >= 0 && j < J;
            const int o = i + j * sj + ko;
            const C ghv = inner ? gh[o] : C(0);
            const C g = ghv - sh[hc - HX] - sh[hc - 1] + C(4) * sh[hc] - sh[hc + 1] - sh[hc + HX];
            S::store(gu + o, g);
            if (inner) {
                const int xi = (ly + 1) * XX + lx + 2, yi = (ly + 2) * YX + lx + 1;
                const C div = sfx[xi] - sfx[xi - 1] + sfy[yi] - sfy[yi - YX];
                S::store(gcoeff + o, -ghv * div);
            }
        }
    }
}

// ---------------------------------------------------------------------------

size_t adjoint_scratch_bytes(int dtype, int sk, int K) {
    const size_t cs = dtype == DT_F64 ? 8 : 4;
    return 2 * (static_cast<size_t>(sk) * K * cs + 256);
}

template <class T, int KMAX>
static void launch_vadv_adjoint_t(const AdjArgs &a, hipStream_t st) {
    const dim3 grid((a.I + 63) / 64, (a.J + 3) / 4);
    if (a.ga || a.gb || a.gc)
        hipLaunchKernelGGL((k_vadv_adjoint<T, KMAX, true>), grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_vadv_adjoint<T, KMAX, false>), grid, dim3(256), 0, st, a);
}

template <class T>
static hipError_t adjoint_run(AdjArgs a, void *scratch, hipStream_t st) {
    using C = typename Storage<T>::C;
    const size_t plane = (static_cast<size_t>(a.sk) * a.K * sizeof(C) + 255) / 256 * 256;
    a.h = scratch;
    a.gh = static_cast<char *>(scratch) + plane;
    HdiffArgs hd{};
    hd.u = a.u;
    hd.coeff = a.coeff;
    hd.out = a.h;
    hd.I = a.I; hd.J = a.J; hd.K = a.K; hd.sj = a.sj; hd.sk = a.sk;
    hipError_t e = launch_hdiff_compute(std::is_same<T, double>::value ? DT_F64
                                        : std::is_same<T, float>::value ? DT_F32 : DT_BF16,
                                        hd, st);
    if (e != hipSuccess) return e;
    if (a.K <= 32) launch_vadv_adjoint_t<T, 32>(a, st);
    else if (a.K <= 64) launch_vadv_adjoint_t<T, 64>(a, st);
    else launch_vadv_adjoint_t<T, 96>(a, st);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nbi = (a.I + 4 + 63) / 64, nbj = (a.J + 4 + 3) / 4;
    hipLaunchKernelGGL((k_hdiff_adjoint<T>), dim3(nbi * nbj, a.K), dim3(256), 0, st, a, nbi);
    return hipGetLastError();
}

hipError_t launch_adjoint(int dtype, const AdjointArgs &x, void *scratch, hipStream_t st) {
    AdjArgs a{};
    a.u = x.u; a.coeff = x.coeff; a.wcon = x.wcon; a.a = x.a; a.b = x.b; a.c = x.c; a.w = x.w;
    a.gu = x.gu; a.gcoeff = x.gcoeff; a.gwcon = x.gwcon;
    a.x = x.x; a.ga = x.ga; a.gb = x.gb; a.gc = x.gc;
    a.I = x.I; a.J = x.J; a.K = x.K; a.sj = x.sj; a.sk = x.sk;
    a.dt = x.dt;
    switch (dtype) {
    case DT_F64: return adjoint_run<double>(a, scratch, st);
    case DT_F32: return adjoint_run<float>(a, scratch, st);
    case DT_BF16: return adjoint_run<uint16_t>(a, scratch, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace stl
