// The "original" optimisation level (Sec. VII-C): no inlining.  Every stencil
// operator of the program is its own kernel, and every temporary it produces
// (Laplacian, the two limited fluxes, h, the right-hand side, the Thomas
// coefficients c' and d') is written to device memory and read back by its
// consumer.  This is the baseline that the fused kernels are compared with.
//
// Each array is addressed as p[i + sj j + sk k] from its interior origin.
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"

namespace stl {

template <class T>
struct Arr {
    T *p;
    int sj, sk;
    __device__ __forceinline__ T &operator()(int i, int j, int k) const {
        return p[i + j * sj + k * sk];
    }
};

// One thread per point of [i_lo, i_lo + ni) x [j_lo, j_lo + nj) at level blockIdx.z.
#define STL_POINT(i_lo, j_lo, ni, nj)                                 \
    const int i = (i_lo) + static_cast<int>(blockIdx.x * 64 + threadIdx.x); \
    const int j = (j_lo) + static_cast<int>(blockIdx.y * 4 + threadIdx.y);  \
    const int k = blockIdx.z;                                         \
    if (i >= (i_lo) + (ni) || j >= (j_lo) + (nj)) return;

// lap = 4u - u(i+1) - u(i-1) - u(j+1) - u(j-1) on [-1, I] x [-1, J].
template <class T, class C>
__global__ __launch_bounds__(256) void k_lap(Arr<const T> u, Arr<C> lap, int I, int J) {
    STL_POINT(-1, -1, I + 2, J + 2);
    using S = Storage<T>;
    const T *c = &u(i, j, k);
    lap(i, j, k) = C(4) * S::load(c) - S::load(c + 1) - S::load(c - 1) - S::load(c + u.sj) -
                   S::load(c - u.sj);
}

// flx(i) = lap(i+1) - lap(i), zeroed when flx (u(i+1) - u(i)) > 0, on
// [-1, I-1] x [0, J); dir = 1 gives fly on [0, I) x [-1, J-1] instead.
template <class T, class C, int DIR>
__global__ __launch_bounds__(256) void k_flux(Arr<const T> u, Arr<const C> lap, Arr<C> f, int I,
                                              int J) {
    STL_POINT(DIR == 0 ? -1 : 0, DIR == 0 ? 0 : -1, DIR == 0 ? I + 1 : I, DIR == 0 ? J : J + 1);
    using S = Storage<T>;
    const int di = DIR == 0 ? 1 : 0, dj = DIR == 0 ? 0 : 1;
    const C v = lap(i + di, j + dj, k) - lap(i, j, k);
    const C du = S::load(&u(i + di, j + dj, k)) - S::load(&u(i, j, k));
    f(i, j, k) = (v * du > C(0)) ? C(0) : v;
}

// h = u - coeff (flx - flx(i-1) + fly - fly(j-1)) on the interior.
template <class T, class C, class H>
__global__ __launch_bounds__(256) void k_update(Arr<const T> u, Arr<const T> coeff,
                                                Arr<const C> fx, Arr<const C> fy, Arr<H> h, int I,
                                                int J) {
    STL_POINT(0, 0, I, J);
    using S = Storage<T>;
    const C div = fx(i, j, k) - fx(i - 1, j, k) + fy(i, j, k) - fy(i, j - 1, k);
    const C v = S::load(&u(i, j, k)) - S::load(&coeff(i, j, k)) * div;
    if constexpr (std::is_same<H, C>::value)
        h(i, j, k) = v;
    else
        S::store(&h(i, j, k), v);
}

// d(k) = h(k) - dt (F(k+1/2) - F(k-1/2)), F(k+1/2) = (w(k)+w(k+1))/2 (h(k)+h(k+1))/2.
template <class T, class C, class H>
__global__ __launch_bounds__(256) void k_rhs(Arr<const H> h, Arr<const T> w, Arr<C> d, int I,
                                             int J, int K, C dt) {
    STL_POINT(0, 0, I, J);
    using S = Storage<T>;
    auto hv = [&](int kk) -> C {
        if constexpr (std::is_same<H, C>::value) return h(i, j, kk);
        else return Storage<H>::load(&h(i, j, kk));
    };
    const C hk = hv(k);
    C fu = C(0), fd = C(0);
    if (k + 1 < K)
        fu = (C(0.5) * (S::load(&w(i, j, k)) + S::load(&w(i, j, k + 1)))) * (C(0.5) * (hk + hv(k + 1)));
    if (k > 0)
        fd = (C(0.5) * (S::load(&w(i, j, k - 1)) + S::load(&w(i, j, k)))) * (C(0.5) * (hv(k - 1) + hk));
    d(i, j, k) = hk - dt * (fu - fd);
}

// Thomas forward elimination per column; c' and d' go to device memory.
template <class T, class C>
__global__ __launch_bounds__(256) void k_thomas_fwd(Arr<const T> a, Arr<const T> b, Arr<const T> c,
                                                    Arr<const C> d, Arr<double> cp,
                                                    Arr<double> dp, int I, int J, int K) {
    const int i = static_cast<int>(blockIdx.x * 64 + threadIdx.x);
    const int j = static_cast<int>(blockIdx.y * 4 + threadIdx.y);
    if (i >= I || j >= J) return;
    using S = Storage<T>;
    double cprev = 0.0, dprev = 0.0;
    for (int k = 0; k < K; ++k) {
        const double av = k > 0 ? static_cast<double>(S::load(&a(i, j, k))) : 0.0;
        const double bv = S::load(&b(i, j, k));
        const double cv = k + 1 < K ? static_cast<double>(S::load(&c(i, j, k))) : 0.0;
        const double m = bv - av * cprev;
        cprev = cv / m;
        dprev = (static_cast<double>(d(i, j, k)) - av * dprev) / m;
        cp(i, j, k) = cprev;
        dp(i, j, k) = dprev;
    }
}

// Back-substitution per column from the stored c', d'.
template <class T>
__global__ __launch_bounds__(256) void k_thomas_bwd(Arr<const double> cp, Arr<const double> dp,
                                                    Arr<T> x, int I, int J, int K) {
    const int i = static_cast<int>(blockIdx.x * 64 + threadIdx.x);
    const int j = static_cast<int>(blockIdx.y * 4 + threadIdx.y);
    if (i >= I || j >= J) return;
    double xn = 0.0;
    for (int k = K - 1; k >= 0; --k) {
        xn = (k == K - 1) ? dp(i, j, k) : dp(i, j, k) - cp(i, j, k) * xn;
        Storage<T>::store_d(&x(i, j, k), xn);
    }
}

// ---------------------------------------------------------------------------

static dim3 grid_for(int ni, int nj, int nk) {
    return dim3((ni + 63) / 64, (nj + 3) / 4, nk);
}

// Scratch layout: lap, fx, fy with a 1-cell halo; h and d dense; c', d' dense.
size_t plain_scratch_bytes(int dtype, int I, int J, int K, bool vadv) {
    const size_t cs = dtype == DT_F64 ? 8 : 4;
    const size_t n1 = static_cast<size_t>(I + 2) * (J + 2) * K, n0 = static_cast<size_t>(I) * J * K;
    size_t bytes = 3 * n1 * cs + 256 * 3;
    if (vadv) bytes += 2 * n0 * cs + 2 * n0 * 8 + 256 * 4;
    return bytes;
}

template <class T>
static hipError_t plain_run(const PlainArgs &a, hipStream_t st) {
    using C = typename Storage<T>::C;
    const int I = a.I, J = a.J, K = a.K;
    char *base = static_cast<char *>(a.scratch);
    auto take = [&](size_t bytes) {
        char *q = base;
        base += (bytes + 255) / 256 * 256;
        return q;
    };
    const int sj1 = I + 2, sk1 = (I + 2) * (J + 2);
    const size_t n1 = static_cast<size_t>(sk1) * K, n0 = static_cast<size_t>(I) * J * K;
    // Halo-1 arrays: the origin is one row and one column in.
    auto halo1 = [&](C *q) { return Arr<C>{q + 1 + sj1, sj1, sk1}; };
    Arr<C> lap = halo1(reinterpret_cast<C *>(take(n1 * sizeof(C))));
    Arr<C> fx = halo1(reinterpret_cast<C *>(take(n1 * sizeof(C))));
    Arr<C> fy = halo1(reinterpret_cast<C *>(take(n1 * sizeof(C))));
    Arr<const T> u{static_cast<const T *>(a.u), a.sj, a.sk};
    Arr<const T> coeff{static_cast<const T *>(a.coeff), a.sj, a.sk};
    const dim3 blk(64, 4);

    if (a.u) {
        hipLaunchKernelGGL((k_lap<T, C>), grid_for(I + 2, J + 2, K), blk, 0, st, u, lap, I, J);
        hipLaunchKernelGGL((k_flux<T, C, 0>), grid_for(I + 1, J, K), blk, 0, st, u,
                           Arr<const C>{lap.p, lap.sj, lap.sk}, fx, I, J);
        hipLaunchKernelGGL((k_flux<T, C, 1>), grid_for(I, J + 1, K), blk, 0, st, u,
                           Arr<const C>{lap.p, lap.sj, lap.sk}, fy, I, J);
    }
    if (!a.vadv) {
        // hdiff alone: the update writes the output field.
        hipLaunchKernelGGL((k_update<T, C, T>), grid_for(I, J, K), blk, 0, st, u, coeff,
                           Arr<const C>{fx.p, fx.sj, fx.sk}, Arr<const C>{fy.p, fy.sj, fy.sk},
                           Arr<T>{static_cast<T *>(a.x), a.sj, a.sk}, I, J);
        return hipGetLastError();
    }
    Arr<C> d{reinterpret_cast<C *>(take(n0 * sizeof(C))), I, I * J};
    Arr<double> cp{reinterpret_cast<double *>(take(n0 * 8)), I, I * J};
    Arr<double> dp{reinterpret_cast<double *>(take(n0 * 8)), I, I * J};
    Arr<const T> w{static_cast<const T *>(a.wcon), a.sj, a.sk};
    const C dt = static_cast<C>(a.dt);
    if (a.u) {
        Arr<C> h{reinterpret_cast<C *>(take(n0 * sizeof(C))), I, I * J};
        hipLaunchKernelGGL((k_update<T, C, C>), grid_for(I, J, K), blk, 0, st, u, coeff,
                           Arr<const C>{fx.p, fx.sj, fx.sk}, Arr<const C>{fy.p, fy.sj, fy.sk}, h,
                           I, J);
        hipLaunchKernelGGL((k_rhs<T, C, C>), grid_for(I, J, K), blk, 0, st,
                           Arr<const C>{h.p, h.sj, h.sk}, w, d, I, J, K, dt);
    } else {
        // vadv alone: h is the input field.
        hipLaunchKernelGGL((k_rhs<T, C, T>), grid_for(I, J, K), blk, 0, st,
                           Arr<const T>{static_cast<const T *>(a.h), a.sj, a.sk}, w, d, I, J, K,
                           dt);
    }
    const dim3 gcol((I + 63) / 64, (J + 3) / 4, 1);
    hipLaunchKernelGGL((k_thomas_fwd<T, C>), gcol, blk, 0, st,
                       Arr<const T>{static_cast<const T *>(a.a), a.sj, a.sk},
                       Arr<const T>{static_cast<const T *>(a.b), a.sj, a.sk},
                       Arr<const T>{static_cast<const T *>(a.c), a.sj, a.sk},
                       Arr<const C>{d.p, d.sj, d.sk}, cp, dp, I, J, K);
    hipLaunchKernelGGL((k_thomas_bwd<T>), gcol, blk, 0, st,
                       Arr<const double>{cp.p, cp.sj, cp.sk}, Arr<const double>{dp.p, dp.sj, dp.sk},
                       Arr<T>{static_cast<T *>(a.x), a.sj, a.sk}, I, J, K);
    return hipGetLastError();
}

hipError_t launch_plain(int dtype, const PlainArgs &a, hipStream_t st) {
    switch (dtype) {
    case DT_F64: return plain_run<double>(a, st);
    case DT_F32: return plain_run<float>(a, st);
    case DT_BF16: return plain_run<uint16_t>(a, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace stl
