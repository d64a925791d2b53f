// Device-side building blocks shared by the stencil kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stl {

// ---------------------------------------------------------------------------
// Storage types.  A field is stored as double, float or bfloat16 (raw bits);
// the stencil arithmetic runs in the compute type C of the storage type and
// the Thomas solve always in double.
// ---------------------------------------------------------------------------
template <class T> struct Storage;

template <> struct Storage<double> {
    using C = double;
    static __device__ __forceinline__ double load(const double *p) { return *p; }
    static __device__ __forceinline__ void store(double *p, double v) { *p = v; }
    static __device__ __forceinline__ void store_d(double *p, double v) { *p = v; }
};

template <> struct Storage<float> {
    using C = float;
    static __device__ __forceinline__ float load(const float *p) { return *p; }
    static __device__ __forceinline__ void store(float *p, float v) { *p = v; }
    static __device__ __forceinline__ void store_d(float *p, double v) { *p = static_cast<float>(v); }
};

// bfloat16: the upper half of an IEEE float.  Loads are exact; stores round
// to nearest, ties to even (NaN stays NaN).
template <> struct Storage<uint16_t> {
    using C = float;
    static __device__ __forceinline__ float load(const uint16_t *p) {
        return __uint_as_float(static_cast<uint32_t>(*p) << 16);
    }
    static __device__ __forceinline__ uint16_t round_bits(uint32_t bits) {
        const uint32_t rne = (bits + 0x7fffu + ((bits >> 16) & 1u)) >> 16;
        const uint32_t nan = (bits >> 16) | 0x40u;
        return static_cast<uint16_t>((bits & 0x7fffffffu) > 0x7f800000u ? nan : rne);
    }
    static __device__ __forceinline__ uint16_t round(float v) { return round_bits(__float_as_uint(v)); }
    static __device__ __forceinline__ void store(uint16_t *p, float v) { *p = round(v); }
    // A double rounded once to bfloat16: first to float with round-to-odd
    // (truncate, then set the last bit if anything was cut off), which keeps
    // the second rounding to nearest-even correct because float carries more
    // than two extra bits.  Truncation steps the nearest float one unit
    // toward zero when it rounded away (its bit pattern minus one: also right
    // for an overflow to infinity); all selects, no branches.
    static __device__ __forceinline__ uint16_t round_d(double v) {
        const float f = static_cast<float>(v);
        uint32_t bits = __float_as_uint(f) - (fabs(static_cast<double>(f)) > fabs(v) ? 1u : 0u);
        bits |= static_cast<double>(__uint_as_float(bits)) != v ? 1u : 0u;
        return round_bits(bits);
    }
    static __device__ __forceinline__ void store_d(uint16_t *p, double v) { *p = round_d(v); }
};

// ---------------------------------------------------------------------------
// Whole-wave lane shifts (DPP wave_shl / wave_shr by one lane): lane_next
// gives lane l the value of lane l + 1, lane_prev that of lane l - 1; the
// lane at the end with no such neighbour (63, resp. 0) gets `edge`.  A lane
// disabled in EXEC supplies no value, so a shift is only meaningful while the
// whole wave is active: callers shift in uniform control flow, never inside an
// operand of ?: (which is evaluated conditionally, so the compiler may branch
// around it), and the empty asm keeps the compiler from sinking a shift into
// the branch of a conditional store that uses it.
// ---------------------------------------------------------------------------
constexpr int DPP_WAVE_SHL1 = 0x130, DPP_WAVE_SHR1 = 0x138;

template <int CTRL>
__device__ __forceinline__ uint32_t lane_move(uint32_t v, uint32_t edge) {
    int r = __builtin_amdgcn_update_dpp(static_cast<int>(edge), static_cast<int>(v), CTRL, 0xf, 0xf, false);
    asm volatile("" : "+v"(r));
    return static_cast<uint32_t>(r);
}
template <int CTRL>
__device__ __forceinline__ float lane_move(float v, float edge) {
    return __uint_as_float(lane_move<CTRL>(__float_as_uint(v), __float_as_uint(edge)));
}
template <int CTRL>
__device__ __forceinline__ double lane_move(double v, double edge) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v), e = __builtin_bit_cast(uint64_t, edge);
    const uint32_t lo = lane_move<CTRL>(static_cast<uint32_t>(b), static_cast<uint32_t>(e));
    const uint32_t hi = lane_move<CTRL>(static_cast<uint32_t>(b >> 32), static_cast<uint32_t>(e >> 32));
    return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}
template <class V> __device__ __forceinline__ V lane_next(V v, V edge) { return lane_move<DPP_WAVE_SHL1>(v, edge); }
template <class V> __device__ __forceinline__ V lane_prev(V v, V edge) { return lane_move<DPP_WAVE_SHR1>(v, edge); }

// Resident workgroups of a kernel with `block` threads on the current device
// (host side; 0 if the runtime cannot say).
int resident_workgroups(const void *kernel, int block);

// ---------------------------------------------------------------------------
// Workgroup -> tile map aware of the 8 XCDs of MI355X.  Consecutive
// workgroup ids are dispatched round-robin over the XCDs, each of which has a
// private L2; this bijection hands each XCD a contiguous range of tiles, so
// tiles that share halo rows are resident in the same L2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int full = nb >> 3, rem = nb & 7;
    const int x = b & 7, q = b >> 3;
    return x * full + min(x, rem) + q;
}

// ---------------------------------------------------------------------------
// The horizontal-diffusion operator for one point, from a staged tile of u.
// `t` points at the centre value; `pitch` is the tile's row length.  The
// Laplacian is recomputed at the centre and its four neighbours (inlining,
// redundant computation instead of stored temporaries), the four fluxes are
// limited with a select, and the update is returned.  The order of the
// floating-point operations follows the operator definitions.
// ---------------------------------------------------------------------------
// Fused multiply-add in the compute type.  The fused kernels evaluate with
// contraction off and write every fused operation out with fmadd, so that
// the rounding sequence is fixed by the source and every schedule and tile
// shape of a kernel gives bitwise the same result.
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <class C, int PITCH>
__device__ __forceinline__ C hdiff_point(const C *t, C cf) {
#pragma clang fp contract(off)
    const C uc = t[0], ue = t[1], uw = t[-1], un = t[PITCH], us = t[-PITCH];
    const C uee = t[2], uww = t[-2], unn = t[2 * PITCH], uss = t[-2 * PITCH];
    const C une = t[PITCH + 1], unw = t[PITCH - 1], use = t[-PITCH + 1], usw = t[-PITCH - 1];
    const C four = C(4);
    // 4 u is exact, so fmadd(4, u, -v) is the rounded 4 u - v.
    const C lc = fmadd(four, uc, -ue) - uw - un - us;
    const C le = fmadd(four, ue, -uee) - uc - une - use;
    const C lw = fmadd(four, uw, -uc) - uww - unw - usw;
    const C ln = fmadd(four, un, -une) - unw - unn - uc;
    const C ls = fmadd(four, us, -use) - usw - uc - uss;
    C fe = le - lc;
    C fw = lc - lw;
    C fn = ln - lc;
    C fs = lc - ls;
    fe = (fe * (ue - uc) > C(0)) ? C(0) : fe;
    fw = (fw * (uc - uw) > C(0)) ? C(0) : fw;
    fn = (fn * (un - uc) > C(0)) ? C(0) : fn;
    fs = (fs * (uc - us) > C(0)) ? C(0) : fs;
    return fmadd(-cf, fe - fw + fn - fs, uc);
}

// ---------------------------------------------------------------------------
// Kernel arguments.  All fields of one call share the strides (sj, sk); each
// pointer is the field's interior origin.
// ---------------------------------------------------------------------------
struct HdiffArgs {
    const void *u, *coeff;  // interior origins
    void *out;
    int I, J, K, sj, sk;
    int nbi, nbj;           // tiles in i and j
    int kc;                 // levels per workgroup (the k range is split into runs of kc)
    uint32_t u_bytes;       // addressable bytes from u's cell (-2, -2, 0)
    uint32_t col_bytes;     // addressable bytes from an interior origin
};

// Column kernels (fused hdiff + vadv, vadv alone); see column.hpp.
struct ColumnArgs {
    const void *u;  // fused: u at interior (-2, -2, 0); vadv alone: h at its origin
    const void *coeff, *wcon, *a, *b, *c;  // interior origins
    void *x;                               // interior origin
    uint32_t u_bytes;                      // addressable bytes from u
    uint32_t col_bytes;                    // addressable bytes from an interior origin
    int I, J, K, sj, sk;
    int nbi, nbj;
    double dt;
    // First column of the first tile (0, or negative so that tiles start on
    // 128-byte lines); columns outside [0, I) are read clamped, never stored.
    int i_lo;
};

}  // namespace stl
