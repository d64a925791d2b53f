// Halo exchange between the shares of a horizontally decomposed grid, and its
// transpose (the reverse halo add of a gradient), on one device.
//
// A grid split into px x py rectangles in (i, j) is the decomposition a
// distributed run would give each GPU one of: vadv and its Thomas solve are
// column-local, so only horizontal diffusion needs data from the neighbours,
// its u halo (Sec. V-B's shape inference gives the width), once per
// application.  Here every share is a separate halo-padded field on the same
// device.
//
// Exchange: for each share s and each of its eight neighbour directions
// (dx, dy) whose neighbour n exists, the halo block of s in that direction
//   i in [-w, 0) / [lo, hi) / [ni, ni + w)   for dx = -1 / 0 / +1  (j alike)
// receives the cells of n at the same grid position.  [lo, hi) is [0, ni)
// grown by w on each side where s lies on the outer boundary of the
// decomposition: there n's own halo holds the whole grid's halo data, which
// s needs in its corner (the 13-point diamond reaches diagonal cells).
// Diagonal corner blocks come straight from the diagonal neighbour, so one
// pass (one launch) fills every halo cell toward a neighbour; halo cells on
// the outer boundary are left alone (they hold the grid's halo data).
//
// Accumulate (the transpose of the exchange): every cell that the exchange
// copies into some neighbour's halo -- interior cells near an inner edge,
// and outer-boundary halo cells next to one -- receives the sum of those
// copies.  It is formulated as a gather on the receiving share, over the
// directions in a fixed order: the cells gathered into (interior and outer
// halo) and the cells read (halo blocks toward neighbours) are disjoint, no
// two threads write one cell, and the result does not depend on scheduling.
// Halo blocks toward neighbours are read, not cleared.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "launch.hpp"

namespace stl {

namespace {

// Neighbour directions in a fixed order.
__constant__ const int kDx[8] = {-1, 1, 0, 0, -1, 1, -1, 1};
__constant__ const int kDy[8] = {0, 0, -1, 1, -1, -1, 1, 1};

struct Block {
    int i0, ni, j0, nj;
};

// Range of share coordinates along one axis that a block with no offset
// along it spans: the interior, grown by w where the share is on the outer
// boundary (lo side: pos == 0, hi side: pos == count - 1).
__device__ __forceinline__ void span(int n, int w, int pos, int count, int *lo, int *hi) {
    *lo = pos == 0 ? -w : 0;
    *hi = pos == count - 1 ? n + w : n;
}

// Halo block of share (p, q) toward direction d, in that share's interior
// coordinates.
__device__ __forceinline__ Block halo_block(const HaloArgs &a, int p, int q, int d) {
    const int ni = a.ni[p], nj = a.nj[q], w = a.w;
    const int dx = kDx[d], dy = kDy[d];
    int ilo, ihi, jlo, jhi;
    span(ni, w, p, a.px, &ilo, &ihi);
    span(nj, w, q, a.py, &jlo, &jhi);
    Block b;
    b.i0 = dx < 0 ? -w : dx > 0 ? ni : ilo;
    b.ni = dx ? w : ihi - ilo;
    b.j0 = dy < 0 ? -w : dy > 0 ? nj : jlo;
    b.nj = dy ? w : jhi - jlo;
    return b;
}

// Offset from a halo cell of share (p, q) in direction d to the same global
// cell in the neighbour's interior coordinates.
__device__ __forceinline__ int shift_i(const HaloArgs &a, int p, int dx) {
    return dx < 0 ? a.ni[p - 1] : dx > 0 ? -a.ni[p] : 0;
}
__device__ __forceinline__ int shift_j(const HaloArgs &a, int q, int dy) {
    return dy < 0 ? a.nj[q - 1] : dy > 0 ? -a.nj[q] : 0;
}

__device__ __forceinline__ long long cell(const HaloShare &s, int i, int j, int k) {
    return static_cast<long long>(i) + static_cast<long long>(j) * s.sj + static_cast<long long>(k) * s.sk;
}

// blockIdx.y = share * 8 + direction; blockIdx.x strides over the block's cells
// (i fastest, then j, then k).
template <class T>
__global__ __launch_bounds__(256) void k_halo_exchange(HaloArgs a) {
    const int sid = blockIdx.y >> 3, d = blockIdx.y & 7;
    const int p = sid % a.px, q = sid / a.px;
    const int pn = p + kDx[d], qn = q + kDy[d];
    if (pn < 0 || pn >= a.px || qn < 0 || qn >= a.py) return;  // outer boundary: untouched
    const Block b = halo_block(a, p, q, d);
    const HaloShare &dst = a.s[sid];
    const HaloShare &src = a.s[pn + a.px * qn];
    const int si = shift_i(a, p, kDx[d]), sjs = shift_j(a, q, kDy[d]);
    const long long plane = static_cast<long long>(b.ni) * b.nj, total = plane * a.K;
    T *out = static_cast<T *>(dst.origin);
    const T *in = static_cast<const T *>(src.origin);
    for (long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; c < total;
         c += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int k = static_cast<int>(c / plane);
        const int r = static_cast<int>(c - k * plane);
        const int j = b.j0 + r / b.ni, i = b.i0 + r % b.ni;
        out[cell(dst, i, j, k)] = in[cell(src, i + si, j + sjs, k)];
    }
}

// Bands of a receiving share along one axis: its range [lo, hi) (interior,
// grown on outer sides) split into [lo, w), [w, n - w), [n - w, hi); with
// n < 2 w the classes are clipped so that every cell falls in one class.
__device__ __forceinline__ void band(int cls, int n, int w, int pos, int count, int *start, int *len) {
    int lo, hi;
    span(n, w, pos, count, &lo, &hi);
    const int a = min(w, n), b = max(n - w, a);
    if (cls == 0) { *start = lo; *len = a - lo; }
    else if (cls == 1) { *start = a; *len = b - a; }
    else { *start = b; *len = hi - b; }
}

// blockIdx.y = share * 8 + region (the eight non-centre regions of the 3 x 3
// partition; the centre, [w, ni - w) x [w, nj - w), is read by no neighbour).
// Each cell of a region adds, in direction order, the halo cells of the
// neighbours whose exchange would have read it.
template <class T>
__global__ __launch_bounds__(256) void k_halo_accumulate(HaloArgs a) {
    using S = Storage<T>;
    using C = typename S::C;
    const int sid = blockIdx.y >> 3, reg = blockIdx.y & 7;
    const int p = sid % a.px, q = sid / a.px;
    const int rr = reg < 4 ? reg : reg + 1;  // skip the centre (class 1, 1)
    const int ci = rr % 3, cj = rr / 3;
    const int ni = a.ni[p], nj = a.nj[q], w = a.w;
    int i0, li, j0, lj;
    band(ci, ni, w, p, a.px, &i0, &li);
    band(cj, nj, w, q, a.py, &j0, &lj);
    const long long plane = static_cast<long long>(li) * lj, total = plane * a.K;
    const HaloShare &me = a.s[sid];
    T *g = static_cast<T *>(me.origin);
    for (long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; c < total;
         c += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int k = static_cast<int>(c / plane);
        const int r = static_cast<int>(c - k * plane);
        const int j = j0 + r / li, i = i0 + r % li;
        C acc = S::load(g + cell(me, i, j, k));
        for (int d = 0; d < 8; ++d) {
            // The sender sits at (p - dx, q - dy); its halo block toward us
            // covers i in [0, w) (dx = +1), [ni - w, ni) (dx = -1), or for
            // dx = 0 this share's whole i range (same column, same span).
            const int dx = kDx[d], dy = kDy[d];
            const int ps = p - dx, qs = q - dy;
            if (ps < 0 || ps >= a.px || qs < 0 || qs >= a.py) continue;
            if ((dx > 0 && (i < 0 || i >= w)) || (dx < 0 && (i < ni - w || i >= ni))) continue;
            if ((dy > 0 && (j < 0 || j >= w)) || (dy < 0 && (j < nj - w || j >= nj))) continue;
            const HaloShare &s = a.s[ps + a.px * qs];
            const int is = i - shift_i(a, ps, dx), js = j - shift_j(a, qs, dy);
            acc = acc + S::load(static_cast<const T *>(s.origin) + cell(s, is, js, k));
        }
        S::store(g + cell(me, i, j, k), acc);
    }
}

template <class T>
hipError_t launch_halo_t(const HaloArgs &a, bool accumulate, hipStream_t st) {
    // Cells of the largest block (a halo strip or a border band); the grid's
    // x dimension covers it, capped so that small strips do not launch
    // thousands of empty workgroups (the loops stride over the rest).
    int maxi = 0, maxj = 0;
    for (int p = 0; p < a.px; ++p) maxi = max(maxi, a.ni[p]);
    for (int q = 0; q < a.py; ++q) maxj = max(maxj, a.nj[q]);
    const long long biggest = static_cast<long long>(max(maxi, maxj) + 2 * a.w) * 2 * a.w * a.K;
    const unsigned gx = static_cast<unsigned>(min(256LL, max(1LL, (biggest + 255) / 256)));
    const dim3 grid(gx, 8u * a.px * a.py);
    if (accumulate)
        hipLaunchKernelGGL(k_halo_accumulate<T>, grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(k_halo_exchange<T>, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_halo(int dtype, const HaloArgs &a, bool accumulate, hipStream_t st) {
    switch (dtype) {
    case DT_F64: return launch_halo_t<double>(a, accumulate, st);
    case DT_F32: return launch_halo_t<float>(a, accumulate, st);
    case DT_BF16: return launch_halo_t<uint16_t>(a, accumulate, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace stl
