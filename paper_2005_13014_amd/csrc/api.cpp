// C ABI of the stencil library: host-side validation and dispatch.
//
// Every entry point validates its descriptors on the host before anything is
// enqueued (the checks a stencil program's asserted ranges and shape inference
// imply: alias-free parameters, Sec. IV-C and IV-D; shape inference,
// Sec. V-B), then launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/stencil.h"
#include "launch.hpp"
#include "program.hpp"

#define STENCIL_API extern "C" __attribute__((visibility("default")))

namespace stl {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(STENCIL_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define TRY(x)                            \
    do {                                  \
        int rc_ = (x);                    \
        if (rc_ != STENCIL_OK) return rc_; \
    } while (0)

// ---------------------------------------------------------------------------
// Library-owned device scratch, one buffer per (device, stream) so that calls
// on different streams never share temporaries.  A lease keeps the lock until
// the kernels that use the buffer are enqueued: a call on another thread that
// grows the same buffer (synchronise, free, allocate) then waits, and its
// synchronisation also covers the kernels enqueued under the lease.
// ---------------------------------------------------------------------------
namespace {
struct Scratch {
    void *p = nullptr;
    size_t bytes = 0;
};
std::mutex g_scratch_mu;
std::map<std::pair<int, hipStream_t>, Scratch> g_scratch;
}  // namespace

struct ScratchLease {
    std::unique_lock<std::mutex> lock;
    void *p = nullptr;
};

// True when `st` is being captured into a graph (then nothing may allocate,
// free or synchronise on it).
int stream_capturing(hipStream_t st, bool *capturing) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    const hipError_t e = hipStreamIsCapturing(st, &cs);
    if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
    *capturing = cs != hipStreamCaptureStatusNone;
    return STENCIL_OK;
}

int scratch_get(hipStream_t st, size_t bytes, ScratchLease *lease) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::unique_lock<std::mutex> lock(g_scratch_mu);
    Scratch &s = g_scratch[{dev, st}];
    if (s.bytes < bytes) {
        bool capturing = false;
        TRY(stream_capturing(st, &capturing));
        if (capturing)
            return fail(STENCIL_E_UNSUPPORTED,
                        "the call needs %zu bytes of library scratch on this stream, which holds %zu; growing it "
                        "would synchronise and allocate inside a stream capture (make the same call once before "
                        "capturing, or use the entry point that allocates nothing)",
                        bytes, s.bytes);
        if (s.p) {
            // Kernels enqueued earlier on this stream may still use the old buffer.
            e = hipStreamSynchronize(st);
            if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
            hipFree(s.p);
            s.p = nullptr;
            s.bytes = 0;
        }
        e = hipMalloc(&s.p, bytes);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(scratch)");
        s.bytes = bytes;
    }
    lease->p = s.p;
    lease->lock = std::move(lock);
    return STENCIL_OK;
}

long long scratch_held_bytes() {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    long long n = 0;
    for (auto &kv : g_scratch) n += static_cast<long long>(kv.second.bytes);
    return n;
}

void scratch_release_all() {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch.empty()) hipDeviceSynchronize();
    for (auto &kv : g_scratch)
        if (kv.second.p) hipFree(kv.second.p);
    g_scratch.clear();
}

// ---------------------------------------------------------------------------
// Descriptor validation
// ---------------------------------------------------------------------------
size_t elem_size(int dtype) {
    return dtype == STENCIL_F64 ? 8 : dtype == STENCIL_F32 ? 4 : 2;
}

bool empty(const stencil_field_t *f) { return f->ni == 0 || f->nj == 0 || f->nk == 0; }

// Element offsets (relative to origin) of the first and last addressable cell.
static void extent(const stencil_field_t *f, long long *lo, long long *hi) {
    *lo = -static_cast<long long>(f->hi) - static_cast<long long>(f->hj) * f->sj;
    *hi = static_cast<long long>(f->ni + f->hi - 1) + static_cast<long long>(f->nj + f->hj - 1) * f->sj +
          static_cast<long long>(f->nk - 1) * f->sk;
}

int check_field(const stencil_field_t *f, const char *name) {
    if (!f) return fail(STENCIL_E_NULL, "%s: descriptor is NULL", name);
    if (f->dtype != STENCIL_F64 && f->dtype != STENCIL_F32 && f->dtype != STENCIL_BF16)
        return fail(STENCIL_E_DTYPE, "%s: unknown dtype %d", name, f->dtype);
    if (f->ni < 0 || f->nj < 0 || f->nk < 0)
        return fail(STENCIL_E_SHAPE, "%s: negative extent (%d, %d, %d)", name, f->ni, f->nj, f->nk);
    if (f->hi < 0 || f->hj < 0) return fail(STENCIL_E_HALO, "%s: negative halo", name);
    if (empty(f)) return STENCIL_OK;
    if (!f->origin) return fail(STENCIL_E_NULL, "%s: origin is NULL", name);
    if (f->sj < static_cast<long long>(f->ni) + 2 * f->hi)
        return fail(STENCIL_E_STRIDE, "%s: sj=%lld < ni + 2 hi = %d", name, (long long)f->sj,
                    f->ni + 2 * f->hi);
    if (f->nk > 1 && f->sk < f->sj * (static_cast<long long>(f->nj) + 2 * f->hj))
        return fail(STENCIL_E_STRIDE, "%s: sk=%lld < sj (nj + 2 hj)", name, (long long)f->sk);
    long long lo, hi;
    extent(f, &lo, &hi);
    if (lo < -2147483647LL || hi > 2147483647LL)
        return fail(STENCIL_E_UNSUPPORTED, "%s: element offsets exceed 32 bits", name);
    return STENCIL_OK;
}

// All fields share dtype, interior extents and strides.
int check_same(const stencil_field_t *const *fs, const char *const *names, int n) {
    const stencil_field_t *r = fs[0];
    for (int q = 1; q < n; ++q) {
        const stencil_field_t *f = fs[q];
        if (f->dtype != r->dtype)
            return fail(STENCIL_E_DTYPE, "%s has dtype %d but %s has %d", names[q], f->dtype,
                        names[0], r->dtype);
        if (f->ni != r->ni || f->nj != r->nj || f->nk != r->nk)
            return fail(STENCIL_E_SHAPE, "%s extents (%d,%d,%d) differ from %s (%d,%d,%d)", names[q],
                        f->ni, f->nj, f->nk, names[0], r->ni, r->nj, r->nk);
        if (!empty(f) && (f->sj != r->sj || (f->nk > 1 && f->sk != r->sk)))
            return fail(STENCIL_E_STRIDE, "%s strides differ from %s", names[q], names[0]);
    }
    return STENCIL_OK;
}

int check_halo(const stencil_field_t *f, const char *name, int need) {
    if (f->hi < need || f->hj < need)
        return fail(STENCIL_E_HALO, "%s: halo (%d, %d) narrower than the access extent %d", name,
                    f->hi, f->hj, need);
    return STENCIL_OK;
}

// Byte ranges of outputs must not overlap any other field of the call.
int check_alias(const stencil_field_t *const *fs, const char *const *names, int n, int nout) {
    struct R {
        uintptr_t lo, hi;
    };
    std::vector<R> r(n);
    for (int q = 0; q < n; ++q) {
        long long lo, hi;
        extent(fs[q], &lo, &hi);
        const size_t es = elem_size(fs[q]->dtype);
        const uintptr_t base = reinterpret_cast<uintptr_t>(fs[q]->origin);
        r[q] = {base + static_cast<intptr_t>(lo * static_cast<long long>(es)),
                base + static_cast<intptr_t>((hi + 1) * static_cast<long long>(es))};
    }
    for (int o = n - nout; o < n; ++o)
        for (int q = 0; q < n; ++q) {
            if (q == o) continue;
            if (r[o].lo < r[q].hi && r[q].lo < r[o].hi)
                return fail(STENCIL_E_ALIAS, "output %s overlaps %s", names[o], names[q]);
        }
    return STENCIL_OK;
}

int check_call(const stencil_field_t *const *fs, const char *const *names, int n, int nout) {
    for (int q = 0; q < n; ++q) TRY(check_field(fs[q], names[q]));
    TRY(check_same(fs, names, n));
    bool any_empty = false;
    for (int q = 0; q < n; ++q) any_empty |= empty(fs[q]);
    if (!any_empty) TRY(check_alias(fs, names, n, nout));
    return STENCIL_OK;
}

static stencil_config_t config_or_default(const stencil_config_t *cfg) {
    stencil_config_t c{};
    if (cfg) c = *cfg;
    return c;
}

static int launch_status(hipError_t e, const char *what) {
    if (e != hipSuccess) return hip_fail(e, what);
    return STENCIL_OK;
}

// Plain-path launch limits (grid y and z).
static int check_plain_dims(int I, int J, int K) {
    if (K > 65535 || (J + 5) / 4 > 65535 || (I + 2) / 64 + 1 > 2147483647)
        return fail(STENCIL_E_UNSUPPORTED, "extents too large for the unfused kernels");
    (void)I;
    return STENCIL_OK;
}

static int run_plain(int dtype, PlainArgs a, hipStream_t st) {
    TRY(check_plain_dims(a.I, a.J, a.K));
    ScratchLease lease;
    TRY(scratch_get(st, plain_scratch_bytes(dtype, a.I, a.J, a.K, a.vadv), &lease));
    a.scratch = lease.p;
    return launch_status(launch_plain(dtype, a, st), "unfused kernels");
}

static hipError_t launch_column(int dtype, bool fused, const ColumnArgs &a, const ColumnVariant &v,
                                hipStream_t st) {
    switch (dtype) {
    case STENCIL_F64: return launch_column_f64(fused, a, v, st);
    case STENCIL_F32: return launch_column_f32(fused, a, v, st);
    default: return launch_column_bf16(fused, a, v, st);
    }
}

static bool column_variant(int dtype, const ColumnVariant &v) {
    switch (dtype) {
    case STENCIL_F64: return column_variant_f64(v);
    case STENCIL_F32: return column_variant_f32(v);
    default: return column_variant_bf16(v);
    }
}

// Resolves the fused variant from the knobs; zero knobs take the fastest
// variant measured at 512 x 512 x 80 (FP32: four rows of 64 columns per half,
// four levels prefetched, non-temporal streams, pipelined schedule).  A
// non-zero knob that names no compiled variant is an error, not a silent
// substitution.
// Grids with fewer columns than this fill fewer than two waves per SIMD at two
// lanes per column; the library then takes four lanes per column.
constexpr long long SMALL_GRID_COLUMNS = 65536;

static int fused_variant(int dtype, const stencil_config_t &cf, const stencil_field_t *u,
                         ColumnVariant *out) {
    ColumnVariant v{};
    if (cf.nontemporal < -1 || cf.nontemporal > 1)
        return fail(STENCIL_E_ARG, "nontemporal must be -1, 0 or 1 (got %d)", cf.nontemporal);
    if (cf.schedule < 0 || cf.schedule > SCHED_FOUR)
        return fail(STENCIL_E_ARG, "schedule must be 0 .. 4 (got %d)", cf.schedule);
    // Four lanes per column: asked for, or the library's choice on a small grid
    // when no other knob is set.  It needs nk >= 8.
    if (cf.tile_i != 0 && cf.tile_i != 64 && cf.tile_i != 128 && cf.tile_i != 256)
        return fail(STENCIL_E_ARG, "tile_i must be 0, 64, 128 or 256 (got %d)", cf.tile_i);
    const bool knobs = cf.tile_j || cf.prefetch || cf.nontemporal || cf.tile_i;
    const bool small = static_cast<long long>(u->ni) * u->nj < SMALL_GRID_COLUMNS;
    if (cf.schedule == SCHED_FOUR || (cf.schedule == 0 && !knobs && small && u->nk >= 8)) {
        v.tile_j = cf.tile_j ? cf.tile_j : 1;
        v.prefetch = cf.prefetch ? cf.prefetch : dtype == STENCIL_F64 ? 2 : 4;
        v.nt = cf.nontemporal >= 0;
        v.sched = SCHED_FOUR;
        if (column_variant(dtype, v) && (u->nk >= 8 || empty(u))) {
            *out = v;
            return STENCIL_OK;
        }
        if (cf.schedule == SCHED_FOUR)
            return fail(STENCIL_E_UNSUPPORTED,
                        "four lanes per column need FP32 or FP64 storage, nk >= 8, tile_j 1, prefetch 4 "
                        "(FP64: 2) and non-temporal streams");
    }
    // FP32 and FP64: 64 x 4 tiles (one 512-lane workgroup per CU, two u rows
    // loaded per lane and level) measured fastest (FP64 at 512 x 512 x 80:
    // 0.179 ms against 0.205 with 64 x 2); bf16: 64 x 2.  An unset tile height
    // takes the preferred one where the other knobs name a compiled variant,
    // else 2.
    const int tjs[2] = {cf.tile_j ? cf.tile_j : dtype == STENCIL_BF16 ? 2 : 4, 2};
    const int ntj = cf.tile_j || tjs[0] == 2 ? 1 : 2;
    v.prefetch = cf.prefetch ? cf.prefetch : dtype == STENCIL_F64 ? 2 : 4;
    v.tile_i = cf.tile_i ? cf.tile_i : 64;
    const bool nts[2] = {true, false};
    const int order[3] = {SCHED_PIPELINED, SCHED_PERSISTENT, SCHED_STAGED};  // library preference
    bool found = false;
    for (int t = 0; t < ntj && !found; ++t) {
        v.tile_j = tjs[t];
        for (int q = 0; q < 2 && !found; ++q) {
            v.nt = nts[q];
            if ((cf.nontemporal > 0 && !v.nt) || (cf.nontemporal < 0 && v.nt)) continue;
            for (int r = 0; r < 3 && !found; ++r) {
                v.sched = cf.schedule ? cf.schedule : order[r];
                found = column_variant(dtype, v);
            }
        }
    }
    if (cf.level != STENCIL_LEVEL_ORIGINAL && !found)
        return fail(STENCIL_E_UNSUPPORTED,
                    "no compiled fused variant tile_i=%d tile_j=%d prefetch=%d nontemporal=%d schedule=%d",
                    v.tile_i, v.tile_j, v.prefetch, cf.nontemporal, cf.schedule);
    *out = v;
    return STENCIL_OK;
}

// Resident workgroups of `kernel` with `block` threads on the current
// device: occupancy per CU (cached per kernel) times the CU count (cached per
// device).  0 if the runtime cannot say.
int resident_workgroups(const void *kernel, int block) {
    static std::mutex mu;
    static std::unordered_map<const void *, int> per_cu;
    static int cus[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    std::lock_guard<std::mutex> lock(mu);
    if (!cus[dev] && hipDeviceGetAttribute(&cus[dev], hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus[dev] = 0;
    auto it = per_cu.find(kernel);
    if (it == per_cu.end()) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, block, 0) != hipSuccess) nb = 0;
        it = per_cu.emplace(kernel, nb).first;
    }
    return it->second * cus[dev];
}

// Column kernels address every field through a raw buffer of < 2^31 bytes.
static bool column_fits(const stencil_field_t *f) {
    const long long cells = static_cast<long long>(f->ni + 3) + static_cast<long long>(f->nj + 3) * f->sj +
                            static_cast<long long>(f->nk - 1) * f->sk + 1;
    return cells * static_cast<long long>(elem_size(f->dtype)) < 2147483647LL;
}

static ColumnArgs column_args(const stencil_field_t *u, const stencil_field_t *coeff,
                              const stencil_field_t *wcon, const stencil_field_t *a,
                              const stencil_field_t *b, const stencil_field_t *c,
                              const stencil_field_t *x, double dt, bool fused) {
    const long long es = static_cast<long long>(elem_size(u->dtype));
    ColumnArgs v{};
    // Fused: u is addressed from its cell (-2, -2, 0), the corner of the ring hdiff reads.
    v.u = fused ? static_cast<const char *>(u->origin) - (2 + 2 * u->sj) * es : u->origin;
    v.coeff = coeff ? coeff->origin : nullptr;
    v.wcon = wcon->origin; v.a = a->origin; v.b = b->origin; v.c = c->origin;
    v.x = x->origin;
    v.u_bytes = static_cast<uint32_t>(((u->ni + 3) + (u->nj + 3) * u->sj + (u->nk - 1) * u->sk + 1) * es);
    v.col_bytes = static_cast<uint32_t>(((u->ni - 1) + (u->nj - 1) * u->sj + (u->nk - 1) * u->sk + 1) * es);
    v.I = u->ni; v.J = u->nj; v.K = u->nk;
    v.sj = static_cast<int>(u->sj); v.sk = static_cast<int>(u->sk);
    v.dt = dt;
    return v;
}


}  // namespace stl

using namespace stl;

// ---------------------------------------------------------------------------
// Entry points
// ---------------------------------------------------------------------------
STENCIL_API int stencil_abi_version(void) { return STENCIL_ABI_VERSION; }

STENCIL_API const char *stencil_last_error(void) { return g_last_error.c_str(); }

STENCIL_API void stencil_shutdown(void) {
    program_release_all();
    scratch_release_all();
}

STENCIL_API int64_t stencil_held_memory(int32_t *programs) {
    int n = 0;
    const long long bytes = program_held_bytes(&n) + scratch_held_bytes();
    if (programs) *programs = n;
    return bytes;
}

STENCIL_API int stencil_hdiff(const stencil_field_t *u, const stencil_field_t *coeff,
                              const stencil_field_t *out, const stencil_config_t *cfg,
                              void *stream) {
    const stencil_field_t *fs[] = {u, coeff, out};
    const char *names[] = {"u", "coeff", "out"};
    TRY(check_call(fs, names, 3, 1));
    TRY(check_halo(u, "u", 2));
    const stencil_config_t c = config_or_default(cfg);
    if (c.level < 0 || c.level > STENCIL_LEVEL_INLINE)
        return fail(STENCIL_E_ARG, "unknown level %d", c.level);
    const int unroll = c.unroll ? c.unroll : 1;
    if (unroll != 1 && unroll != 2 && unroll != 4)
        return fail(STENCIL_E_ARG, "unroll must be 1, 2 or 4 (got %d)", c.unroll);
    if (empty(u)) return STENCIL_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // The inlined kernel addresses u, coeff and out through raw buffers of
    // < 2^31 bytes; larger fields take the unfused kernels (element offsets,
    // checked above, stay 32-bit there), unless the inlined level is asked for.
    const bool fits = column_fits(u);
    if (!fits && c.level == STENCIL_LEVEL_INLINE)
        return fail(STENCIL_E_UNSUPPORTED, "the inlined hdiff kernel supports fields below 2 GiB");
    if (c.level == STENCIL_LEVEL_ORIGINAL || !fits) {
        PlainArgs a{};
        a.u = u->origin;
        a.coeff = coeff->origin;
        a.x = out->origin;
        a.I = u->ni; a.J = u->nj; a.K = u->nk;
        a.sj = static_cast<int>(u->sj); a.sk = static_cast<int>(u->sk);
        a.vadv = false;
        return run_plain(u->dtype, a, st);
    }
    HdiffArgs a{};
    a.u = u->origin;
    a.coeff = coeff->origin;
    a.out = out->origin;
    a.I = u->ni; a.J = u->nj; a.K = u->nk;
    a.sj = static_cast<int>(u->sj); a.sk = static_cast<int>(u->sk);
    return launch_status(launch_hdiff(u->dtype, a, unroll, st), "hdiff kernel");
}

static int check_dt(double dt) {
    if (!std::isfinite(dt)) return fail(STENCIL_E_ARG, "dt must be finite");
    return STENCIL_OK;
}

STENCIL_API int stencil_vadv(const stencil_field_t *h, const stencil_field_t *wcon,
                             const stencil_field_t *a, const stencil_field_t *b,
                             const stencil_field_t *c, double dt, const stencil_field_t *x,
                             const stencil_config_t *cfg, void *stream) {
    const stencil_field_t *fs[] = {h, wcon, a, b, c, x};
    const char *names[] = {"h", "wcon", "a", "b", "c", "x"};
    TRY(check_call(fs, names, 6, 1));
    TRY(check_dt(dt));
    const stencil_config_t cf = config_or_default(cfg);
    if (cf.level < 0 || cf.level > STENCIL_LEVEL_INLINE)
        return fail(STENCIL_E_ARG, "unknown level %d", cf.level);
    if (empty(h)) return STENCIL_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int dtype = h->dtype;
    if (cf.level == STENCIL_LEVEL_ORIGINAL || h->nk > KMAX_COLUMN || !column_fits(h)) {
        PlainArgs p{};
        p.h = h->origin; p.wcon = wcon->origin; p.a = a->origin; p.b = b->origin; p.c = c->origin;
        p.x = x->origin;
        p.I = h->ni; p.J = h->nj; p.K = h->nk;
        p.sj = static_cast<int>(h->sj); p.sk = static_cast<int>(h->sk);
        p.dt = dt;
        p.vadv = true;
        return run_plain(dtype, p, st);
    }
    const ColumnArgs v = column_args(h, nullptr, wcon, a, b, c, x, dt, false);
    return launch_status(launch_column(dtype, false, v, ColumnVariant{}, st), "vadv kernel");
}

STENCIL_API int stencil_hdiff_vadv(const stencil_field_t *u, const stencil_field_t *coeff,
                                   const stencil_field_t *wcon, const stencil_field_t *a,
                                   const stencil_field_t *b, const stencil_field_t *c, double dt,
                                   const stencil_field_t *x, const stencil_config_t *cfg,
                                   void *stream) {
    const stencil_field_t *fs[] = {u, coeff, wcon, a, b, c, x};
    const char *names[] = {"u", "coeff", "wcon", "a", "b", "c", "x"};
    TRY(check_call(fs, names, 7, 1));
    TRY(check_halo(u, "u", 2));
    TRY(check_dt(dt));
    const stencil_config_t cf = config_or_default(cfg);
    if (cf.level < 0 || cf.level > STENCIL_LEVEL_INLINE)
        return fail(STENCIL_E_ARG, "unknown level %d", cf.level);
    const int dtype = u->dtype;
    ColumnVariant var{};
    TRY(fused_variant(dtype, cf, u, &var));
    if (empty(u)) return STENCIL_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (cf.level == STENCIL_LEVEL_ORIGINAL || u->nk > KMAX_COLUMN || !column_fits(u)) {
        if (cf.level == STENCIL_LEVEL_INLINE)
            return fail(STENCIL_E_UNSUPPORTED,
                        "fused kernel supports nk <= %d and fields below 2 GiB", KMAX_COLUMN);
        PlainArgs p{};
        p.u = u->origin; p.coeff = coeff->origin;
        p.wcon = wcon->origin; p.a = a->origin; p.b = b->origin; p.c = c->origin;
        p.x = x->origin;
        p.I = u->ni; p.J = u->nj; p.K = u->nk;
        p.sj = static_cast<int>(u->sj); p.sk = static_cast<int>(u->sk);
        p.dt = dt;
        p.vadv = true;
        return run_plain(dtype, p, st);
    }
    const ColumnArgs v = column_args(u, coeff, wcon, a, b, c, x, dt, true);
    return launch_status(launch_column(dtype, true, v, var, st), "fused hdiff+vadv kernel");
}

namespace stl {

// The reverse pass behind stencil_hdiff_vadv_adjoint and its variant that
// allocates nothing: without `fixed` it takes the (device, stream) scratch
// buffer (which may grow); with it, the fixed device array of
// ADJOINT_FIXED_SCRATCH_BYTES, and a call that needs more is refused before
// anything touches the device.
int adjoint_entry(const stencil_field_t *u, const stencil_field_t *coeff, const stencil_field_t *wcon,
                  const stencil_field_t *a, const stencil_field_t *b, const stencil_field_t *c, double dt,
                  const stencil_field_t *w, const stencil_field_t *gu, const stencil_field_t *gcoeff,
                  const stencil_field_t *gwcon, const stencil_field_t *xf, const stencil_field_t *ga,
                  const stencil_field_t *gb, const stencil_field_t *gc, const stencil_config_t *cfg,
                  void *stream, bool fixed) {
    // Inputs first, outputs last (the alias check takes the last nout as outputs).
    const stencil_field_t *fs[15];
    const char *names[15];
    int n = 0, nout = 0;
    auto add = [&](const stencil_field_t *f, const char *name) { fs[n] = f; names[n++] = name; };
    add(u, "u"); add(coeff, "coeff"); add(wcon, "wcon"); add(a, "a"); add(b, "b"); add(c, "c");
    add(w, "w");
    const bool matrix = ga || gb || gc;
    if (matrix && !xf) return fail(STENCIL_E_NULL, "x (the forward result) is required for ga, gb, gc");
    if (matrix) add(xf, "x");
    const int nin = n;
    add(gu, "gu"); add(gcoeff, "gcoeff"); add(gwcon, "gwcon");
    if (ga) add(ga, "ga");
    if (gb) add(gb, "gb");
    if (gc) add(gc, "gc");
    nout = n - nin;
    TRY(check_call(fs, names, n, nout));
    TRY(check_halo(u, "u", 2));
    TRY(check_halo(gu, "gu", 2));
    TRY(check_dt(dt));
    if (cfg && cfg->schedule != 0 && cfg->schedule != 1)
        return fail(STENCIL_E_ARG, "adjoint schedule must be 0 (register strips) or 1 (LDS tiles), got %d",
                    cfg->schedule);
    if (cfg && ((cfg->tile_j != 0 && cfg->tile_j != 4 && cfg->tile_j != 8 && cfg->tile_j != 12) ||
                (cfg->tile_j > 4 && u->dtype == STENCIL_F64) || cfg->prefetch < 0 || cfg->prefetch > 2 ||
                (cfg->tile_j == 12 && cfg->prefetch == 2)))
        return fail(STENCIL_E_ARG,
                    "adjoint register strips take tile_j 4 or 8 with prefetch 1 or 2, or tile_j 12 with prefetch "
                    "1 (FP64: tile_j 4) (got %d, %d)",
                    cfg->tile_j, cfg->prefetch);
    if (empty(u)) return STENCIL_OK;
    if (u->nk > KMAX_ADJOINT)
        return fail(STENCIL_E_UNSUPPORTED, "adjoint supports nk <= %d", KMAX_ADJOINT);
    {
        // 32-bit buffer offsets, also into the compute-type scratch (FP32 for bfloat16 storage)
        const long long cells = static_cast<long long>(u->ni + 3) + static_cast<long long>(u->nj + 3) * u->sj +
                                static_cast<long long>(u->nk - 1) * u->sk + 1;
        if (cells * (u->dtype == STENCIL_F64 ? 8 : 4) >= 2147483647LL)
            return fail(STENCIL_E_UNSUPPORTED, "adjoint supports fields below 2 GiB (in the compute type)");
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    AdjointArgs x{};
    x.u = u->origin; x.coeff = coeff->origin; x.wcon = wcon->origin;
    x.a = a->origin; x.b = b->origin; x.c = c->origin; x.w = w->origin;
    x.gu = gu->origin; x.gcoeff = gcoeff->origin; x.gwcon = gwcon->origin;
    x.x = matrix ? xf->origin : nullptr;
    x.ga = ga ? ga->origin : nullptr;
    x.gb = gb ? gb->origin : nullptr;
    x.gc = gc ? gc->origin : nullptr;
    x.I = u->ni; x.J = u->nj; x.K = u->nk;
    x.sj = static_cast<int>(u->sj); x.sk = static_cast<int>(u->sk);
    x.dt = dt;
    x.hdiff_schedule = cfg ? cfg->schedule : 0;
    x.hdiff_tile_j = cfg ? cfg->tile_j : 0;
    x.hdiff_prefetch = cfg ? cfg->prefetch : 0;
    const size_t need = adjoint_scratch_bytes(u->dtype, x.sk, x.K);
    if (fixed) {
        if (need > ADJOINT_FIXED_SCRATCH_BYTES)
            return fail(STENCIL_E_UNSUPPORTED,
                        "the call needs %zu bytes of scratch; the fixed scratch array of the entry point that "
                        "allocates nothing holds %zu",
                        need, static_cast<size_t>(ADJOINT_FIXED_SCRATCH_BYTES));
        void *p = nullptr;
        const hipError_t e = adjoint_fixed_scratch(&p);
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(adjoint scratch)");
        return launch_status(launch_adjoint(u->dtype, x, p, st), "adjoint kernels");
    }
    ScratchLease lease;
    TRY(scratch_get(st, need, &lease));
    return launch_status(launch_adjoint(u->dtype, x, lease.p, st), "adjoint kernels");
}

}  // namespace stl

STENCIL_API int stencil_hdiff_vadv_adjoint(const stencil_field_t *u, const stencil_field_t *coeff,
                                           const stencil_field_t *wcon, const stencil_field_t *a,
                                           const stencil_field_t *b, const stencil_field_t *c,
                                           double dt, const stencil_field_t *w,
                                           const stencil_field_t *gu, const stencil_field_t *gcoeff,
                                           const stencil_field_t *gwcon, const stencil_field_t *xf,
                                           const stencil_field_t *ga, const stencil_field_t *gb,
                                           const stencil_field_t *gc, const stencil_config_t *cfg,
                                           void *stream) {
    return adjoint_entry(u, coeff, wcon, a, b, c, dt, w, gu, gcoeff, gwcon, xf, ga, gb, gc, cfg, stream, false);
}

STENCIL_API int stencil_hdiff_vadv_adjoint_noalloc(const stencil_field_t *u, const stencil_field_t *coeff,
                                                   const stencil_field_t *wcon, const stencil_field_t *a,
                                                   const stencil_field_t *b, const stencil_field_t *c,
                                                   double dt, const stencil_field_t *w,
                                                   const stencil_field_t *gu, const stencil_field_t *gcoeff,
                                                   const stencil_field_t *gwcon, const stencil_field_t *xf,
                                                   const stencil_field_t *ga, const stencil_field_t *gb,
                                                   const stencil_field_t *gc, const stencil_config_t *cfg,
                                                   void *stream) {
    return adjoint_entry(u, coeff, wcon, a, b, c, dt, w, gu, gcoeff, gwcon, xf, ga, gb, gc, cfg, stream, true);
}

STENCIL_API int stencil_hdiff_vadv_jvp(const stencil_field_t *u, const stencil_field_t *coeff,
                                       const stencil_field_t *wcon, const stencil_field_t *a,
                                       const stencil_field_t *b, const stencil_field_t *c, double dt,
                                       const stencil_field_t *xf, const stencil_field_t *du,
                                       const stencil_field_t *dcoeff, const stencil_field_t *dwcon,
                                       const stencil_field_t *da, const stencil_field_t *db,
                                       const stencil_field_t *dc, const stencil_field_t *dx,
                                       const stencil_config_t *cfg, void *stream) {
    // Inputs first, the output last (the alias check takes the last nout as outputs).
    const stencil_field_t *fs[14];
    const char *names[14];
    int n = 0;
    auto add = [&](const stencil_field_t *f, const char *name) { fs[n] = f; names[n++] = name; };
    add(u, "u"); add(coeff, "coeff"); add(wcon, "wcon"); add(a, "a"); add(b, "b"); add(c, "c");
    const bool matrix = da || db || dc;
    if (matrix && !xf) return fail(STENCIL_E_NULL, "x (the forward result) is required for da, db, dc");
    if (matrix) add(xf, "x");
    if (du) add(du, "du");
    if (dcoeff) add(dcoeff, "dcoeff");
    if (dwcon) add(dwcon, "dwcon");
    if (da) add(da, "da");
    if (db) add(db, "db");
    if (dc) add(dc, "dc");
    add(dx, "dx");
    TRY(check_call(fs, names, n, 1));
    TRY(check_halo(u, "u", 2));
    if (du) TRY(check_halo(du, "du", 2));
    TRY(check_dt(dt));
    (void)cfg;
    if (empty(u)) return STENCIL_OK;
    if (u->nk > KMAX_JVP) return fail(STENCIL_E_UNSUPPORTED, "jvp supports nk <= %d", KMAX_JVP);
    if (!column_fits(u)) return fail(STENCIL_E_UNSUPPORTED, "jvp supports fields below 2 GiB");
    JvpArgs v{};
    v.u = u->origin; v.coeff = coeff->origin; v.wcon = wcon->origin;
    v.a = a->origin; v.b = b->origin; v.c = c->origin;
    v.x = matrix ? xf->origin : nullptr;
    v.du = du ? du->origin : nullptr;
    v.dcoeff = dcoeff ? dcoeff->origin : nullptr;
    v.dwcon = dwcon ? dwcon->origin : nullptr;
    v.da = da ? da->origin : nullptr;
    v.db = db ? db->origin : nullptr;
    v.dc = dc ? dc->origin : nullptr;
    v.dx = dx->origin;
    v.I = u->ni; v.J = u->nj; v.K = u->nk;
    v.sj = static_cast<int>(u->sj); v.sk = static_cast<int>(u->sk);
    v.dt = dt;
    return launch_status(launch_jvp(u->dtype, v, static_cast<hipStream_t>(stream)), "jvp kernel");
}

namespace stl {

// Validation and launch shared by the halo exchange and its transpose.
static int halo_entry(const stencil_field_t *shares, int px, int py, int width, void *stream, bool accumulate) {
    if (!shares) return fail(STENCIL_E_NULL, "shares: array is NULL");
    if (px < 1 || py < 1 || static_cast<long long>(px) * py > HALO_MAX_SHARES)
        return fail(STENCIL_E_ARG, "px x py = %d x %d shares; 1 to %d are supported", px, py, HALO_MAX_SHARES);
    if (width < 1) return fail(STENCIL_E_ARG, "halo width %d < 1", width);
    const int n = px * py;
    std::vector<const stencil_field_t *> fs(n);
    std::vector<std::string> nm(n);
    std::vector<const char *> names(n);
    for (int s = 0; s < n; ++s) {
        fs[s] = &shares[s];
        nm[s] = "shares[" + std::to_string(s) + "]";
        names[s] = nm[s].c_str();
        TRY(check_field(fs[s], names[s]));
    }
    for (int s = 0; s < n; ++s) {
        const stencil_field_t *f = fs[s], *r = fs[0];
        const int p = s % px, q = s / px;
        if (f->dtype != r->dtype)
            return fail(STENCIL_E_DTYPE, "%s has dtype %d but shares[0] has %d", names[s], f->dtype, r->dtype);
        if (f->nk != r->nk) return fail(STENCIL_E_SHAPE, "%s has nk=%d but shares[0] has %d", names[s], f->nk, r->nk);
        if (f->ni != fs[p]->ni)
            return fail(STENCIL_E_SHAPE, "%s has ni=%d but the share at the top of its column has %d", names[s],
                        f->ni, fs[p]->ni);
        if (f->nj != fs[q * px]->nj)
            return fail(STENCIL_E_SHAPE, "%s has nj=%d but the first share of its row has %d", names[s], f->nj,
                        fs[q * px]->nj);
        if ((px > 1 && f->hi < width) || (py > 1 && f->hj < width))
            return fail(STENCIL_E_HALO, "%s: halo (%d, %d) narrower than the exchanged width %d", names[s], f->hi,
                        f->hj, width);
        if (f->nk > 0 && ((px > 1 && f->ni < width) || (py > 1 && f->nj < width)))
            return fail(STENCIL_E_SHAPE, "%s: interior %d x %d narrower than the exchanged width %d", names[s],
                        f->ni, f->nj, width);
    }
    if (fs[0]->nk == 0 || n == 1) return STENCIL_OK;
    // Every share is read by its neighbours and written: no two may overlap.
    TRY(check_alias(fs.data(), names.data(), n, n));
    HaloArgs a{};
    for (int s = 0; s < n; ++s) a.s[s] = {shares[s].origin, shares[s].sj, shares[s].sk};
    for (int p = 0; p < px; ++p) a.ni[p] = fs[p]->ni;
    for (int q = 0; q < py; ++q) a.nj[q] = fs[q * px]->nj;
    a.px = px;
    a.py = py;
    a.w = width;
    a.K = fs[0]->nk;
    return launch_status(launch_halo(fs[0]->dtype, a, accumulate, static_cast<hipStream_t>(stream)),
                         accumulate ? "halo accumulate kernel" : "halo exchange kernel");
}

}  // namespace stl

STENCIL_API int stencil_halo_exchange(const stencil_field_t *shares, int32_t px, int32_t py, int32_t width,
                                      void *stream) {
    return halo_entry(shares, px, py, width, stream, false);
}

STENCIL_API int stencil_halo_accumulate(const stencil_field_t *shares, int32_t px, int32_t py, int32_t width,
                                        void *stream) {
    return halo_entry(shares, px, py, width, stream, true);
}

STENCIL_API int stencil_probe_copy(const void *src, void *dst, int64_t nbytes, void *stream) {
    if (!src || !dst) return fail(STENCIL_E_NULL, "probe_copy: NULL pointer");
    if (nbytes < 0 || nbytes % 16 || reinterpret_cast<uintptr_t>(src) % 16 ||
        reinterpret_cast<uintptr_t>(dst) % 16)
        return fail(STENCIL_E_ARG, "probe_copy: nbytes and pointers must be 16-byte aligned");
    const uintptr_t s = reinterpret_cast<uintptr_t>(src), d = reinterpret_cast<uintptr_t>(dst);
    if (s < d + nbytes && d < s + nbytes) return fail(STENCIL_E_ALIAS, "probe_copy: ranges overlap");
    return launch_status(launch_probe_copy(src, dst, nbytes, static_cast<hipStream_t>(stream)),
                         "copy kernel");
}

STENCIL_API int stencil_probe_streams(const void *const *src, int32_t nsrc, void *dst, int64_t nbytes,
                                      void *stream) {
    if (!src || !dst) return fail(STENCIL_E_NULL, "probe_streams: NULL pointer");
    if (nsrc < 1 || nsrc > 8) return fail(STENCIL_E_ARG, "probe_streams: nsrc must be 1 .. 8 (got %d)", nsrc);
    if (nbytes < 0 || nbytes % 16 || reinterpret_cast<uintptr_t>(dst) % 16)
        return fail(STENCIL_E_ARG, "probe_streams: nbytes and pointers must be 16-byte aligned");
    const uintptr_t d = reinterpret_cast<uintptr_t>(dst);
    for (int f = 0; f < nsrc; ++f) {
        if (!src[f]) return fail(STENCIL_E_NULL, "probe_streams: source %d is NULL", f);
        const uintptr_t s = reinterpret_cast<uintptr_t>(src[f]);
        if (s % 16) return fail(STENCIL_E_ARG, "probe_streams: nbytes and pointers must be 16-byte aligned");
        if (s < d + nbytes && d < s + nbytes) return fail(STENCIL_E_ALIAS, "probe_streams: source %d overlaps dst", f);
    }
    return launch_status(launch_probe_streams(src, nsrc, dst, nbytes, static_cast<hipStream_t>(stream)),
                         "streams kernel");
}

STENCIL_API int stencil_probe_read(const void *src, int64_t nbytes, uint32_t key, void *sink, void *stream) {
    if (!src || !sink) return fail(STENCIL_E_NULL, "probe_read: NULL pointer");
    if (nbytes < 0 || nbytes % 16 || reinterpret_cast<uintptr_t>(src) % 16 ||
        reinterpret_cast<uintptr_t>(sink) % 4)
        return fail(STENCIL_E_ARG, "probe_read: nbytes and src must be 16-byte aligned, sink 4-byte");
    return launch_status(launch_probe_read(src, nbytes, key, sink, static_cast<hipStream_t>(stream)),
                         "read kernel");
}
