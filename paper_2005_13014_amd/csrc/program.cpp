// Batched timestep program: stencil_program_run.
//
// A program applies the stage chain hdiff -> vadv [-> vdiff [-> hgrad]] to
// every field of every subdomain.  Shape inference (Sec. V-B) grows the
// domain of the column stages by one cell when hgrad follows, since hgrad
// reads y on the interior and its 1-cell ring.  Planning:
//   - the column stages (hdiff + vadv, with vdiff folded into the
//     back-substitution) run as batched launches, one per register bucket of
//     the column height, each over a table of up to BATCH_SUBS subdomains x
//     BATCH_FIELDS fields (the table rides in the kernel arguments);
//   - with hgrad, y goes to library-owned scratch and a batched 7-point
//     kernel writes z.
// With STENCIL_PROGRAM_AUTOTUNE the compiled (tile_j, prefetch, level-loop
// schedule) variants of the column kernel are timed once per program
// signature and the fastest is kept; otherwise the preferred one runs.  With STENCIL_PROGRAM_GRAPH the launches are captured once per
// signature into a hipGraph that later calls replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <list>
#include <memory>
#include <mutex>
#include <vector>

#include "../../include/stencil.h"
#include "launch.hpp"
#include "program.hpp"
#include "program_kernels.hpp"

#define STENCIL_API extern "C" __attribute__((visibility("default")))

namespace stl {

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int check_field(const stencil_field_t *f, const char *name);
int check_same(const stencil_field_t *const *fs, const char *const *names, int n);
int check_halo(const stencil_field_t *f, const char *name, int need);
size_t elem_size(int dtype);
bool empty(const stencil_field_t *f);

hipError_t launch_column_batch_f64(const ColumnBatch &, int, int, int, int, int, int, int, hipStream_t);
hipError_t launch_column_batch_f32(const ColumnBatch &, int, int, int, int, int, int, int, hipStream_t);
hipError_t launch_column_batch_bf16(const ColumnBatch &, int, int, int, int, int, int, int, hipStream_t);
hipError_t launch_hgrad_batch_f64(const HgradBatch &, int, hipStream_t);
hipError_t launch_hgrad_batch_f32(const HgradBatch &, int, hipStream_t);
hipError_t launch_hgrad_batch_bf16(const HgradBatch &, int, hipStream_t);
bool batch_variant_f64(int, int, int, int);
bool batch_variant_f32(int, int, int, int);
bool batch_variant_bf16(int, int, int, int);

#define TRY(x)                             \
    do {                                   \
        int rc_ = (x);                     \
        if (rc_ != STENCIL_OK) return rc_; \
    } while (0)

namespace {

// A column-kernel variant: rows per tile, levels prefetched, level loop
// (1 staged, 2 software-pipelined), fields of one tile per workgroup (the
// compiled kernels take one; the planner counts tiles with it).
struct Variant {
    int tj, pf, sched, fpw;
};

// Compiled variants, the library's preference first (the choice without
// autotuning); staged_only keeps the staged level loop alone.
std::vector<Variant> variants_for(int dtype, bool staged_only) {
    std::vector<Variant> v;
    const Variant all[] = {{2, 4, 2, 1}, {2, 4, 1, 1}, {4, 4, 2, 1}, {4, 4, 1, 1}, {2, 2, 1, 1}};
    for (const Variant &c : all) {
        if (staged_only && c.sched != 1) continue;
        const bool ok = dtype == STENCIL_F64   ? batch_variant_f64(c.tj, c.pf, c.sched, c.fpw)
                        : dtype == STENCIL_F32 ? batch_variant_f32(c.tj, c.pf, c.sched, c.fpw)
                                               : batch_variant_bf16(c.tj, c.pf, c.sched, c.fpw);
        if (ok) v.push_back(c);
    }
    return v;
}

int kh_bucket(int K) {
    const int m = (K + 1) / 2;
    for (int kh : PROGRAM_BUCKETS)
        if (m <= kh) return kh;
    return PROGRAM_BUCKETS[sizeof(PROGRAM_BUCKETS) / sizeof(PROGRAM_BUCKETS[0]) - 1];
}

// One batched launch of the column stages, and of hgrad.
struct ColumnLaunch {
    ColumnBatch b;
    int kh, ntiles, tj_nbj_rows;  // tj_nbj_rows: TJ the tile counts were computed for
};

// The planned program: everything a replay needs, pointers included.
struct Plan {
    int dtype = 0;
    int vdiff = 0;  // 0 none, 1 explicit, 2 implicit vertical diffusion
    bool hgrad = false;
    std::vector<ColumnLaunch> col;
    std::vector<HgradBatch> hg;
    std::vector<int> hg_tiles;
    size_t scratch_bytes = 0;
};

// A device buffer of y scratch, shared by the cached programs on the same
// device and stream that need the same number of bytes: their launches are
// ordered by that stream, so they never use it at the same time.
struct Buffer {
    int dev = 0;
    hipStream_t st = nullptr;
    size_t bytes = 0;
    void *p = nullptr;
    int refs = 0;
};

struct Entry {
    std::vector<unsigned char> key;  // the full signature, compared byte for byte
    uint64_t hash = 0;
    int dev = 0;
    hipStream_t st = nullptr;
    Plan plan;
    Buffer *buf = nullptr;
    Variant var{0, 0, 0, 1};
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
};

// Cached programs, most recently used first, at most PROGRAM_CACHE_MAX.
constexpr size_t PROGRAM_CACHE_MAX = 16;
std::mutex g_mu;
std::list<std::unique_ptr<Entry>> g_lru;
std::vector<std::unique_ptr<Buffer>> g_bufs;

uint64_t fnv(uint64_t h, const void *p, size_t n) {
    const unsigned char *c = static_cast<const unsigned char *>(p);
    for (size_t q = 0; q < n; ++q) {
        h ^= c[q];
        h *= 1099511628211ULL;
    }
    return h;
}

// Everything a cached plan or graph depends on: device, stream, stages,
// flags (they choose the kernel variant), parameters and every descriptor.
std::vector<unsigned char> signature(const stencil_program_t *prog, int dev, hipStream_t st) {
    std::vector<unsigned char> k;
    auto put = [&](const void *p, size_t n) {
        const unsigned char *c = static_cast<const unsigned char *>(p);
        k.insert(k.end(), c, c + n);
    };
    put(&dev, sizeof(dev));
    put(&st, sizeof(st));
    put(&prog->nsub, sizeof(prog->nsub));
    put(&prog->stages, sizeof(prog->stages));
    put(&prog->flags, sizeof(prog->flags));
    put(&prog->dt, sizeof(double));
    put(&prog->kappa, sizeof(double));
    put(&prog->beta_h, sizeof(double));
    put(&prog->beta_v, sizeof(double));
    for (int s = 0; s < prog->nsub; ++s) {
        const stencil_subdomain_t &sd = prog->sub[s];
        for (const stencil_field_t *f : {&sd.coeff, &sd.wcon, &sd.a, &sd.b, &sd.c}) put(f, sizeof(*f));
        put(&sd.nfields, sizeof(sd.nfields));
        for (int q = 0; q < sd.nfields; ++q) put(&sd.u[q], sizeof(stencil_field_t));
        for (int q = 0; q < sd.nfields; ++q) put(&sd.z[q], sizeof(stencil_field_t));
    }
    return k;
}

int buffer_get(int dev, hipStream_t st, size_t bytes, Buffer **out) {
    *out = nullptr;
    if (!bytes) return STENCIL_OK;
    for (auto &b : g_bufs)
        if (b->dev == dev && b->st == st && b->bytes == bytes) {
            ++b->refs;
            *out = b.get();
            return STENCIL_OK;
        }
    std::unique_ptr<Buffer> b(new Buffer);
    b->dev = dev;
    b->st = st;
    b->bytes = bytes;
    const hipError_t e = hipMalloc(&b->p, bytes);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(program scratch)");
    b->refs = 1;
    *out = b.get();
    g_bufs.push_back(std::move(b));
    return STENCIL_OK;
}

// Drops an entry: waits for its stream (launches in flight may still use the
// graph and the scratch), then frees the graph and, with its last user, the
// scratch buffer.
void entry_release(Entry &en) {
    int cur = 0;
    const bool have_cur = hipGetDevice(&cur) == hipSuccess;
    if (have_cur && cur != en.dev) hipSetDevice(en.dev);
    hipStreamSynchronize(en.st);
    if (en.exec) hipGraphExecDestroy(en.exec);
    if (en.graph) hipGraphDestroy(en.graph);
    en.exec = nullptr;
    en.graph = nullptr;
    if (en.buf && --en.buf->refs == 0) {
        hipFree(en.buf->p);
        for (size_t q = 0; q < g_bufs.size(); ++q)
            if (g_bufs[q].get() == en.buf) {
                g_bufs.erase(g_bufs.begin() + static_cast<long>(q));
                break;
            }
    }
    en.buf = nullptr;
    if (have_cur && cur != en.dev) hipSetDevice(cur);
}

int check_program(const stencil_program_t *prog, int *dtype_out) {
    if (!prog) return fail(STENCIL_E_NULL, "program is NULL");
    if (prog->nsub < 0) return fail(STENCIL_E_ARG, "nsub < 0");
    if (prog->nsub > 0 && !prog->sub) return fail(STENCIL_E_NULL, "program subdomains are NULL");
    const int st = prog->stages;
    const int chain1 = STENCIL_STAGE_HDIFF | STENCIL_STAGE_VADV;
    const int chain2 = chain1 | STENCIL_STAGE_VDIFF, chain2i = chain1 | STENCIL_STAGE_VDIFF_IMPLICIT;
    const int chain3 = chain2 | STENCIL_STAGE_HGRAD, chain3i = chain2i | STENCIL_STAGE_HGRAD;
    if (st != chain1 && st != chain2 && st != chain3 && st != chain2i && st != chain3i)
        return fail(STENCIL_E_ARG, "stages must be HDIFF|VADV[|VDIFF or VDIFF_IMPLICIT[|HGRAD]] (got %d)", st);
    if (prog->flags & ~(STENCIL_PROGRAM_GRAPH | STENCIL_PROGRAM_AUTOTUNE | STENCIL_PROGRAM_STAGED))
        return fail(STENCIL_E_ARG, "unknown program flags %d", prog->flags);
    if (!std::isfinite(prog->dt) || !std::isfinite(prog->kappa) || !std::isfinite(prog->beta_h) ||
        !std::isfinite(prog->beta_v))
        return fail(STENCIL_E_ARG, "program parameters must be finite");
    const int e = (st & STENCIL_STAGE_HGRAD) ? 1 : 0;
    int dtype = -1;
    struct Range {
        uintptr_t lo, hi;
        bool out;
    };
    std::vector<Range> ranges;
    for (int s = 0; s < prog->nsub; ++s) {
        const stencil_subdomain_t &sd = prog->sub[s];
        if (sd.nfields < 0) return fail(STENCIL_E_ARG, "subdomain %d: nfields < 0", s);
        if (sd.nfields > 0 && (!sd.u || !sd.z))
            return fail(STENCIL_E_NULL, "subdomain %d: field arrays are NULL", s);
        std::vector<const stencil_field_t *> fs = {&sd.coeff, &sd.wcon, &sd.a, &sd.b, &sd.c};
        std::vector<const char *> names = {"coeff", "wcon", "a", "b", "c"};
        for (int f = 0; f < sd.nfields; ++f) {
            fs.push_back(&sd.u[f]);
            names.push_back("u");
        }
        for (int f = 0; f < sd.nfields; ++f) {
            fs.push_back(&sd.z[f]);
            names.push_back("z");
        }
        for (size_t q = 0; q < fs.size(); ++q) TRY(check_field(fs[q], names[q]));
        TRY(check_same(fs.data(), names.data(), static_cast<int>(fs.size())));
        if (dtype < 0) dtype = sd.coeff.dtype;
        if (sd.coeff.dtype != dtype) return fail(STENCIL_E_DTYPE, "subdomains differ in dtype");
        if (empty(&sd.coeff) || sd.nfields == 0) continue;
        for (int q = 0; q < 5; ++q) TRY(check_halo(fs[q], names[q], e));
        for (int f = 0; f < sd.nfields; ++f) TRY(check_halo(&sd.u[f], "u", 2 + e));
        if (sd.coeff.nk > KMAX_COLUMN)
            return fail(STENCIL_E_UNSUPPORTED, "program columns support nk <= %d", KMAX_COLUMN);
        const long long es = static_cast<long long>(elem_size(dtype));
        const long long span = (sd.coeff.ni + 5) + (sd.coeff.nj + 5) * sd.coeff.sj +
                               (sd.coeff.nk - 1) * sd.coeff.sk + 1;
        if (span * es >= 2147483647LL)
            return fail(STENCIL_E_UNSUPPORTED, "subdomain %d: fields of 2 GiB or more", s);
        for (size_t q = 0; q < fs.size(); ++q) {
            const stencil_field_t *f = fs[q];
            const long long lo = -f->hi - static_cast<long long>(f->hj) * f->sj;
            const long long hi = (f->ni + f->hi - 1) + static_cast<long long>(f->nj + f->hj - 1) * f->sj +
                                 static_cast<long long>(f->nk - 1) * f->sk;
            const uintptr_t base = reinterpret_cast<uintptr_t>(f->origin);
            ranges.push_back({base + static_cast<intptr_t>(lo * es), base + static_cast<intptr_t>((hi + 1) * es),
                              q >= 5 + static_cast<size_t>(sd.nfields)});
        }
    }
    for (size_t o = 0; o < ranges.size(); ++o) {
        if (!ranges[o].out) continue;
        for (size_t q = 0; q < ranges.size(); ++q)
            if (q != o && ranges[o].lo < ranges[q].hi && ranges[q].lo < ranges[o].hi)
                return fail(STENCIL_E_ALIAS, "a program output overlaps another field");
    }
    *dtype_out = dtype < 0 ? STENCIL_F32 : dtype;
    return STENCIL_OK;
}

// ColumnArgs of a subdomain's column stages on its interior grown by e.
ColumnArgs column_args_ext(const stencil_field_t &cf, const stencil_subdomain_t &sd, int e,
                           double dt, int tj) {
    const long long es = static_cast<long long>(elem_size(cf.dtype));
    const long long shift = (e + e * cf.sj) * es;
    auto sh = [&](const void *p) { return static_cast<const void *>(static_cast<const char *>(p) - shift); };
    ColumnArgs a{};
    a.coeff = sh(sd.coeff.origin);
    a.wcon = sh(sd.wcon.origin);
    a.a = sh(sd.a.origin);
    a.b = sh(sd.b.origin);
    a.c = sh(sd.c.origin);
    a.I = cf.ni + 2 * e;
    a.J = cf.nj + 2 * e;
    a.K = cf.nk;
    a.sj = static_cast<int>(cf.sj);
    a.sk = static_cast<int>(cf.sk);
    a.u_bytes = static_cast<uint32_t>(((a.I + 3) + (a.J + 3) * cf.sj + (a.K - 1) * cf.sk + 1) * es);
    a.col_bytes = static_cast<uint32_t>(((a.I - 1) + (a.J - 1) * cf.sj + (a.K - 1) * cf.sk + 1) * es);
    a.nbi = (a.I + 63) / 64;
    a.nbj = (a.J + tj - 1) / tj;
    a.dt = dt;
    return a;
}

// First column of a subdomain's first column-kernel tile, in the coordinates
// of its domain grown by e: a tile that starts at the start of a 128-byte line
// of the coefficient fields reads each tile row of every field in whole lines
// (a tile starting one element into a line touches one more line per row), so
// the tiles start on the last line start at or before the domain's first
// column, unless that takes more tiles than starting at column 0.
int tile_origin(const stencil_field_t &cf, int e, long long es) {
    const long long L = 128 / es;
    const uintptr_t addr = reinterpret_cast<uintptr_t>(cf.origin);
    if (addr % static_cast<uintptr_t>(es) != 0) return 0;
    const long long a = static_cast<long long>((addr / es) % L);  // interior column 0 is element a of its line
    long long first = -a;                                         // interior column of a line start
    while (first > -e) first -= L;
    const int lo = static_cast<int>(first) + e;
    const int I = cf.ni + 2 * e;
    return (I - lo + 63) / 64 <= (I + 63) / 64 ? lo : 0;
}

// Builds the launch tables for a given column-kernel tile height and number
// of fields per workgroup.  Scratch offsets for y are laid out when
// `scratch` is null (sizing pass).
int build_plan(const stencil_program_t *prog, int dtype, int tj, int fpw, char *scratch, Plan *plan) {
    plan->dtype = dtype;
    plan->vdiff = (prog->stages & STENCIL_STAGE_VDIFF_IMPLICIT) ? 2 : (prog->stages & STENCIL_STAGE_VDIFF) ? 1 : 0;
    plan->hgrad = (prog->stages & STENCIL_STAGE_HGRAD) != 0;
    plan->col.clear();
    plan->hg.clear();
    plan->hg_tiles.clear();
    const int e = plan->hgrad ? 1 : 0;
    const long long es = static_cast<long long>(elem_size(dtype));
    size_t off = 0;
    // Scratch y per (subdomain, field), same strides as the subdomain.
    std::vector<std::vector<char *>> ys(prog->nsub);
    for (int s = 0; s < prog->nsub; ++s) {
        const stencil_subdomain_t &sd = prog->sub[s];
        if (!plan->hgrad || empty(&sd.coeff) || sd.nfields == 0) continue;
        // y's origin at least one row and one column in, so the 1-cell ring is
        // addressable, and placed so that the column tiles' rows of y start on
        // 128-byte lines, as their rows of the input fields do (tile_origin).
        const int lo = tile_origin(sd.coeff, e, es);
        const long long ring = (sd.coeff.sj + 1) * es;
        const long long want = ((-(lo - e) * es) % 128 + 128) % 128;
        const long long pad = ring + ((want - ring % 128) % 128 + 128) % 128;
        for (int f = 0; f < sd.nfields; ++f) {
            const size_t bytes = static_cast<size_t>(static_cast<long long>(sd.coeff.nk) * sd.coeff.sk * es + pad + ring);
            ys[s].push_back(scratch ? scratch + off + pad : nullptr);
            off += (bytes + 255) / 256 * 256;
        }
    }
    plan->scratch_bytes = off;

    for (int bucket : PROGRAM_BUCKETS) {
        ColumnLaunch cl{};
        cl.kh = bucket;
        cl.tj_nbj_rows = tj;
        int tiles = 0;
        auto flush = [&]() {
            if (cl.b.nsub > 0) {
                cl.ntiles = tiles;
                cl.b.kappa = prog->kappa;
                plan->col.push_back(cl);
            }
            cl.b = ColumnBatch{};
            tiles = 0;
        };
        cl.b = ColumnBatch{};
        for (int s = 0; s < prog->nsub; ++s) {
            const stencil_subdomain_t &sd = prog->sub[s];
            if (empty(&sd.coeff) || sd.nfields == 0 || kh_bucket(sd.coeff.nk) != bucket) continue;
            ColumnArgs a = column_args_ext(sd.coeff, sd, e, prog->dt, tj);
            a.i_lo = tile_origin(sd.coeff, e, es);
            a.nbi = (a.I - a.i_lo + 63) / 64;
            const long long shift = (e + e * sd.coeff.sj) * es;
            for (int f0 = 0; f0 < sd.nfields; f0 += BATCH_FIELDS) {
                if (cl.b.nsub == BATCH_SUBS) flush();
                ColumnBatchSub &sb = cl.b.sub[cl.b.nsub++];
                sb.a = a;
                sb.nfields = sd.nfields - f0 < BATCH_FIELDS ? sd.nfields - f0 : BATCH_FIELDS;
                sb.tile0 = tiles;
                for (int f = 0; f < sb.nfields; ++f) {
                    // u addressed from cell (-2, -2) of the grown domain
                    sb.u[f] = static_cast<const char *>(sd.u[f0 + f].origin) - shift - (2 + 2 * sd.coeff.sj) * es;
                    void *out = plan->hgrad ? static_cast<void *>(ys[s][f0 + f]) : sd.z[f0 + f].origin;
                    sb.x[f] = out ? static_cast<char *>(out) - shift : nullptr;
                }
                tiles += a.nbi * a.nbj * ((sb.nfields + fpw - 1) / fpw);
            }
        }
        flush();
    }
    if (plan->hgrad) {
        HgradBatch hb{};
        int tiles = 0;
        auto flush = [&]() {
            if (hb.nsub > 0) {
                hb.kc = HGRAD_RUN;
                hb.beta_h = prog->beta_h;
                hb.beta_v = prog->beta_v;
                plan->hg.push_back(hb);
                plan->hg_tiles.push_back(tiles);
            }
            hb = HgradBatch{};
            tiles = 0;
        };
        for (int s = 0; s < prog->nsub; ++s) {
            const stencil_subdomain_t &sd = prog->sub[s];
            if (empty(&sd.coeff) || sd.nfields == 0) continue;
            const stencil_field_t &cf = sd.coeff;
            for (int f0 = 0; f0 < sd.nfields; f0 += BATCH_FIELDS) {
                if (hb.nsub == BATCH_SUBS) flush();
                HgradSub &h = hb.sub[hb.nsub++];
                h.I = cf.ni; h.J = cf.nj; h.K = cf.nk;
                h.sj = static_cast<int>(cf.sj); h.sk = static_cast<int>(cf.sk);
                h.nbi = (cf.ni + 63) / 64;
                h.nbj = (cf.nj + HGRAD_ROWS - 1) / HGRAD_ROWS;
                h.ngroups = (h.nbi * h.nbj + 3) / 4;
                h.nruns = (cf.nk + HGRAD_RUN - 1) / HGRAD_RUN;
                h.nfields = sd.nfields - f0 < BATCH_FIELDS ? sd.nfields - f0 : BATCH_FIELDS;
                h.tile0 = tiles;
                h.y_bytes = static_cast<uint32_t>(((cf.ni + 1) + (cf.nj + 1) * cf.sj + (cf.nk - 1) * cf.sk + 1) * es);
                h.z_bytes = static_cast<uint32_t>(((cf.ni - 1) + (cf.nj - 1) * cf.sj + (cf.nk - 1) * cf.sk + 1) * es);
                for (int f = 0; f < h.nfields; ++f) {
                    h.y[f] = ys[s][f0 + f];
                    h.z[f] = sd.z[f0 + f].origin;
                }
                tiles += h.ngroups * h.nruns * h.nfields;
            }
        }
        flush();
    }
    return STENCIL_OK;
}

hipError_t enqueue(const Plan &plan, Variant v, hipStream_t st, bool columns_only = false) {
    for (const ColumnLaunch &cl : plan.col) {
        hipError_t e;
        switch (plan.dtype) {
        case STENCIL_F64:
            e = launch_column_batch_f64(cl.b, plan.vdiff, cl.kh, v.tj, v.pf, v.sched, v.fpw, cl.ntiles, st);
            break;
        case STENCIL_F32:
            e = launch_column_batch_f32(cl.b, plan.vdiff, cl.kh, v.tj, v.pf, v.sched, v.fpw, cl.ntiles, st);
            break;
        default:
            e = launch_column_batch_bf16(cl.b, plan.vdiff, cl.kh, v.tj, v.pf, v.sched, v.fpw, cl.ntiles, st);
            break;
        }
        if (e != hipSuccess) return e;
    }
    if (columns_only) return hipSuccess;
    for (size_t q = 0; q < plan.hg.size(); ++q) {
        hipError_t e;
        switch (plan.dtype) {
        case STENCIL_F64: e = launch_hgrad_batch_f64(plan.hg[q], plan.hg_tiles[q], st); break;
        case STENCIL_F32: e = launch_hgrad_batch_f32(plan.hg[q], plan.hg_tiles[q], st); break;
        default: e = launch_hgrad_batch_bf16(plan.hg[q], plan.hg_tiles[q], st); break;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Times the column launches of each compiled variant: after one warm-up
// launch each, five rounds that time every candidate once (interleaved, so
// that clock and cache drift hit all of them alike); the median decides.
int autotune(const stencil_program_t *prog, int dtype, char *scratch, hipStream_t st, Variant *best) {
    const std::vector<Variant> cands = variants_for(dtype, (prog->flags & STENCIL_PROGRAM_STAGED) != 0);
    constexpr int ROUNDS = 5;
    *best = cands.front();
    hipEvent_t e0, e1;
    hipError_t he = hipEventCreate(&e0);
    if (he != hipSuccess) return hip_fail(he, "hipEventCreate");
    he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        hipEventDestroy(e0);
        return hip_fail(he, "hipEventCreate");
    }
    std::vector<Plan> plans(cands.size());
    std::vector<std::vector<float>> ms(cands.size());
    hipError_t e = hipSuccess;
    for (size_t c = 0; c < cands.size() && e == hipSuccess; ++c) {
        build_plan(prog, dtype, cands[c].tj, cands[c].fpw, scratch, &plans[c]);
        e = enqueue(plans[c], cands[c], st, true);
    }
    for (int r = 0; r < ROUNDS && e == hipSuccess; ++r)
        for (size_t c = 0; c < cands.size() && e == hipSuccess; ++c) {
            e = hipEventRecord(e0, st);
            if (e == hipSuccess) e = enqueue(plans[c], cands[c], st, true);
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float t = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
            ms[c].push_back(t);
        }
    int rc = STENCIL_OK;
    if (e != hipSuccess) {
        rc = hip_fail(e, "autotune");
    } else {
        float best_ms = 1e30f;
        for (size_t c = 0; c < cands.size(); ++c) {
            std::vector<float> v = ms[c];
            std::nth_element(v.begin(), v.begin() + v.size() / 2, v.end());
            if (v[v.size() / 2] < best_ms) {
                best_ms = v[v.size() / 2];
                *best = cands[c];
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return rc;
}

}  // namespace

void program_release_all() {
    std::lock_guard<std::mutex> lock(g_mu);
    for (auto &en : g_lru) entry_release(*en);
    g_lru.clear();
    for (auto &b : g_bufs)
        if (b->p) hipFree(b->p);
    g_bufs.clear();
}

long long program_held_bytes(int *programs) {
    std::lock_guard<std::mutex> lock(g_mu);
    long long n = 0;
    for (auto &b : g_bufs) n += static_cast<long long>(b->bytes);
    if (programs) *programs = static_cast<int>(g_lru.size());
    return n;
}

int stream_capturing(hipStream_t st, bool *capturing);

}  // namespace stl

using namespace stl;

STENCIL_API int stencil_program_run(const stencil_program_t *prog, void *stream) {
    int dtype = 0;
    TRY(check_program(prog, &dtype));
    bool work = false;
    for (int s = 0; s < prog->nsub; ++s)
        work |= prog->sub[s].nfields > 0 && !empty(&prog->sub[s].coeff);
    if (!work) return STENCIL_OK;  // nothing to run: no allocation, no launch
    hipStream_t st = static_cast<hipStream_t>(stream);
    bool capturing = false;
    TRY(stream_capturing(st, &capturing));
    // Capture needs a real stream; on the null stream the program runs
    // eagerly.  Inside the caller's own capture the kernels are enqueued
    // into it directly.
    const bool graph = (prog->flags & STENCIL_PROGRAM_GRAPH) && st != nullptr && !capturing;
    const bool tune = (prog->flags & STENCIL_PROGRAM_AUTOTUNE) != 0;
    int dev = 0;
    hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess) return hip_fail(he, "hipGetDevice");
    std::vector<unsigned char> key = signature(prog, dev, st);
    const uint64_t hash = fnv(1469598103934665603ULL, key.data(), key.size());

    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_lru.begin();
    for (; it != g_lru.end(); ++it)
        if ((*it)->hash == hash && (*it)->key == key) break;
    if (it != g_lru.end()) {
        g_lru.splice(g_lru.begin(), g_lru, it);  // most recently used first
    } else {
        if (capturing)
            return fail(STENCIL_E_UNSUPPORTED,
                        "the first run of a program allocates its scratch%s; run it once before capturing the "
                        "stream",
                        tune ? " and synchronises to autotune" : "");
        std::unique_ptr<Entry> en(new Entry);
        en->key = std::move(key);
        en->hash = hash;
        en->dev = dev;
        en->st = st;
        Plan sizing;
        build_plan(prog, dtype, 2, 1, nullptr, &sizing);
        // Make room first, so that an evicted entry's scratch can be reused.
        while (g_lru.size() >= PROGRAM_CACHE_MAX) {
            entry_release(*g_lru.back());
            g_lru.pop_back();
        }
        TRY(buffer_get(dev, st, sizing.scratch_bytes, &en->buf));
        char *scratch = en->buf ? static_cast<char *>(en->buf->p) : nullptr;
        const std::vector<Variant> cands = variants_for(dtype, (prog->flags & STENCIL_PROGRAM_STAGED) != 0);
        en->var = cands.front();
        if (tune && cands.size() > 1) {
            const int rc = autotune(prog, dtype, scratch, st, &en->var);
            if (rc != STENCIL_OK) {
                entry_release(*en);
                return rc;
            }
        }
        build_plan(prog, dtype, en->var.tj, en->var.fpw, scratch, &en->plan);
        g_lru.push_front(std::move(en));
    }
    Entry &en = *g_lru.front();
    if (!graph) {
        const hipError_t e = enqueue(en.plan, en.var, st);
        return e == hipSuccess ? STENCIL_OK : hip_fail(e, "program kernels");
    }
    if (!en.exec) {
        hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        const hipError_t le = enqueue(en.plan, en.var, st);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(st, &g);
        if (le != hipSuccess || e != hipSuccess) {
            if (g) hipGraphDestroy(g);
            return hip_fail(le != hipSuccess ? le : e, "graph capture");
        }
        hipGraphExec_t x = nullptr;
        e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            hipGraphDestroy(g);
            return hip_fail(e, "hipGraphInstantiate");
        }
        en.graph = g;
        en.exec = x;
    }
    const hipError_t e = hipGraphLaunch(en.exec, st);
    return e == hipSuccess ? STENCIL_OK : hip_fail(e, "hipGraphLaunch");
}
