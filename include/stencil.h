/*
 * stencil.h -- C ABI of the MI355X (gfx950) stencil library.
 *
 * The library executes the stencil program that the Open Earth Compiler's two
 * optimisations produce (arXiv 2005.13014): horizontal diffusion
 * (Laplacian -> limited fluxes -> update, the hdiffsa benchmark of Sec. VII-B,
 * Table II) fused with vertical advection (a per-column tridiagonal solve by
 * the Thomas algorithm, the implicit vertical integration named in
 * Sec. VII-B).  Stencil inlining (Sec. V-A) becomes one fused kernel that
 * keeps every temporary on chip; stencil unrolling (Sec. V-A) becomes a
 * j-unroll factor of the horizontal-diffusion kernel.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All field pointers are DEVICE addresses owned by the caller.  The library
 *    never frees or reallocates them.
 *  - Index convention (the paper's range notation, Sec. IV-B): the origin is
 *    the first interior point; element (i, j, k) of a field lives at
 *    origin[i + sj * j + sk * k] (element strides, the i stride is 1).
 *    Interior: 0 <= i < ni, 0 <= j < nj, 0 <= k < nk.  A halo of hi (hj)
 *    cells on each side in i (j) may be addressed with negative indices or
 *    indices >= ni (nj).  There is no halo in k.
 *  - All fields of one call must have the same dtype, the same interior
 *    extents and the same strides (sj, sk).
 *  - Only the interior of an output is written; its halo is never touched.
 *  - Outputs must not overlap any input or other output (stencil programs are
 *    alias-free, Sec. IV-C and IV-D); overlap of the addressed byte ranges is rejected.
 *  - Input halos must be at least the access extent that shape inference
 *    derives for the call (Sec. V-B); otherwise STENCIL_E_HALO.
 *  - Calls validate on the host, then enqueue asynchronously on the given HIP
 *    stream (a hipStream_t passed as void*; NULL = the null stream).
 *    Validation errors return before anything is enqueued.
 *  - Synchronisation and allocation.  No call synchronises, allocates or frees
 *    device memory except these, and only in the case named:
 *      (1) calls that use library scratch -- stencil_hdiff, stencil_vadv and
 *          stencil_hdiff_vadv when they run the unfused kernels (level
 *          ORIGINAL, or a size the fused kernels do not take), and
 *          stencil_hdiff_vadv_adjoint -- when they need more scratch than the
 *          stream's buffer holds (the first such call on a stream, or a
 *          larger one): the stream is synchronised, the old buffer freed and
 *          a larger one allocated (stencil_hdiff_vadv_adjoint_noalloc, on
 *          fixed scratch, never does);
 *      (2) stencil_program_run on the first run of a program signature: it
 *          allocates the program's scratch (shared with cached programs of
 *          the same size on the same stream), with STENCIL_PROGRAM_AUTOTUNE
 *          synchronises the stream to time the candidates, and when the
 *          cache is full evicts the least recently used program (waiting for
 *          that program's stream, then freeing its graph and scratch);
 *      (3) stencil_shutdown (synchronises the device, frees everything).
 *    On a stream that is being captured into a graph such a call returns
 *    STENCIL_E_UNSUPPORTED instead of allocating (make it once before the
 *    capture, so the scratch exists); every other call captures normally.
 *  - Empty interiors (ni, nj or nk == 0) are valid no-ops.
 *  - Every element offset must fit in a signed 32-bit integer.
 *  - Return value: STENCIL_OK or an error code; stencil_last_error() gives a
 *    message for the calling thread's last error.
 */
#ifndef STENCIL_H
#define STENCIL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STENCIL_ABI_VERSION 2

typedef enum {
    STENCIL_F64 = 0,  /* storage and arithmetic in double */
    STENCIL_F32 = 1,  /* storage and stencil arithmetic in float; the Thomas
                         elimination and back-substitution in double */
    STENCIL_BF16 = 2  /* bfloat16 storage (raw uint16 bit patterns), float
                         stencil arithmetic, double Thomas solve; stores round
                         to nearest even */
} stencil_dtype;

typedef enum {
    STENCIL_OK = 0,
    STENCIL_E_NULL = 1,        /* a required pointer is NULL */
    STENCIL_E_DTYPE = 2,       /* unknown dtype, or dtypes differ within a call */
    STENCIL_E_SHAPE = 3,       /* negative extents, or extents differ within a call */
    STENCIL_E_STRIDE = 4,      /* strides cannot hold extents + halo, or differ within a call */
    STENCIL_E_HALO = 5,        /* an input halo is narrower than the access extent */
    STENCIL_E_ALIAS = 6,       /* an output overlaps an input or another output */
    STENCIL_E_UNSUPPORTED = 7, /* size or option the library does not implement */
    STENCIL_E_HIP = 8,         /* HIP runtime or launch error */
    STENCIL_E_ARG = 9          /* invalid scalar argument or configuration */
} stencil_status;

/* A halo-padded 3D field (the paper's !stencil.field with its asserted range,
 * Sec. IV-A).  `origin` is the device address of interior element (0,0,0). */
typedef struct {
    void *origin;
    int32_t dtype;       /* stencil_dtype */
    int32_t ni, nj, nk;  /* interior extents */
    int32_t hi, hj;      /* halo cells available on each side in i and j */
    int64_t sj, sk;      /* element strides of j and k; sj >= ni + 2 hi,
                            sk >= sj * (nj + 2 hj) */
} stencil_field_t;

/* Optimisation level, the levels compared in Sec. VII-C. */
typedef enum {
    STENCIL_LEVEL_DEFAULT = 0,  /* the library's choice (fused) */
    STENCIL_LEVEL_ORIGINAL = 1, /* one kernel per stencil operator; every
                                   temporary (lap, fluxes, h, rhs, Thomas
                                   coefficients) goes through device memory */
    STENCIL_LEVEL_INLINE = 2    /* all operators fused into one kernel;
                                   temporaries stay on chip */
} stencil_level;

/* Optional tuning knobs; pass NULL for defaults.  Zero fields mean default. */
typedef struct {
    int32_t level;    /* stencil_level */
    int32_t unroll;   /* j-unroll factor of stencil_hdiff: 1, 2 or 4 (Sec. V-A) */
    int32_t tile_j;   /* rows of columns per workgroup: 1, 2 or 4 (fused kernels) */
    int32_t prefetch; /* k-levels loaded ahead of use: 2, 4 or 8 */
    int32_t nontemporal; /* read-once inputs and the output use non-temporal
                            loads and stores: 1 on, -1 off, 0 the library's
                            choice (on wherever the variant is compiled) */
    int32_t schedule; /* level loop of the fused kernel: 1 staged (each level
                         is staged, evaluated and eliminated in turn), 2
                         pipelined (hdiff of level s overlaps the elimination
                         of level s-2), 3 pipelined on a persistent grid (a
                         workgroup walks several tiles and requests the next
                         tile's first levels before storing the current
                         one), 4 four lanes per column, partitioned (for
                         grids with few columns; FP32 and FP64, nk >= 8),
                         0 the library's choice (four lanes below 65536
                         columns when no other knob is set) */
    int32_t tile_i;   /* columns per tile row of the pipelined fused kernels:
                         64, 128 or 256 where compiled (0: 64) */
} stencil_config_t;

/* Horizontal diffusion, per level k and interior point (i, j):
 *   lap = 4u - u(i+1) - u(i-1) - u(j+1) - u(j-1)
 *   flx = lap(i+1) - lap(i), set to 0 when flx * (u(i+1) - u(i)) > 0
 *   fly = lap(j+1) - lap(j), set to 0 when fly * (u(j+1) - u(j)) > 0
 *   out = u - coeff * (flx - flx(i-1) + fly - fly(j-1))
 * The paper names this benchmark (Sec. VII-B, Table II: four stencil
 * operators, a min-style limiter) without printing its formula; the limiter is
 * branch-free control flow inside the operator (Sec. IV-E).
 * Inputs: u (halo >= 2 in i and j), coeff (interior read only).
 * Output: out (interior written).  cfg: level, unroll.  Fields whose
 * addressed span is 2 GiB or more run the unfused kernels (library scratch);
 * level INLINE then returns STENCIL_E_UNSUPPORTED. */
int stencil_hdiff(const stencil_field_t *u, const stencil_field_t *coeff,
                  const stencil_field_t *out, const stencil_config_t *cfg, void *stream);

/* Vertical advection of h, per column (i, j):
 *   F(k+1/2) = (w(k) + w(k+1))/2 * (h(k) + h(k+1))/2,  F(-1/2) = F(nk-1/2) = 0
 *   d(k)     = h(k) - dt * (F(k+1/2) - F(k-1/2))
 *   a(k) x(k-1) + b(k) x(k) + c(k) x(k+1) = d(k)   (a(0), c(nk-1) ignored)
 * solved by Thomas forward elimination and back-substitution in double
 * precision whatever the storage dtype (Sec. VII-B names the Thomas algorithm
 * for implicit vertical integration).  All inputs are read on the interior
 * only; the system must be non-singular (e.g. diagonally dominant).
 * Inputs: h, wcon, a, b, c.  Output: x.  Scalar: dt (finite). */
int stencil_vadv(const stencil_field_t *h, const stencil_field_t *wcon,
                 const stencil_field_t *a, const stencil_field_t *b,
                 const stencil_field_t *c, double dt, const stencil_field_t *x,
                 const stencil_config_t *cfg, void *stream);

/* The fused program x = vadv(hdiff(u, coeff), wcon, a, b, c, dt): stencil
 * inlining (Sec. V-A) of the two stages.  With level ORIGINAL it runs one
 * kernel per operator through library-owned device scratch instead.
 * Inputs: u (halo >= 2), coeff, wcon, a, b, c (interior read only).
 * Output: x.  cfg: level, tile_j, prefetch, nontemporal, schedule. */
int stencil_hdiff_vadv(const stencil_field_t *u, const stencil_field_t *coeff,
                       const stencil_field_t *wcon, const stencil_field_t *a,
                       const stencil_field_t *b, const stencil_field_t *c, double dt,
                       const stencil_field_t *x, const stencil_config_t *cfg, void *stream);

/* Reverse mode of stencil_hdiff_vadv for the loss L = sum over the interior
 * of w * x.  With the limiter decisions of the forward pass frozen (their
 * derivative is taken as zero):
 *   lam = T^-T w              (transposed Thomas solve, double)
 *   Fhat(k+1/2) = -dt (lam(k) - lam(k+1))
 *   gh(k) = lam(k) + sum over faces f of k of Fhat(f) * wbar(f) / 2
 *   gwcon(k) = sum over faces f of k of Fhat(f) * hbar(f) / 2
 *   gcoeff = -gh * (flx - flx(i-1) + fly - fly(j-1))
 *   gu = gh + masked transposed flux and Laplacian stencils applied to gh
 * and, optionally, the gradients of the tridiagonal matrix
 *   ga(k) = -lam(k) x(k-1), gb(k) = -lam(k) x(k), gc(k) = -lam(k) x(k+1)
 *                             (ga(0) = gc(K-1) = 0: those entries lie outside
 *                             the matrix)
 * Inputs: u (halo >= 2), coeff, wcon, a, b, c, w (interior read only); x,
 * the forward result x = vadv(hdiff(u)) (interior read only), needed only
 * for ga, gb, gc.
 * Outputs: gu (needs halo >= 2: its interior and 2-cell ring are
 * overwritten; the four 3-cell corner notches of the ring receive 0),
 * gcoeff and gwcon (interior); optionally ga, gb, gc (interior; NULL skips
 * each, and x may be NULL when all three are NULL).  Uses library-owned
 * device scratch: one field-sized plane of the compute type (FP64 storage:
 * two), see the synchronisation rules above.  nk <= 96 and fields below
 * 2 GiB in the compute type (FP32 for bfloat16 storage);
 * STENCIL_E_UNSUPPORTED otherwise.  cfg (may be NULL): schedule 1 evaluates
 * the hdiff adjoint with LDS-staged tiles, 0 with register strips whose
 * neighbours in i come from cross-lane shifts (the default; the same
 * operations, so the same bits); for the strips, tile_j is the rows per
 * strip and prefetch the levels in flight: 4 or 8 rows with 1 or 2 levels,
 * or 12 rows with 1 (FP64: 4 rows); 0 takes the default (12 rows and 1
 * level; FP64 4 and 1); other values STENCIL_E_ARG; the other fields are
 * ignored. */
int stencil_hdiff_vadv_adjoint(const stencil_field_t *u, const stencil_field_t *coeff,
                               const stencil_field_t *wcon, const stencil_field_t *a,
                               const stencil_field_t *b, const stencil_field_t *c, double dt,
                               const stencil_field_t *w, const stencil_field_t *gu,
                               const stencil_field_t *gcoeff, const stencil_field_t *gwcon,
                               const stencil_field_t *x, const stencil_field_t *ga,
                               const stencil_field_t *gb, const stencil_field_t *gc,
                               const stencil_config_t *cfg, void *stream);

/* stencil_hdiff_vadv_adjoint for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, kernels and results, but the scratch is a
 * fixed array of 128 MiB (134217728 bytes) inside the library's code object
 * instead of a growing per-stream buffer, so the call never allocates, frees
 * or synchronises.  Each device the library runs on holds its own copy of
 * the array until the process ends.  The scratch a call needs is one
 * field-sized plane of the compute type (FP64 storage: two), 256-byte
 * aligned per plane (256x256x80 FP64 or 512x512x80 FP32 with a halo of 2
 * fit); a larger call returns STENCIL_E_UNSUPPORTED before anything is
 * enqueued.  All calls on one device share that device's array: calls that
 * overlap in time on one device (on different streams, or from different
 * threads without ordering) race on it and their results are undefined. */
int stencil_hdiff_vadv_adjoint_noalloc(const stencil_field_t *u, const stencil_field_t *coeff,
                                       const stencil_field_t *wcon, const stencil_field_t *a,
                                       const stencil_field_t *b, const stencil_field_t *c, double dt,
                                       const stencil_field_t *w, const stencil_field_t *gu,
                                       const stencil_field_t *gcoeff, const stencil_field_t *gwcon,
                                       const stencil_field_t *x, const stencil_field_t *ga,
                                       const stencil_field_t *gb, const stencil_field_t *gc,
                                       const stencil_config_t *cfg, void *stream);

/* Forward mode of stencil_hdiff_vadv: the tangent dx = J v in the direction
 * v = (du, dcoeff, dwcon, da, db, dc), with the limiter decisions of the
 * forward pass (a zeroed flux has a zero tangent):
 *   dh = du - dcoeff * div - coeff * ddiv   (ddiv: div of the masked fluxes
 *                                             of lap(du))
 *   dF(k+1/2) = dwbar * hbar + wbar * dhbar, zero at the bottom and top
 *   dd(k) = dh(k) - dt (dF(k+1/2) - dF(k-1/2))
 *   T dx = dd - (da(k) x(k-1) + db(k) x(k) + dc(k) x(k+1))   (double)
 * which follows from T x = d by differentiating every stage (Sec. V-A's
 * inlining applied to the derivative: one fused kernel).
 * Inputs: u (halo >= 2), coeff, wcon, a, b, c (interior read only); x, the
 * forward result (interior; needed only when da, db or dc is given, else
 * may be NULL); the tangents du (halo >= 2 when given), dcoeff, dwcon, da,
 * db, dc (interior), each NULL for a zero tangent.  Output: dx (interior).
 * nk <= 96 (STENCIL_E_UNSUPPORTED beyond).  cfg is unused (may be NULL). */
int stencil_hdiff_vadv_jvp(const stencil_field_t *u, const stencil_field_t *coeff,
                           const stencil_field_t *wcon, const stencil_field_t *a,
                           const stencil_field_t *b, const stencil_field_t *c, double dt,
                           const stencil_field_t *x, const stencil_field_t *du,
                           const stencil_field_t *dcoeff, const stencil_field_t *dwcon,
                           const stencil_field_t *da, const stencil_field_t *db,
                           const stencil_field_t *dc, const stencil_field_t *dx,
                           const stencil_config_t *cfg, void *stream);

/* ---- batched timestep program ------------------------------------------ */

/* Stages of a timestep program, applied in this order to every field. */
enum {
    STENCIL_STAGE_HDIFF = 1,
    STENCIL_STAGE_VADV = 2,
    STENCIL_STAGE_VDIFF = 4,  /* y(k) = x(k) + kappa (x(k+1) - 2x(k) + x(k-1)),
                                 zero flux through the bottom and top faces */
    STENCIL_STAGE_HGRAD = 8,  /* z = y - beta_h ((y(i+1)-y(i-1))/2 + (y(j+1)-y(j-1))/2)
                                 - beta_v Dk y, Dk centred inside the column and
                                 one-sided at its two ends */
    STENCIL_STAGE_VDIFF_IMPLICIT = 16 /* in place of VDIFF: y solves
                                 y(k) - kappa (y(k+1) - 2y(k) + y(k-1)) = x(k),
                                 zero flux through the bottom and top faces (a
                                 second tridiagonal solve per column, FP64) */
};

/* One subdomain: nfields prognostic fields sharing coeff, wcon, a, b, c. */
typedef struct {
    stencil_field_t coeff, wcon, a, b, c;
    int32_t nfields;
    const stencil_field_t *u;  /* nfields inputs */
    const stencil_field_t *z;  /* nfields outputs */
} stencil_subdomain_t;

/* A timestep program over independent subdomains of different sizes
 * (a stencil program with eager program-level control, Sec. IV-E).
 * stages: HDIFF|VADV, HDIFF|VADV|VDIFF or HDIFF|VADV|VDIFF|HGRAD, or either
 * of the last two with VDIFF_IMPLICIT in place of VDIFF.
 * Shape inference (Sec. V-B) derives the halos: with HGRAD the earlier stages
 * run on the interior grown by one cell, so u needs halo >= 3 and the shared
 * coefficient fields halo >= 1; otherwise u needs 2 and the coefficients 0. */
typedef struct {
    int32_t nsub;
    const stencil_subdomain_t *sub;
    int32_t stages;
    int32_t flags;  /* STENCIL_PROGRAM_* */
    double dt, kappa, beta_h, beta_v;
} stencil_program_t;

enum {
    STENCIL_PROGRAM_GRAPH = 1,    /* capture the launches in a hipGraph cached on
                                     the program signature and replay it */
    STENCIL_PROGRAM_AUTOTUNE = 2, /* time the candidate kernel configurations on
                                     first use (synchronises the stream once) */
    STENCIL_PROGRAM_STAGED = 4    /* only the staged level loop for the column
                                     stages (same results; for comparisons) */
};

/* Runs the program.  All fields of one subdomain share dtype, extents and
 * strides; subdomains may differ in size and layout.  Output z of each field
 * is written on its interior.  The plan, the tuned variant, the scratch and
 * the graph are cached on the program's full signature (device, stream,
 * stages, flags, parameters and every descriptor, compared exactly); the
 * cache holds the 16 most recently used programs.  Programs on the same
 * stream whose scratch has the same size share it.  See the
 * synchronisation rules above for the first run of a signature. */
int stencil_program_run(const stencil_program_t *prog, void *stream);

/* ---- run-time compiled stencil programs ---------------------------------- */

/* The stencil-program front end (Python, paper_2005_13014_amd/frontend.py)
 * turns a program of stencil applies into one inlined, unrolled kernel whose
 * extents and strides are compile-time constants (Sec. IV-B), as HIP source.
 * stencil_rtc_compile builds it for gfx950 with hipRTC (the library's own
 * code-generation flags) and returns an opaque handle owned by the caller
 * (release with stencil_rtc_release).  source: NUL-terminated HIP source;
 * kernel_name: its extern "C" __global__ function.  Compile errors return
 * STENCIL_E_ARG with the compiler log in stencil_last_error(). */
int stencil_rtc_compile(const char *source, const char *kernel_name, void **handle);

/* Launches a compiled kernel on `stream`: grid[3] workgroups of block[3]
 * threads (at most 1024), args[q] pointing at the q-th kernel argument's
 * value (hipModuleLaunchKernel convention).  An empty grid is a no-op. */
int stencil_rtc_launch(void *handle, const uint32_t grid[3], const uint32_t block[3], void **args,
                       void *stream);

/* Unloads a compiled kernel; NULL is a no-op. */
int stencil_rtc_release(void *handle);

/* ---- horizontal domain decomposition ------------------------------------ */

/* A grid split into px x py rectangles in (i, j) -- the shares that separate
 * GPUs would own -- held here as separate halo-padded fields on one device.
 * vadv and its Thomas solve are column-local; only horizontal diffusion reads
 * across a share's edge, through the u halo whose width shape inference
 * derives (Sec. V-B: 2 for hdiff, 3 for the timestep chain).  The paper
 * itself runs on one GPU; the decomposition is this library's.
 * shares: px * py descriptors, share (p, q) at shares[p + px q], p along i
 * and q along j; share (p, q)'s interior follows share (p - 1, q)'s in i and
 * share (p, q - 1)'s in j.  All shares have one dtype and nk; shares in one
 * column p have the same ni, shares in one row q the same nj; strides may
 * differ.  Shares must not overlap (STENCIL_E_ALIAS).  width: cells
 * exchanged (1 <= width; every share's halo at least width wide and, where
 * it has neighbours in that direction, its interior too).  1 <= px * py <= 64.
 * The halo blocks on the outer boundary of the decomposition are never
 * written: they hold the whole grid's halo data. */

/* Fills each share's halo blocks toward its up to eight neighbours (edges and
 * corners, width cells deep) with the neighbours' interior cells at the same
 * grid position: afterwards every share holds, on its interior and halo, what
 * the undivided grid holds there.  One launch on `stream`. */
int stencil_halo_exchange(const stencil_field_t *shares, int32_t px, int32_t py, int32_t width,
                          void *stream);

/* The transpose of stencil_halo_exchange, for gradients: every interior cell
 * that the exchange copies into neighbours' halos receives the sum of those
 * halo cells (added to its own value, in a fixed order of directions, in the
 * compute type).  Applied to per-share gradients with respect to u (interior
 * plus halo ring, as stencil_hdiff_vadv_adjoint writes them), it yields the
 * undivided grid's gradient on every share's interior, and on the outer
 * boundary's halo cells.  Halos are read, not cleared.  One launch. */
int stencil_halo_accumulate(const stencil_field_t *shares, int32_t px, int32_t py, int32_t width,
                            void *stream);

/* ---- library management and measurement --------------------------------- */

/* Message describing the calling thread's last nonzero return code. */
const char *stencil_last_error(void);

/* Device memory the library holds on all devices (scratch buffers and
 * cached programs), in bytes; *programs (if not NULL) receives the number
 * of cached programs. */
int64_t stencil_held_memory(int32_t *programs);

/* STENCIL_ABI_VERSION of the loaded library. */
int stencil_abi_version(void);

/* Releases all library-owned device memory and cached graphs.  The library
 * stays usable; resources are re-created on demand.  Must not race with
 * calls in flight on other threads. */
void stencil_shutdown(void);

/* Bandwidth probe: copies nbytes (a multiple of 16, both pointers 16-byte
 * aligned) from src to dst with a plain streaming kernel.  Measures the
 * achievable HBM copy rate that the stencil kernels are compared against. */
int stencil_probe_copy(const void *src, void *dst, int64_t nbytes, void *stream);

/* Bandwidth probe: reads nbytes (a multiple of 16, src 16-byte aligned) and
 * folds them into per-lane XOR checksums; writes one 32-bit word (the
 * checksum) to sink only if the checksum of some lane equals key (pass a key
 * the data cannot produce: then nothing is written).  Measures the achievable
 * HBM read rate. */
int stencil_probe_read(const void *src, int64_t nbytes, uint32_t key, void *sink, void *stream);

/* Bandwidth probe: reads nsrc (1 .. 8) arrays of nbytes each (a multiple of
 * 16, pointers 16-byte aligned) and writes their element-wise XOR to dst
 * (nbytes, not overlapping any source), all streamed non-temporally.  With
 * six sources it has the traffic mix of the fused kernel: six field streams
 * in, one out. */
int stencil_probe_streams(const void *const *src, int32_t nsrc, void *dst, int64_t nbytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* STENCIL_H */
