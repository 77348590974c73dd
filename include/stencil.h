/*
 * stencil.h -- C ABI of the MI355X stencil-sweep library (libstencil.so).
 *
 * The library runs structured-grid stencil sweeps -- the data-parallel
 * innermost loop bodies that ACC Saturator (arXiv 2306.13002) rewrites --
 * as hand-written HIP kernels for gfx950, each in two forms:
 *
 *   STENCIL_PLAIN      the loop body translated directly: one thread per
 *                      point, every operand loaded from memory, terms added
 *                      in the written order (the paper's "original" code);
 *   STENCIL_SATURATED  the body after the paper's rewrites (Sec. "Rewriting
 *                      Rules", Sec. "Code Generation"): common subexpressions
 *                      shared, shared coefficients factored, FMA chains,
 *                      constants folded, temporaries kept in registers, loads
 *                      issued early ("bulk load") and reused along the z axis
 *                      through a register queue and LDS-staged xy tiles.
 *
 * Memory layout (every kind): a padded grid, x contiguous.  Element (x,y,z)
 * of the padded grid is at  base + z*pitch_z + y*pitch_y + x  (elements);
 * the interior point (i,j,k), 0 <= i < n[0], ... sits at (i+r, j+r, k+r)
 * where r is the halo width.  pitch_y >= n[0]+2r, pitch_z >= pitch_y*(n[1]+2r);
 * 0 selects the dense pitch.  2-D kinds ignore z.  The halo holds boundary
 * values; under STENCIL_BC_DIRICHLET it is never written.
 *
 * Ownership: every grid pointer is a DEVICE pointer owned by the caller; the
 * library never frees or reallocates caller memory.  Arrays in the descriptor
 * (coef, tap_off, tap_cid) are HOST pointers, copied at plan time.  A plan
 * owns only small device buffers (residual partials, tap tables, graphs),
 * released by stencil_destroy.
 *
 * Errors: every entry returns a stencil_status.  All validation happens
 * before anything is enqueued; on error nothing is enqueued, output handles
 * are left NULL and stencil_last_error() (thread-local, never NULL)
 * describes the failure.  Launch failures map to STENCIL_E_DEVICE.  The
 * library never aborts and prints nothing unless STENCIL_LOG is set.
 *
 * Streams: a `stream` argument is a hipStream_t passed as void* (NULL = the
 * null stream).  stencil_run is asynchronous; stencil_residual synchronizes
 * the stream it is given, which must be the stream of the preceding run (or
 * ordered after it).  Calls that share one plan must not overlap.
 */
#ifndef STENCIL_H
#define STENCIL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stencil_plan_s *stencil_plan_t;

typedef enum {
    STENCIL_OK = 0,
    STENCIL_E_INVAL = -1,       /* bad descriptor or argument */
    STENCIL_E_UNSUPPORTED = -2, /* valid but not offered (kind/dtype/bc/tile combination) */
    STENCIL_E_NOMEM = -3,       /* host or device allocation failed */
    STENCIL_E_DEVICE = -4,      /* no usable GPU, or a HIP call/launch failed */
    STENCIL_E_STATE = -5        /* call out of order (e.g. residual before any sweep) */
} stencil_status;

/* Stencil kinds.  Definitions per interior point (src -> dst):
 *
 * HEAT2D5   dst = c[0]*u + c[1]*u(-x) + c[1]*u(+x) + c[1]*u(-y) + c[1]*u(+y);
 *           r = 1, F64; coef = {centre, neighbour}.  Jacobi heat sweep, the
 *           paper's Jacobi class ("ostencil" in its SPEC ACCEL table).
 *           PLAIN with zblock k > 1 (Dirichlet only) fuses up to k sweeps per
 *           launch: each block loads its output tile and a k-cell ring into
 *           LDS and runs the sweeps there (the ring recomputed by every block
 *           that needs it), with the plain body's operands and order, so the
 *           grid equals k single-sweep launches bit for bit (the residual is
 *           the same sum taken in another order).  A run of T sweeps makes
 *           ceil(T/k) launches, the first doing T mod k when that is not 0;
 *           each launch writes its destination's boundary ring, so the run
 *           makes no separate halo copy (fields[1] ends with the same ring).
 * HEAT3D7   the same with -z, +z added; r = 1, F64.
 * POISSON19 19-point variable-coefficient pressure relaxation (the halo-3D
 *           CFD class of the paper's NPB/SPEC tables), F32 storage, FP64
 *           arithmetic, r = 1, with (i,j,k) = (x,y,z) and every coefficient
 *           read at the point itself:
 *             s0 = a0*p(i+1,j,k) + a1*p(i,j+1,k) + a2*p(i,j,k+1)
 *                + b0*(p(i+1,j+1,k) - p(i+1,j-1,k) - p(i-1,j+1,k) + p(i-1,j-1,k))
 *                + b1*(p(i,j+1,k+1) - p(i,j-1,k+1) - p(i,j+1,k-1) + p(i,j-1,k-1))
 *                + b2*(p(i+1,j,k+1) - p(i-1,j,k+1) - p(i+1,j,k-1) + p(i-1,j,k-1))
 *                + c0*p(i-1,j,k) + c1*p(i,j-1,k) + c2*p(i,j,k-1) + wrk1
 *             ss = (s0*a3 - p)*bnd ;  p' = p + omega*ss ;  residual = sum ss^2.
 *           Its saturated kernels (SATURATED, SATURATED_T2) address a plane
 *           with 32-bit byte offsets: pitch_z*4 above 0xFFFFFFF0 bytes is
 *           E_UNSUPPORTED for them and makes AUTO choose PLAIN.
 * WAVE25    radius-4 star, second order in time (leapfrog), F64, r = 4:
 *             L(u) = sum over x,y,z of [c0*u + sum_{q=1..4} c_q*(u(+q) + u(-q))]
 *             u_next = 2u - u_prev + vsq*L(u);   coef = {c0,c1,c2,c3,c4}.
 *           Its SATURATED kernel addresses a plane with 32-bit byte offsets:
 *           pitch_z*8 above 0xFFFFFFF0 bytes is E_UNSUPPORTED for SATURATED
 *           and makes AUTO choose PLAIN, which takes every plane size.
 * GENERIC   u'(x) = sum_t coef[cid_t] * u(x + delta_t), 3-D, radius 1..4,
 *           F32 or F64, taps given by tap_off/tap_cid.  Its saturated
 *           kernels are generated and launched through the module API,
 *           which limits them to ny, nz <= 65535 (E_UNSUPPORTED above;
 *           PLAIN takes every extent up to 2^24).
 */
typedef enum {
    STENCIL_HEAT2D5 = 1,
    STENCIL_HEAT3D7 = 2,
    STENCIL_POISSON19 = 3,
    STENCIL_WAVE25 = 4,
    STENCIL_GENERIC = 5
} stencil_kind;

typedef enum { STENCIL_F32 = 1, STENCIL_F64 = 2 } stencil_dtype; /* storage type */
/* PLAIN and SATURATED are the two forms (see the top of this file); AUTO lets
 * the plan choose between them and, where a kind offers them, the multi-sweep
 * saturated forms below (FIXED tuning: SATURATED).  The per-point ablation forms of the paper's
 * evaluation (Sec. Evaluation: CSE, CSE+SAT, CSE+BULK, ACCSAT) exist for WAVE25
 * and POISSON19, one thread per point with every operand from memory (CSE is
 * PLAIN: no address is loaded twice in these bodies):
 *   CSE_SAT       the saturated arithmetic, loads where first used;
 *   CSE_BULK      all loads first in ascending address order, plain arithmetic
 *                 (bit-identical to PLAIN);
 *   ACCSAT_POINT  both (bit-identical to CSE_SAT and to SATURATED, which adds
 *                 the z-streaming register queue and LDS tile).
 * They use the plain launch shapes and are never picked by the tuners.
 *
 * SATURATED_T2 (POISSON19 and HEAT3D7, Dirichlet; single and batched plans):
 * the saturated form with two sweeps per pass over memory -- the first sweep
 * is recomputed on a one-cell ring around each tile so the second can follow
 * it plane by plane, and every input stream is read once per two sweeps.
 * Bit-identical to SATURATED at the same tile, z-block and tile map (an odd
 * sweep count starts with one SATURATED sweep).  EXHAUSTIVE and MODEL tuning
 * of AUTO consider it beside PLAIN and SATURATED (the model's form feature
 * tells the forms apart; its target is the time per sweep in every form).
 *
 * SATURATED_T3 (HEAT3D7, Dirichlet; single and batched plans): three sweeps
 * per pass, one thread per column of a region two cells wider on every side
 * than the output tile (tile_x, tile_y = 28 x 28, 28 x 20, 28 x 12 or 60 x 12);
 * the first and second sweeps are recomputed on the ring, and every input
 * stream is read once per three sweeps.  Bit-identical to SATURATED (a sweep
 * count that is not a multiple of three starts with one launch of the
 * remainder's sweeps in the same form).  EXHAUSTIVE and MODEL tuning of AUTO
 * weigh it (the model's form feature tells the four forms apart). */
typedef enum {
    STENCIL_PLAIN = 0,
    STENCIL_SATURATED = 1,
    STENCIL_AUTO = 2,
    STENCIL_CSE_SAT = 3,
    STENCIL_CSE_BULK = 4,
    STENCIL_ACCSAT_POINT = 5,
    STENCIL_SATURATED_T2 = 6,
    STENCIL_SATURATED_T3 = 7
} stencil_variant;
/* How a plan picks variant and tile when variant == AUTO or a tile field is 0:
 * FIXED uses library defaults; EXHAUSTIVE times every candidate on the device
 * (results cached per size class); MODEL asks the learned cost model. */
typedef enum { STENCIL_TUNE_FIXED = 0, STENCIL_TUNE_EXHAUSTIVE = 1, STENCIL_TUNE_MODEL = 2 } stencil_tune;
/* DIRICHLET: halo fixed.  PERIODIC (heat kinds): before every sweep the halo
 * is filled from the opposite side of the interior (the halo is written). */
typedef enum { STENCIL_BC_DIRICHLET = 0, STENCIL_BC_PERIODIC = 1 } stencil_bc;

typedef struct {
    uint32_t struct_size;   /* = sizeof(stencil_desc) (ABI versioning) */
    int32_t kind;           /* stencil_kind */
    int32_t dtype;          /* stencil_dtype */
    int32_t variant;        /* stencil_variant */
    int32_t tune;           /* stencil_tune */
    int32_t bc;             /* stencil_bc */
    int32_t ndim;           /* 2 (HEAT2D5) or 3 */
    int32_t radius;         /* halo width: 1 (heat, poisson19), 4 (wave25), 1..4 (generic) */
    int64_t n[3];           /* INTERIOR extents; n[0] = x (contiguous); n[2] ignored for 2-D */
    int64_t pitch_y;        /* elements per padded row; 0 = n[0]+2r */
    int64_t pitch_z;        /* elements per padded plane; 0 = pitch_y*(n[1]+2r) */
    const double *coef;     /* host: HEAT {centre, neighbour}; WAVE25 {c0..c4};
                               GENERIC one value per coefficient id; POISSON19 unused */
    int32_t n_coef;
    int32_t n_taps;         /* GENERIC: number of taps */
    const int32_t *tap_off; /* GENERIC: n_taps triples (dx,dy,dz), |d| <= radius */
    const int32_t *tap_cid; /* GENERIC: coefficient id per tap, 0 <= id < n_coef */
    double omega;           /* POISSON19 relaxation factor */
    int32_t tile_x;         /* threads along x per block; 0 = let the plan decide */
    int32_t tile_y;         /* rows per block tile; 0 = let the plan decide */
    int32_t zblock;         /* z planes per block (saturated forms); 0 = let the plan decide.
                               HEAT2D5 PLAIN: sweeps fused per launch (1..16); with more than one,
                               tile_x = tile_y is the square output tile: 16 or 32 (default 32), or
                               any size with tile_x + 2 * zblock <= 32 (one region cell per thread) */
    int32_t tile_map;       /* saturated forms, order of blocks over tiles: 0 = let the plan decide,
                               1 = natural (x fastest), 2 = XCD-chunked (each of the 8 XCDs gets one
                               contiguous run of tiles, so neighbours share an L2) */
} stencil_desc;

/* Build a plan: validate d (host only, no device call before validation
 * passes), choose variant and tile, allocate the plan's small buffers.
 * Paper: the choice it stands for is the paper's -- run the loop body as
 * written or in its rewritten form (Sec. Methodology Overview: the tool
 * swaps the rewritten kernel into the directive code at compile time). 
 * On success *out is a new plan; on error *out = NULL. */
stencil_status stencil_plan(const stencil_desc *d, stencil_plan_t *out);

/* Build one plan over `count` independent grids (HEAT3D7, Dirichlet), run
 * together (a serving extension; the paper defines no batched launch): problems are grouped into size classes by their largest
 * interior edge (<= 64, then buckets of 32); each class gets one form and
 * launch shape -- when ds[0].tune is not FIXED and ds[0] leaves the form or
 * shape open, by timing the class's own work-list kernel over all its
 * problems (on scratch grids the library allocates for the tuning and frees;
 * on E_NOMEM for those, by tuning its largest problem alone), else the
 * defaults or ds[0]'s fields -- and a work-list kernel over (problem,
 * tile) items, one block per item.  stencil_batch_problem_config reports each
 * problem's class and shape.  stencil_run on a
 * batch plan takes fields = {p0.fields[0], p0.fields[1], p1.fields[0], ...}
 * and replays one hipGraph per (iterations, field pointers): halo copies, the
 * class chains as parallel branches, tail copies.  Each problem's result is
 * bit-identical to its own single plan with the same form and shape. */
stencil_status stencil_plan_batch(const stencil_desc *ds, int32_t count, stencil_plan_t *out);

/* Run `iterations` sweeps asynchronously on `stream`.  Paper: one sweep is
 * the data-parallel loop nest whose innermost body the paper rewrites (Sec.
 * Program Representation, E-Graph Creation), in the plain form or after the
 * rewrites of Sec. Optimization with Saturation and Code Generation.
 * fields (device pointers):
 *   HEAT*, GENERIC, POISSON19: fields[0] = state (in/out), fields[1] = a
 *     scratch grid of the same layout; the library first copies the halo of
 *     fields[0] into fields[1] and ping-pongs; the result ends in fields[0].
 *   WAVE25: fields[0] = u^{n-1}, fields[1] = u^n; each step overwrites the
 *     interior of the older level in place, so after T steps the newest
 *     level u^{n+T} is in fields[T % 2 == 1 ? 0 : 1] and the other holds
 *     u^{n+T-1}.  Each buffer keeps its own halo.
 * coef_arrays (device pointers): POISSON19: 12 F32 grids of the state's
 *   layout in the order a0 a1 a2 a3 b0 b1 b2 c0 c1 c2 bnd wrk1;
 *   WAVE25: {vsq} (F64 grid); others: NULL.
 * Every pointer must be aligned to its element size.  iterations == 0 is a
 * no-op.  The residual of the last sweep is kept for stencil_residual.
 * With graphs enabled (stencil_plan_use_graphs), a run that repeats the
 * previous run's iteration count and pointers is captured into HIP graphs
 * (halo copy, sweeps, final copy) and replayed from them while the same
 * runs keep arriving: the same kernels and results. */
stencil_status stencil_run(stencil_plan_t p, void *const *fields, const void *const *coef_arrays,
                           int32_t iterations, void *stream);

/* Allocation-free run, for callers that cannot allocate device or host
 * memory during the call: code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation.  The same sweeps, kernels and results as
 * stencil_run (eagerly; graph replay is not used), but the per-block residual
 * partials of the last sweep and the first pass of their reduction go to a
 * fixed scratch array inside the library (one per GPU, 2^17 + 256 doubles,
 * about 1 MiB, resident until the process ends), and the FP64 residual --
 * the value stencil_residual would report -- is written to residual_dev, a
 * DEVICE pointer owned by the caller (8 bytes, 8-byte aligned; NULL skips the
 * reduction).  Only kernel launches are enqueued on `stream`; the call never
 * synchronizes, allocates nothing and leaves the plan's own residual state
 * (stencil_residual) as the last stencil_run left it.
 * Limits: a plan whose sweep launch has more than 2^17 blocks (see
 * stencil_plan_config; small tiles on large grids), batched plans and GENERIC
 * plans running generated saturated kernels: E_UNSUPPORTED, checked before
 * anything is enqueued.  Every call on one GPU shares that GPU's scratch and
 * it keeps the last call's contents (each call writes every slot it reads):
 * calls that overlap on one GPU -- concurrent streams, threads or graph
 * replays -- race and must be serialized by the caller. */
stencil_status stencil_run_noalloc(stencil_plan_t p, void *const *fields, const void *const *coef_arrays,
                                   int32_t iterations, double *residual_dev, void *stream);

/* Residual of the last sweep of the last run, FP64: sum over the interior of
 * (new - old)^2 (POISSON19: sum of ss^2).  Paper: not defined there (it
 * rewrites loop bodies and reports kernel times); this is the FP64 sum of
 * squared updates a Jacobi-type solver checks for convergence.  Reduces the per-block partials in
 * a fixed order (bitwise reproducible) into a pinned host word of the plan
 * and synchronizes `stream`.  E_STATE if no sweep has run on this plan. */
stencil_status stencil_residual(stencil_plan_t p, double *host_out, void *stream);

/* Per-problem residuals of the last run of a batch plan (count = number of
 * problems; a single plan takes count = 1).  stencil_residual on a batch
 * plan returns their sum in problem order.  Synchronizes `stream`. */
stencil_status stencil_residuals(stencil_plan_t p, double *host_out, int32_t count, void *stream);

/* Chosen configuration of a plan (any output pointer may be NULL).
 * tile_map is reported as 1 (natural) or 2 (XCD-chunked). */
stencil_status stencil_plan_config(stencil_plan_t p, int32_t *variant, int32_t *tile_x, int32_t *tile_y,
                                   int32_t *zblock, int32_t *tile_map);

/* Size class and launch configuration of problem `problem` (0-based, in the
 * order given to stencil_plan_batch) of a batch plan; any output pointer may
 * be NULL.  size_class numbers the plan's non-empty classes from the
 * smallest edge bucket up; variant, tile and z-block are that class's.
 * E_INVAL if p is not a batch plan or problem is out of range. */
stencil_status stencil_batch_problem_config(stencil_plan_t p, int32_t problem, int32_t *size_class, int32_t *variant,
                                            int32_t *tile_x, int32_t *tile_y, int32_t *zblock);

/* Graph replay of repeated runs for a single plan (off by default; GENERIC
 * and batched plans: E_UNSUPPORTED, batches always run as graphs).  One
 * graph launch replaces a launch per sweep, which saves host time when the
 * caller cannot stay ahead of the GPU; on MI355X the graph's sweeps run no
 * faster than the same launches on a stream.  A capture failure leaves the
 * plan running eagerly. */
stencil_status stencil_plan_use_graphs(stencil_plan_t p, int32_t enable);

/* Iteration count of the run a single plan replays from captured graphs (see
 * stencil_run), or 0 if it holds none. */
stencil_status stencil_plan_graph(stencil_plan_t p, int32_t *iterations);

/* Sweep timing.  When enabled, stencil_run records HIP events on its stream
 * around its sweep launches (after the halo copy, before any tail copy);
 * stencil_profile_read waits for the last run's end event and returns its
 * elapsed milliseconds and sweep count. */
stencil_status stencil_profile_enable(stencil_plan_t p, int32_t enable);
stencil_status stencil_profile_read(stencil_plan_t p, double *sweep_ms, int32_t *sweeps);

/* ---- cost model (learned launch-shape picker, used by STENCIL_TUNE_MODEL) ----
 * The model is an FP32 MLP 24 -> 64 -> 64 -> 1 (ReLU) predicting the log of
 * seconds per sweep from 24 static features of a (stencil, form, shape).  A
 * model is 24 feature means, 24 standard deviations and 5825 parameters (W1
 * 64x24 row-major by unit, b1, W2 64x64, b2, w3, b3).  MODEL tuning loads a
 * JSON model file ("mean", "std", "params" arrays) from STENCIL_COST_MODEL or
 * cost_model.json beside libstencil.so, scores every candidate on the device
 * and keeps the lowest prediction; without a usable file it falls back to
 * exhaustive tuning. */

/* The candidates the tuners consider for d (fields of d left 0 / AUTO are
 * open).  Writes up to max rows of 5 ints (variant, tile_x, tile_y, zblock,
 * tile_map) to out (host) and the total count to *n.  Host only. */
stencil_status stencil_candidates(const stencil_desc *d, int32_t max, int32_t *out, int32_t *n);

/* The 24 features of d run with one candidate, into out[24] (host).  Host only. */
stencil_status stencil_features(const stencil_desc *d, int32_t variant, int32_t tile_x, int32_t tile_y,
                                int32_t zblock, int32_t tile_map, float *out);

/* Train on the device: X (n x 24 raw features, row-major, host), y (n log
 * seconds, host), init (5825 initial parameters, host).  Features are
 * standardized with the rows' mean and standard deviation (0 -> 1), then
 * `epochs` full-batch Adam steps (lr; beta1 0.9, beta2 0.999, eps 1e-8) on the
 * mean squared error run as a replayed hipGraph of one epoch.  Writes the
 * model (24 + 24 + 5825 floats) to model_out and, if loss_out is not NULL,
 * the loss before each step.  Synchronizes `stream`. */
stencil_status stencil_mlp_train(const float *X, const float *y, int32_t n, const float *init, int32_t epochs,
                                 float lr, float *model_out, float *loss_out, void *stream);

/* Predictions (log seconds) of a model for n rows of raw features (host in,
 * host out).  Synchronizes `stream`. */
stencil_status stencil_mlp_predict(const float *model, const float *X, int32_t n, float *y_out, void *stream);

/* GENERIC saturated plans run kernels generated for their taps and compiled
 * with hipRTC when the plan is made (one per tile shape; cached per process
 * and, if STENCIL_RTC_CACHE names a directory, as code objects there;
 * STENCIL_GENERIC_TABLE=1 selects the precompiled table-driven kernel).
 * stencil_prepare compiles, concurrently, every generated kernel the tuners
 * may try for d so later plans find them cached.  Other kinds: no-op. */
stencil_status stencil_prepare(const stencil_desc *d);

/* Streaming kernel of known traffic: the HBM ceiling of the sweeps' access
 * shapes (and the known-size kernel that calibrates byte counters).  It is a
 * measurement aid beside the sweeps, defined by the bytes it moves:
 *   op 0: d[i] = a[i]                          (8 B read, 8 B written per element)
 *   op 1: d[i] = fma(c[i], a[i], 2*a[i] - b[i])  (24 B read, 8 B written) --
 *         the leapfrog step's shape: three FP64 grids read, one written, and
 *         d may be b (written in place, as WAVE25 overwrites u^{n-1}).
 * a, b, c, d: DEVICE pointers to n doubles each (b, c unused by op 0), owned
 * by the caller, aligned to 8*width bytes; d must not overlap a or c, nor b
 * unless d == b.  width: doubles per lane and access (1: 8-byte loads and
 * stores, 2: 16-byte).  flags: bit 0 nontemporal loads, bit 1 nontemporal
 * stores.  grid: blocks of 256 threads in a grid-stride loop; 0 = enough
 * blocks for one element group per thread.  Asynchronous on `stream`;
 * E_INVAL for bad arguments (nothing enqueued), E_DEVICE for no GPU or a
 * failed launch. */
stencil_status stencil_stream(int32_t op, const double *a, const double *b, const double *c, double *d, int64_t n,
                              int32_t width, int32_t flags, int32_t grid, void *stream);

/* Release a plan and its buffers (waits for nothing; the caller must not
 * destroy a plan while its work is in flight).  NULL is accepted.
 * (Library plumbing; no paper passage.) */
stencil_status stencil_destroy(stencil_plan_t p);

/* Description of the last error on this thread; never NULL.  (Library
 * plumbing; no paper passage.) */
const char *stencil_last_error(void);

/* Library version string, e.g. "0.1.0 gfx950". */
const char *stencil_version(void);

#ifdef __cplusplus
}
#endif

#endif /* STENCIL_H */
