/*
 * stencil.h -- C ABI of the MI355X (gfx950) engine for iterated stencil sweeps.
 *
 * The operation (Section 1 of Li et al., "An Efficient Vectorization Scheme
 * for Stencil Computation", arXiv 2103.08825): a d-dimensional grid is
 * updated T times; at each step every point becomes a weighted sum of its
 * order-r neighbourhood at the previous step (2r+1 points per direction),
 * with the time loop outermost.  Section 3.3 fixes Jacobi semantics (the new
 * values are computed from the old ones only, two arrays) and introduces
 * computing several time steps per pass over the data (unroll-and-jam of the
 * time loop); this library does the GPU analogue: k fused steps per kernel
 * launch.
 *
 *   u_{t+1}[x] = sum_j c_j * g(u_t, x + o_j)
 *   g(u, y)    = u[y] inside the grid; 0 outside (STENCIL_BC_ZERO);
 *                u[y mod N] per axis (STENCIL_BC_PERIODIC)
 *
 * Offsets.  STENCIL_STAR = {0} U {+-j e_i : 1 <= j <= r}, 2*d*r+1 points;
 * STENCIL_BOX = {o : max_i |o_i| <= r}, (2r+1)^d points.
 * Coefficient order ("canonical"): the offset tuples (o_0, ..., o_{d-1}) in
 * lexicographic order, axis 0 most significant, each component ascending
 * from -r to +r.  stencil_offsets() lists it.
 * Layout.  Grids are dense row-major arrays, shape given slowest axis first,
 * the last axis unit-stride, element type the plan's dtype.
 * Precision.  STENCIL_F64 computes in FP64.  STENCIL_F32 stores and
 * accumulates in FP32 with coefficients rounded to FP32.  STENCIL_BF16 and
 * STENCIL_F16 store 16-bit values, load them into FP32, accumulate in FP32
 * with FP32 coefficients and round to nearest even on every store to memory;
 * values kept on chip between fused steps stay FP32.
 *
 * Status codes.  Every function returning int returns STENCIL_OK (0) or a
 * negative code, never aborts and never throws.  stencil_last_error() gives a
 * message for the calling thread's last failure.
 *
 * Asynchrony and ownership.  Device pointers are caller-owned HIP device
 * memory.  Run calls enqueue work on `stream` (a hipStream_t; NULL = the
 * null stream) and return; argument errors are reported synchronously, device
 * faults at the caller's next synchronisation.  A plan owns its ping-pong
 * scratch field(s), allocated on the current HIP device at the first run (or
 * by stencil_plan_prepare); one plan must not be used by two streams at once.
 */
#ifndef STENCIL_H
#define STENCIL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STENCIL_VERSION 1
#define STENCIL_MAX_DIM 3
#define STENCIL_MAX_RADIUS 4

enum stencil_status {
    STENCIL_OK = 0,
    STENCIL_E_INVALID = -1,     /* bad argument */
    STENCIL_E_UNSUPPORTED = -2, /* valid but not implemented (e.g. 16-bit adjoint) */
    STENCIL_E_NOMEM = -3,       /* device or host allocation failed */
    STENCIL_E_DEVICE = -4       /* a HIP call failed */
};
enum stencil_kind { STENCIL_STAR = 0, STENCIL_BOX = 1 };
enum stencil_bc { STENCIL_BC_ZERO = 0, STENCIL_BC_PERIODIC = 1 };
enum stencil_dtype { STENCIL_F64 = 0, STENCIL_F32 = 1, STENCIL_BF16 = 2, STENCIL_F16 = 3 };

/* How stencil_run executes (stencil_opts.method). */
enum stencil_method {
    STENCIL_METHOD_AUTO = 0,    /* fused when a fused kernel fits the plan, else plain */
    STENCIL_METHOD_PLAIN = 1,   /* one time step per launch (the fused kernel with k = 1) */
    STENCIL_METHOD_FUSED = 2,   /* k time steps per launch */
    STENCIL_METHOD_GENERIC = 3, /* reference kernel: any d, r <= 4, one step per launch,
                                   every neighbour read straight from memory */
    STENCIL_METHOD_TESSELLATE = 4 /* 3D only: k steps per pass without recomputing a y
                                   halo, as the two stages of the tessellated tiling of
                                   Section 3.4 (trapezoids along y, then the inverted
                                   trapezoids around the cuts, in two launches; the
                                   intermediate rows the second stage needs go through
                                   a plan-owned slope buffer).  Same results as
                                   STENCIL_METHOD_FUSED, bit for bit.  Needs a y extent
                                   of at least 2(k+1)r; STENCIL_E_UNSUPPORTED when no
                                   tessellated kernel is compiled for the stencil. */
};

typedef struct stencil_plan stencil_plan;   /* opaque, library-owned */
typedef struct stencil_batch stencil_batch; /* opaque, library-owned */

/* Plan options; a NULL pointer means all zero (automatic choices). */
typedef struct stencil_opts {
    int method;   /* enum stencil_method */
    int fused_k;  /* steps per launch for STENCIL_METHOD_FUSED; 0 = choose */
    int variant;  /* fused tile variant id (stencil_plan_info lists them); 0 = choose */
    int autotune; /* nonzero: time the candidate (variant, k, chunk) choices on the first
                     run (or on stencil_autotune) and keep the fastest */
    int chunk;    /* 2D/3D fused kernels: output planes per workgroup along axis 0;
                     0 = choose (the measured default; for k >= 2 otherwise the
                     chunk count that minimises rounds of resident workgroups x
                     stream length, from the kernel's occupancy on the current
                     device) */
    int graph;    /* nonzero: stencil_run records the launches of a (d_in, d_out, T)
                     triple into a HIP graph on its first call and replays the graph
                     while later calls repeat the triple (a new triple, autotuning or
                     a device change re-records); for launch-bound small grids */
    int inplace;  /* nonzero: fused passes update one field in place instead of
                     ping-ponging with a second one (Section 3.3, last paragraph:
                     with every pass ending at the same time level, the input's
                     space can hold the output).  The points a pass's other
                     workgroups still read (the bands of every output tile) go
                     through a plan-owned side buffer and are copied in by a
                     second kernel per pass; the plan holds no ping-pong field,
                     and d_in == d_out needs no copy of the input.  Results are
                     bitwise those of the ping-pong plan.  Fused and plain methods
                     only; STENCIL_E_UNSUPPORTED when no in-place kernel is
                     compiled for the plan's stencil, variant and depth. */
} stencil_opts;

/* What a plan resolved to (stencil_plan_info). */
typedef struct stencil_plan_desc {
    int dim, radius, kind, bc, dtype, npts;
    int64_t shape[STENCIL_MAX_DIM];
    int64_t points;       /* prod(shape) */
    int method;           /* resolved method (never AUTO) */
    int fused_k;          /* steps per launch (1 for PLAIN and GENERIC) */
    int variant;          /* fused tile variant id, 0 if none */
    int tile[3];          /* output tile of the fused kernel: x, y, z-chunk (0 = unused) */
    int elem_bytes;       /* bytes per stored element */
    int64_t scratch_bytes;/* device memory the plan holds once prepared */
    int tuned;            /* 1 once autotuning has run */
} stencil_plan_desc;

/* --- plans ------------------------------------------------------------------ */

/* Points of a d-dimensional star (2*d*r+1) or box ((2r+1)^d) stencil of
 * order r (Section 1), or STENCIL_E_INVALID for dim outside 1..3, r < 1 or
 * an unknown kind. */
int stencil_num_points(int dim, int radius, int kind);

/* Writes the offset set in canonical order to out[npts*dim] (host memory,
 * offset j at out[j*dim .. j*dim+dim-1]).  Returns npts or a negative code.
 * The offset sets are those of Section 1 (star and box of order r); the paper
 * fixes no order for the weights, so the canonical order is this library's. */
int stencil_offsets(int dim, int radius, int kind, int32_t *out);

/* Creates a plan for the operation of Section 1 (one constant weight per
 * offset) on one grid; the fused depth k is the time-loop unroll of
 * Section 3.3.  shape: dim extents (host, slowest first, each >= 1).
 * coeffs: ncoeffs = stencil_num_points(dim, radius, kind) doubles in
 * canonical order (host; copied).  r must be 1..STENCIL_MAX_RADIUS.
 * Allocates no device memory.  On failure *out is set to NULL. */
int stencil_plan_create(stencil_plan **out, int dim, const int64_t *shape, int radius, int kind,
                        const double *coeffs, int ncoeffs, int bc, int dtype,
                        const stencil_opts *opts);

/* Frees the plan and its device memory (NULL-safe).  Waits for nothing: the
 * caller must have synchronised any stream still using the plan.  (Library
 * housekeeping; no passage of the paper.) */
void stencil_plan_destroy(stencil_plan *p);

/* Fills *out with the plan's resolved configuration (library housekeeping). */
int stencil_plan_info(const stencil_plan *p, stencil_plan_desc *out);

/* Allocates the plan's device scratch on the current device now (otherwise
 * done by the first run).  Needed before capturing stencil_run in a graph.
 * (Library housekeeping.) */
int stencil_plan_prepare(stencil_plan *p, void *stream);

/* Times every candidate (variant, k, chunk) of the plan on its own scratch
 * buffers, on `stream`, and keeps the fastest.  Synchronises the stream.
 * The paper tunes its block sizes and k by hand (Section 4.1) and leaves
 * tuning to future work; this is the library's extension.  The result is
 * cached under a signature of the device architecture, the stencil, the
 * grid and the options that narrow the candidates, in memory and in the file
 * named by STENCIL_TUNE_CACHE (unset: $XDG_CACHE_HOME or ~/.cache,
 * paper_2103_08825_amd/autotune.txt; empty: memory only); entries a plan
 * cannot run, and unreadable or corrupt files, are ignored.  Plans created
 * with the tessellated method or in place keep their measured choice. */
int stencil_autotune(stencil_plan *p, void *stream);

/* --- sweeps ------------------------------------------------------------------- */

/* u_T = T steps of the plan's stencil applied to u_0 (Section 1), k steps
 * per pass over the data (Section 3.3, Algorithm 1: the multistep update).
 * d_in: u_0 (read only); d_out: u_T; both prod(shape) elements of the plan's
 * dtype in device memory.  d_in == d_out is allowed (the input is copied to
 * scratch first).  T == 0 copies d_in to d_out.  The T steps run as
 * floor(T/k) passes of k fused steps plus one pass of T mod k steps. */
int stencil_run(stencil_plan *p, const void *d_in, void *d_out, int64_t T, void *stream);

/* n independent sweeps, each with its own plan (2D plans, any r <= 2, star or
 * box, any bc, same dtype across the batch), input, output and step count,
 * executed by one persistent kernel launch.  Not in the paper: the library's
 * extension for many small, uneven grids.  d_in[i] and d_out[i] must not
 * alias any buffer of another batch member, and d_in[i] != d_out[i].
 * Equivalent to stencil_batch_create + stencil_batch_launch + destroy. */
int stencil_run_batched(stencil_plan *const *plans, int n, const void *const *d_in,
                        void *const *d_out, const int64_t *T, void *stream);

/* Builds the work list of a batch once (host), uploads it, and captures the
 * counter reset and the persistent kernel into a HIP graph (the batched
 * extension, not in the paper).  The plans and
 * buffers must outlive the batch.  Each replay recomputes the outputs from the
 * inputs.  Per grid, a pass runs the plan's requested fused depth (opts.fused_k),
 * one step for plans created with the plain or generic method, else the deepest
 * depth the batched kernel compiles (12 for r = 1, 4 for r = 2), or the tuned
 * depth when flags bit 0 is set; a pass splits into work items of opts.chunk
 * rows (default 128).  flags: bit 0 = autotune each distinct plan first and
 * take its tuned depth; bit 1 = tune the items instead on this batch's own
 * persistent kernel: a coordinate search over the depth of each stencil class
 * present (order 1: 6, 8, 10, 12; order 2: 2, 3, 4) and then over the rows per
 * item (64, 96, 128, 192, 256), timing whole replays, so creation runs the
 * batch several times (reading d_in, overwriting d_out) on `stream`; a plan's
 * requested fused_k, method or chunk still wins, and the choice is cached
 * in-process per workload and device architecture.  Other bits:
 * STENCIL_E_INVALID. */
int stencil_batch_create(stencil_batch **out, stencil_plan *const *plans, int n,
                         const void *const *d_in, void *const *d_out, const int64_t *T,
                         int flags, void *stream);
/* The item shape a batch runs (batched extension): depths[0..3] = fused steps
 * per item for order-1 star, order-1 box, order-2 star, order-2 box grids
 * whose plan requests no depth (0 for a class the batch does not hold), and
 * *chunk = rows per item for grids whose plan requests no chunk.  Either
 * pointer may be NULL.  STENCIL_E_INVALID for a NULL batch. */
int stencil_batch_choice(const stencil_batch *b, int *depths, int *chunk);
/* Replays the captured graph on `stream` (batched extension). */
int stencil_batch_launch(stencil_batch *b, void *stream);
/* Frees the batch (NULL-safe); the caller must have synchronised its stream
 * (batched extension). */
void stencil_batch_destroy(stencil_batch *b);
/* Number of work items and of persistent workgroups of a batch (batched
 * extension). */
int stencil_batch_info(const stencil_batch *b, int64_t *items, int64_t *workgroups);
/* Synchronises `stream` and reports whether the last replay completed every
 * work item (batched extension): STENCIL_E_DEVICE if a work item gave up waiting for its
 * predecessor (a bounded wait; it cannot happen with a well-formed list). */
int stencil_batch_status(const stencil_batch *b, void *stream);
/* How long a work item of the batch polls for the previous pass of its grid
 * before it gives up (batched extension, housekeeping).  limit_us: microseconds,
 * >= 0; 0 gives up at the first wait that is not already satisfied.  The
 * default is 1,000,000 (about one second of the device's 100 MHz clock).  A
 * give-up sets the batch's error flag, every later wait of that replay gives up
 * at once (the kernel still ends), and stencil_batch_status reports
 * STENCIL_E_DEVICE; each replay starts with the flag cleared.  The value is
 * written to device memory on `stream`, so it applies to replays launched on
 * that stream afterwards.  Errors: STENCIL_E_INVALID for a NULL batch or a
 * negative limit, STENCIL_E_DEVICE if the write fails. */
int stencil_batch_set_wait_limit(stencil_batch *b, int64_t limit_us, void *stream);

/* --- derivative --------------------------------------------------------------- */

/* Reverse-mode derivative of u_T = stencil_run(u_0, T).  Not in the paper:
 * the library's extension for gradients through the sweep of Section 1.  Given
 * d_gT = dL/du_T (device, plan dtype), writes d_grad_u0 = dL/du_0 (device,
 * plan dtype) and d_grad_coeffs[j] = dL/dc_j (device, ncoeffs doubles,
 * overwritten).  The adjoint step is the mirrored stencil (weight c_j at
 * offset -o_j, same boundary rule); dL/dc_j sums lambda_{t+1}[x]*u_t[x+o_j]
 * over x and t with FP64 partials.  Forward states are checkpointed every
 * checkpoint_every steps and recomputed per segment (device memory: about
 * (ceil(T/ckpt) + ckpt + 2) fields, or + 2 ckpt where the fused adjoint pass
 * applies: it rebuilds the next segment on a second stream owned by the plan
 * while the current one runs, and `stream` waits for that stream before the
 * call's work ends).  The workspace comes stream-ordered from a memory pool
 * the library keeps per device, which holds up to 8 GiB of freed blocks for
 * later calls instead of returning them to the system at the next
 * synchronisation.  One call at a time per plan.  F64 and F32
 * plans only (STENCIL_E_UNSUPPORTED otherwise). */
int stencil_adjoint(stencil_plan *p, const void *d_u0, const void *d_gT, int64_t T,
                    int64_t checkpoint_every, void *d_grad_u0, double *d_grad_coeffs,
                    void *stream);

/* --- FP64 reductions ---------------------------------------------------------- */

/* Reduces n elements of dtype at d_u (and d_ref if not NULL, same dtype) in
 * FP64 into d_out[6] (device doubles) -- checksums and norms of results, a
 * library extension (the paper has no reduction):
 *   [0] sum u   [1] sum u^2   [2] max |u|
 *   [3] sum (u-ref)^2   [4] max |u-ref|   [5] max |ref|   (0 when d_ref is NULL)
 * The result is deterministic for a given n and pointer alignment (fixed
 * partial layout; vector loads when both pointers are 4-element aligned).
 * Its 96 KiB of partials come stream-ordered from the library's per-device
 * memory pool (see stencil_adjoint). */
int stencil_reduce(int dtype, const void *d_u, const void *d_ref, int64_t n, double *d_out,
                   void *stream);

/* The same reduction without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Arguments, result and determinism are those of
 * stencil_reduce (the same kernels; bitwise the same result).  The partial
 * rows live in a fixed 96 KiB device array (2048 rows of 6 doubles), one per
 * GPU, held until the process ends; a reduction never needs more rows,
 * whatever n, so no n is rejected for size.  Every call on a GPU shares that
 * array: calls that overlap on one GPU (two streams, or two threads) race and
 * must be serialised by the caller. */
int stencil_reduce_noalloc(int dtype, const void *d_u, const void *d_ref, int64_t n, double *d_out,
                           void *stream);

/* --- errors ------------------------------------------------------------------ */

/* Message of the calling thread's last failure ("" if none).  The pointer
 * stays valid until the thread's next library call.  (Library housekeeping.) */
const char *stencil_last_error(void);

/* STENCIL_VERSION of the built library (library housekeeping). */
int stencil_version(void);

#ifdef __cplusplus
}
#endif

#endif /* STENCIL_H */
