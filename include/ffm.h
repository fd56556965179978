/*
 * ffm.h -- C ABI of the MI355X (gfx950) Fast Free Memory library.
 *
 * The library evaluates the discrete convolution of Aussal & Bakry,
 * "The Fast and Free Memory Method for the efficient computation of
 * convolution kernels" (arXiv:1909.05600), Sec. 1 eqs. (convolution_discrete)
 * and (convolution_matrix):
 *
 *     v_i = sum_j  G(x_i - y_j) * wu_j ,      wu_j = w_j u_j,
 *
 * to a prescribed accuracy eps, for the Laplace kernel 1/(4 pi r)
 * (Sec. 4.1, eq. laplaceGreenKernel) and the Helmholtz kernel
 * e^{ikr}/(4 pi r) (Sec. 2.2.3, eq. helmholtzKernel).  Pairs of coincident
 * points (r == 0) contribute nothing.
 *
 * The method (Sec. 2) builds two octrees whose root cubes have the same edge
 * d_0 (Sec. 2.2.1), descends them once (descent-only, Sec. 2.1 and the
 * remark closing Sec. 2.2.3), compresses every admissible box pair at the
 * level where it first becomes admissible (Sec. 2.2.2: Lagrange
 * interpolation on Chebyshev nodes; Sec. 2.2.3: Gegenbauer plane-wave
 * expansion for oscillatory Helmholtz levels), and sums the remaining leaf
 * pairs densely (Sec. 2.2.4).
 *
 * Conventions for every entry point:
 *   - all pointers named as device pointers must be HIP device memory of the
 *     current device; host pointers are plain host memory;
 *   - coordinates are FP64, n x 3, row-major (x0 y0 z0 x1 y1 z1 ...);
 *   - complex data is interleaved (re, im);
 *   - a hip_stream argument is a hipStream_t (NULL = the null stream);
 *   - every call returns an ffm_status_t; nothing throws across the ABI; on
 *     FFM_EINVAL nothing is written; ffm_last_error() gives a message
 *     (thread-local, valid until the next call on the same thread).
 */
#ifndef FFM_H
#define FFM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ffm_plan_s *ffm_plan_t;

/* Kernels.  The _DN kernels are the normal derivative at the target, dG/dn_x (x, y) = n_x . grad_x G(x - y), of
 * the adjoint double-layer operator (Sec. 4.2.1, eq. doubleLayer); they need options.target_normals.  The _DL
 * kernels are the normal derivative at the source, dG/dn_y (x, y) = n_y . grad_y G(x - y), of the double-layer
 * operator (same equation); they need options.source_normals and run their Lagrange transfers in FP32 whatever
 * options.precision asks.  The _GRAD kernels are the gradient at the target, grad_x G(x - y), three components
 * per target (the vector kernels the integral operators of Sec. 4.2.2 are built from): their products v hold
 * n_x x 3 values, v[3 i + c] the derivative along axis c at target i.  Where a plane-wave level's differentiated
 * transform takes the ring-pair or the grid form it runs once per axis (k s . n = sum_c k s_c n_c). */
typedef enum {
    FFM_LAPLACE = 0, FFM_HELMHOLTZ = 1, FFM_LAPLACE_DN = 2, FFM_HELMHOLTZ_DN = 3, FFM_LAPLACE_DL = 4,
    FFM_HELMHOLTZ_DL = 5, FFM_LAPLACE_GRAD = 6, FFM_HELMHOLTZ_GRAD = 7
} ffm_kernel_t;

typedef enum {
    FFM_OK = 0,
    FFM_EINVAL = -1,     /* invalid argument (null pointer, NaN coordinate, eps, k, sizes) */
    FFM_ENOMEM = -2,     /* a device or host allocation failed; nothing is leaked           */
    FFM_EDEVICE = -3,    /* a HIP runtime call failed; the message names it                 */
    FFM_EBUSY = -4,      /* the plan still has applies in flight                            */
    FFM_EINTERNAL = -5   /* an internal consistency check failed                           */
} ffm_status_t;

/* Element type of the input vector wu. */
typedef enum { FFM_C64 = 0, FFM_F32 = 1, FFM_F64 = 2, FFM_C128 = 3 } ffm_dtype_t;

/* Precision of the compressed transfers (the near field is always FP32). */
typedef enum {
    FFM_PREC_FP32 = 0,   /* FP32 everywhere, FP64 geometry and coarse-level phase reduction   */
    FFM_PREC_MIXED = 1   /* Lagrange transfers on FP16 MFMA with FP32 accumulation            */
} ffm_precision_t;

/* Plan options; an all-zero struct (or NULL) selects the defaults. */
typedef struct {
    int32_t n_leaf;       /* stopping rule: stop when the average box occupancy <= n_leaf (64)  */
    int32_t precision;    /* ffm_precision_t (FFM_PREC_FP32)                                    */
    double  kd_switch;    /* Helmholtz levels use the Gegenbauer form iff k d_l >= kd_switch (pi) */
    int32_t r1_override;  /* > 0: Chebyshev nodes per axis at every Lagrange level              */
    int32_t max_level;    /* depth cap, 1..20 (20)                                              */
    uint32_t flags;       /* FFM_FLAG_* bits; other bits must be 0                              */
    const double *target_normals;   /* _DN kernels: device, FP64 [n_x][3] unit normals at the targets in the
                                       caller's order, read while the plan is built; otherwise NULL     */
    const double *source_normals;   /* _DL kernels: device, FP64 [n_y][3] unit normals at the sources in the
                                       caller's order, read while the plan is built; read for no other
                                       kernel                                                          */
} ffm_options_t;

/* options.flags: record HIP events between the phases of every apply (see ffm_plan_timing). */
#define FFM_FLAG_TIMING 1u
/* options.flags: form of the plane-wave transforms of the Gegenbauer levels (Sec. 2.2.3).  By
 * default the planner picks, per level, the cheaper of the direct sums (every point against every
 * quadrature direction) and the grid form (points spread onto a uniform grid with a smooth kernel,
 * separable sums from the grid to the directions, the kernel's Fourier transform divided out: the
 * fast evaluation the remark closing Sec. 2.2.3 calls for).  These bits force one form. */
#define FFM_FLAG_DIRECT_TRANSFORMS 2u
#define FFM_FLAG_GRID_TRANSFORMS   4u
/* options.flags: adaptive cross approximation of the Lagrange transfer matrices (Sec. 2.2.2, eq.
 * ffmACAmatvec: T ~ A B^T, applied as A (B^T u~)), at relative tolerance eps / 4.  By default the planner
 * uses it at FP32 Lagrange levels with at least 5 Chebyshev nodes per axis where the ranks save a quarter of
 * the transfer work; FFM_FLAG_NO_ACA never uses it, FFM_FLAG_ACA uses it at every FP32 Lagrange level. */
#define FFM_FLAG_NO_ACA 8u
#define FFM_FLAG_ACA    16u
/* options.flags: per-pair leaf rule (beyond the global stopping rule of Sec. 2.2.4): a near pair whose two boxes
 * both hold at most n_leaf points is summed densely at its level instead of being refined, and a level where
 * no near pair is left to refine is the leaf.  For clouds of uneven density (a dense cluster beside a sparse
 * surface) the sparse regions stop descending early. */
#define FFM_FLAG_ADAPTIVE_LEAVES 32u

/*
 * ffm_plan -- build the two octrees, the descent lists and the transfer
 * tables (Sec. 2.2.1-2.2.4; translations shared per class as in the proof
 * of Prop. 1).
 *   X      device, FP64 [n_x][3]: targets x_i.
 *   Y      device, FP64 [n_y][3]: sources y_j.  Y == X with n_y == n_x means
 *          the same set: one tree serves both.
 *   kernel FFM_LAPLACE or FFM_HELMHOLTZ, or their normal derivatives at the
 *          targets FFM_LAPLACE_DN, FFM_HELMHOLTZ_DN or at the sources
 *          FFM_LAPLACE_DL, FFM_HELMHOLTZ_DL, or their gradients at the targets
 *          FFM_LAPLACE_GRAD, FFM_HELMHOLTZ_GRAD; k >= 0 is the wavenumber
 *          (ignored for Laplace; Helmholtz with k = 0 equals Laplace).
 *   eps    prescribed accuracy, 1e-7 <= eps < 0.5.
 *   opts   host pointer or NULL.
 *   hip_stream  stream for the planning kernels.
 *   out    host pointer receiving the plan handle.
 * When it returns, X and Y may be freed (every read of them is complete).  The
 * plan's last tables and launch lists may still be in flight on hip_stream:
 * ffm_apply on any stream is ordered after them on the device (a stream wait,
 * no host synchronisation), and the other calls that use the plan's device
 * data (export, set_tiles, batch_create, server_submit, destroy) wait for them
 * on the host.  The plan owns its device memory until ffm_destroy.  n_x == 0
 * or n_y == 0 gives a plan whose apply writes zeros.  Limits: n_x, n_y < 2^31.
 */
ffm_status_t ffm_plan(const double *X, int64_t n_x, const double *Y, int64_t n_y,
                      ffm_kernel_t kernel, double k, double eps, const ffm_options_t *opts,
                      void *hip_stream, ffm_plan_t *out);

/*
 * ffm_apply -- v = G W u, the matrix-vector product of Sec. 1 eq.
 * (convolution_matrix), evaluated as Sec. 2.2 describes: one descent over the
 * plan's levels (per level: source transform, transfer between the admissible
 * box pairs, target transform; Sec. 2.2.2 and 2.2.3, the descent-only form of
 * the remark closing Sec. 2.2.3) and the dense near field of the leaf level
 * (Sec. 2.2.4).
 *   wu     device, n_y elements of in_dtype, in the caller's source order:
 *          the products w_j u_j of eq. (convolution_discrete).  Real inputs
 *          are taken as complex with zero imaginary part.
 *   v      device, complex64 [n_x] ([n_x][3] for the _GRAD kernels), in the
 *          caller's target order; overwritten.
 * Asynchronous on hip_stream: the caller keeps wu and v alive until the
 * stream passes the apply.  One apply per plan may be in flight at a time
 * (the plan's workspace is reused); a second apply on the same stream is
 * ordered after the first.  No allocation happens inside apply.  Errors:
 * FFM_EINVAL (NULL plan, NULL wu or v with a non-empty set, unknown dtype;
 * nothing is enqueued), FFM_EDEVICE (a launch failed).
 */
ffm_status_t ffm_apply(ffm_plan_t plan, const void *wu, ffm_dtype_t in_dtype, void *v, void *hip_stream);

/*
 * ffm_destroy -- release the plan and all its device memory.  Not in the
 * paper, whose implementation rebuilds every structure at each product and
 * keeps nothing between calls (its linear storage bound, Sec. 3); here a plan stays
 * resident until this call.  FFM_EBUSY (and nothing released) if an apply on
 * it, or a batched apply that includes it, has not completed yet, if it
 * belongs to a batch (ffm_batch_create), or if server requests of it are
 * pending.  NULL is accepted.
 */
ffm_status_t ffm_destroy(ffm_plan_t plan);

/*
 * ffm_apply_batched -- v[i] = FFM_i(wu[i]) for n >= 1 distinct plans in one
 * pass of merged launches (one launch per step kind for all instances,
 * replayed from a HIP graph).  Not in the paper, which evaluates one product
 * at a time; each instance computes bitwise what ffm_apply computes for it.
 *   plans   host array of n plan handles (no plan twice, none in a batch made
 *           by ffm_batch_create).
 *   wu, v   host arrays of n device pointers with the layouts of ffm_apply;
 *           wu[i] is complex64 (FFM_C64) [n_y of plan i].
 * Asynchronous on hip_stream.  The merged launches are built on the first
 * call for a plan set (host-synchronous, allocates) and kept for the next
 * call with the same plans in the same order; a call with another set, and
 * ffm_destroy, ffm_plan_set_tiles or ffm_batch_create on one of the plans,
 * releases them.  While a batched apply is in flight, none of its plans may
 * be applied on its own (they share the plan's workspace).  Errors:
 * FFM_EINVAL (NULL arrays or entries, n <= 0, a repeated plan), FFM_EBUSY (a
 * plan belongs to a batch), FFM_ENOMEM.
 */
ffm_status_t ffm_apply_batched(const ffm_plan_t *plans, const void *const *wu, void *const *v, int32_t n,
                               void *hip_stream);

/* Message of the last failing call on this thread ("" if none).  Not in the
 * paper. */
const char *ffm_last_error(void);

/* Library version string.  Not in the paper. */
const char *ffm_version(void);

/* ---------------------------------------------------------------- statistics */
#define FFM_MAX_LEVELS 21

typedef struct {
    int32_t leaf;                          /* leaf level                                  */
    int32_t same_set;                      /* 1 if sources and targets are one set        */
    double  d0;                            /* root cube edge                              */
    double  corner_x[3], corner_y[3];      /* root cube corners of the two sets           */
    int64_t nbox_x[FFM_MAX_LEVELS], nbox_y[FFM_MAX_LEVELS];
    int64_t nfar[FFM_MAX_LEVELS];          /* far pairs first admissible at level l        */
    int64_t nnear[FFM_MAX_LEVELS];         /* near pairs of level l                        */
    int32_t method[FFM_MAX_LEVELS];        /* 0 none, 1 Lagrange, 2 Gegenbauer             */
    int32_t order[FFM_MAX_LEVELS];         /* r1 (Lagrange) or L (Gegenbauer)              */
    int32_t tform[FFM_MAX_LEVELS];         /* Gegenbauer transforms: 1 direction pairs, 2 ring pairs, 3 grid form */
    int32_t prec[FFM_MAX_LEVELS];          /* transfer arithmetic: 0 FP32, 1 FP16 MFMA with FP32 accumulation */
    int32_t phase64[FFM_MAX_LEVELS];       /* Gegenbauer in-plane phases in FP64 (1) or FP32 (0) */
    int32_t nclass[FFM_MAX_LEVELS];        /* distinct translations at level l             */
    int64_t nq[FFM_MAX_LEVELS];            /* quadrature directions (Gegenbauer levels)    */
    double  fwd_points[FFM_MAX_LEVELS];    /* points of the source boxes transformed at level l */
    double  bwd_points[FFM_MAX_LEVELS];    /* points of the target boxes transformed at level l */
    double  transform_terms;               /* sum over Gegenbauer levels of points x n_Q, both transforms */
    double  transfer_macs;                 /* complex multiply-adds of all transfers      */
    double  near_pairs;                    /* point pairs of the leaf near field          */
    double  plan_bytes;                    /* device memory held by the plan              */
    double  workspace_bytes;               /* device memory of the apply workspace        */
    int32_t grid_nodes[FFM_MAX_LEVELS];    /* grid form: nodes p per axis of each box's grid, else 0 */
    int64_t fwd_boxes[FFM_MAX_LEVELS];     /* source boxes transformed at level l         */
    int64_t bwd_boxes[FFM_MAX_LEVELS];     /* target boxes transformed at level l         */
    int32_t grid_width[FFM_MAX_LEVELS];    /* grid form: spreading kernel width w in nodes, else 0 */
    double  grid_beta[FFM_MAX_LEVELS];     /* grid form: kernel shape beta, else 0 (the grid spacing is
                                              h = d_l / (grid_nodes - 1 - grid_width))               */
    double  grid_alias[FFM_MAX_LEVELS];    /* grid form: bound on the aliasing error of spreading one plane
                                              wave along one axis, relative, for every direction, else 0 */
    int32_t aca[FFM_MAX_LEVELS];           /* 1 if the level's transfers use the ACA factors                 */
    double  aca_rank[FFM_MAX_LEVELS];      /* mean ACA rank over the level's classes where it was evaluated  */
    int64_t nearly[FFM_MAX_LEVELS];        /* near pairs the per-pair leaf rule sums densely at level l      */
} ffm_stats_t;

/* ffm_plan_stats -- copy the plan's sizes and work counters to host memory.
 * The counts are those of Sec. 3 (boxes per level, far and near pairs,
 * translation classes of the proof of Prop. 1, quadrature sizes of eq.
 * (gegenbauerQuadrature)); the byte counts are not in the paper. */
ffm_status_t ffm_plan_stats(ffm_plan_t plan, ffm_stats_t *out);

/*
 * ffm_plan_export -- copy tree and list data to host memory for bit-exact
 * comparison (tests): the octrees of Sec. 2.2.1 and the far and near lists of
 * the descent of Sec. 2.2.2.  what selects the array; set 0 = targets, 1 = sources;
 * level l.  Returns the element count in *count; if dst is non-NULL it must
 * hold that many elements of the listed type.
 *   FFM_EXPORT_KEYS      uint64  sorted Morton keys (set)
 *   FFM_EXPORT_PERM      int64   sorted position -> caller index (set)
 *   FFM_EXPORT_BOX_START int64   [nbox+1] point ranges of level l (set)
 *   FFM_EXPORT_BOX_IJK   int32   [nbox][3] integer box coordinates (set, l)
 *   FFM_EXPORT_BOX_CTR   double  [nbox][3] box centres (set, l)
 *   FFM_EXPORT_FAR       int64   [nfar][5] (t, s, ox, oy, oz) sorted by (t, s) (l)
 *   FFM_EXPORT_NEAR      int64   [nnear][2] (t, s) sorted by (t, s) (l)
 *   FFM_EXPORT_ACA_RANK  int64   [ncls][4] (ox, oy, oz, rank) of an ACA level l (count 0 elsewhere)
 *   FFM_EXPORT_EARLY     int64   [nearly][2] (t, s) the per-pair leaf rule sums at level l, sorted by (t, s)
 */
typedef enum {
    FFM_EXPORT_KEYS = 0, FFM_EXPORT_PERM = 1, FFM_EXPORT_BOX_START = 2, FFM_EXPORT_BOX_IJK = 3,
    FFM_EXPORT_BOX_CTR = 4, FFM_EXPORT_FAR = 5, FFM_EXPORT_NEAR = 6, FFM_EXPORT_ACA_RANK = 7, FFM_EXPORT_EARLY = 8
} ffm_export_t;

ffm_status_t ffm_plan_export(ffm_plan_t plan, int32_t what, int32_t set, int32_t level,
                             void *dst, int64_t *count);

/*
 * ffm_plan_timing -- not in the paper: per-phase durations (milliseconds, HIP events on the
 * apply's stream) of the most recent apply of a plan made with
 * FFM_FLAG_TIMING; waits for that apply to finish.  ms has n >= 64 slots:
 *   [0] input permutation, [1 + 3(l-1) + 0/1/2] level l source transform /
 *   transfer / target transform, [61] near field, [62] output permutation.
 * Phases that did not run read 0.  FFM_EINVAL without FFM_FLAG_TIMING.
 */
#define FFM_TIMING_SLOTS 64
ffm_status_t ffm_plan_timing(ffm_plan_t plan, float *ms, int32_t n);

/*
 * ffm_plan_launch_timing -- not in the paper: the kernel launches of the most recent apply of a
 * plan made with FFM_FLAG_TIMING, in launch order, each timed by its own pair
 * of HIP events on the apply's stream; waits for that apply to finish.  The
 * first min(n, launches) records are written to out (host memory); *count
 * receives the number of launches.  kernel, variant_a and variant_b name the
 * kernel (ffm_kernel_name); level is the level the launch works on (0 for the
 * permutations and the near field); blocks its thread blocks.  FFM_EINVAL
 * without FFM_FLAG_TIMING or with NULL out (n > 0) or count.
 */
typedef struct {
    int32_t kernel, variant_a, variant_b, level;
    int64_t blocks;
    float   ms;
    int32_t reserved;
} ffm_launch_t;
ffm_status_t ffm_plan_launch_timing(ffm_plan_t plan, ffm_launch_t *out, int32_t n, int32_t *count);

/*
 * ffm_kernel_name -- not in the paper: the symbol of a launch's kernel as profilers print it
 * (template arguments included, namespaces and parameters left out), e.g.
 * "k_grid_phi_s<4>", written NUL-terminated into buf (host, n bytes, cut to
 * fit).  Returns the full length, or -1 for an unknown kernel.
 */
int32_t ffm_kernel_name(int32_t kernel, int32_t variant_a, int32_t variant_b, char *buf, int32_t n);

/* Device bytes held by the plan, and by its apply workspace (every part
 * aligned to 256 bytes; the same figure as ffm_stats_t.workspace_bytes and
 * the server's admission).  The paper's storage bound is Sec. 3, Prop. 1. */
size_t ffm_plan_bytes(ffm_plan_t plan);
size_t ffm_workspace_bytes(ffm_plan_t plan);

/* Device bytes the library holds in live allocations (plans, batches, server
 * workspaces), not counting freed blocks it keeps cached for reuse.  Not in
 * the paper: memory accounting for callers, and the check that a failed call
 * (FFM_ENOMEM included) leaves nothing allocated. */
size_t ffm_device_bytes_live(void);

/*
 * ffm_apply_static -- ffm_apply over a workspace the library holds in static
 * device memory instead of the plan's own: for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  It calls no allocating routine; it copies its I/O entry and
 * launches the plan's kernels, computing bitwise what ffm_apply computes.
 * The workspace is FFM_STATIC_WORKSPACE_BYTES on every device the library
 * runs on, held until the process ends; a plan whose apply workspace
 * (ffm_workspace_bytes) is larger is rejected with FFM_EINVAL and a message
 * naming both sizes.  Every call on a device shares that device's workspace,
 * which keeps the last call's contents (the kernels clear what must start at
 * zero): calls that overlap on one device, for the same plan or different
 * plans, race; calls on one stream are ordered.  Arguments, layouts and
 * stream semantics as ffm_apply.
 */
#define FFM_STATIC_WORKSPACE_BYTES ((size_t)128 << 20)
ffm_status_t ffm_apply_static(ffm_plan_t plan, const void *wu, ffm_dtype_t in_dtype, void *v, void *hip_stream);

/* ------------------------------------------------------------------ tiles and batches
 * Not in the paper: the paper evaluates one product at a time.  These entry
 * points apply many independent plans together (one launch per step kind for
 * all of them, optionally captured in a HIP graph) and choose the tile shapes
 * of the plane-wave transform kernels (Sec. 2.2.3) by timing them.
 */

/* Tile choice of the ring-pair plane-wave kernels: ring_g groups of four
 * quadrature directions per thread in the source transform (2 or 4), bwd_pt
 * target points per thread in the target transform (1 or 2).  Default {4, 2}.
 * Results do not depend on bwd_pt; ring_g can change how a box's points are
 * split into partial sums, so results with different ring_g agree to
 * rounding, not bitwise. */
typedef struct {
    int32_t ring_g;
    int32_t bwd_pt;
} ffm_tiles_t;

/* Rebuild a plan's launches for a tile choice.  Waits for the plan's last
 * apply.  FFM_EINVAL for other values; FFM_EBUSY while the plan belongs to a
 * batch. */
ffm_status_t ffm_plan_set_tiles(ffm_plan_t plan, const ffm_tiles_t *tiles, void *hip_stream);
ffm_status_t ffm_plan_get_tiles(ffm_plan_t plan, ffm_tiles_t *tiles);

typedef struct ffm_batch_s *ffm_batch_t;

#define FFM_BATCH_GRAPH    1u   /* capture the merged launches once in a HIP graph; apply replays it */
#define FFM_BATCH_AUTOTUNE 2u   /* time the tile candidates on this batch and keep the fastest */

/*
 * ffm_batch_create -- group n >= 1 distinct plans for joint application.
 *   plans       host array of n plan handles.  The batch borrows them: while it
 *               exists ffm_destroy and ffm_plan_set_tiles on them return
 *               FFM_EBUSY, a plan belongs to at most one batch, and a plan must
 *               not be applied on its own while a batch apply is in flight
 *               (both use the plan's workspace).
 *   flags       FFM_BATCH_GRAPH | FFM_BATCH_AUTOTUNE.
 *   tile_cache  NULL, or the path of a JSON file {"<signature>": {"ring_g": G,
 *               "bwd_pt": PT, "ms": T}, ...}: with FFM_BATCH_AUTOTUNE a
 *               recorded choice for this batch's shapes is used without timing,
 *               and a new one is added.  The signature hashes each instance's
 *               kernel, sizes, depth and per-level method, order and box count.
 *   hip_stream  stream for the set-up work (autotuning runs the batch on it).
 * Autotuning sets the chosen tiles on every plan of the batch.  Host-
 * synchronous.  Errors: FFM_EINVAL (NULL, n <= 0, repeated plan, unknown
 * flags, unwritable cache), FFM_EBUSY (a plan already in a batch).
 */
ffm_status_t ffm_batch_create(const ffm_plan_t *plans, int32_t n, uint32_t flags, const char *tile_cache,
                              void *hip_stream, ffm_batch_t *out);

/*
 * ffm_batch_apply -- v[i] = FFM_i(wu[i]) for every instance i of the batch, as
 * ffm_apply would give it with the same tiles (bitwise).  wu, in_dtype and v
 * are host arrays of n entries; wu[i] and v[i] are device pointers with the
 * layouts of ffm_apply.  Asynchronous on hip_stream; the pointer table is
 * copied in stream order, so the caller may reuse the host arrays on return.
 */
ffm_status_t ffm_batch_apply(ffm_batch_t batch, const void *const *wu, const ffm_dtype_t *in_dtype, void *const *v,
                             void *hip_stream);

typedef struct {
    int32_t n;             /* instances                                          */
    int32_t launches;      /* kernel launches per apply                          */
    int32_t graph;         /* 1 if applies replay a HIP graph                    */
    int32_t tuned;         /* 0 plans' own tiles, 1 timed at creation, 2 from the cache */
    ffm_tiles_t tiles;     /* tiles in use                                       */
    float tuned_ms[4];     /* timings of {4,2}, {4,1}, {2,2}, {2,1} (tuned == 1) */
    int64_t work_items;    /* thread blocks per apply                            */
} ffm_batch_info_t;

ffm_status_t ffm_batch_info(ffm_batch_t batch, ffm_batch_info_t *out);

/* Free a batch (not its plans).  FFM_EBUSY if an apply is in flight. */
ffm_status_t ffm_batch_destroy(ffm_batch_t batch);

/* ------------------------------------------------------------------ serving
 * Not in the paper (its applications call the product repeatedly inside an
 * iterative solver, Sec. 4.2).  A server keeps plans resident and runs apply
 * requests submitted from any host thread: a scheduler thread admits queued
 * requests in submission order as soon as one of `slots` HIP streams is free
 * and the request's apply workspace (ffm_stats_t.workspace_bytes of its plan)
 * fits in the part of `budget_bytes` not held by running requests.  Each
 * running request owns its workspace, so requests of different plans, or of
 * the same plan, run concurrently; each computes bitwise what ffm_apply
 * computes for its plan.
 */
typedef struct ffm_server_s *ffm_server_t;

typedef struct {
    int32_t slots;          /* concurrent requests (streams), 1..16; 0 = 4        */
    int32_t reserved;       /* must be 0                                          */
    double  budget_bytes;   /* device memory for request workspaces; 0 = 80% of the free memory at creation */
} ffm_server_options_t;

/* Start a server on the current device.  opts may be NULL (defaults). */
ffm_status_t ffm_server_create(const ffm_server_options_t *opts, ffm_server_t *out);

/*
 * ffm_server_submit -- queue v = FFM(wu) for a plan; returns at once with a
 * ticket.  wu and v are device pointers with the layouts of ffm_apply, valid
 * until the request completes.  hip_stream is the caller's stream that
 * produces wu: an event recorded on it at submission orders the request after
 * everything enqueued there before this call (a device-side wait, no host
 * synchronisation).  v is complete once ffm_server_wait returns, or
 * ffm_server_poll reports the request done.  The plan may not be destroyed or retiled while it
 * has pending requests (FFM_EBUSY).  FFM_ENOMEM if the workspace exceeds the
 * whole budget.  Thread-safe.
 */
ffm_status_t ffm_server_submit(ffm_server_t server, ffm_plan_t plan, const void *wu, ffm_dtype_t in_dtype, void *v,
                               void *hip_stream, int64_t *ticket);

/* Block until the request completes; *latency_ms (nullable) receives the
 * time from submission to observed completion.  Each ticket is waited for
 * once; returns the request's own error status if it failed. */
ffm_status_t ffm_server_wait(ffm_server_t server, int64_t ticket, double *latency_ms);

/* *done = 1 if the request has completed (the ticket stays valid until waited for). */
ffm_status_t ffm_server_poll(ffm_server_t server, int64_t ticket, int32_t *done);

typedef struct {
    int32_t slots;
    int32_t running, peak_running;
    int32_t reserved;
    int64_t completed, failed, queued;
    double  budget_bytes, in_use_bytes, peak_in_use_bytes;
    double  points;         /* sum of target counts of completed requests */
    double  p50_ms, p99_ms, max_ms;   /* latency quantiles of completed requests */
} ffm_server_stats_t;

ffm_status_t ffm_server_stats(ffm_server_t server, ffm_server_stats_t *out);

/* Finish every queued and running request, then stop the server. */
ffm_status_t ffm_server_destroy(ffm_server_t server);

#ifdef __cplusplus
}
#endif
#endif
