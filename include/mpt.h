/*
 * mpt.h - C ABI of the MI355X (gfx950) batched Min-Path-Tracing solver.
 *
 * The library solves, for every candidate path of a batch, the small
 * nonlinear minimisation of Sec. III-B of the paper (Eqs. (8)-(12)): the
 * unknowns are the interaction points X_1..X_n (n <= 5) on the listed objects
 * (planes and quadric surfaces reflect, straight and circular edges
 * diffract); the cost stacks the reflection law (Eq. 8), the Keller-cone
 * diffraction law (Eq. 9) and the implicit object equations (Eq. 11).  A path
 * exists iff the minimum is zero (Eq. 12); it is kept iff the cost is below
 * a threshold and every point lies on the finite object (Alg. 1, the
 * acceptance test after find_minimum_path).
 *
 * Conventions
 *  - Every function returns an mpt_status; no C++ exception crosses the ABI.
 *    On failure mpt_last_error() describes the problem.
 *  - A bad *path* is not a call error: it gets a per-solve status code.
 *  - Units are metres in a right-handed world frame.  The signs of normals
 *    and edge directions are irrelevant (Eq. 1 is even in n, Eq. 3 flips
 *    both sides).
 *  - Scene memory belongs to the context.  Batch and output buffers are
 *    device pointers owned by the caller and never freed by the library.
 *  - Work is enqueued on the context's HIP stream and is asynchronous unless
 *    a function says it synchronises.  One context per host thread.
 */
#ifndef MPT_H
#define MPT_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mpt_ctx mpt_ctx;

typedef enum {
    MPT_OK = 0,
    MPT_E_INVALID_ARG = 1,   /* null pointer, bad size, non-finite scene value */
    MPT_E_NOMEM = 2,         /* device allocation failed or over the ctx cap    */
    MPT_E_DEVICE = 3,        /* a HIP call failed                               */
    MPT_E_NO_SCENE = 4,      /* solve/accept before mpt_scene_upload            */
    MPT_E_UNSUPPORTED = 5,   /* option value not implemented                    */
    MPT_E_NO_MODEL = 6,      /* learned start requested without a network       */
    MPT_E_CAPACITY = 7       /* output arrays smaller than the result           */
} mpt_status;

/* Per-solve status codes (uint8).  Bit 7 (MPT_PATH_FALLBACK) marks a solve
 * that was re-solved by the plain FP64 solver after the FP32 stage. */
enum {
    MPT_PATH_CONVERGED = 0,  /* stationary with |R|_inf <= tau_root: a root     */
    MPT_PATH_MAXITER = 1,    /* iteration cap reached                           */
    MPT_PATH_STALLED = 2,    /* damping grew past 1e12 x max diag(J^T J)        */
    MPT_PATH_DIVERGED = 3,   /* start point outside the guard box               */
    MPT_PATH_DEGENERATE = 4, /* zero-length segment, zero gradient, circle axis */
    MPT_PATH_BAD_INPUT = 5,  /* order outside 1..5, bad id, non-finite input    */
    MPT_PATH_LOCALMIN = 6,   /* stationary but |R|_inf > tau_root: no path;
                                also, with 0 iterations and an infinite cost,
                                a path with a plane reflection whose previous
                                and next points lie strictly on opposite sides
                                of the plane for every position they can take
                                (TX or RX, or a plane or straight edge exactly
                                parallel to it): the law returns a ray to its
                                own side, so no root exists                     */
    MPT_PATH_OUTSIDE = 7,    /* FP32 stage only: the FP32 end point is a root of
                                the infinite objects (residual below the polish
                                gate) but some point lies outside its object's
                                finite extent by more than extent_skip + 100
                                |R|_inf metres; the FP64 polish and fallback
                                stay next to it, so it is not polished and is
                                never accepted (x holds the FP32 end point)    */
    MPT_PATH_FALLBACK = 0x80
};

enum { MPT_PLANE = 0, MPT_LINE = 1, MPT_QUADRIC = 2, MPT_CIRCLE = 3 };
enum { MPT_MAX_ORDER = 5 };
/* Point arrays (start points, solver outputs, network predictions, training
 * targets) hold one row of MPT_ROW doubles per solve: the 3 * order
 * coordinates x1, y1, z1, x2, ... of its points, then zeros.  A row is 128
 * bytes, so a solve's points fill one cache line and a path's store or load
 * is one contiguous access. */
enum { MPT_ROW = 16 };

/* Record widths (doubles) of the host scene arrays. */
enum { MPT_PLANE_W = 13, MPT_LINE_W = 8, MPT_QUADRIC_W = 17, MPT_CIRCLE_W = 7, MPT_WEDGE_W = 7 };
/* Kind of a straight edge's wedge: no solid, the outer corner of a solid,
 * an inner corner (the free space is the wedge between the faces). */
enum { MPT_WEDGE_NONE = 0, MPT_WEDGE_OUTER = 1, MPT_WEDGE_INNER = 2 };

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * enqueue on (for example the caller's current stream), or NULL for a
 * context-owned stream.  *out receives the context. */
mpt_status mpt_create(int device, void *hip_stream, mpt_ctx **out);
/* Release every device buffer of the context (synchronises its stream). */
mpt_status mpt_destroy(mpt_ctx *ctx);
/* Text of the last error on this context; valid until the next call. */
const char *mpt_last_error(const mpt_ctx *ctx);
/* Replace the stream work is enqueued on (NULL: the context's own). */
mpt_status mpt_set_stream(mpt_ctx *ctx, void *hip_stream);
/* Block until all work enqueued by the context has finished. */
mpt_status mpt_synchronize(mpt_ctx *ctx);

/*
 * Scene: the object database D of Alg. 1 (Sec. II: one implicit equation per
 * object, infinite first, the finite extent kept for validation) and the
 * transmitter (the paper's BS).  Host FP64 arrays, row-major records:
 *   planes   [n_planes][13]   n(3) unit normal, d (n.x = d), o(3) corner,
 *                             eu(3), ev(3) rectangle sides (full length)
 *   lines    [n_lines][8]     p(3), e(3) unit direction, s0, s1 (extent)
 *   quadrics [n_quadrics][17] p(3) anchor, A(6) = xx,xy,xz,yy,yz,zz,
 *                             b(3), c with f = (x-p)^T A (x-p) + b^T(x-p) + c,
 *                             ax(3) patch axis, r_ap patch radius about ax
 *   circles  [n_circles][7]   c(3) centre, n(3) unit plane normal, R
 *   wedges   [n_lines][7]     optional (NULL: none): m1(3), m2(3) unit
 *                             normals of the two faces meeting at the edge,
 *                             pointing into free space, kind (MPT_WEDGE_*)
 *   sides    [n_planes]       optional (NULL: all 0): the side of each facet
 *                             that faces free space, +1 along n, -1 against
 *                             n, 0 both (a thin two-sided surface)
 * Global primitive ids are type-major: planes, lines, quadrics, circles.
 * aabb_lo/hi bound the scene; the guard box is that box scaled 10x about
 * its centre plus 1 m.  The arrays are copied (and packed by a device
 * kernel into the solver's FP64 and TX-local FP32 records); the caller keeps
 * ownership.  Errors: MPT_E_INVALID_ARG for non-finite values, non-unit
 * directions (|1-|v|| > 1e-9), a non-positive radius, a wedge kind other
 * than 0, 1, 2 or a side other than -1, 0, 1.  Synchronises. */
typedef struct {
    double tx[3];
    double aabb_lo[3], aabb_hi[3];
    int32_t n_planes, n_lines, n_quadrics, n_circles;
    const double *planes, *lines, *quadrics, *circles;
    const double *wedges;  /* [n_lines][7] or NULL (validation, visibility)     */
    const double *sides;   /* [n_planes] or NULL (visibility matrix only)        */
    const double *refraction; /* [n_planes][2] or NULL: the refractive indices
                              of a facet that refracts instead of reflecting
                              (Sec. VI: Snell's law as one more law equation):
                              the index on the side its normal points to,
                              then the other side's; (0, 0) marks a mirror.
                              Both positive or both 0, else
                              MPT_E_INVALID_ARG                               */
} mpt_scene_desc;
mpt_status mpt_scene_upload(mpt_ctx *ctx, const mpt_scene_desc *scene);

/*
 * A batch of candidate paths: the interaction lists L of Sec. II (one per
 * solve) with their receiver (the paper's UE).  All pointers are DEVICE
 * pointers owned by the caller:
 *   rx        [n_rx][3] FP64 receiver positions
 *   rx_index  [n] int32 receiver of each solve
 *   order     [n] int32 number of interactions n_t, 1..5
 *   prim      [5][n] int32 global primitive ids (component-major; entries
 *             beyond the order are ignored)
 *   x0        [n][MPT_ROW] FP64 start points for MPT_INIT_USER, else NULL
 */
typedef struct {
    int64_t n;
    int32_t n_rx;
    const double *rx;
    const int32_t *rx_index;
    const int32_t *order;
    const int32_t *prim;
    const double *x0;
} mpt_batch_desc;

enum { MPT_FP64_PLAIN = 0, MPT_FP32_POLISH64 = 1 };
/* MPT_INIT_LEARNED: the network's points for the paths that touch a curved
 * object (paraboloid or circle), the straight-line start for the others
 * (planes and straight edges converge from any start, paper Sec. III-B);
 * MPT_INIT_LEARNED_ALL: the network's points for every path.
 * MPT_INIT_RANDOM: the random start of Alg. 1 - each interaction's point is
 * the projection onto its object of a point drawn uniformly in the scene box
 * (aabb_lo..aabb_hi).  Draw number c = 15 i + 3 k + axis of solve i,
 * interaction k is the (c+1)-th output of SplitMix64 (Steele, Lea & Flood,
 * OOPSLA 2014) started from state opts.seed, as u = (output >> 11) * 2^-53.
 * Restarts are further solves of the same candidate (other i) or other
 * seeds. */
enum { MPT_INIT_LINE = 0, MPT_INIT_USER = 1, MPT_INIT_LEARNED = 2, MPT_INIT_LEARNED_ALL = 3,
       MPT_INIT_RANDOM = 4 };
enum { MPT_FALLBACK_NONE = 0, MPT_FALLBACK_GPU_FP64 = 1 };
/* Formulation of the minimisation (paper Sec. III-B). */
enum { MPT_FORM_IMPLICIT = 0, MPT_FORM_PARAMETRIC = 1, MPT_FORM_AUTO = 2 };
/* MPT_SCHED_PERSISTENT: one persistent launch runs every order's bin;
 * MPT_SCHED_PER_ORDER: one persistent launch per order, with its own
 * register budget, all five running concurrently on forked streams;
 * MPT_SCHED_SPLIT: one persistent launch for orders 1-3 (the register
 * budget of order 3) and one launch each for orders 4 and 5 beside it.
 * Every schedule gives the same results.  A scene with a refracting facet
 * always runs MPT_SCHED_PERSISTENT (the only kernel compiled with the rows
 * of such facets). */
enum { MPT_SCHED_PER_ORDER = 0, MPT_SCHED_PERSISTENT = 1, MPT_SCHED_AUTO = 2, MPT_SCHED_SPLIT = 3 };

/* Solver options; mpt_default_opts fills the defaults noted here. */
typedef struct {
    int32_t precision;     /* MPT_FP32_POLISH64                                 */
    int32_t init;          /* MPT_INIT_LINE: the projection onto each object of
                              the point k/(n+1) of the way from TX to RX        */
    int32_t max_iter;      /* 200  FP64 Levenberg-Marquardt cap                 */
    int32_t max_iter32;    /* 100  FP32 stage cap                               */
    int32_t polish_steps;  /* 5    FP64 Gauss-Newton polish steps at most       */
    int32_t fallback;      /* MPT_FALLBACK_GPU_FP64                             */
    int32_t plateau_win;   /* 10   window of the plateau test (0: off)          */
    int32_t sched;         /* MPT_SCHED_AUTO: the autotuner's choice            */
    int32_t block;         /* 0: the autotuner's threads per block (64..256)    */
    int32_t grid;          /* 0: all blocks that fit on the device at once      */
    int32_t max_iter_fb;   /* 50   FP64 fallback cap (it restarts from the FP32
                              end point, which is already root-like)          */
    int32_t graph;         /* 0: launch directly; 1: capture the whole solve in
                              a HIP graph once per (batch, options, outputs,
                              scene) and replay it (stage timings unavailable) */
    double plateau_frac;   /* 0.999 the cost must fall below frac x its value
                              one window earlier, else the descent ends         */
    double tol_step;       /* 1e-12 stop when |dx|_inf <= tol_step (1+|x|_inf)  */
    double tol_res;        /* 1e-13 stop when |R|_inf <= tol_res (metres)       */
    double tau_root;       /* 1e-9  a stationary point is a root iff |R|_inf <= */
    double lambda0;        /* 1e-3  initial damping / max diag(J^T J)           */
    double tol_step32;     /* 1e-6  FP32 stage step tolerance (relative)        */
    double tol_res32;      /* 1e-5  FP32 stage residual tolerance (metres)      */
    double tau_root32;     /* 1e-4  an FP32 end point this close is a root: if
                              its FP64 polish fails, FP64 re-solves the path    */
    double polish_gate;    /* 1e-2  FP32 end points with |R|_inf above this are
                              final (no path); below it they are polished       */
    uint64_t seed;         /* 0     state of the MPT_INIT_RANDOM draws          */
    int32_t spill;         /* -1: the autotuner's choice; 0: off; 1..64: once an
                              order's queue is empty, a wave with at most this
                              many busy lanes parks them for a second, densely
                              packed launch (results are unchanged)           */
    int32_t form;          /* MPT_FORM_IMPLICIT: the points are the unknowns
                              (Eq. 12); MPT_FORM_PARAMETRIC: 2 parameters per
                              surface, 1 per edge (Eqs. 13-15), for the first
                              LM pass (the polish and the fallback stay
                              implicit).  Paraboloids must be of revolution
                              (A = k (I - ax ax^T), b = -ax, c = 0); another
                              quadric makes its paths MPT_PATH_BAD_INPUT.
                              MPT_FORM_AUTO: parametric when every object
                              of the scene has a parametric expression
                              (every quadric is a paraboloid of
                              revolution), else implicit; a property of the
                              scene, never a timing choice (the forms can
                              accept different paths: about 1 in 10^5 hard
                              chains of planes and straight edges ends at a
                              non-root point in one form and not the other) */
    double stat_tol;       /* 0.02  paths of planes and straight edges only
                              (their root is unique and reached from any
                              start, Sec. III-B): the descent has stalled,
                              and the path is classified by its residual,
                              when the damped model's predicted decrease is
                              below stat_tol x the cost ...                 */
    int32_t stat_win;      /* 4     ... this many iterations in a row (0: off) */
    int32_t refill;        /* 16    a wave takes new paths once at least this
                              many of its 64 lanes are idle (1..64): each
                              refill stalls the wave on the new paths' loads */
    int32_t max_iter32_planar; /* 80  FP32 stage cap for paths of planes and
                              straight edges (1..max_iter32, else
                              MPT_E_INVALID_ARG): their descents converge in
                              a few iterations from any start, so one still
                              running after this many is slow; it is
                              polished when its residual is below
                              polish_gate, else re-solved by the FP64
                              fallback from its FP32 end point               */
    double extent_skip;    /* 0.05 FP32 end points farther than this (plus
                              100 |R|_inf) outside a finite extent end as
                              MPT_PATH_OUTSIDE without the FP64 polish (the
                              acceptance test would reject them); 0: off     */
    double learned_gain;   /* 1.0  the learned starts: the network's points
                              (projected onto the objects) replace the
                              straight-line start only where their FP64 cost
                              is below learned_gain x the straight-line
                              start's cost (the solver judges the network) */
} mpt_solve_opts;
void mpt_default_opts(mpt_solve_opts *opts);

/* Outputs, DEVICE pointers owned by the caller:
 *   x           [n][MPT_ROW] FP64 points (zero beyond 3*order)
 *   cost        [n] FP64 final cost C = |R|^2 (Eq. 12 with the rescaled rows)
 *   iters       [n] int32 iterations run (FP32 + polish + fallback)
 *   status      [n] uint8 MPT_PATH_* code, bit 7 = fallback used
 *   stage_iters [4][n] int32 or NULL: iterations of the first LM pass (FP32
 *               or plain FP64), polish steps, fallback iterations, and the
 *               part of the first count run by the straggler launch        */
typedef struct {
    double *x;
    double *cost;
    int32_t *iters;
    uint8_t *status;
    int32_t *stage_iters;
} mpt_solve_out;

/*
 * find_minimum_path of Alg. 1 for every solve of the batch (Sec. III-B,
 * Eq. 12): Levenberg-Marquardt on the rescaled residual, in FP64
 * (MPT_FP64_PLAIN) or in FP32 in a frame centred on TX followed by an FP64
 * Gauss-Newton polish (MPT_FP32_POLISH64), with the plain FP64 solver as
 * fallback for solves the FP32 stage leaves ambiguous.  Solves are binned by
 * order and run by one persistent launch.  Asynchronous.
 * Errors: MPT_E_NO_SCENE, MPT_E_INVALID_ARG (null pointer, n < 0, n_rx < 1),
 * MPT_E_NO_MODEL (learned start without a network), MPT_E_NOMEM.
 */
mpt_status mpt_solve_batch(mpt_ctx *ctx, const mpt_batch_desc *batch, const mpt_solve_opts *opts,
                           const mpt_solve_out *out);

/*
 * mpt_solve_batch without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results as
 * mpt_solve_batch with spill = 0.  Its counters and lists live in a static
 * device scratch array of the library, sized for at most
 * MPT_NOALLOC_MAX_SOLVES solves (37.8 MB, held by every GPU the library
 * runs on until the process ends); the counters are cleared by a fill
 * kernel at the start of every call.  Every call on one GPU shares that
 * scratch, so calls that overlap on one GPU (other contexts or streams)
 * race: the caller serialises them.  It calls no hipMalloc, hipFree or
 * other allocating routine and reads no tuning cache file (tuned choices
 * already in the context are used).
 * Errors: those of mpt_solve_batch; MPT_E_INVALID_ARG when n exceeds
 * MPT_NOALLOC_MAX_SOLVES; MPT_E_UNSUPPORTED for the learned starts (their
 * start points need the context's workspace) and for graph = 1 (graph
 * instantiation allocates); MPT_E_DEVICE when the scratch's device address
 * could not be found when the context was created.
 */
enum { MPT_NOALLOC_MAX_SOLVES = 1 << 20 };
mpt_status mpt_solve_batch_noalloc(mpt_ctx *ctx, const mpt_batch_desc *batch, const mpt_solve_opts *opts,
                                   const mpt_solve_out *out);

/*
 * Autotuner of the launch choices that do not change results (the schedule -
 * one mixed-order launch or concurrent per-order launches -, the block size,
 * the grid divisor of the per-order launches and the straggler threshold
 * `spill`) in the form the options resolve to: runs whole solves of the
 * given batch back to back with each candidate (writing the outputs; the
 * median of three groups of runs), keeps the fastest and uses it for later
 * solves of the same precision, form, size class (floor log2 n) and scene
 * (a hash of the uploaded records, TX and box).  best_form receives the
 * form.  With the
 * environment variable MPT_AUTOTUNE_CACHE set to a file path, choices are
 * loaded from and saved to that file (one line per entry).  Synchronises.
 * best_* (host, may be NULL) receive the choice and its time per solve in
 * ms.
 */
mpt_status mpt_autotune(mpt_ctx *ctx, const mpt_batch_desc *batch, const mpt_solve_opts *opts,
                        const mpt_solve_out *out, int32_t *best_sched, int32_t *best_block, float *best_ms,
                        int32_t *best_gdiv, int32_t *best_spill, int32_t *best_form);

/*
 * The acceptance test of Alg. 1 ("C < threshold and X is valid") in FP64 on
 * solve outputs: accept[i] = 1 iff status is CONVERGED (bit 7 ignored),
 * |R(x)|_inf <= tau_res, every segment is at least min_seg long and every
 * point lies in its finite extent (closed sets: rectangle, edge segment,
 * paraboloid patch radius; a circle is its own extent) and no reflection
 * grazes its surface (|cos| between the incoming direction and the normal
 * at least 1e-9: a grazing ray passes along the surface unchanged, so the
 * point could slide along it).  Writes accept [n]
 * uint8, the accepted ids in increasing order into accepted_idx [n] int32 and
 * their count into d_count (device int32).  If h_count is not NULL the call
 * synchronises and stores the count there.  All array pointers are device
 * pointers owned by the caller.
 */
mpt_status mpt_accept(mpt_ctx *ctx, const mpt_batch_desc *batch, const mpt_solve_out *in,
                      double tau_res, double min_seg, uint8_t *accept, int32_t *accepted_idx,
                      int32_t *d_count, int64_t *h_count);

/*
 * Physical validation of the accepted paths (Alg. 1 keeps a path whose points
 * are valid; between interactions a ray travels in free space, Sec. II): a
 * path stays when none of its segments crosses a rectangle facet or a
 * paraboloid patch other than the objects it starts and ends on, more than
 * min_seg (metres) inside its ends.  Edges and circles have no area and
 * block nothing; a segment parallel to a facet is not blocked.  At a
 * straight edge with a wedge (scene upload) both segments must leave the
 * edge point X into free space: with d the direction to the neighbouring
 * point, an outer corner blocks d when <d,m1> < 0 and <d,m2> < 0, an inner
 * corner when either is negative.  accept [n]
 * uint8 (from mpt_accept) selects the paths; writes visible [n] uint8 (0 for
 * the others) and their count into d_count (device int32); with h_count not
 * NULL the call synchronises and stores the count there.  The arithmetic is
 * IEEE FP64 without contraction.  Device pointers owned by the caller.
 */
mpt_status mpt_visible(mpt_ctx *ctx, const mpt_batch_desc *batch, const mpt_solve_out *in, const uint8_t *accept,
                       double min_seg, uint8_t *visible, int32_t *d_count, int64_t *h_count);

/*
 * Candidate generation (Alg. 1, before the solves; Sec. II-C, Figs. 3-4): the
 * visibility matrix of the objects, the adjacency matrix that adds BS (TX)
 * and UE (RX), and every simple path BS -> objects -> UE through at most
 * max_order objects as an interaction list.
 *
 * Object i sees object j (i != j) when some segment between a sample point
 * of i and a sample point of j leaves both objects strictly into free space
 * (a facet with a side: towards that side; a two-sided facet or a
 * paraboloid: not tangent; an edge with a wedge: strictly outside the solid;
 * other edges and circles: any direction) and crosses no other facet or
 * paraboloid patch more than min_seg inside its ends.  BS sees j, and j sees
 * a receiver, by the same rule with the single point.  Sample points, k per
 * side (1 <= k <= 16): a rectangle's k x k cell centres o + u eu + v ev with
 * u, v = (2a+1)/(2k); an edge's points s0 + (2a+1)/(2k) (s1 - s0); a
 * paraboloid of revolution's points (2a+1-k)/k r_ap of the k x k grid
 * across its axis with (2a+1-k)^2 + (2b+1-k)^2 < k^2, lifted onto the
 * surface (another quadric: its anchor point); a circle's 2k rational points
 * c + R (x u1 + y u2), (x, y) = ((1-t^2), 2t)/(1+t^2), t = (2a+1-k)/k, and
 * their antipodes, (u1, u2) the pair of Duff et al. (JCGT 2017) across n.
 * All in IEEE FP64 without contraction.
 *
 * Bit matrices: W = (n_all + 31) / 32 words per row; bit j of a row is word
 * j / 32, bit j % 32.  All array pointers are device pointers owned by the
 * caller; scene objects are limited to 4096.
 *
 * mpt_visibility: vis [n_all][W] (symmetric, zero diagonal) and the BS row
 *   bs [W].  mpt_visibility_rx: ue [n_rx][W] (row r: the objects that see
 *   receiver r, rx [n_rx][3] FP64) and los [n_rx] uint8 (TX sees RX; may be
 *   NULL).
 * mpt_candidates: the paths of every receiver, receiver by receiver, order
 *   1..max_order, each order in increasing object ids (lexicographic);
 *   with edge_last, an edge (straight or circular) is only allowed as the
 *   last interaction (the pruning of Fig. 4).  *h_total receives the number
 *   of paths (the call synchronises).  With cap >= total the paths are
 *   written: rx_index [cap], order [cap], prim [5][cap] (stride cap, -1
 *   beyond the order), ready as a batch of cap == total solves; with cap ==
 *   0 only the total is returned; with 0 < cap < total nothing is written and
 *   the status is MPT_E_CAPACITY.
 */
mpt_status mpt_visibility(mpt_ctx *ctx, int32_t k, double min_seg, uint32_t *vis, uint32_t *bs);
mpt_status mpt_visibility_rx(mpt_ctx *ctx, const double *rx, int32_t n_rx, int32_t k, double min_seg,
                             uint32_t *ue, uint8_t *los);
mpt_status mpt_candidates(mpt_ctx *ctx, const uint32_t *vis, const uint32_t *bs, const uint32_t *ue, int32_t n_rx,
                          int32_t max_order, int32_t edge_last, int64_t cap, int32_t *rx_index, int32_t *order,
                          int32_t *prim, int64_t *h_total);

/*
 * Learned warm start (replaces the random guess of Alg. 1 by a network's
 * prediction).  Network: 96 features -> 256 -> 256 -> 256 -> 15 with GELU,
 * BF16 weights and activations, FP32 accumulation on the matrix cores; FP32
 * master weights and Adam state live in the context.  Features are built on
 * the device in a frame centred on TX and scaled by 1/|RX-TX|; the outputs
 * are the points in that frame.
 */
/* Initialise the network with seeded random weights. */
mpt_status mpt_mlp_init(mpt_ctx *ctx, uint64_t seed);
/* One Adam step (FP32 master weights, beta 0.9 / 0.999, eps 1e-8) on the
 * masked mean-squared error between the predicted and the target points,
 * in frame units, of the minibatch `rows` (device int32 [n_rows] ids into the
 * batch; NULL = every solve).  target_x: [n][MPT_ROW] FP64 device, for example the
 * solver's converged points; coordinates beyond a path's order and solves
 * whose `use` flag (uint8 [n], NULL = all) is zero are masked out.
 * *d_loss (device FP32, may be NULL) receives the loss before the step.  */
mpt_status mpt_mlp_train_step(mpt_ctx *ctx, const mpt_batch_desc *batch, const double *target_x,
                              const uint8_t *use, const int32_t *rows, int32_t n_rows, float lr,
                              float *d_loss);
/* The same loss and its gradient with respect to every parameter, without
 * an update: d_grad (device FP32, mpt_mlp_param_count values, in the order
 * of the saved blob's weights).  For gradient checks. */
mpt_status mpt_mlp_grad(mpt_ctx *ctx, const mpt_batch_desc *batch, const double *target_x,
                        const uint8_t *use, const int32_t *rows, int32_t n_rows, float *d_loss,
                        float *d_grad);
/* mpt_mlp_grad with the network run in FP32 throughout (FP32 master
 * weights, FP32 features and activations, FP32 vector-ALU products) instead
 * of BF16 on the matrix cores: a check of the backward pass without BF16
 * rounding.  Same arguments, layout and errors. */
mpt_status mpt_mlp_grad_fp32(mpt_ctx *ctx, const mpt_batch_desc *batch, const double *target_x,
                             const uint8_t *use, const int32_t *rows, int32_t n_rows, float *d_loss,
                             float *d_grad);
/* The 96 input features of every solve, FP32 [n][96] device (before the
 * BF16 rounding the network applies). */
mpt_status mpt_mlp_features(mpt_ctx *ctx, const mpt_batch_desc *batch, float *d_feat);
/* Number of FP32 parameters (W1 [256][96], b1, W2 [256][256], b2, W3, b3,
 * W4 [16][256] with row 15 unused, b4 [16]). */
mpt_status mpt_mlp_param_count(size_t *count);
/* Check of the matrix-core GEMM the network uses: C = A B with A [M][K]
 * (a_trans: stored [K][M]) and B [K][N] (b_trans: stored [N][K]), FP32
 * device inputs rounded to BF16, FP32 accumulation, K split `splits` ways.
 * Synchronises. */
mpt_status mpt_gemm_bf16_check(mpt_ctx *ctx, int32_t M, int32_t N, int32_t K, const float *A,
                               int32_t a_trans, const float *B, int32_t b_trans, float *C,
                               int32_t splits);
/* Predicted points [n][MPT_ROW] FP64 world frame (device, caller-owned). */
mpt_status mpt_mlp_predict(mpt_ctx *ctx, const mpt_batch_desc *batch, double *x_out);
/* The same prediction through the layer-by-layer GEMM kernels training
 * uses (activations in device memory) instead of the fused kernel; for
 * checking the fused kernel. */
mpt_status mpt_mlp_predict_unfused(mpt_ctx *ctx, const mpt_batch_desc *batch, double *x_out);
/* Serialise / restore the network (FP32 master weights and Adam state).
 * mpt_mlp_save with blob = NULL stores the needed size in *bytes. */
mpt_status mpt_mlp_save(mpt_ctx *ctx, void *blob, size_t *bytes);
mpt_status mpt_mlp_load(mpt_ctx *ctx, const void *blob, size_t bytes);

/* Algorithmic floating-point work of the solver for one path of `order`
 * interactions whose primitive types are types[0..order-1] (MPT_PLANE ..
 * MPT_CIRCLE), counted on the host by running the solver's own arithmetic
 * with a counting scalar that skips operations on structural zeros:
 *   out[0] one Levenberg-Marquardt iteration (residual, Jacobian, banded
 *          normal equations, damping, banded Cholesky, solve, trial cost)
 *   out[1] one Gauss-Newton polish step (no trial cost)
 *   out[2] one residual evaluation (the acceptance test's arithmetic)
 *   out[3] square roots and divisions inside out[0]
 * With form = MPT_FORM_PARAMETRIC, out[0], out[2] and out[3] are those of the
 * parametric form (out[1], the polish, is implicit in both).
 * Host only (no device work).  MPT_E_INVALID_ARG for a bad order, type or
 * form. */
mpt_status mpt_flops_per_iter(int order, const int32_t *types, int32_t form, int64_t out[4]);

/* The part of out[0] of mpt_flops_per_iter that builds the residual, the
 * Jacobian and the banded normal equations and gradient (Sec. III-B, Eq. 12
 * with the rescaled rows; Eq. 15 with form = MPT_FORM_PARAMETRIC), in *out.
 * After a rejected step the point has not moved, so the FP32 solver of
 * orders 1-3 keeps these from the previous iteration and runs only the rest
 * of out[0] (damping, banded Cholesky, solve, trial cost); counts of the
 * algorithmic work charge such iterations out[0] minus this figure.
 * Host only.  MPT_E_INVALID_ARG as mpt_flops_per_iter. */
mpt_status mpt_flops_assembly(int order, const int32_t *types, int32_t form, int64_t *out);

/* Stage timing of mpt_solve_batch, on (1) by default: each solve then
 * records 7 HIP events at its stage boundaries (a few microseconds each on
 * the stream) for mpt_last_timings and mpt_last_lm_timings.  Off (0): no
 * events, and those two calls fail until a timed solve.  Graph replays are
 * never timed.  Host only.  MPT_E_INVALID_ARG for a null context. */
mpt_status mpt_set_timing(mpt_ctx *ctx, int32_t on);
/* Per-stage timings of the last mpt_solve_batch in milliseconds (HIP events
 * on the context's stream; synchronises): [0] order binning, [1] learned
 * start, [2] first LM pass (FP32 or plain FP64), [3] its straggler launch,
 * [4] FP64 polish, [5] FP64 fallback.  MPT_E_INVALID_ARG when the last solve
 * was not timed. */
mpt_status mpt_last_timings(mpt_ctx *ctx, float ms[6]);
/* Durations (ms) of the per-order kernels of the first LM pass of the last
 * mpt_solve_batch run with MPT_SCHED_PER_ORDER, index = order - 1 (HIP
 * events on the forked streams; synchronises). */
mpt_status mpt_last_lm_timings(mpt_ctx *ctx, float ms[5]);
/* The launch the last mpt_solve_batch used for its first LM pass, after the
 * tuner's table and the options were applied: out[0] schedule (MPT_SCHED_*),
 * out[1] block size, out[2] grid divisor, out[3] straggler threshold,
 * out[4] form (MPT_FORM_IMPLICIT or MPT_FORM_PARAMETRIC, never AUTO).
 * Host only, no device work.  MPT_E_INVALID_ARG before the first solve. */
mpt_status mpt_last_launch(mpt_ctx *ctx, int32_t out[5]);

#ifdef __cplusplus
}
#endif
#endif
