/*
 * FP64 CPU oracle for the Min-Path-Tracing per-path minimisation.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, obviously correct
 * reference used by the tests, by smoke() and by the CPU-baseline leg of the
 * benchmark.  The product path never links, loads or calls it.  It shares no
 * code with the HIP library.
 *
 * What it computes (paper Sec. III-B, Eqs. (8)-(12)): for one candidate path
 * (TX = X_0, RX = X_{n+1}, interaction list L_1..L_n), the points
 * X_1..X_n that minimise C = |I(X)|^2 + |F(X)|^2, where I stacks the
 * reflection (Eq. 8) and diffraction (Eq. 9) residuals and F the implicit
 * object equations (Eq. 11).  A path exists iff the minimum is 0 (Eq. 12),
 * and it is kept iff the cost is below a threshold and every point lies on
 * the finite object (Alg. 1, the acceptance test).
 *
 * Readings of the paper taken here (each also listed in the design notes):
 *  - the reflection rows are S_k (r^ - (i^ - 2<i^,n^>n^)) and the
 *    diffraction row S_k <i^ - r^, e^>, with S_k the mean length of the two
 *    segments at X_k: Eq. (8) is |i| times the unit form and Eq. (9) the
 *    unit form itself, so this is the "rescaling" Sec. III-B allows, chosen
 *    to keep every row in metres, to avoid the spurious zeros of |i| = 0 and
 *    to make the cost grow away from the scene;
 *  - a surface adds one row f(X) (plane n.X - d; quadric scaled so that
 *    |grad f| = 1 at its vertex); an edge adds two rows (a straight edge:
 *    the two coordinates across the line; a circle: distance to its plane
 *    and (|X-c|^2 - R^2)/(2R));
 *  - the minimiser is Levenberg-Marquardt with Marquardt's diagonal scaling
 *    (the paper only says "gradient descent"); a descent ends at a root
 *    (small step or small residual), at a plateau of the cost (every 10
 *    iterations the cost must fall below 0.999 of its value 10 iterations
 *    before), when the damping blows up, or at the iteration cap;
 *  - initial points: each object's projection of the point k/(n+1) of the
 *    way along the TX -> RX segment, or of a point drawn uniformly in the
 *    scene box (the random start of Alg. 1, SplitMix64 counter draws), or
 *    caller-given points.
 *
 * Parity status: every function here is pinned by the CPU tests (closed
 * forms of the image method and of the Keller point, the paper's Fig. 5
 * example, Fermat-length invariants, finite-difference Jacobians, shooting
 * constructions and brute force).  No function is parity-unpinned.
 */
#ifndef MPT_ORACLE_H
#define MPT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_CONVERGED = 0, ORC_MAXITER = 1, ORC_STALLED = 2, ORC_DIVERGED = 3,
       ORC_DEGENERATE = 4, ORC_BAD_INPUT = 5, ORC_LOCALMIN = 6 };

typedef struct {
    double tx[3];
    double lo[3], hi[3];           /* scene box; the guard box is 10x it plus 1 m:
                                      trial points outside it are rejected, a start
                                      point outside it is DIVERGED */
    int32_t n_pl, n_ln, n_q, n_c;  /* counts; global ids are type-major */
    const double *pl;              /* [n_pl][13] n, d, o, eu, ev            */
    const double *ln;              /* [n_ln][8]  p, e, s0, s1               */
    const double *q;               /* [n_q][17]  p, A(6), b, c, ax, r_ap     */
    const double *c;               /* [n_c][7]   c, n, R                    */
    const double *wd;              /* [n_ln][7]  wedge of each straight edge:
                                      m1, m2 face normals into free space, kind
                                      (0 none, 1 outer corner, 2 inner corner);
                                      NULL: no wedges                          */
    const double *sd;              /* [n_pl] side of each facet that faces free
                                      space: +1 along n, -1 against n, 0 both;
                                      NULL: every facet two-sided              */
    const double *rf;              /* [n_pl][2] refractive indices of a facet
                                      that refracts: (index on the side n
                                      points to, index on the other side);
                                      (0, 0) or NULL: the facet reflects      */
} orc_scene;

typedef struct {
    int32_t max_iter;      /* 200 */
    double  tol_step;      /* converged when |dx|_inf <= tol_step*(1+|x|_inf) */
    double  tol_res;       /* converged when |R|_inf <= tol_res */
    double  tau_root;      /* a converged point is a root iff |R|_inf <= tau_root */
    double  lambda0;       /* initial damping relative to max diag(J^T J) */
    int32_t plateau_win;   /* every plateau_win iterations the cost must have */
    double  plateau_frac;  /* dropped below plateau_frac x its value before   */
} orc_lm_opts;

/* Residual rows (and, if J != NULL, the dense Jacobian, row-major
 * [rows][3n]) at the points X (x1,y1,z1,x2,...).  Returns the row count,
 * or -1 when a direction is undefined (zero-length segment, zero gradient,
 * point on a circle's axis). */
int orc_residual(const orc_scene *s, const double rx[3], int n, const int32_t *ids,
                 const double *X, double *R, double *J);

/* Straight-line initial points (3n values). */
void orc_init_line(const orc_scene *s, const double rx[3], int n, const int32_t *ids, double *X);

/* Random initial points (3n values) of solve `sid`: each object's projection
 * of a point uniform in the scene box, drawn with SplitMix64 from `seed`
 * (counter 15 sid + 3 k + axis).  orc_splitmix64 is the generator's output
 * number c+1 from state seed.  The batch form writes [15][nb], zero past
 * 3 order (and for invalid paths). */
uint64_t orc_splitmix64(uint64_t seed, uint64_t c);
void orc_init_random(const orc_scene *s, uint64_t seed, int64_t sid, int n, const int32_t *ids, double *X);
void orc_init_random_batch(const orc_scene *s, uint64_t seed, int64_t nb, const int32_t *order,
                           const int32_t *prim, double *x);

/* One solve; x0 may be NULL (straight-line start).  Returns the status. */
int orc_solve_one(const orc_scene *s, const double rx[3], int n, const int32_t *ids,
                  const double *x0, const orc_lm_opts *o, double *X, double *cost, int32_t *iters);

/* Parametric form (Eqs. (13)-(15)): unknowns are 2 parameters per surface
 * and 1 per edge, only the law rows remain.  orc_param_residual returns the
 * law rows at X(U) and J = dI/dU ([rows][nu]), and X(U) in Xout (may be
 * NULL).  orc_solve_one_param solves from the parameters of the start
 * points x0 (or of the straight-line start) with the same Levenberg-
 * Marquardt rules, and returns X(U).  Paraboloids must be of revolution
 * (A = kappa (I - ax ax^T), b = -ax, c = 0); other quadrics give
 * ORC_BAD_INPUT. */
int orc_param_residual(const orc_scene *s, const double rx[3], int n, const int32_t *ids, const double *U,
                       double *R, double *J, double *Xout);
int orc_solve_one_param(const orc_scene *s, const double rx[3], int n, const int32_t *ids,
                        const double *x0, const orc_lm_opts *o, double *X, double *cost, int32_t *iters);
void orc_solve_batch_param(const orc_scene *s, int64_t nb, const double *rx, const int32_t *rx_index,
                           const int32_t *order, const int32_t *prim, const double *x0,
                           const orc_lm_opts *o, double *x, double *cost, int32_t *iters,
                           uint8_t *status, int nthreads);

/* Smallest |cos| between a reflection's incoming direction and the surface
 * normal that acceptance allows. */
#define ORC_GRAZE 1e-9

/* Finite-object acceptance of a solved path (1 accepted / 0 rejected):
 * CONVERGED, |R|_inf <= tau_res, segments >= min_seg, points in their
 * extents, and no grazing reflection (|cos| < ORC_GRAZE). */
int orc_accept_one(const orc_scene *s, const double rx[3], int n, const int32_t *ids,
                   const double *X, int status, double tau_res, double min_seg);

/* Physical validation of an accepted path (1 visible / 0 blocked): no
 * segment may cross a rectangle facet or paraboloid patch other than the
 * objects it starts and ends on, more than min_seg inside its ends, and no
 * segment at a straight edge with a wedge may leave it into the solid. */
int orc_visible_one(const orc_scene *s, const double rx[3], int n, const int32_t *ids, const double *X,
                    double min_seg);
void orc_visible_batch(const orc_scene *s, int64_t nb, const double *rx, const int32_t *rx_index,
                       const int32_t *order, const int32_t *prim, const double *x, const uint8_t *accept,
                       double min_seg, uint8_t *visible, int nthreads);

/* Candidate generation (Alg. 1: visibility matrix, adjacency matrix, all
 * simple paths from BS to UE).  orc_samples writes the sample points of
 * object g (at most k*k + 2k) and returns their count.  orc_visibility
 * fills V [n][n] (symmetric, zero diagonal) and the BS row B [n];
 * orc_visibility_rx fills U [n_rx][n] (object j sees receiver r) and the
 * line of sight los [n_rx].  orc_candidates enumerates, receiver by
 * receiver, order by order, in increasing object ids, the simple paths
 * with 1..max_order objects (edges only last when edge_last); it writes the
 * first min(total, cap) into rx_index, order [cap] and prim [5][cap] and
 * returns the total (-1 for bad arguments). */
int orc_samples(const orc_scene *s, int g, int k, double *pts);
void orc_visibility(const orc_scene *s, int k, double min_seg, uint8_t *V, uint8_t *B, int nthreads);
void orc_visibility_rx(const orc_scene *s, const double *rx, int n_rx, int k, double min_seg, uint8_t *U,
                       uint8_t *los, int nthreads);
int64_t orc_candidates(const orc_scene *s, const uint8_t *V, const uint8_t *B, const uint8_t *U, int n_rx,
                       int max_order, int edge_last, int64_t cap, int32_t *rx_index, int32_t *order, int32_t *prim);

/* Batched forms, component-major [15][nb] point arrays; OpenMP over solves.
 * x0 may be NULL. */
void orc_solve_batch(const orc_scene *s, int64_t nb, const double *rx, const int32_t *rx_index,
                     const int32_t *order, const int32_t *prim, const double *x0,
                     const orc_lm_opts *o, double *x, double *cost, int32_t *iters,
                     uint8_t *status, int nthreads);
void orc_accept_batch(const orc_scene *s, int64_t nb, const double *rx, const int32_t *rx_index,
                      const int32_t *order, const int32_t *prim, const double *x,
                      const uint8_t *status, double tau_res, double min_seg, uint8_t *accept,
                      int nthreads);

#ifdef __cplusplus
}
#endif
#endif
