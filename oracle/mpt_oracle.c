/*
 * FP64 CPU oracle for the Min-Path-Tracing per-path minimisation.
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline timing); the
 * product path never uses it.  See mpt_oracle.h for what is computed and
 * which reading of the paper each piece takes.
 *
 * Deliberately plain: the residual is a dense vector, the Jacobian a dense
 * rows x 3n matrix, the normal equations a dense 3n x 3n matrix solved by
 * textbook Cholesky.  No blocking, no band structure, no fusion.
 */
#include "mpt_oracle.h"
#include <math.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXN 5
#define MAXU (3 * MAXN)
#define MAXR (4 * MAXN)

enum { TP = 0, TL = 1, TQ = 2, TC = 3 };

/* ------------------------------------------------------------ small algebra */
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static double norm3(const double *a) { return sqrt(dot3(a, a)); }
static void sub3(const double *a, const double *b, double *o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
/* C = A B for 3x3 */
static void mm3(double A[3][3], double B[3][3], double C[3][3])
{
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0;
            for (int k = 0; k < 3; k++) s += A[i][k] * B[k][j];
            C[i][j] = s;
        }
}
/* P(u) = (I - u^ u^T)/|u| : derivative of u/|u| with respect to u */
static void unit_jac(const double *uh, double len, double P[3][3])
{
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) P[i][j] = ((i == j ? 1.0 : 0.0) - uh[i] * uh[j]) / len;
}

/* ------------------------------------------------------------ primitives */
static int prim_type(const orc_scene *s, int id, const double **rec)
{
    if (id < 0) return -1;
    if (id < s->n_pl) { *rec = s->pl + 13 * (size_t)id; return TP; }
    id -= s->n_pl;
    if (id < s->n_ln) { *rec = s->ln + 8 * (size_t)id; return TL; }
    id -= s->n_ln;
    if (id < s->n_q) { *rec = s->q + 17 * (size_t)id; return TQ; }
    id -= s->n_q;
    if (id < s->n_c) { *rec = s->c + 7 * (size_t)id; return TC; }
    return -1;
}

static void quad_A(const double *q, double A[3][3])
{
    A[0][0] = q[3]; A[0][1] = q[4]; A[0][2] = q[5];
    A[1][0] = q[4]; A[1][1] = q[6]; A[1][2] = q[7];
    A[2][0] = q[5]; A[2][1] = q[7]; A[2][2] = q[8];
}

/* Implicit value and gradient of a surface (Eq. 11 row, Eq. 2 gradient). */
static void surface_eval(int t, const double *r, const double *X, double *f, double g[3], double H[3][3])
{
    if (t == TP) {
        *f = dot3(r, X) - r[3];
        for (int i = 0; i < 3; i++) g[i] = r[i];
        memset(H, 0, 9 * sizeof(double));
    } else {
        double A[3][3], w[3];
        quad_A(r, A);
        sub3(X, r, w);
        double Aw[3];
        for (int i = 0; i < 3; i++) Aw[i] = A[i][0] * w[0] + A[i][1] * w[1] + A[i][2] * w[2];
        *f = dot3(w, Aw) + dot3(r + 9, w) + r[12];
        for (int i = 0; i < 3; i++) g[i] = 2.0 * Aw[i] + r[9 + i];
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) H[i][j] = 2.0 * A[i][j];
    }
}

/* Orthonormal pair across a unit direction e (any such pair gives the same
 * normal equations, only the rows rotate). */
static void across(const double *e, double u1[3], double u2[3])
{
    double a[3] = {0, 0, 0};
    double ax = fabs(e[0]), ay = fabs(e[1]), az = fabs(e[2]);
    if (ax <= ay && ax <= az) a[0] = 1; else if (ay <= az) a[1] = 1; else a[2] = 1;
    cross3(e, a, u1);
    double l = norm3(u1);
    for (int i = 0; i < 3; i++) u1[i] /= l;
    cross3(e, u1, u2);
}

/* Edge direction e^ at X and its derivative (Eq. 4; circle: tangent field). */
static int edge_dir(int t, const double *r, const double *X, double e[3], double E[3][3])
{
    if (t == TL) {
        for (int i = 0; i < 3; i++) e[i] = r[3 + i];
        memset(E, 0, 9 * sizeof(double));
        return 0;
    }
    double d[3], w[3];
    sub3(X, r, d);
    cross3(r + 3, d, w);
    double lw = norm3(w);
    if (!(lw > 0)) return -1;
    for (int i = 0; i < 3; i++) e[i] = w[i] / lw;
    const double *nc = r + 3;
    double K[3][3] = {{0, -nc[2], nc[1]}, {nc[2], 0, -nc[0]}, {-nc[1], nc[0], 0}};
    double P[3][3];
    unit_jac(e, lw, P);
    mm3(P, K, E);
    return 0;
}

/* Two rows that vanish exactly on the edge curve, with their gradients. */
static void edge_rows(int t, const double *r, const double *X, double f[2], double df[2][3])
{
    double d[3];
    if (t == TL) {
        double u1[3], u2[3];
        across(r + 3, u1, u2);
        sub3(X, r, d);
        f[0] = dot3(d, u1);
        f[1] = dot3(d, u2);
        for (int i = 0; i < 3; i++) { df[0][i] = u1[i]; df[1][i] = u2[i]; }
    } else {
        sub3(X, r, d);
        double R = r[6];
        f[0] = dot3(d, r + 3);
        f[1] = (dot3(d, d) - R * R) / (2.0 * R);
        for (int i = 0; i < 3; i++) { df[0][i] = r[3 + i]; df[1][i] = d[i] / R; }
    }
}

/* Refractive indices of facet `id` (a plane id): 1 with (front, back) when
 * the facet refracts (Sec. VI: Snell's law as one more law equation), else
 * 0 - the facet reflects. */
static int refracts(const orc_scene *s, int id, double *nf, double *nb)
{
    if (!s->rf || id < 0 || id >= s->n_pl) return 0;
    *nf = s->rf[2 * (size_t)id];
    *nb = s->rf[2 * (size_t)id + 1];
    return *nf > 0.0 && *nb > 0.0;
}

/* ------------------------------------------------------------ residual */
/*
 * Rows of interaction k, in metres:
 *   reflection  S_k (r^ - (i^ - 2<i^,n^>n^))      3 rows  (Eq. 8 rescaled)
 *               f_k(X_k)                          1 row   (Eq. 11)
 *   refraction  S_k (n_t r^_t - n_i i^_t)         3 rows  (Snell's law on a
 *               f_k(X_k)                          1 row    refracting facet)
 *     where v_t = v - <v,n^> n^ is the part along the facet, n_i the index of
 *     the side the ray arrives from (the side n^ points to when <i^,n^> < 0)
 *     and n_t the other side's; the law rows hold for any ray that keeps its
 *     tangential slowness, so acceptance also checks that it crosses
 *   diffraction S_k <i^ - r^, e^>                 1 row   (Eq. 9 rescaled)
 *               two rows vanishing on the edge    2 rows  (Eq. 11 for edges)
 * with i = X_k - X_{k-1}, r = X_{k+1} - X_k and S_k = (|i| + |r|)/2.  Eq. (8)
 * equals |i| times the unit form; the mean length keeps the rows in metres
 * without the spurious zeros |i| = 0 would create, and it grows away from
 * the scene so that the cost has no descent towards infinity.
 */
int orc_residual(const orc_scene *s, const double rx[3], int n, const int32_t *ids,
                 const double *X, double *R, double *J)
{
    int nu = 3 * n, row = 0;
    if (J) memset(J, 0, sizeof(double) * (size_t)MAXR * nu);
    for (int k = 0; k < n; k++) {
        const double *rec;
        int t = prim_type(s, ids[k], &rec);
        const double *Xp = (k == 0) ? s->tx : X + 3 * (k - 1);
        const double *Xk = X + 3 * k;
        const double *Xn = (k == n - 1) ? rx : X + 3 * (k + 1);
        double a[3], b[3];
        sub3(Xk, Xp, a);
        sub3(Xn, Xk, b);
        double la = norm3(a), lb = norm3(b);
        if (!(la > 0) || !(lb > 0)) return -1;
        double ih[3], rh[3];
        for (int i = 0; i < 3; i++) { ih[i] = a[i] / la; rh[i] = b[i] / lb; }
        double Pa[3][3], Pb[3][3];
        unit_jac(ih, la, Pa);
        unit_jac(rh, lb, Pb);
        /* unit-form law rows u and their derivatives with respect to
         * X_{k-1}, X_k, X_{k+1}: Up, Uk, Un (nl rows each) */
        double u[3], Up[3][3], Uk[3][3], Un[3][3];
        int nl;
        double obj[2], dobj[2][3];
        int no;
        if (t == TP || t == TQ) {
            double f, g[3], H[3][3];
            surface_eval(t, rec, Xk, &f, g, H);
            double lg = norm3(g);
            if (!(lg > 0)) return -1;
            double nh[3];
            for (int i = 0; i < 3; i++) nh[i] = g[i] / lg;
            double sdot = dot3(ih, nh);
            double nf, nb;
            if (t == TP && refracts(s, ids[k], &nf, &nb)) {
                /* u = n_t Pn r^ - n_i Pn i^ with Pn = I - n n^T (constant on a
                 * plane): dU/dX_{k-1} = n_i Pn Pa, dU/dX_{k+1} = n_t Pn Pb */
                double ni = (sdot < 0.0) ? nf : nb, nt = (sdot < 0.0) ? nb : nf;
                double sr = dot3(rh, nh);
                double PnPa[3][3], PnPb[3][3], Pn[3][3];
                for (int i = 0; i < 3; i++) {
                    u[i] = nt * (rh[i] - sr * nh[i]) - ni * (ih[i] - sdot * nh[i]);
                    for (int j = 0; j < 3; j++) Pn[i][j] = (i == j ? 1.0 : 0.0) - nh[i] * nh[j];
                }
                mm3(Pn, Pa, PnPa);
                mm3(Pn, Pb, PnPb);
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++) {
                        Up[i][j] = ni * PnPa[i][j];
                        Un[i][j] = nt * PnPb[i][j];
                        Uk[i][j] = -Up[i][j] - Un[i][j];
                    }
            } else {
                for (int i = 0; i < 3; i++) u[i] = rh[i] - ih[i] + 2.0 * sdot * nh[i];
                double Q[3][3], QPa[3][3], Nm[3][3], Pn[3][3], T[3][3], TN[3][3];
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++) {
                        Q[i][j] = (i == j ? 1.0 : 0.0) - 2.0 * nh[i] * nh[j];
                        Pn[i][j] = (i == j ? 1.0 : 0.0) - nh[i] * nh[j];
                    }
                mm3(Q, Pa, QPa);
                mm3(Pn, H, Nm); /* d n^ / dX = (I - n n^T) H / |g| */
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++) Nm[i][j] /= lg;
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++) T[i][j] = 2.0 * (nh[i] * ih[j] + (i == j ? sdot : 0.0));
                mm3(T, Nm, TN);
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++) {
                        Up[i][j] = QPa[i][j];
                        Un[i][j] = Pb[i][j];
                        Uk[i][j] = -Pb[i][j] - QPa[i][j] + TN[i][j];
                    }
            }
            nl = 3;
            obj[0] = f;
            for (int j = 0; j < 3; j++) dobj[0][j] = g[j];
            no = 1;
        } else if (t == TL || t == TC) {
            double e[3], E[3][3];
            if (edge_dir(t, rec, Xk, e, E)) return -1;
            double dv[3];
            for (int i = 0; i < 3; i++) dv[i] = ih[i] - rh[i];
            u[0] = dot3(dv, e);
            for (int j = 0; j < 3; j++) {
                double ePa = 0, ePb = 0, dE = 0;
                for (int i = 0; i < 3; i++) {
                    ePa += e[i] * Pa[i][j];
                    ePb += e[i] * Pb[i][j];
                    dE += dv[i] * E[i][j];
                }
                Up[0][j] = -ePa;
                Un[0][j] = -ePb;
                Uk[0][j] = ePa + ePb + dE;
            }
            nl = 1;
            edge_rows(t, rec, Xk, obj, dobj);
            no = 2;
        } else {
            return -1;
        }
        /* scale the law rows by S = (|i| + |r|)/2 (product rule for J) */
        double S = 0.5 * (la + lb);
        double dSp[3], dSk[3], dSn[3];
        for (int j = 0; j < 3; j++) {
            dSp[j] = -0.5 * ih[j];
            dSk[j] = 0.5 * (ih[j] - rh[j]);
            dSn[j] = 0.5 * rh[j];
        }
#define JAC(rw, blk, col) J[(size_t)(rw) * nu + 3 * (blk) + (col)]
        for (int i = 0; i < nl; i++) {
            R[row + i] = S * u[i];
            if (J)
                for (int j = 0; j < 3; j++) {
                    if (k > 0) JAC(row + i, k - 1, j) += S * Up[i][j] + u[i] * dSp[j];
                    if (k < n - 1) JAC(row + i, k + 1, j) += S * Un[i][j] + u[i] * dSn[j];
                    JAC(row + i, k, j) += S * Uk[i][j] + u[i] * dSk[j];
                }
        }
        for (int i = 0; i < no; i++) {
            R[row + nl + i] = obj[i];
            if (J)
                for (int j = 0; j < 3; j++) JAC(row + nl + i, k, j) += dobj[i][j];
        }
#undef JAC
        row += nl + no;
    }
    return row;
}

/* ------------------------------------------------------------ start points */
static void project(int t, const double *r, const double *P, double *X)
{
    if (t == TP) {
        double f = dot3(r, P) - r[3];
        for (int i = 0; i < 3; i++) X[i] = P[i] - f * r[i];
    } else if (t == TL) {
        double d[3];
        sub3(P, r, d);
        double sp = dot3(d, r + 3);
        for (int i = 0; i < 3; i++) X[i] = r[i] + sp * r[3 + i];
    } else if (t == TQ) {
        /* one Newton projection step onto f = 0 */
        double f, g[3], H[3][3];
        surface_eval(t, r, P, &f, g, H);
        double gg = dot3(g, g);
        for (int i = 0; i < 3; i++) X[i] = (gg > 0) ? P[i] - f * g[i] / gg : P[i];
    } else {
        /* nearest point of the circle: drop onto its plane, push to radius R */
        double d[3], w[3];
        sub3(P, r, d);
        double h = dot3(d, r + 3);
        for (int i = 0; i < 3; i++) w[i] = d[i] - h * r[3 + i];
        double lw = norm3(w);
        if (!(lw > 0)) {
            double u2[3];
            across(r + 3, w, u2);
            lw = 1.0;
        }
        for (int i = 0; i < 3; i++) X[i] = r[i] + r[6] * w[i] / lw;
    }
}

void orc_init_line(const orc_scene *s, const double rx[3], int n, const int32_t *ids, double *X)
{
    for (int k = 0; k < n; k++) {
        const double *rec;
        int t = prim_type(s, ids[k], &rec);
        double a = (double)(k + 1) / (double)(n + 1), P[3], nf, nb;
        /* a refracting facet is crossed: where the TX -> RX segment meets its
         * plane, when it does */
        if (t == TP && refracts(s, ids[k], &nf, &nb)) {
            double dd[3];
            sub3(rx, s->tx, dd);
            double den = dot3(rec, dd);
            double c = (den != 0.0) ? (rec[3] - dot3(rec, s->tx)) / den : -1.0;
            if (c > 0.0 && c < 1.0) a = c;
        }
        for (int i = 0; i < 3; i++) P[i] = s->tx[i] + a * (rx[i] - s->tx[i]);
        project(t, rec, P, X + 3 * k);
    }
}

/* Random start of Alg. 1 (the paper draws X_0 at random).  Reading: each
 * interaction's point is the projection onto its object of a point drawn
 * uniformly in the scene box, the same projection the straight-line start
 * uses.  The draws come from SplitMix64 (Steele, Lea & Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014) used as a counter
 * generator: value c (0-based) is the generator's (c+1)-th output from state
 * `seed`; a uniform double is its top 53 bits times 2^-53.  Solve i,
 * interaction k, axis j uses counter 15 i + 3 k + j. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + (c + 1u) * 0x9e3779b97f4a7c15ull;  /* state after c+1 steps */
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

static double uniform01(uint64_t seed, uint64_t c)
{
    return (double)(orc_splitmix64(seed, c) >> 11) * (1.0 / 9007199254740992.0);
}

void orc_init_random(const orc_scene *s, uint64_t seed, int64_t sid, int n, const int32_t *ids, double *X)
{
    for (int k = 0; k < n; k++) {
        const double *rec;
        int t = prim_type(s, ids[k], &rec);
        double P[3];
        for (int j = 0; j < 3; j++) {
            double u = uniform01(seed, 15u * (uint64_t)sid + 3u * (uint64_t)k + (uint64_t)j);
            P[j] = s->lo[j] + u * (s->hi[j] - s->lo[j]);
        }
        project(t, rec, P, X + 3 * k);
    }
}

void orc_init_random_batch(const orc_scene *s, uint64_t seed, int64_t nb, const int32_t *order,
                           const int32_t *prim, double *x)
{
    for (int64_t i = 0; i < nb; i++) {
        int n = order[i];
        double X[15] = {0};
        int32_t ids[5] = {-1, -1, -1, -1, -1};
        int ok = n >= 1 && n <= 5;
        for (int k = 0; ok && k < n; k++) {
            const double *rec;
            ids[k] = prim[(size_t)k * nb + i];
            ok = prim_type(s, ids[k], &rec) >= 0;
        }
        if (ok) orc_init_random(s, seed, i, n, ids, X);
        for (int j = 0; j < 15; j++) x[(size_t)j * nb + i] = (ok && j < 3 * n) ? X[j] : 0.0;
    }
}

/* ------------------------------------------------------------ LM */
/* In-place Cholesky of the dense SPD matrix M (lower triangle); 0 on success. */
static int cholesky(double *M, int m)
{
    for (int j = 0; j < m; j++) {
        double d = M[j * m + j];
        for (int k = 0; k < j; k++) d -= M[j * m + k] * M[j * m + k];
        if (!(d > 0)) return -1;
        d = sqrt(d);
        M[j * m + j] = d;
        for (int i = j + 1; i < m; i++) {
            double v = M[i * m + j];
            for (int k = 0; k < j; k++) v -= M[i * m + k] * M[j * m + k];
            M[i * m + j] = v / d;
        }
    }
    return 0;
}

static void chol_solve(const double *L, int m, const double *b, double *x)
{
    double y[MAXU];
    for (int i = 0; i < m; i++) {
        double v = b[i];
        for (int k = 0; k < i; k++) v -= L[i * m + k] * y[k];
        y[i] = v / L[i * m + i];
    }
    for (int i = m - 1; i >= 0; i--) {
        double v = y[i];
        for (int k = i + 1; k < m; k++) v -= L[k * m + i] * x[k];
        x[i] = v / L[i * m + i];
    }
}

static double inf_norm(const double *v, int m)
{
    double r = 0;
    for (int i = 0; i < m; i++) r = fmax(r, fabs(v[i]));
    return r;
}

static int outside_guard(const orc_scene *s, const double *X, int n)
{
    for (int k = 0; k < n; k++)
        for (int i = 0; i < 3; i++) {
            double c = 0.5 * (s->lo[i] + s->hi[i]);
            double h = 10.0 * 0.5 * (s->hi[i] - s->lo[i]) + 1.0;
            if (!(fabs(X[3 * k + i] - c) <= h)) return 1;
        }
    return 0;
}

static int ids_ok(const orc_scene *s, int n, const int32_t *ids)
{
    int tot = s->n_pl + s->n_ln + s->n_q + s->n_c;
    if (n < 1 || n > MAXN) return 0;
    for (int k = 0; k < n; k++)
        if (ids[k] < 0 || ids[k] >= tot) return 0;
    return 1;
}

/* normal equations A = J^T J, g = J^T R (dense) */
static void normal_eq(const double *J, const double *R, int m, int nu, double *A, double *g)
{
    for (int i = 0; i < nu; i++) {
        double gi = 0;
        for (int r = 0; r < m; r++) gi += J[r * nu + i] * R[r];
        g[i] = gi;
        for (int j = 0; j < nu; j++) {
            double a = 0;
            for (int r = 0; r < m; r++) a += J[r * nu + i] * J[r * nu + j];
            A[i * nu + j] = a;
        }
    }
}

int orc_solve_one(const orc_scene *s, const double rx[3], int n, const int32_t *ids,
                  const double *x0, const orc_lm_opts *o, double *X, double *cost, int32_t *iters)
{
    int nu = 3 * n;
    *iters = 0;
    *cost = INFINITY;
    if (!ids_ok(s, n, ids)) return ORC_BAD_INPUT;
    for (int i = 0; i < 3; i++)
        if (!isfinite(rx[i])) return ORC_BAD_INPUT;
    if (x0) {
        for (int i = 0; i < nu; i++) {
            X[i] = x0[i];
            if (!isfinite(X[i])) return ORC_BAD_INPUT;
        }
    } else {
        orc_init_line(s, rx, n, ids, X);
    }
    double R[MAXR], J[MAXR * MAXU], A[MAXU * MAXU], g[MAXU], M[MAXU * MAXU], dx[MAXU], mg[MAXU];
    double Xt[MAXU], Rt[MAXR];
    double lam = 0, C = INFINITY, C_ref = INFINITY, rinf = INFINITY;
    int status = ORC_MAXITER, small = 0;
    if (outside_guard(s, X, n)) return ORC_DIVERGED;
    for (int it = 1; it <= o->max_iter; it++) {
        *iters = it;
        /* linearise at the current points */
        int m = orc_residual(s, rx, n, ids, X, R, J);
        if (m < 0) { status = ORC_DEGENERATE; break; }
        C = 0;
        for (int r = 0; r < m; r++) C += R[r] * R[r];
        rinf = inf_norm(R, m);
        normal_eq(J, R, m, nu, A, g);
        double dmax = 0;
        for (int i = 0; i < nu; i++) dmax = fmax(dmax, A[i * nu + i]);
        if (it == 1) { lam = o->lambda0 * dmax; C_ref = C; }
        if (rinf <= o->tol_res) { small = 1; break; }
        /* plateau: too small a decrease of the cost over a window ends the
         * descent; the point is then classified by its residual */
        if (o->plateau_win > 0 && it > 1 && (it - 1) % o->plateau_win == 0) {
            if (C > o->plateau_frac * C_ref) { small = 1; break; }
            C_ref = C;
        }
        /* (J^T J + lambda diag(J^T J)) dx = -J^T R, diag floored at 1e-12 max */
        for (int i = 0; i < nu * nu; i++) M[i] = A[i];
        for (int i = 0; i < nu; i++) M[i * nu + i] += lam * fmax(A[i * nu + i], 1e-12 * dmax);
        if (cholesky(M, nu)) {
            lam *= 10.0;
            if (lam > 1e12 * dmax) { status = ORC_STALLED; break; }
            continue;
        }
        for (int i = 0; i < nu; i++) mg[i] = -g[i];
        chol_solve(M, nu, mg, dx);
        for (int i = 0; i < nu; i++) Xt[i] = X[i] + dx[i];
        int is_small = inf_norm(dx, nu) <= o->tol_step * (1.0 + inf_norm(X, nu));
        /* a trial point outside the guard box counts as a cost increase */
        int mt = outside_guard(s, Xt, n) ? -1 : orc_residual(s, rx, n, ids, Xt, Rt, NULL);
        double Ct = INFINITY;
        if (mt == m) {
            Ct = 0;
            for (int r = 0; r < m; r++) Ct += Rt[r] * Rt[r];
        }
        if (Ct < C) {
            for (int i = 0; i < nu; i++) X[i] = Xt[i];
            C = Ct;
            rinf = inf_norm(Rt, m);
            lam = fmax(lam / 10.0, 1e-15 * dmax);
            if (is_small) { small = 1; break; }
        } else {
            if (is_small) { small = 1; break; }
            lam *= 10.0;
            if (lam > 1e12 * dmax) { status = ORC_STALLED; break; }
        }
    }
    *cost = C;
    if (small) status = (rinf <= o->tau_root) ? ORC_CONVERGED : ORC_LOCALMIN;
    return status;
}

/* ------------------------------------------------------------ parametric form */
/*
 * Eqs. (13)-(15): with a parametric expression of every object the points
 * are functions X(U) of 2 parameters per surface and 1 per edge, the object
 * rows vanish identically and only the law rows of Eqs. (8), (9) remain.
 * Parameters (all in metres):
 *   plane      (s, t)  X = o + s e1 + t e2,  e1 = eu/|eu|, e2 = n x e1
 *   line       (s)     X = p + s e
 *   paraboloid (s, t)  X = p + s e1 + t e2 + kappa (s^2 + t^2) ax, with
 *                      (e1, e2) orthonormal across the axis; the record must
 *                      be a paraboloid of revolution, A = kappa (I - ax ax^T),
 *                      b = -ax, c = 0, so kappa = trace(A)/2
 *   circle     (phi)   X = c + R (cos(phi/R) u1 + sin(phi/R) u2), arc length
 * Any orthonormal pair gives the same points (the objects are symmetric
 * about their axis / normal), only the parameter origin turns; the pair is
 * Duff et al.'s construction.
 */
static int param_dim(int t) { return (t == TP || t == TQ) ? 2 : 1; }

/* Orthonormal pair across a unit vector a, by the branch-free construction
 * of Duff et al., "Building an Orthonormal Basis, Revisited" (JCGT 2017). */
static void onb_duff(const double *a, double u1[3], double u2[3])
{
    double sg = a[2] >= 0.0 ? 1.0 : -1.0;
    double q = -1.0 / (sg + a[2]);
    double b = a[0] * a[1] * q;
    u1[0] = 1.0 + sg * a[0] * a[0] * q;
    u1[1] = sg * b;
    u1[2] = -sg * a[0];
    u2[0] = b;
    u2[1] = sg + a[1] * a[1] * q;
    u2[2] = -a[1];
}

/* Frame of an object's parameters; -1 if the record cannot be parametrised. */
static int param_frame(int t, const double *r, double o[3], double e1[3], double e2[3], double *k)
{
    if (t == TP) {
        double l = norm3(r + 7);
        if (!(l > 0)) return -1;
        for (int i = 0; i < 3; i++) { o[i] = r[4 + i]; e1[i] = r[7 + i] / l; }
        cross3(r, e1, e2);
        *k = 0.0;
    } else if (t == TL) {
        for (int i = 0; i < 3; i++) { o[i] = r[i]; e1[i] = r[3 + i]; e2[i] = 0.0; }
        *k = 0.0;
    } else if (t == TQ) {
        const double *ax = r + 13;
        double kap = 0.5 * (r[3] + r[6] + r[8]);
        double A[3][3], err = fabs(r[12]);
        quad_A(r, A);
        for (int i = 0; i < 3; i++) {
            err = fmax(err, fabs(r[9 + i] + ax[i]));
            for (int j = 0; j < 3; j++)
                err = fmax(err, fabs(A[i][j] - kap * ((i == j ? 1.0 : 0.0) - ax[i] * ax[j])));
        }
        if (!(kap > 0) || err > 1e-9 * (1.0 + kap)) return -1;
        for (int i = 0; i < 3; i++) o[i] = r[i];
        onb_duff(ax, e1, e2);
        *k = kap;
    } else {
        for (int i = 0; i < 3; i++) o[i] = r[i];
        onb_duff(r + 3, e1, e2);
        *k = r[6];
    }
    return 0;
}

/* X(U) and its tangent columns dX/dU (T[.][1] unused for edges). */
static int param_map(int t, const double *r, const double *U, double X[3], double T[3][2])
{
    double o[3], e1[3], e2[3], k;
    if (param_frame(t, r, o, e1, e2, &k)) return -1;
    if (t == TP) {
        for (int i = 0; i < 3; i++) {
            X[i] = o[i] + U[0] * e1[i] + U[1] * e2[i];
            T[i][0] = e1[i];
            T[i][1] = e2[i];
        }
    } else if (t == TL) {
        for (int i = 0; i < 3; i++) {
            X[i] = o[i] + U[0] * e1[i];
            T[i][0] = e1[i];
            T[i][1] = 0.0;
        }
    } else if (t == TQ) {
        const double *ax = r + 13;
        double h = k * (U[0] * U[0] + U[1] * U[1]);
        for (int i = 0; i < 3; i++) {
            X[i] = o[i] + U[0] * e1[i] + U[1] * e2[i] + h * ax[i];
            T[i][0] = e1[i] + 2.0 * k * U[0] * ax[i];
            T[i][1] = e2[i] + 2.0 * k * U[1] * ax[i];
        }
    } else {
        double R = k, a = U[0] / R, ca = cos(a), sa = sin(a);
        for (int i = 0; i < 3; i++) {
            X[i] = o[i] + R * (ca * e1[i] + sa * e2[i]);
            T[i][0] = -sa * e1[i] + ca * e2[i];
            T[i][1] = 0.0;
        }
    }
    return 0;
}

/* Parameters of a point (the start points are first put on the object). */
static int param_of(int t, const double *r, const double X[3], double U[2])
{
    double o[3], e1[3], e2[3], k, d[3];
    if (param_frame(t, r, o, e1, e2, &k)) return -1;
    sub3(X, o, d);
    U[1] = 0.0;
    if (t == TP || t == TQ) {
        U[0] = dot3(d, e1);
        U[1] = dot3(d, e2);
    } else if (t == TL) {
        U[0] = dot3(d, e1);
    } else {
        U[0] = k * atan2(dot3(d, e2), dot3(d, e1));
    }
    return 0;
}

/* Law rows at X(U) and J = dI/dU ([rows][nu], nu = sum of the dims), built
 * from the implicit residual's law rows and its Jacobian by the chain rule;
 * returns the row count, or -1 (degenerate or not parametrisable). */
int orc_param_residual(const orc_scene *s, const double rx[3], int n, const int32_t *ids, const double *U,
                       double *R, double *J, double *Xout)
{
    double X[MAXU], T[MAXN][3][2];
    int off[MAXN + 1], ty[MAXN];
    off[0] = 0;
    for (int k = 0; k < n; k++) {
        const double *rec;
        ty[k] = prim_type(s, ids[k], &rec);
        if (ty[k] < 0 || param_map(ty[k], rec, U + off[k], X + 3 * k, T[k])) return -1;
        off[k + 1] = off[k] + param_dim(ty[k]);
    }
    int nu = off[n];
    double Rf[MAXR], Jf[MAXR * MAXU];
    int mf = orc_residual(s, rx, n, ids, X, Rf, J ? Jf : NULL);
    if (mf < 0) return -1;
    if (J) memset(J, 0, sizeof(double) * (size_t)MAXR * nu);
    int row = 0, rowf = 0;
    for (int k = 0; k < n; k++) {
        int surf = (ty[k] == TP || ty[k] == TQ);
        int nl = surf ? 3 : 1, no = surf ? 1 : 2;
        for (int i = 0; i < nl; i++, row++) {
            R[row] = Rf[rowf + i];
            if (!J) continue;
            for (int b = k - 1; b <= k + 1; b++) {
                if (b < 0 || b >= n) continue;
                for (int c = 0; c < param_dim(ty[b]); c++) {
                    double v = 0.0;
                    for (int j = 0; j < 3; j++) v += Jf[(size_t)(rowf + i) * (3 * n) + 3 * b + j] * T[b][j][c];
                    J[(size_t)row * nu + off[b] + c] = v;
                }
            }
        }
        rowf += nl + no;
    }
    if (Xout)
        for (int j = 0; j < 3 * n; j++) Xout[j] = X[j];
    return row;
}

int orc_solve_one_param(const orc_scene *s, const double rx[3], int n, const int32_t *ids,
                        const double *x0, const orc_lm_opts *o, double *X, double *cost, int32_t *iters)
{
    *iters = 0;
    *cost = INFINITY;
    if (!ids_ok(s, n, ids)) return ORC_BAD_INPUT;
    for (int i = 0; i < 3; i++)
        if (!isfinite(rx[i])) return ORC_BAD_INPUT;
    double X0[MAXU], U[MAXU];
    if (x0) {
        for (int i = 0; i < 3 * n; i++) {
            X0[i] = x0[i];
            if (!isfinite(X0[i])) return ORC_BAD_INPUT;
        }
    } else {
        orc_init_line(s, rx, n, ids, X0);
    }
    int nu = 0;
    for (int k = 0; k < n; k++) {
        const double *rec;
        int t = prim_type(s, ids[k], &rec);
        if (param_of(t, rec, X0 + 3 * k, U + nu)) return ORC_BAD_INPUT;
        nu += param_dim(t);
    }
    double R[MAXR], J[MAXR * MAXU], A[MAXU * MAXU], g[MAXU], M[MAXU * MAXU], du[MAXU], mg[MAXU];
    double Ut[MAXU], Rt[MAXR], Xt[MAXU];
    double lam = 0, C = INFINITY, C_ref = INFINITY, rinf = INFINITY;
    int status = ORC_MAXITER, small = 0;
    for (int k = 0, off = 0; k < n; k++) {
        const double *rec;
        int t = prim_type(s, ids[k], &rec);
        double T[3][2];
        param_map(t, rec, U + off, X + 3 * k, T);
        off += param_dim(t);
    }
    if (outside_guard(s, X, n)) return ORC_DIVERGED;
    for (int it = 1; it <= o->max_iter; it++) {
        *iters = it;
        int m = orc_param_residual(s, rx, n, ids, U, R, J, X);
        if (m < 0) { status = ORC_DEGENERATE; break; }
        C = 0;
        for (int r = 0; r < m; r++) C += R[r] * R[r];
        rinf = inf_norm(R, m);
        normal_eq(J, R, m, nu, A, g);
        double dmax = 0;
        for (int i = 0; i < nu; i++) dmax = fmax(dmax, A[i * nu + i]);
        if (it == 1) { lam = o->lambda0 * dmax; C_ref = C; }
        if (rinf <= o->tol_res) { small = 1; break; }
        if (o->plateau_win > 0 && it > 1 && (it - 1) % o->plateau_win == 0) {
            if (C > o->plateau_frac * C_ref) { small = 1; break; }
            C_ref = C;
        }
        for (int i = 0; i < nu * nu; i++) M[i] = A[i];
        for (int i = 0; i < nu; i++) M[i * nu + i] += lam * fmax(A[i * nu + i], 1e-12 * dmax);
        if (cholesky(M, nu)) {
            lam *= 10.0;
            if (lam > 1e12 * dmax) { status = ORC_STALLED; break; }
            continue;
        }
        for (int i = 0; i < nu; i++) mg[i] = -g[i];
        chol_solve(M, nu, mg, du);
        for (int i = 0; i < nu; i++) Ut[i] = U[i] + du[i];
        int is_small = inf_norm(du, nu) <= o->tol_step * (1.0 + inf_norm(U, nu));
        int mt = orc_param_residual(s, rx, n, ids, Ut, Rt, NULL, Xt);
        if (mt == m && outside_guard(s, Xt, n)) mt = -1;
        double Ct = INFINITY;
        if (mt == m) {
            Ct = 0;
            for (int r = 0; r < m; r++) Ct += Rt[r] * Rt[r];
        }
        if (Ct < C) {
            for (int i = 0; i < nu; i++) U[i] = Ut[i];
            for (int j = 0; j < 3 * n; j++) X[j] = Xt[j];
            C = Ct;
            rinf = inf_norm(Rt, m);
            lam = fmax(lam / 10.0, 1e-15 * dmax);
            if (is_small) { small = 1; break; }
        } else {
            if (is_small) { small = 1; break; }
            lam *= 10.0;
            if (lam > 1e12 * dmax) { status = ORC_STALLED; break; }
        }
    }
    *cost = C;
    if (small) status = (rinf <= o->tau_root) ? ORC_CONVERGED : ORC_LOCALMIN;
    return status;
}

/* ------------------------------------------------------------ acceptance */
static int in_extent(int t, const double *r, const double *X)
{
    double d[3];
    if (t == TP) {
        sub3(X, r + 4, d);
        double a = dot3(d, r + 7), b = dot3(d, r + 10);
        return a >= 0.0 && a <= dot3(r + 7, r + 7) && b >= 0.0 && b <= dot3(r + 10, r + 10);
    }
    if (t == TL) {
        sub3(X, r, d);
        double sp = dot3(d, r + 3);
        return sp >= r[6] && sp <= r[7];
    }
    if (t == TQ) {
        sub3(X, r, d);
        double h = dot3(d, r + 13), w[3];
        for (int i = 0; i < 3; i++) w[i] = d[i] - h * r[13 + i];
        return dot3(w, w) <= r[16] * r[16];
    }
    return 1; /* a circle is its own finite extent */
}

int orc_accept_one(const orc_scene *s, const double rx[3], int n, const int32_t *ids,
                   const double *X, int status, double tau_res, double min_seg)
{
    if (status != ORC_CONVERGED || !ids_ok(s, n, ids)) return 0;
    double R[MAXR];
    int m = orc_residual(s, rx, n, ids, X, R, NULL);
    if (m < 0 || !(inf_norm(R, m) <= tau_res)) return 0;
    for (int k = 0; k <= n; k++) {
        const double *P = (k == 0) ? s->tx : X + 3 * (k - 1);
        const double *Q = (k == n) ? rx : X + 3 * k;
        double d[3];
        sub3(Q, P, d);
        if (!(norm3(d) >= min_seg)) return 0;
    }
    double medium = 0.0; /* index of the medium the ray travels in (0: not yet known) */
    for (int k = 0; k < n; k++) {
        const double *rec;
        int t = prim_type(s, ids[k], &rec);
        if (!in_extent(t, rec, X + 3 * k)) return 0;
        /* a grazing reflection is degenerate: the ray passes along the
           surface unchanged, so the point can slide along it */
        if (t == TP || t == TQ) {
            const double *P = (k == 0) ? s->tx : X + 3 * (k - 1);
            double d[3], nr[3];
            sub3(X + 3 * k, P, d);
            if (t == TP) {
                for (int i = 0; i < 3; i++) nr[i] = rec[i];
            } else {
                const double A[3][3] = {{rec[3], rec[4], rec[5]}, {rec[4], rec[6], rec[7]}, {rec[5], rec[7], rec[8]}};
                double w[3];
                sub3(X + 3 * k, rec, w);
                for (int i = 0; i < 3; i++) nr[i] = 2.0 * (A[i][0] * w[0] + A[i][1] * w[1] + A[i][2] * w[2]) + rec[9 + i];
            }
            if (!(fabs(dot3(d, nr)) >= ORC_GRAZE * norm3(d) * norm3(nr))) return 0;
            /* a refracting facet passes the ray to its other side, and the
             * ray arrives in the medium the previous refracting facet of the
             * path sent it into */
            double nf, nb;
            if (t == TP && refracts(s, ids[k], &nf, &nb)) {
                const double *Q = (k == n - 1) ? rx : X + 3 * (k + 1);
                double e[3];
                sub3(Q, X + 3 * k, e);
                if (!(dot3(d, nr) * dot3(e, nr) > 0.0)) return 0;
                const double in = (dot3(d, nr) < 0.0) ? nf : nb, out = (dot3(d, nr) < 0.0) ? nb : nf;
                if (medium > 0.0 && in != medium) return 0;
                medium = out;
            }
        }
    }
    return 1;
}

/* ------------------------------------------------------------ physical validation */
/*
 * Alg. 1 keeps a path when its points are valid "a posteriori" (Sec. II):
 * beyond the finite extent of each interaction object (the acceptance test
 * above), no segment of the path may pass through another object.  A
 * segment P -> Q is blocked by a rectangle facet or a paraboloid patch it
 * crosses strictly inside, more than min_seg from both ends.  The objects a
 * segment starts or ends on are not tested; edges and circles have no area
 * and block nothing; a segment parallel to a facet's plane is not blocked.
 */
static int seg_hits_plane(const double *r, const double P[3], const double d[3], double tmin, double tmax)
{
    double den = dot3(r, d);
    if (den == 0.0) return 0;
    double t = (r[3] - dot3(r, P)) / den;
    if (!(t > tmin && t < tmax)) return 0;
    double w[3];
    for (int i = 0; i < 3; i++) w[i] = (P[i] + t * d[i]) - r[4 + i];
    double a = dot3(w, r + 7), b = dot3(w, r + 10);
    return a >= 0.0 && a <= dot3(r + 7, r + 7) && b >= 0.0 && b <= dot3(r + 10, r + 10);
}

static int in_patch(const double *r, const double H[3])
{
    double w[3];
    sub3(H, r, w);
    double h = dot3(w, r + 13), v[3];
    for (int i = 0; i < 3; i++) v[i] = w[i] - h * r[13 + i];
    return dot3(v, v) <= r[16] * r[16];
}

/* f(P + t d) = a t^2 + b t + c for a quadric; its roots inside (tmin, tmax)
 * that lie on the patch block the segment. */
static int seg_hits_quadric(const double *r, const double P[3], const double d[3], double tmin, double tmax)
{
    double A[3][3], w[3], Ad[3], Aw[3];
    quad_A(r, A);
    sub3(P, r, w);
    for (int i = 0; i < 3; i++) {
        Ad[i] = A[i][0] * d[0] + A[i][1] * d[1] + A[i][2] * d[2];
        Aw[i] = A[i][0] * w[0] + A[i][1] * w[1] + A[i][2] * w[2];
    }
    double a = dot3(d, Ad);
    double b = 2.0 * dot3(w, Ad) + dot3(r + 9, d);
    double c = dot3(w, Aw) + dot3(r + 9, w) + r[12];
    double ts[2];
    int nt = 0;
    if (a == 0.0) {
        if (b != 0.0) ts[nt++] = -c / b;
    } else {
        double disc = b * b - 4.0 * a * c;
        if (disc < 0.0) return 0;
        double sq = sqrt(disc);
        /* the stable pair of roots: q = -(b + sign(b) sq)/2, t = q/a, c/q */
        double q = -0.5 * (b + (b >= 0.0 ? sq : -sq));
        ts[nt++] = q / a;
        if (q != 0.0) ts[nt++] = c / q;
    }
    for (int j = 0; j < nt; j++) {
        double t = ts[j];
        if (!(t > tmin && t < tmax)) continue;
        double H[3];
        for (int i = 0; i < 3; i++) H[i] = P[i] + t * d[i];
        if (in_patch(r, H)) return 1;
    }
    return 0;
}

/* A diffracted ray leaves its edge into free space (Sec. II: rays travel in
   free space between interactions).  The faces meeting at the edge bound the
   solid near the edge point X: with their normals m1, m2 pointing into free
   space, the direction d from X towards a neighbouring point of the path
   enters the solid when both <d,m1> and <d,m2> are negative at an outer
   corner (kind 1), or when either is negative at an inner corner (kind 2). */
static int wedge_blocks(const double *w, const double *X, const double *Q)
{
    double d[3];
    sub3(Q, X, d);
    double a1 = dot3(d, w), a2 = dot3(d, w + 3);
    if (w[6] == 1.0) return a1 < 0.0 && a2 < 0.0;
    if (w[6] == 2.0) return a1 < 0.0 || a2 < 0.0;
    return 0;
}

int orc_visible_one(const orc_scene *s, const double rx[3], int n, const int32_t *ids, const double *X,
                    double min_seg)
{
    if (!ids_ok(s, n, ids)) return 0;
    if (s->wd)
        for (int k = 0; k < n; k++) {
            int j = ids[k] - s->n_pl;
            if (j < 0 || j >= s->n_ln) continue;
            const double *P = (k == 0) ? s->tx : X + 3 * (k - 1);
            const double *Q = (k == n - 1) ? rx : X + 3 * (k + 1);
            const double *w = s->wd + 7 * (size_t)j;
            if (wedge_blocks(w, X + 3 * k, P) || wedge_blocks(w, X + 3 * k, Q)) return 0;
        }
    for (int k = 0; k <= n; k++) {
        const double *P = (k == 0) ? s->tx : X + 3 * (k - 1);
        const double *Q = (k == n) ? rx : X + 3 * k;
        const int ip = (k == 0) ? -1 : ids[k - 1], iq = (k == n) ? -1 : ids[k];
        double d[3];
        sub3(Q, P, d);
        double L = norm3(d);
        if (!(L > 0.0)) return 0;
        double tmin = min_seg / L, tmax = 1.0 - tmin;
        for (int j = 0; j < s->n_pl; j++)
            if (j != ip && j != iq && seg_hits_plane(s->pl + 13 * (size_t)j, P, d, tmin, tmax)) return 0;
        for (int j = 0; j < s->n_q; j++) {
            int gid = s->n_pl + s->n_ln + j;
            if (gid != ip && gid != iq && seg_hits_quadric(s->q + 17 * (size_t)j, P, d, tmin, tmax)) return 0;
        }
    }
    return 1;
}

/* ------------------------------------------------------------ batches */
void orc_solve_batch(const orc_scene *s, int64_t nb, const double *rx, const int32_t *rx_index,
                     const int32_t *order, const int32_t *prim, const double *x0,
                     const orc_lm_opts *o, double *x, double *cost, int32_t *iters,
                     uint8_t *status, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < nb; i++) {
        int n = order[i];
        int32_t ids[MAXN];
        double X[MAXU], X0[MAXU];
        for (int k = 0; k < MAXN; k++) ids[k] = prim[k * nb + i];
        if (x0)
            for (int j = 0; j < MAXU; j++) X0[j] = x0[j * nb + i];
        for (int j = 0; j < MAXU; j++) X[j] = 0.0;
        double c;
        int32_t it;
        int st = (n >= 1 && n <= MAXN)
                     ? orc_solve_one(s, rx + 3 * (size_t)rx_index[i], n, ids, x0 ? X0 : NULL, o, X, &c, &it)
                     : ORC_BAD_INPUT;
        if (!(n >= 1 && n <= MAXN)) { c = INFINITY; it = 0; }
        for (int j = 0; j < MAXU; j++) x[j * nb + i] = (j < 3 * n) ? X[j] : 0.0;
        cost[i] = c;
        iters[i] = it;
        status[i] = (uint8_t)st;
    }
}

void orc_solve_batch_param(const orc_scene *s, int64_t nb, const double *rx, const int32_t *rx_index,
                           const int32_t *order, const int32_t *prim, const double *x0,
                           const orc_lm_opts *o, double *x, double *cost, int32_t *iters,
                           uint8_t *status, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < nb; i++) {
        int n = order[i];
        int32_t ids[MAXN];
        double X[MAXU], X0[MAXU];
        for (int k = 0; k < MAXN; k++) ids[k] = prim[k * nb + i];
        if (x0)
            for (int j = 0; j < MAXU; j++) X0[j] = x0[j * nb + i];
        for (int j = 0; j < MAXU; j++) X[j] = 0.0;
        double c = INFINITY;
        int32_t it = 0;
        int st = (n >= 1 && n <= MAXN)
                     ? orc_solve_one_param(s, rx + 3 * (size_t)rx_index[i], n, ids, x0 ? X0 : NULL, o, X, &c, &it)
                     : ORC_BAD_INPUT;
        for (int j = 0; j < MAXU; j++) x[j * nb + i] = (n >= 1 && n <= MAXN && j < 3 * n) ? X[j] : 0.0;
        cost[i] = c;
        iters[i] = it;
        status[i] = (uint8_t)st;
    }
}

void orc_visible_batch(const orc_scene *s, int64_t nb, const double *rx, const int32_t *rx_index,
                       const int32_t *order, const int32_t *prim, const double *x, const uint8_t *accept,
                       double min_seg, uint8_t *visible, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < nb; i++) {
        int n = order[i];
        int32_t ids[MAXN];
        double X[MAXU];
        for (int k = 0; k < MAXN; k++) ids[k] = prim[k * nb + i];
        for (int j = 0; j < MAXU; j++) X[j] = x[j * nb + i];
        visible[i] = (accept[i] && n >= 1 && n <= MAXN)
                         ? (uint8_t)orc_visible_one(s, rx + 3 * (size_t)rx_index[i], n, ids, X, min_seg)
                         : 0;
    }
}

void orc_accept_batch(const orc_scene *s, int64_t nb, const double *rx, const int32_t *rx_index,
                      const int32_t *order, const int32_t *prim, const double *x,
                      const uint8_t *status, double tau_res, double min_seg, uint8_t *accept,
                      int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < nb; i++) {
        int n = order[i];
        int32_t ids[MAXN];
        double X[MAXU];
        for (int k = 0; k < MAXN; k++) ids[k] = prim[k * nb + i];
        for (int j = 0; j < MAXU; j++) X[j] = x[j * nb + i];
        accept[i] = (n >= 1 && n <= MAXN)
                        ? (uint8_t)orc_accept_one(s, rx + 3 * (size_t)rx_index[i], n, ids, X, status[i], tau_res, min_seg)
                        : 0;
    }
}

/* ------------------------------------------------------------ candidate generation
 * Alg. 1 starts from a visibility matrix of the objects and an adjacency
 * matrix that adds BS (TX) and UE (RX), and takes every simple path from BS
 * to UE through at most n_t objects as an interaction list (Sec. II-C,
 * Figs. 3-4).  Object i sees object j when some segment between a sample
 * point of i and one of j leaves both objects into free space and crosses
 * no other facet or paraboloid patch.  Sample points, per side count k:
 *   rectangle   the k x k cell centres o + u eu + v ev, u, v = (2a+1)/(2k)
 *   edge        s0 + (2a+1)/(2k) (s1 - s0) along the edge
 *   paraboloid  the points of the k x k grid (2a+1-k)/k r_ap across the axis
 *               strictly inside the aperture, lifted onto the surface (a
 *               quadric of another kind: its anchor point only)
 *   circle      2k points from the rational parametrisation of the circle,
 *               t = (2a+1-k)/k and the antipodes
 * Each is computed in the order written here, in IEEE FP64 without
 * contraction. */
static int obj_type(const orc_scene *s, int g)
{
    if (g < s->n_pl) return TP;
    if (g < s->n_pl + s->n_ln) return TL;
    if (g < s->n_pl + s->n_ln + s->n_q) return TQ;
    return TC;
}

static const double *obj_rec(const orc_scene *s, int g)
{
    if (g < s->n_pl) return s->pl + 13 * (size_t)g;
    g -= s->n_pl;
    if (g < s->n_ln) return s->ln + 8 * (size_t)g;
    g -= s->n_ln;
    if (g < s->n_q) return s->q + 17 * (size_t)g;
    return s->c + 7 * (size_t)(g - s->n_q);
}

/* A paraboloid of revolution (A = kap (I - ax ax^T), b = -ax, c = 0):
   returns kap, or -1 for another quadric. */
static double revolution_kappa(const double *r)
{
    const double *ax = r + 13;
    double kap = 0.5 * (r[3] + r[6] + r[8]);
    const double A[3][3] = {{r[3], r[4], r[5]}, {r[4], r[6], r[7]}, {r[5], r[7], r[8]}};
    double err = fabs(r[12]);
    for (int i = 0; i < 3; i++) {
        err = fmax(err, fabs(r[9 + i] + ax[i]));
        for (int j = 0; j < 3; j++) err = fmax(err, fabs(A[i][j] - kap * ((i == j ? 1.0 : 0.0) - ax[i] * ax[j])));
    }
    return (kap > 0.0 && err <= 1e-9 * (1.0 + kap)) ? kap : -1.0;
}

int orc_samples(const orc_scene *s, int g, int k, double *pts)
{
    const double *r = obj_rec(s, g);
    int t = obj_type(s, g), m = 0;
    if (t == TP) {
        for (int a = 0; a < k; a++)
            for (int b = 0; b < k; b++) {
                double u = (double)(2 * a + 1) / (double)(2 * k), v = (double)(2 * b + 1) / (double)(2 * k);
                for (int c = 0; c < 3; c++) pts[3 * m + c] = (r[4 + c] + u * r[7 + c]) + v * r[10 + c];
                m++;
            }
    } else if (t == TL) {
        for (int a = 0; a < k; a++) {
            double f = (double)(2 * a + 1) / (double)(2 * k);
            double sp = r[6] + f * (r[7] - r[6]);
            for (int c = 0; c < 3; c++) pts[3 * m + c] = r[c] + sp * r[3 + c];
            m++;
        }
    } else if (t == TQ) {
        double kap = revolution_kappa(r);
        if (kap < 0.0) {
            for (int c = 0; c < 3; c++) pts[c] = r[c];
            return 1;
        }
        double e1[3], e2[3];
        onb_duff(r + 13, e1, e2);
        for (int a = 0; a < k; a++)
            for (int b = 0; b < k; b++) {
                int ia = 2 * a + 1 - k, ib = 2 * b + 1 - k;
                if (ia * ia + ib * ib >= k * k) continue;
                double u = r[16] * ((double)ia / (double)k), v = r[16] * ((double)ib / (double)k);
                double h = kap * (u * u + v * v);
                for (int c = 0; c < 3; c++) pts[3 * m + c] = ((r[c] + u * e1[c]) + v * e2[c]) + h * r[13 + c];
                m++;
            }
    } else {
        double u1[3], u2[3];
        onb_duff(r + 3, u1, u2);
        for (int a = 0; a < k; a++) {
            double tt = (double)(2 * a + 1 - k) / (double)k;
            double den = 1.0 + tt * tt;
            double x = (1.0 - tt * tt) / den, y = (2.0 * tt) / den;
            for (int c = 0; c < 3; c++) {
                pts[3 * m + c] = r[c] + r[6] * (x * u1[c] + y * u2[c]);
                pts[3 * (m + 1) + c] = r[c] + r[6] * ((-x) * u1[c] + (-y) * u2[c]);
            }
            m += 2;
        }
    }
    return m;
}

/* Does a segment from the point X of object g in direction d leave g into
   free space (strictly)?  A facet with a side: d points to that side; a
   two-sided facet or a paraboloid: d is not tangent; an edge with a wedge:
   d points strictly outside the solid; other edges and circles: always. */
static int leaves_obj(const orc_scene *s, int g, const double *X, const double *d)
{
    int t = obj_type(s, g);
    const double *r = obj_rec(s, g);
    if (t == TP) {
        double a = dot3(d, r), sd = s->sd ? s->sd[g] : 0.0;
        if (sd > 0.0) return a > 0.0;
        if (sd < 0.0) return a < 0.0;
        return a != 0.0;
    }
    if (t == TL) {
        if (!s->wd) return 1;
        const double *w = s->wd + 7 * (size_t)(g - s->n_pl);
        double a1 = dot3(d, w), a2 = dot3(d, w + 3);
        if (w[6] == 1.0) return a1 > 0.0 || a2 > 0.0;
        if (w[6] == 2.0) return a1 > 0.0 && a2 > 0.0;
        return 1;
    }
    if (t == TQ) {
        const double A[3][3] = {{r[3], r[4], r[5]}, {r[4], r[6], r[7]}, {r[5], r[7], r[8]}};
        double w[3], gr[3];
        sub3(X, r, w);
        for (int i = 0; i < 3; i++) gr[i] = 2.0 * (A[i][0] * w[0] + A[i][1] * w[1] + A[i][2] * w[2]) + r[9 + i];
        return dot3(d, gr) != 0.0;
    }
    return 1;
}

/* The segment P -> Q crosses a facet or paraboloid patch other than gi, gj
   strictly inside (more than min_seg from its ends). */
static int seg_blocked(const orc_scene *s, const double *P, const double *Q, int gi, int gj, double min_seg)
{
    double d[3];
    sub3(Q, P, d);
    double L = norm3(d);
    if (!(L > 0.0)) return 1;
    double tmin = min_seg / L, tmax = 1.0 - tmin;
    for (int j = 0; j < s->n_pl; j++)
        if (j != gi && j != gj && seg_hits_plane(s->pl + 13 * (size_t)j, P, d, tmin, tmax)) return 1;
    for (int j = 0; j < s->n_q; j++) {
        int gid = s->n_pl + s->n_ln + j;
        if (gid != gi && gid != gj && seg_hits_quadric(s->q + 17 * (size_t)j, P, d, tmin, tmax)) return 1;
    }
    return 0;
}

#define SAMPLE_CAP(k) ((k) * (k) + 2 * (k))

void orc_visibility(const orc_scene *s, int k, double min_seg, uint8_t *V, uint8_t *B, int nthreads)
{
    int n = s->n_pl + s->n_ln + s->n_q + s->n_c;
    memset(V, 0, (size_t)n * n);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int i = 0; i < n; i++) {
        double Si[3 * SAMPLE_CAP(16)], Sj[3 * SAMPLE_CAP(16)];
        int mi = orc_samples(s, i, k, Si);
        /* BS row: a segment from BS to a sample of i */
        B[i] = 0;
        for (int a = 0; a < mi && !B[i]; a++) {
            double d[3];
            sub3(s->tx, Si + 3 * a, d);
            if (leaves_obj(s, i, Si + 3 * a, d) && !seg_blocked(s, s->tx, Si + 3 * a, -1, i, min_seg)) B[i] = 1;
        }
        for (int j = i + 1; j < n; j++) {
            int mj = orc_samples(s, j, k, Sj), vis = 0;
            for (int a = 0; a < mi && !vis; a++)
                for (int b = 0; b < mj && !vis; b++) {
                    const double *p = Si + 3 * a, *q = Sj + 3 * b;
                    double d[3], e[3];
                    sub3(q, p, d);
                    sub3(p, q, e);
                    if (leaves_obj(s, i, p, d) && leaves_obj(s, j, q, e) && !seg_blocked(s, p, q, i, j, min_seg))
                        vis = 1;
                }
            V[(size_t)i * n + j] = V[(size_t)j * n + i] = (uint8_t)vis;
        }
    }
}

void orc_visibility_rx(const orc_scene *s, const double *rx, int n_rx, int k, double min_seg, uint8_t *U,
                       uint8_t *los, int nthreads)
{
    int n = s->n_pl + s->n_ln + s->n_q + s->n_c;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int ri = 0; ri < n_rx; ri++) {
        const double *R = rx + 3 * (size_t)ri;
        double S[3 * SAMPLE_CAP(16)];
        los[ri] = (uint8_t)!seg_blocked(s, s->tx, R, -1, -1, min_seg);
        for (int j = 0; j < n; j++) {
            int m = orc_samples(s, j, k, S), vis = 0;
            for (int a = 0; a < m && !vis; a++) {
                double d[3];
                sub3(R, S + 3 * a, d);
                if (leaves_obj(s, j, S + 3 * a, d) && !seg_blocked(s, S + 3 * a, R, j, -1, min_seg)) vis = 1;
            }
            U[(size_t)ri * n + j] = (uint8_t)vis;
        }
    }
}

/* Depth-first enumeration in increasing object id of the simple paths
   BS -> v1 -> ... -> v_ord -> UE of one receiver. */
typedef struct {
    int n, ord, edge_last;
    const uint8_t *V, *B, *U, *edge;
    int32_t path[MAXN];
    int64_t count, cap;
    int32_t rxi, *rx_index, *order, *prim;
} orc_dfs;

static void dfs_step(orc_dfs *D, int depth)
{
    for (int v = 0; v < D->n; v++) {
        if (depth == 0) {
            if (!D->B[v]) continue;
        } else {
            int u = D->path[depth - 1];
            if (!D->V[(size_t)u * D->n + v] || (D->edge_last && D->edge[u])) continue;
            int seen = 0;
            for (int q = 0; q < depth; q++) seen |= D->path[q] == v;
            if (seen) continue;
        }
        D->path[depth] = v;
        if (depth + 1 < D->ord) {
            dfs_step(D, depth + 1);
        } else if (D->U[v]) {
            if (D->count < D->cap) {
                D->rx_index[D->count] = D->rxi;
                D->order[D->count] = D->ord;
                for (int q = 0; q < MAXN; q++) D->prim[(size_t)q * D->cap + D->count] = q < D->ord ? D->path[q] : -1;
            }
            D->count++;
        }
    }
}

int64_t orc_candidates(const orc_scene *s, const uint8_t *V, const uint8_t *B, const uint8_t *U, int n_rx,
                       int max_order, int edge_last, int64_t cap, int32_t *rx_index, int32_t *order, int32_t *prim)
{
    int n = s->n_pl + s->n_ln + s->n_q + s->n_c;
    uint8_t edge[4096];
    if (n > 4096 || max_order < 1 || max_order > MAXN) return -1;
    for (int g = 0; g < n; g++) edge[g] = (uint8_t)(obj_type(s, g) == TL || obj_type(s, g) == TC);
    orc_dfs D;
    D.n = n;
    D.V = V;
    D.B = B;
    D.edge = edge;
    D.edge_last = edge_last;
    D.count = 0;
    D.cap = cap;
    D.rx_index = rx_index;
    D.order = order;
    D.prim = prim;
    for (int ri = 0; ri < n_rx; ri++) {
        D.U = U + (size_t)ri * n;
        D.rxi = ri;
        for (int o = 1; o <= max_order; o++) {
            D.ord = o;
            dfs_step(&D, 0);
        }
    }
    return D.count;
}
