// Geometric tests of physical validation and of candidate generation, in
// plain IEEE FP64 in a fixed order with no contraction, so that each
// decision is the one a plain FP64 implementation of the same test takes.
#pragma once
#include "mpt_internal.hpp"

namespace mpt {

// A kept path's segments may not pass through another object: a rectangle
// facet or a paraboloid patch crossed strictly inside a segment (more than
// min_seg from its ends) blocks it; the objects a segment starts or ends on
// are not tested; edges and circles have no area.  The arithmetic is plain
// IEEE FP64 in a fixed order with no contraction, so each decision is the
// one a plain FP64 implementation of the same test takes.
__device__ __forceinline__ double vdot(const double *a, const double *b)
{
#pragma clang fp contract(off)
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

__device__ __forceinline__ bool vis_plane(const double *r, const double P[3], const double d[3], double tmin, double tmax)
{
#pragma clang fp contract(off)
    const double den = vdot(r, d);
    if (den == 0.0) return false;
    const double t = (r[3] - vdot(r, P)) / den;
    if (!(t > tmin && t < tmax)) return false;
    double w[3];
    for (int i = 0; i < 3; i++) w[i] = (P[i] + t * d[i]) - r[4 + i];
    const double a = vdot(w, r + 7), b = vdot(w, r + 10);
    return a >= 0.0 && a <= vdot(r + 7, r + 7) && b >= 0.0 && b <= vdot(r + 10, r + 10);
}

__device__ __forceinline__ bool vis_quadric(const double *r, const double P[3], const double d[3], double tmin, double tmax)
{
#pragma clang fp contract(off)
    const double A[3][3] = {{r[3], r[4], r[5]}, {r[4], r[6], r[7]}, {r[5], r[7], r[8]}};
    const double w[3] = {P[0] - r[0], P[1] - r[1], P[2] - r[2]};
    double Ad[3], Aw[3];
    for (int i = 0; i < 3; i++) {
        Ad[i] = A[i][0] * d[0] + A[i][1] * d[1] + A[i][2] * d[2];
        Aw[i] = A[i][0] * w[0] + A[i][1] * w[1] + A[i][2] * w[2];
    }
    const double a = vdot(d, Ad);
    const double b = 2.0 * vdot(w, Ad) + vdot(r + 9, d);
    const double c = vdot(w, Aw) + vdot(r + 9, w) + r[12];
    double ts[2];
    int nt = 0;
    if (a == 0.0) {
        if (b != 0.0) ts[nt++] = -c / b;
    } else {
        const double disc = b * b - 4.0 * a * c;
        if (disc < 0.0) return false;
        const double sq = sqrt(disc);
        const double q = -0.5 * (b + (b >= 0.0 ? sq : -sq));
        ts[nt++] = q / a;
        if (q != 0.0) ts[nt++] = c / q;
    }
    for (int j = 0; j < nt; j++) {
        const double t = ts[j];
        if (!(t > tmin && t < tmax)) continue;
        double v[3];
        for (int i = 0; i < 3; i++) v[i] = (P[i] + t * d[i]) - r[i];
        const double h = vdot(v, r + 13);
        for (int i = 0; i < 3; i++) v[i] = v[i] - h * r[13 + i];
        if (vdot(v, v) <= r[16] * r[16]) return true;
    }
    return false;
}

// A segment at a straight edge with a wedge may not leave the edge point X
// into the solid: m1, m2 are the normals of the faces meeting at the edge,
// pointing into free space; at an outer corner (kind 1) the solid is where
// both <d, m> are negative, at an inner corner (kind 2) where either is.
__device__ __forceinline__ bool vis_wedge(const double *w, const double X[3], const double Q[3])
{
#pragma clang fp contract(off)
    const double d[3] = {Q[0] - X[0], Q[1] - X[1], Q[2] - X[2]};
    const double a1 = vdot(d, w), a2 = vdot(d, w + 3);
    if (w[6] == 1.0) return a1 < 0.0 && a2 < 0.0;
    if (w[6] == 2.0) return a1 < 0.0 || a2 < 0.0;
    return false;
}


// ------------------------------------------------------------------ candidate generation
// Sample points of object g, k per side (at most k*k + 2k):
//   rectangle   the k x k cell centres o + u eu + v ev, u, v = (2a+1)/(2k)
//   edge        s0 + (2a+1)/(2k) (s1 - s0) along the edge
//   paraboloid  the points (2a+1-k)/k r_ap of the k x k grid across the axis
//               strictly inside the aperture (an integer test), lifted onto
//               the surface; a quadric of another kind: its anchor point
//   circle      the rational points ((1-t^2), 2t)/(1+t^2), t = (2a+1-k)/k,
//               and their antipodes
__host__ __device__ constexpr int sample_cap(int k) { return k * k + 2 * k; }

// Orthonormal pair across a unit vector (Duff et al., JCGT 2017), without
// contraction.
__device__ __forceinline__ void duff_frame(const double *a, double u1[3], double u2[3])
{
#pragma clang fp contract(off)
    const double sg = a[2] >= 0.0 ? 1.0 : -1.0;
    const double q = -1.0 / (sg + a[2]);
    const double b = a[0] * a[1] * q;
    u1[0] = 1.0 + sg * a[0] * a[0] * q;
    u1[1] = sg * b;
    u1[2] = -sg * a[0];
    u2[0] = b;
    u2[1] = sg + a[1] * a[1] * q;
    u2[2] = -a[1];
}

// kappa of a paraboloid of revolution (A = kappa (I - ax ax^T), b = -ax,
// c = 0), or -1 for another quadric.
__device__ __forceinline__ double revolution_kappa(const double *r)
{
#pragma clang fp contract(off)
    const double *ax = r + 13;
    const double kap = 0.5 * (r[3] + r[6] + r[8]);
    const double A[3][3] = {{r[3], r[4], r[5]}, {r[4], r[6], r[7]}, {r[5], r[7], r[8]}};
    double err = fabs(r[12]);
    for (int i = 0; i < 3; i++) {
        err = fmax(err, fabs(r[9 + i] + ax[i]));
        for (int j = 0; j < 3; j++) err = fmax(err, fabs(A[i][j] - kap * ((i == j ? 1.0 : 0.0) - ax[i] * ax[j])));
    }
    return (kap > 0.0 && err <= 1e-9 * (1.0 + kap)) ? kap : -1.0;
}

__device__ inline int obj_samples(const SceneDev &s, int g, int k, double *pts)
{
#pragma clang fp contract(off)
    const double *r = s.rec64 + (size_t)g * kRec;
    const int t = prim_type(g, s.n_pl, s.n_pl_ln, s.n_pl_ln_q);
    int m = 0;
    if (t == TP) {
        for (int a = 0; a < k; a++)
            for (int b = 0; b < k; b++) {
                const double u = (double)(2 * a + 1) / (double)(2 * k), v = (double)(2 * b + 1) / (double)(2 * k);
                for (int c = 0; c < 3; c++) pts[3 * m + c] = (r[4 + c] + u * r[7 + c]) + v * r[10 + c];
                m++;
            }
    } else if (t == TL) {
        for (int a = 0; a < k; a++) {
            const double f = (double)(2 * a + 1) / (double)(2 * k);
            const double sp = r[6] + f * (r[7] - r[6]);
            for (int c = 0; c < 3; c++) pts[3 * m + c] = r[c] + sp * r[3 + c];
            m++;
        }
    } else if (t == TQ) {
        const double kap = revolution_kappa(r);
        if (kap < 0.0) {
            for (int c = 0; c < 3; c++) pts[c] = r[c];
            return 1;
        }
        double e1[3], e2[3];
        duff_frame(r + 13, e1, e2);
        for (int a = 0; a < k; a++)
            for (int b = 0; b < k; b++) {
                const int ia = 2 * a + 1 - k, ib = 2 * b + 1 - k;
                if (ia * ia + ib * ib >= k * k) continue;
                const double u = r[16] * ((double)ia / (double)k), v = r[16] * ((double)ib / (double)k);
                const double h = kap * (u * u + v * v);
                for (int c = 0; c < 3; c++) pts[3 * m + c] = ((r[c] + u * e1[c]) + v * e2[c]) + h * r[13 + c];
                m++;
            }
    } else {
        double u1[3], u2[3];
        duff_frame(r + 3, u1, u2);
        for (int a = 0; a < k; a++) {
            const double tt = (double)(2 * a + 1 - k) / (double)k;
            const double den = 1.0 + tt * tt;
            const double x = (1.0 - tt * tt) / den, y = (2.0 * tt) / den;
            for (int c = 0; c < 3; c++) {
                pts[3 * m + c] = r[c] + r[6] * (x * u1[c] + y * u2[c]);
                pts[3 * (m + 1) + c] = r[c] + r[6] * ((-x) * u1[c] + (-y) * u2[c]);
            }
            m += 2;
        }
    }
    return m;
}

// Does a segment from the point X of object g in direction d leave g into
// free space (strictly)?  A facet with a side: d points to that side; a
// two-sided facet or a paraboloid: d is not tangent; an edge with a wedge:
// d points strictly outside the solid; other edges and circles: always.
__device__ __forceinline__ bool leaves_obj(const SceneDev &s, int g, const double X[3], const double d[3])
{
#pragma clang fp contract(off)
    const double *r = s.rec64 + (size_t)g * kRec;
    const int t = prim_type(g, s.n_pl, s.n_pl_ln, s.n_pl_ln_q);
    if (t == TP) {
        const double a = vdot(d, r), sd = s.side ? s.side[g] : 0.0;
        if (sd > 0.0) return a > 0.0;
        if (sd < 0.0) return a < 0.0;
        return a != 0.0;
    }
    if (t == TL) {
        if (!s.wedge) return true;
        const double *w = s.wedge + 7 * (size_t)(g - s.n_pl);
        const double a1 = vdot(d, w), a2 = vdot(d, w + 3);
        if (w[6] == 1.0) return a1 > 0.0 || a2 > 0.0;
        if (w[6] == 2.0) return a1 > 0.0 && a2 > 0.0;
        return true;
    }
    if (t == TQ) {
        const double A[3][3] = {{r[3], r[4], r[5]}, {r[4], r[6], r[7]}, {r[5], r[7], r[8]}};
        const double w[3] = {X[0] - r[0], X[1] - r[1], X[2] - r[2]};
        double gr[3];
        for (int i = 0; i < 3; i++) gr[i] = 2.0 * (A[i][0] * w[0] + A[i][1] * w[1] + A[i][2] * w[2]) + r[9 + i];
        return vdot(d, gr) != 0.0;
    }
    return true;
}

// The segment P -> Q crosses a facet or paraboloid patch other than gi, gj
// strictly inside (more than min_seg from its ends).  prec / qrec: the
// plane and quadric records (possibly staged in LDS).
__device__ __forceinline__ bool seg_blocked(const SceneDev &s, const double *prec, const double *qrec,
                                            const double P[3], const double Q[3], int gi, int gj, double min_seg)
{
#pragma clang fp contract(off)
    const double d[3] = {Q[0] - P[0], Q[1] - P[1], Q[2] - P[2]};
    const double L = sqrt(vdot(d, d));
    if (!(L > 0.0)) return true;
    const double tmin = min_seg / L, tmax = 1.0 - tmin;
    for (int j = 0; j < s.n_pl; j++)
        if (j != gi && j != gj && vis_plane(prec + (size_t)j * kRec, P, d, tmin, tmax)) return true;
    const int nq = s.n_pl_ln_q - s.n_pl_ln;
    for (int j = 0; j < nq; j++) {
        const int gid = s.n_pl_ln + j;
        if (gid != gi && gid != gj && vis_quadric(qrec + (size_t)j * kRec, P, d, tmin, tmax)) return true;
    }
    return false;
}

}  // namespace mpt
