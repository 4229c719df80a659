// Device-side math of the batched Min-Path-Tracing solve (gfx950).
//
// One lane owns one candidate path.  Everything a Levenberg-Marquardt
// iteration needs lives in that lane's registers: the points X_1..X_N, the
// block-banded normal equations and their Cholesky factor.  The order N is a
// template parameter so every loop unrolls and every index is a constant.
//
// Paper, Sec. III-B: the residual of interaction k depends on X_{k-1}, X_k,
// X_{k+1} only, so J is block-tridiagonal and J^T J block-pentadiagonal with
// 3x3 blocks (the tridiagonal structure the conclusion suggests exploiting).
// Only the 93 (N = 5) in-band entries of J^T J are ever touched.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpt {

constexpr int kRec = 18;        // doubles / floats per packed primitive record
constexpr int kMaxN = 5;
constexpr int kRow = 16;        // doubles per solve in a point array (3 kMaxN coordinates, then zeros)

enum : int { TP = 0, TL = 1, TQ = 2, TC = 3 };
enum : int { ST_CONV = 0, ST_MAXIT = 1, ST_STALL = 2, ST_DIVERGED = 3, ST_DEGEN = 4,
             ST_BAD = 5, ST_LOCALMIN = 6, ST_OUTSIDE = 7, ST_PARKED = 250, ST_RUNNING = 255 };

// Packed record layout (kRec wide), written by the scene pack kernel:
//  plane   : n[0..2] d[3] o[4..6] eu[7..9] ev[10..12] e1[13..15] (eu/|eu|, the
//            parametric frame) n_front[16] n_back[17] (refractive indices of a
//            refracting facet; 0 for a mirror)
//  line    : p[0..2] e[3..5] s0[6] s1[7] u1[8..10] u2[11..13]
//  quadric : p[0..2] A[3..8] (xx xy xz yy yz zz) b[9..11] c[12] ax[13..15] rap[16]
//  circle  : c[0..2] n[3..5] R[6]

template <typename T>
struct SceneT {
    const T *rec;      // [n_prims][kRec]
    int n_pl, n_pl_ln, n_pl_ln_q, n_all;
    T tx[3];           // transmitter in this frame (0 in the TX-local frame)
    T glo[3], ghi[3];  // guard box
};

__host__ __device__ __forceinline__ int prim_type(int id, int a, int b, int c)
{
    return (id < a) ? TP : (id < b) ? TL : (id < c) ? TQ : TC;
}

__host__ __device__ __forceinline__ double dsqrt(double x) { return sqrt(x); }
__host__ __device__ __forceinline__ float dsqrt(float x) { return __builtin_sqrtf(x); }

// Reciprocal and reciprocal square root.  FP32: the hardware approximations
// (about 1 ulp; the FP32 pass only has to land close to a root, the FP64
// polish restores full accuracy).  FP64: the hardware seed refined by
// Newton steps (each doubles the number of correct bits) to within a few ulp,
// instead of the IEEE division and square-root sequences.
__host__ __device__ __forceinline__ float drcp(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}
__host__ __device__ __forceinline__ double drcp(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(x);
    r = r * (2.0 - x * r);
    r = r * (2.0 - x * r);
    return r;
#else
    return 1.0 / x;
#endif
}
__host__ __device__ __forceinline__ float drsqrt(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rsqf(x);
#else
    return 1.0f / sqrtf(x);
#endif
}
__host__ __device__ __forceinline__ double drsqrt(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rsq(x);
    r = r * (1.5 - 0.5 * x * r * r);
    r = r * (1.5 - 0.5 * x * r * r);
    return r;
#else
    return 1.0 / sqrt(x);
#endif
}

template <typename T>
__host__ __device__ __forceinline__ T dot3(const T *a, const T *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// -------------------------------------------------------------------------
// Rows of one interaction (5 slots: 0..2 law rows, 3..4 object rows; unused
// slots are exactly zero with zero derivatives).  Law rows are the unit-form
// laws scaled by S = (|i| + |r|)/2 (metres):
//   reflection  S (r^ - i^ + 2 <i^,n^> n^)                (Eqs. 1, 2, 8)
//   diffraction S <i^ - r^, e^>                           (Eqs. 3, 4, 9)
// object rows: f(X) for a surface; for a straight edge the two coordinates
// across the line; for a circle the distance to its plane and
// (|X-c|^2 - R^2)/(2R)                                     (Eq. 11)
// Derivative blocks: Jp = d/dX_{k-1} (law rows), Jk = d/dX_k (all rows),
// Jn = d/dX_{k+1} (law rows).
// Returns false when a direction is undefined (degenerate).  REFR = false
// compiles the refracting-facet rows out (scenes without such facets).
// -------------------------------------------------------------------------
template <typename T, bool WITH_J, bool REFR = true>
__host__ __device__ __forceinline__ bool interaction_rows(int t, const T *__restrict__ r, const T *Xp, const T *Xk,
                                                 const T *Xn, T u[5], T Jp[3][3], T Jk[5][3], T Jn[3][3])
{
    // No early exits: an undefined direction sets valid = false and the
    // arithmetic continues on a harmless substitute value.
    bool valid = true;
    T a[3], b[3];
#pragma unroll
    for (int i = 0; i < 3; i++) { a[i] = Xk[i] - Xp[i]; b[i] = Xn[i] - Xk[i]; }
    T la2 = dot3(a, a), lb2 = dot3(b, b);
    valid = valid && (la2 > T(0)) && (lb2 > T(0));
    la2 = (la2 > T(0)) ? la2 : T(1);
    lb2 = (lb2 > T(0)) ? lb2 : T(1);
    const T ia = drsqrt(la2), ib = drsqrt(lb2);
    const T la = la2 * ia, lb = lb2 * ib;
    T ih[3], rh[3];
#pragma unroll
    for (int i = 0; i < 3; i++) { ih[i] = a[i] * ia; rh[i] = b[i] * ib; }
    const T S = T(0.5) * (la + lb);
    if (t == TP || t == TQ) {
        // plane: g = n, f = n.X - d.  quadric: w = X - p, g = 2 A w + b,
        // f = w^T A w + b^T w + c, with A = [[a0 a1 a2][a1 a3 a4][a2 a4 a5]]
        T g[3], f;
        if (t == TQ) {
            const T w0 = Xk[0] - r[0], w1 = Xk[1] - r[1], w2 = Xk[2] - r[2];
            const T Aw0 = r[3] * w0 + r[4] * w1 + r[5] * w2;
            const T Aw1 = r[4] * w0 + r[6] * w1 + r[7] * w2;
            const T Aw2 = r[5] * w0 + r[7] * w1 + r[8] * w2;
            f = w0 * Aw0 + w1 * Aw1 + w2 * Aw2 + r[9] * w0 + r[10] * w1 + r[11] * w2 + r[12];
            g[0] = T(2) * Aw0 + r[9];
            g[1] = T(2) * Aw1 + r[10];
            g[2] = T(2) * Aw2 + r[11];
        } else {
            f = r[0] * Xk[0] + r[1] * Xk[1] + r[2] * Xk[2] - r[3];
            g[0] = r[0];
            g[1] = r[1];
            g[2] = r[2];
        }
        T lg2 = dot3(g, g);
        valid = valid && (lg2 > T(0));
        lg2 = (lg2 > T(0)) ? lg2 : T(1);
        const T ig = drsqrt(lg2);
        const T nh[3] = {g[0] * ig, g[1] * ig, g[2] * ig};
        const T s = dot3(ih, nh);
        // a refracting facet (record entries 16, 17: the indices of the side
        // the normal points to and of the other side): Snell's law, the part
        // of n r^ along the facet equals that of n i^ (Sec. VI), with n_i the
        // index of the side the ray arrives from
        const bool refr = REFR && (t == TP) && (r[16] > T(0));
        const T n_i = refr ? ((s < T(0)) ? r[16] : r[17]) : T(0);
        const T n_t = refr ? ((s < T(0)) ? r[17] : r[16]) : T(0);
        const T sr = dot3(rh, nh);
        T ul[3];
#pragma unroll
        for (int i = 0; i < 3; i++)
            ul[i] = refr ? n_t * (rh[i] - sr * nh[i]) - n_i * (ih[i] - s * nh[i]) : rh[i] - ih[i] + T(2) * s * nh[i];
#pragma unroll
        for (int i = 0; i < 3; i++) u[i] = S * ul[i];
        u[3] = f;
        u[4] = T(0);
        if (WITH_J) {
            // (Q Pa)_ij = Pa_ij - nh_i m_j with m = 2 (nh - s ih)/|a|
            T m[3];
#pragma unroll
            for (int j = 0; j < 3; j++) m[j] = T(2) * (nh[j] - s * ih[j]) * ia;
            // curvature of a quadric: Nm = (I - nh nh^T) B, B = 2A/|g|;
            // TN = 2 (nh ih^T + s I) Nm = 2 nh q^T + 2 s (B - nh v^T),
            // v = B nh, q = B ih - s v.  A plane has no curvature.
            T TN[3][3];
            if (t == TQ) {
                const T c2 = T(2) * ig;
                const T b0 = c2 * r[3], b1 = c2 * r[4], b2 = c2 * r[5], b3 = c2 * r[6], b4 = c2 * r[7],
                        b5 = c2 * r[8];
                const T v[3] = {b0 * nh[0] + b1 * nh[1] + b2 * nh[2], b1 * nh[0] + b3 * nh[1] + b4 * nh[2],
                                b2 * nh[0] + b4 * nh[1] + b5 * nh[2]};
                const T q[3] = {b0 * ih[0] + b1 * ih[1] + b2 * ih[2] - s * v[0],
                                b1 * ih[0] + b3 * ih[1] + b4 * ih[2] - s * v[1],
                                b2 * ih[0] + b4 * ih[1] + b5 * ih[2] - s * v[2]};
                const T Bm[3][3] = {{b0, b1, b2}, {b1, b3, b4}, {b2, b4, b5}};
                const T s2 = T(2) * s;
#pragma unroll
                for (int i = 0; i < 3; i++)
#pragma unroll
                    for (int j = 0; j < 3; j++) TN[i][j] = T(2) * nh[i] * q[j] + s2 * (Bm[i][j] - nh[i] * v[j]);
            } else {
#pragma unroll
                for (int i = 0; i < 3; i++)
#pragma unroll
                    for (int j = 0; j < 3; j++) TN[i][j] = T(0);
            }
            if (refr) {
                // u = n_t Pn r^ - n_i Pn i^, Pn = I - n n^T constant on a plane:
                // dU/dX_{k-1} = n_i Pn Pa, dU/dX_{k+1} = n_t Pn Pb, dU/dX_k = -(both)
                T ma[3], mb[3];
#pragma unroll
                for (int j = 0; j < 3; j++) {
                    ma[j] = (nh[j] - s * ih[j]) * ia;
                    mb[j] = (nh[j] - sr * rh[j]) * ib;
                }
#pragma unroll
                for (int i = 0; i < 3; i++) {
#pragma unroll
                    for (int j = 0; j < 3; j++) {
                        const T pa = ((i == j) ? ia : T(0)) - ih[i] * ih[j] * ia;
                        const T pb = ((i == j) ? ib : T(0)) - rh[i] * rh[j] * ib;
                        const T up = n_i * (pa - nh[i] * ma[j]);
                        const T un = n_t * (pb - nh[i] * mb[j]);
                        Jp[i][j] = S * up - T(0.5) * ul[i] * ih[j];
                        Jn[i][j] = S * un + T(0.5) * ul[i] * rh[j];
                        Jk[i][j] = -S * (up + un) + T(0.5) * ul[i] * (ih[j] - rh[j]);
                    }
                }
            } else {
#pragma unroll
                for (int i = 0; i < 3; i++) {
#pragma unroll
                    for (int j = 0; j < 3; j++) {
                        const T pa = ((i == j) ? ia : T(0)) - ih[i] * ih[j] * ia;
                        const T pb = ((i == j) ? ib : T(0)) - rh[i] * rh[j] * ib;
                        const T qpa = pa - nh[i] * m[j];
                        // product rule with dS: dS/dX_{k-1} = -ih/2, dS/dX_k = (ih - rh)/2, dS/dX_{k+1} = rh/2
                        Jp[i][j] = S * qpa - T(0.5) * ul[i] * ih[j];
                        Jn[i][j] = S * pb + T(0.5) * ul[i] * rh[j];
                        Jk[i][j] = S * (TN[i][j] - pb - qpa) + T(0.5) * ul[i] * (ih[j] - rh[j]);
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < 3; j++) { Jk[3][j] = g[j]; Jk[4][j] = T(0); }
        }
    } else {
        const T d[3] = {Xk[0] - r[0], Xk[1] - r[1], Xk[2] - r[2]};
        const T dv[3] = {ih[0] - rh[0], ih[1] - rh[1], ih[2] - rh[2]};
        T e[3], go0[3], go1[3], o0, o1, iw = T(0);
        if (t == TL) {
            // straight edge: fixed e, rows across the line
#pragma unroll
            for (int j = 0; j < 3; j++) {
                e[j] = r[3 + j];
                go0[j] = r[8 + j];
                go1[j] = r[11 + j];
            }
            o0 = dot3(d, go0);
            o1 = dot3(d, go1);
        } else {
            // circle: e = n x d / |n x d|, rows <d,n> and (|d|^2 - R^2)/(2R)
            const T w[3] = {r[4] * d[2] - r[5] * d[1], r[5] * d[0] - r[3] * d[2], r[3] * d[1] - r[4] * d[0]};
            T lw2 = dot3(w, w);
            valid = valid && (lw2 > T(0));
            lw2 = (lw2 > T(0)) ? lw2 : T(1);
            iw = drsqrt(lw2);
            const T R = r[6], iR = drcp(R);
#pragma unroll
            for (int j = 0; j < 3; j++) {
                e[j] = w[j] * iw;
                go0[j] = r[3 + j];
                go1[j] = d[j] * iR;
            }
            o0 = dot3(d, go0);
            o1 = (dot3(d, d) - R * R) * (T(0.5) * iR);
        }
        const T u0 = dot3(dv, e);
        u[0] = S * u0;
        u[1] = T(0);
        u[2] = T(0);
        u[3] = o0;
        u[4] = o1;
        if (WITH_J) {
            // circle: dv^T de/dX = (dv x n - <dv,e> (e x n)) / |w|; straight edge: 0
            T dvE[3] = {T(0), T(0), T(0)};
            if (t == TC) {
                const T n0 = r[3], n1 = r[4], n2 = r[5];
                const T dxn[3] = {dv[1] * n2 - dv[2] * n1, dv[2] * n0 - dv[0] * n2, dv[0] * n1 - dv[1] * n0};
                const T exn[3] = {e[1] * n2 - e[2] * n1, e[2] * n0 - e[0] * n2, e[0] * n1 - e[1] * n0};
#pragma unroll
                for (int j = 0; j < 3; j++) dvE[j] = (dxn[j] - u0 * exn[j]) * iw;
            }
            const T ei = dot3(e, ih), er = dot3(e, rh);
#pragma unroll
            for (int j = 0; j < 3; j++) {
                const T ePa = (e[j] - ei * ih[j]) * ia;
                const T ePb = (e[j] - er * rh[j]) * ib;
                Jp[0][j] = -S * ePa - T(0.5) * u0 * ih[j];
                Jn[0][j] = -S * ePb + T(0.5) * u0 * rh[j];
                Jk[0][j] = S * (ePa + ePb + dvE[j]) + T(0.5) * u0 * (ih[j] - rh[j]);
#pragma unroll
                for (int i = 1; i < 3; i++) { Jp[i][j] = T(0); Jn[i][j] = T(0); Jk[i][j] = T(0); }
                Jk[3][j] = go0[j];
                Jk[4][j] = go1[j];
            }
        }
    }
    return valid;
}

// ------------------------------------------------------------------ band
// Packed lower band of J^T J for N interactions of B unknowns each (B = 3:
// the points, B = 2: the parameters of the parametric form); an interaction's
// rows couple its own block and its two neighbours, so block (I, J) is
// nonzero only for |I - J| <= 2.
template <int N, int B = 3>
struct Band {
    static constexpr int M = B * N;
    static constexpr int SIZE = M * (M + 1) / 2;
    __host__ __device__ static constexpr bool in(int i, int j) { return i >= j && (i / B - j / B) <= 2; }
    __host__ __device__ static constexpr int at(int i, int j) { return i * (i + 1) / 2 + j; }
};

// Per-solve inputs as seen by the solver (in the solver's frame).
template <typename T, int N>
struct PathIn {
    T rx[3];
    int id[N];
    int ty[N];
    bool planar;  // planes and straight edges only (a unique root)
};

// Points of interaction k for the residual evaluated at X + dx (dx may be
// null): X_0 = TX, X_{N+1} = RX.
template <typename T, int N>
__host__ __device__ __forceinline__ void point_at(int k, const T *X, const T *dx, const T *tx, const T *rx, T out[3])
{
    if (k < 0) { out[0] = tx[0]; out[1] = tx[1]; out[2] = tx[2]; return; }
    if (k >= N) { out[0] = rx[0]; out[1] = rx[1]; out[2] = rx[2]; return; }
#pragma unroll
    for (int i = 0; i < 3; i++) out[i] = X[3 * k + i] + (dx ? dx[3 * k + i] : T(0));
}

// Residual cost and inf-norm at X (+dx).  Returns false if degenerate.
template <typename T, int N, bool REFR = true>
__host__ __device__ __forceinline__ bool eval_cost(const SceneT<T> &sc, const PathIn<T, N> &p, const T *X, const T *dx,
                                          T &C, T &rinf)
{
    C = T(0);
    rinf = T(0);
    bool ok = true;
#pragma unroll
    for (int k = 0; k < N; k++) {
        T Xp[3], Xk[3], Xn[3], u[5];
        point_at<T, N>(k - 1, X, dx, sc.tx, p.rx, Xp);
        point_at<T, N>(k, X, dx, sc.tx, p.rx, Xk);
        point_at<T, N>(k + 1, X, dx, sc.tx, p.rx, Xn);
        const bool okk = interaction_rows<T, false, REFR>(p.ty[k], sc.rec + (size_t)p.id[k] * kRec, Xp, Xk, Xn, u,
                                                    nullptr, nullptr, nullptr);
        ok = ok && okk;
#pragma unroll
        for (int i = 0; i < 5; i++) {
            C += u[i] * u[i];
            rinf = fmax(rinf, fabs(u[i]));
        }
    }
    return ok;
}

// Residual, J^T J (in-band, packed lower) and g = J^T R at X.
template <typename T, int N, bool REFR = true>
__host__ __device__ __forceinline__ bool assemble(const SceneT<T> &sc, const PathIn<T, N> &p, const T *X,
                                         T *A, T *g, T &C, T &rinf)
{
    constexpr int M = 3 * N;
#pragma unroll
    for (int i = 0; i < M; i++)
#pragma unroll
        for (int j = 0; j <= i; j++)
            if (Band<N>::in(i, j)) A[Band<N>::at(i, j)] = T(0);
#pragma unroll
    for (int i = 0; i < M; i++) g[i] = T(0);
    C = T(0);
    rinf = T(0);
    bool ok = true;
#pragma unroll
    for (int k = 0; k < N; k++) {
        T Xp[3], Xk[3], Xn[3], u[5], Jp[3][3], Jk[5][3], Jn[3][3];
        point_at<T, N>(k - 1, X, nullptr, sc.tx, p.rx, Xp);
        point_at<T, N>(k, X, nullptr, sc.tx, p.rx, Xk);
        point_at<T, N>(k + 1, X, nullptr, sc.tx, p.rx, Xn);
        const bool okk = interaction_rows<T, true, REFR>(p.ty[k], sc.rec + (size_t)p.id[k] * kRec, Xp, Xk, Xn, u, Jp, Jk, Jn);
        ok = ok && okk;
#pragma unroll
        for (int i = 0; i < 5; i++) {
            C += u[i] * u[i];
            rinf = fmax(rinf, fabs(u[i]));
        }
        // law rows couple blocks k-1, k, k+1
#pragma unroll
        for (int row = 0; row < 3; row++) {
            T jr[9];
#pragma unroll
            for (int c = 0; c < 3; c++) { jr[c] = Jp[row][c]; jr[3 + c] = Jk[row][c]; jr[6 + c] = Jn[row][c]; }
#pragma unroll
            for (int bi = 0; bi < 3; bi++) {
                const int Bi = k - 1 + bi;
                if (Bi < 0 || Bi >= N) continue;
#pragma unroll
                for (int ci = 0; ci < 3; ci++) {
                    const int gi = 3 * Bi + ci;
                    g[gi] += jr[3 * bi + ci] * u[row];
#pragma unroll
                    for (int bj = 0; bj < 3; bj++) {
                        const int Bj = k - 1 + bj;
                        if (Bj < 0 || Bj >= N) continue;
#pragma unroll
                        for (int cj = 0; cj < 3; cj++) {
                            const int gj = 3 * Bj + cj;
                            if (gj > gi) continue;
                            A[Band<N>::at(gi, gj)] += jr[3 * bi + ci] * jr[3 * bj + cj];
                        }
                    }
                }
            }
        }
        // object rows touch block k only
#pragma unroll
        for (int row = 3; row < 5; row++) {
#pragma unroll
            for (int ci = 0; ci < 3; ci++) {
                const int gi = 3 * k + ci;
                g[gi] += Jk[row][ci] * u[row];
#pragma unroll
                for (int cj = 0; cj <= ci; cj++) A[Band<N>::at(gi, 3 * k + cj)] += Jk[row][ci] * Jk[row][cj];
            }
        }
    }
    return ok;
}

// ------------------------------------------------------------------ parametric form
// Eqs. (13)-(15): two parameters per interaction (metres), the points are
// X(U) and only the law rows remain.  An edge has one parameter; its second
// slot is a placeholder with a zero Jacobian column.
//   plane      X = o + s e1 + t e2          (e1 packed in slots 13..15, e2 = n x e1)
//   line       X = p + s e
//   paraboloid X = p + s e1 + t e2 + kappa (s^2 + t^2) ax, (e1, e2) across the
//              axis, kappa packed in slot 17 (negative: not parametrisable)
//   circle     X = c + R (cos(s/R) u1 + sin(s/R) u2), (u1, u2) packed in slots 7..12
// Returns false if the record has no such parametrisation.
template <typename T>
__host__ __device__ __forceinline__ void across_dir(const T *a, T u1[3], T u2[3])
{
    // branch-free orthonormal pair across a unit vector (Duff et al. 2017)
    const T sg = a[2] >= T(0) ? T(1) : T(-1);
    const T q = T(-1) / (sg + a[2]);
    const T b = a[0] * a[1] * q;
    u1[0] = T(1) + sg * a[0] * a[0] * q;
    u1[1] = sg * b;
    u1[2] = -sg * a[0];
    u2[0] = b;
    u2[1] = sg + a[1] * a[1] * q;
    u2[2] = -a[1];
}

// sin and cos of a (radians) in FP32 for the FP32 solver, which evaluates
// them in every iteration of a circle path.  Cody-Waite reduction by pi/2,
// split into three floats of 8, 11 and 24 significant bits (k p1 and k p2
// are exact for |k| < 4096, |a| < 6400), then the Taylor series of sin to
// r^9 and cos to r^8 on |r| <= pi/4 (truncation error below 3e-8).  The
// library routine's wide-range reduction raised the register budget of
// every parametric FP32 kernel (order 5: 80 -> 64 bytes of spill per lane).
__host__ __device__ __forceinline__ void sincos32(float a, float &s, float &c)
{
    const float k = rintf(a * 0x1.45f306p-1f);  // a / (pi/2), rounded
    float r = fmaf(-k, 0x1.92p0f, a);
    r = fmaf(-k, 0x1.fb4p-12f, r);
    r = fmaf(-k, 0x1.4442d2p-24f, r);
    const float r2 = r * r;
    const float sp = r + r * r2 * (-1.0f / 6.0f + r2 * (1.0f / 120.0f + r2 * (-1.0f / 5040.0f + r2 * (1.0f / 362880.0f))));
    const float cp = 1.0f + r2 * (-0.5f + r2 * (1.0f / 24.0f + r2 * (-1.0f / 720.0f + r2 * (1.0f / 40320.0f))));
    const int q = (int)k & 3;  // a = k pi/2 + r
    s = (q == 0) ? sp : (q == 1) ? cp : (q == 2) ? -sp : -cp;
    c = (q == 0) ? cp : (q == 1) ? -sp : (q == 2) ? -cp : sp;
}

template <typename T>
__host__ __device__ __forceinline__ bool param_map(int t, const T *__restrict__ r, T s, T u, T X[3], T Tm[3][2])
{
    bool ok = true;
    if (t == TP) {
        const T e2[3] = {r[1] * r[15] - r[2] * r[14], r[2] * r[13] - r[0] * r[15], r[0] * r[14] - r[1] * r[13]};
#pragma unroll
        for (int i = 0; i < 3; i++) {
            X[i] = r[4 + i] + s * r[13 + i] + u * e2[i];
            Tm[i][0] = r[13 + i];
            Tm[i][1] = e2[i];
        }
    } else if (t == TL) {
#pragma unroll
        for (int i = 0; i < 3; i++) {
            X[i] = r[i] + s * r[3 + i];
            Tm[i][0] = r[3 + i];
            Tm[i][1] = T(0);
        }
    } else if (t == TQ) {
        T e1[3], e2[3];
        across_dir(r + 13, e1, e2);
        const T k = r[17];
        ok = k > T(0);
        const T h = k * (s * s + u * u), k2 = T(2) * k;
#pragma unroll
        for (int i = 0; i < 3; i++) {
            X[i] = r[i] + s * e1[i] + u * e2[i] + h * r[13 + i];
            Tm[i][0] = e1[i] + k2 * s * r[13 + i];
            Tm[i][1] = e2[i] + k2 * u * r[13 + i];
        }
    } else {
        const T R = r[6], a = s * drcp(R);
        T ca, sa;
        if constexpr (sizeof(T) == 4) {
            sincos32(a, sa, ca);
        } else {
            ca = cos(a);
            sa = sin(a);
        }
#pragma unroll
        for (int i = 0; i < 3; i++) {
            X[i] = r[i] + R * (ca * r[7 + i] + sa * r[10 + i]);
            Tm[i][0] = -sa * r[7 + i] + ca * r[10 + i];
            Tm[i][1] = T(0);
        }
    }
    return ok;
}

// The angle of a circle's start point, out of line: inlined, the FP64
// arctangent's registers count in every solver kernel (whose start code
// holds it) whether or not a circle is solved; called, it costs a register
// save only on the paths that take it.  Order-5 parametric FP32 kernel:
// 236 -> 80 bytes of spill per lane.
__host__ __device__ __attribute__((noinline)) inline double circle_angle(double y, double x) { return atan2(y, x); }

// Parameters of a point of an object (the start points, already put on it).
__host__ __device__ __forceinline__ bool param_of(int t, const double *__restrict__ r, const double X[3],
                                                  double U[2])
{
    U[1] = 0.0;
    if (t == TP) {
        const double d[3] = {X[0] - r[4], X[1] - r[5], X[2] - r[6]};
        const double e2[3] = {r[1] * r[15] - r[2] * r[14], r[2] * r[13] - r[0] * r[15], r[0] * r[14] - r[1] * r[13]};
        U[0] = d[0] * r[13] + d[1] * r[14] + d[2] * r[15];
        U[1] = dot3(d, e2);
        return true;
    }
    const double d[3] = {X[0] - r[0], X[1] - r[1], X[2] - r[2]};
    if (t == TL) {
        U[0] = d[0] * r[3] + d[1] * r[4] + d[2] * r[5];
        return true;
    }
    if (t == TQ) {
        double e1[3], e2[3];
        across_dir(r + 13, e1, e2);
        U[0] = dot3(d, e1);
        U[1] = dot3(d, e2);
        return r[17] > 0.0;
    }
    U[0] = r[6] * circle_angle(d[0] * r[10] + d[1] * r[11] + d[2] * r[12], d[0] * r[7] + d[1] * r[8] + d[2] * r[9]);
    return true;
}

// Law rows of the parametric form at X(U + dU) (dU may be null): cost, inf
// norm, and whether every trial point stays in the guard box.
template <typename T, int N, bool REFR = true>
__host__ __device__ __forceinline__ bool eval_cost_param(const SceneT<T> &sc, const PathIn<T, N> &p, const T *U,
                                                const T *dU, T &C, T &rinf, bool &guard)
{
    // points k-1, k, k+1 in a rolling window (slot j % 3): point j is mapped
    // just before the rows that first need it, so at most three are live
    T Xw[3][3], Tm[3][2];
    bool ok = true;
    guard = true;
    auto map = [&](int j) {
        const T s = U[2 * j] + (dU ? dU[2 * j] : T(0)), u = U[2 * j + 1] + (dU ? dU[2 * j + 1] : T(0));
        ok = param_map<T>(p.ty[j], sc.rec + (size_t)p.id[j] * kRec, s, u, Xw[j % 3], Tm) && ok;
#pragma unroll
        for (int i = 0; i < 3; i++) guard = guard && (Xw[j % 3][i] >= sc.glo[i]) && (Xw[j % 3][i] <= sc.ghi[i]);
    };
    map(0);
    C = T(0);
    rinf = T(0);
#pragma unroll
    for (int k = 0; k < N; k++) {
        if (k + 1 < N) map(k + 1);
        T u[5];
        const T *Xp = (k == 0) ? sc.tx : Xw[(k + 2) % 3];
        const T *Xn = (k + 1 < N) ? Xw[(k + 1) % 3] : p.rx;
        const bool okk = interaction_rows<T, false, REFR>(p.ty[k], sc.rec + (size_t)p.id[k] * kRec, Xp, Xw[k % 3], Xn,
                                                          u, nullptr, nullptr, nullptr);
        ok = ok && okk;
#pragma unroll
        for (int i = 0; i < 3; i++) {
            C += u[i] * u[i];
            rinf = fmax(rinf, fabs(u[i]));
        }
    }
    return ok;
}

// Normal equations of the parametric form: band of J^T J (2 x 2 blocks) and
// J^T I, with J = dI/dX . dX/dU by the chain rule.
template <typename T, int N, bool REFR = true>
__host__ __device__ __forceinline__ bool assemble_param(const SceneT<T> &sc, const PathIn<T, N> &p, const T *U, T *A,
                                               T *g, T &C, T &rinf)
{
    constexpr int M = 2 * N;
#pragma unroll
    for (int i = 0; i < M; i++)
#pragma unroll
        for (int j = 0; j <= i; j++)
            if (Band<N, 2>::in(i, j)) A[Band<N, 2>::at(i, j)] = T(0);
#pragma unroll
    for (int i = 0; i < M; i++) g[i] = T(0);
    // points and parametrisation Jacobians of interactions k-1, k, k+1 in a
    // rolling window (slot j % 3), mapped just before the rows that first
    // need them: at most three are live instead of all N
    T Xw[3][3], Tw[3][3][2];
    bool ok = true;
    auto map = [&](int j) {
        ok = param_map<T>(p.ty[j], sc.rec + (size_t)p.id[j] * kRec, U[2 * j], U[2 * j + 1], Xw[j % 3], Tw[j % 3]) &&
             ok;
    };
    map(0);
    C = T(0);
    rinf = T(0);
#pragma unroll
    for (int k = 0; k < N; k++) {
        if (k + 1 < N) map(k + 1);
        T u[5], Jp[3][3], Jk[5][3], Jn[3][3];
        const T *Xp = (k == 0) ? sc.tx : Xw[(k + 2) % 3];
        const T *Xn = (k + 1 < N) ? Xw[(k + 1) % 3] : p.rx;
        const bool okk = interaction_rows<T, true, REFR>(p.ty[k], sc.rec + (size_t)p.id[k] * kRec, Xp, Xw[k % 3], Xn,
                                                         u, Jp, Jk, Jn);
        ok = ok && okk;
#pragma unroll
        for (int row = 0; row < 3; row++) {
            C += u[row] * u[row];
            rinf = fmax(rinf, fabs(u[row]));
            // the row's derivatives with respect to the parameters of
            // interactions k-1, k, k+1
            T jr[6];
#pragma unroll
            for (int c = 0; c < 2; c++) {
                T vp = T(0), vk = T(0), vn = T(0);
#pragma unroll
                for (int j = 0; j < 3; j++) {
                    if (k > 0) vp += Jp[row][j] * Tw[(k + 2) % 3][j][c];
                    vk += Jk[row][j] * Tw[k % 3][j][c];
                    if (k + 1 < N) vn += Jn[row][j] * Tw[(k + 1) % 3][j][c];
                }
                jr[c] = vp;
                jr[2 + c] = vk;
                jr[4 + c] = vn;
            }
#pragma unroll
            for (int bi = 0; bi < 3; bi++) {
                const int Bi = k - 1 + bi;
                if (Bi < 0 || Bi >= N) continue;
#pragma unroll
                for (int ci = 0; ci < 2; ci++) {
                    const int gi = 2 * Bi + ci;
                    g[gi] += jr[2 * bi + ci] * u[row];
#pragma unroll
                    for (int bj = 0; bj < 3; bj++) {
                        const int Bj = k - 1 + bj;
                        if (Bj < 0 || Bj >= N) continue;
#pragma unroll
                        for (int cj = 0; cj < 2; cj++) {
                            const int gj = 2 * Bj + cj;
                            if (gj > gi) continue;
                            A[Band<N, 2>::at(gi, gj)] += jr[2 * bi + ci] * jr[2 * bj + cj];
                        }
                    }
                }
            }
        }
    }
    return ok;
}

// In-place banded Cholesky of the packed lower band; false if not SPD.  The
// diagonal slots receive the INVERSE of L's diagonal (the solves multiply).
template <typename T, int N, int B = 3>
__host__ __device__ __forceinline__ bool chol_band(T *A)
{
    constexpr int M = B * N;
    bool ok = true;
#pragma unroll
    for (int j = 0; j < M; j++) {
        T d = A[Band<N, B>::at(j, j)];
#pragma unroll
        for (int k = 0; k < j; k++)
            if (Band<N, B>::in(j, k)) d -= A[Band<N, B>::at(j, k)] * A[Band<N, B>::at(j, k)];
        ok = ok && (d > T(0));
        const T inv = drsqrt(d > T(0) ? d : T(1));
        A[Band<N, B>::at(j, j)] = inv;
#pragma unroll
        for (int i = j + 1; i < M; i++) {
            if (!Band<N, B>::in(i, j)) continue;
            T v = A[Band<N, B>::at(i, j)];
#pragma unroll
            for (int k = 0; k < j; k++)
                if (Band<N, B>::in(i, k) && Band<N, B>::in(j, k)) v -= A[Band<N, B>::at(i, k)] * A[Band<N, B>::at(j, k)];
            A[Band<N, B>::at(i, j)] = v * inv;
        }
    }
    return ok;
}

// Solve L L^T x = b in place (b -> x); the diagonal holds 1 / L_ii.
// Returns |y|^2 of the forward substitution L y = b: with b = -g this is
// -g^T x, the decrease the damped model predicts for the step x.
template <typename T, int N, int B = 3>
__host__ __device__ __forceinline__ T chol_solve_band(const T *L, T *b)
{
    constexpr int M = B * N;
    T ysq = T(0);
#pragma unroll
    for (int i = 0; i < M; i++) {
        T v = b[i];
#pragma unroll
        for (int k = 0; k < i; k++)
            if (Band<N, B>::in(i, k)) v -= L[Band<N, B>::at(i, k)] * b[k];
        b[i] = v * L[Band<N, B>::at(i, i)];
        ysq += b[i] * b[i];
    }
#pragma unroll
    for (int i = M - 1; i >= 0; i--) {
        T v = b[i];
#pragma unroll
        for (int k = i + 1; k < M; k++)
            if (Band<N, B>::in(k, i)) v -= L[Band<N, B>::at(k, i)] * b[k];
        b[i] = v * L[Band<N, B>::at(i, i)];
    }
    return ysq;
}

}  // namespace mpt
