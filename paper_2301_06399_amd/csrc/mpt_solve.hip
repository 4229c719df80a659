// Solver kernels of the batched Min-Path-Tracing solve (gfx950, wave64).
//
//  k_pack            scene records -> packed FP64 world + FP32 TX-local records
//  k_bin_count       histogram of path orders (invalid solves finished here)
//  k_bin_scatter     solve ids grouped by order (one bin per order)
//  k_lm              persistent Levenberg-Marquardt over the bins, one lane per
//                    path, lanes refilled from a per-wave chunk of the bin as
//                    soon as their path finishes (FP64 plain, FP32 stage or FP64
//                    fallback)
//  k_polish          FP64 Gauss-Newton polish of the FP32 end points
//  k_accept_*        FP64 acceptance test and ordered compaction
#include "mpt_internal.hpp"

namespace mpt {

// ------------------------------------------------------------------ pack
// Ortho-normal pair across a unit vector (Duff et al., "Building an
// orthonormal basis, revisited", JCGT 2017).
__global__ void k_pack(const double *__restrict__ raw, const double *__restrict__ refr, int n_pl, int n_ln, int n_q,
                       int n_c, double tx0, double tx1, double tx2, double *__restrict__ rec64,
                       float *__restrict__ rec32)
{
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    const int n_all = n_pl + n_ln + n_q + n_c;
    if (id >= n_all) return;
    const double tx[3] = {tx0, tx1, tx2};
    double o[kRec];
#pragma unroll
    for (int i = 0; i < kRec; i++) o[i] = 0.0;
    // raw arrays are concatenated type-major with their own widths
    const int t = prim_type(id, n_pl, n_pl + n_ln, n_pl + n_ln + n_q);
    size_t off;
    if (t == TP) off = (size_t)id * 13;
    else if (t == TL) off = (size_t)n_pl * 13 + (size_t)(id - n_pl) * 8;
    else if (t == TQ) off = (size_t)n_pl * 13 + (size_t)n_ln * 8 + (size_t)(id - n_pl - n_ln) * 17;
    else off = (size_t)n_pl * 13 + (size_t)n_ln * 8 + (size_t)n_q * 17 + (size_t)(id - n_pl - n_ln - n_q) * 7;
    const double *r = raw + off;
    const int w = (t == TP) ? 13 : (t == TL) ? 8 : (t == TQ) ? 17 : 7;
    for (int i = 0; i < w; i++) o[i] = r[i];
    if (t == TL) across_dir(r + 3, o + 8, o + 11);
    // frames of the parametric form
    if (t == TP) {
        const double l = sqrt(r[7] * r[7] + r[8] * r[8] + r[9] * r[9]);
        for (int i = 0; i < 3; i++) o[13 + i] = l > 0.0 ? r[7 + i] / l : 0.0;
        // refractive indices of a refracting facet (0, 0: a mirror)
        if (refr) {
            o[16] = refr[2 * (size_t)id];
            o[17] = refr[2 * (size_t)id + 1];
        }
    }
    if (t == TC) across_dir(r + 3, o + 7, o + 10);
    if (t == TQ) {
        // a paraboloid of revolution: A = kappa (I - ax ax^T), b = -ax, c = 0
        const double kap = 0.5 * (r[3] + r[6] + r[8]);
        const double *ax = r + 13;
        const double Am[3][3] = {{r[3], r[4], r[5]}, {r[4], r[6], r[7]}, {r[5], r[7], r[8]}};
        double err = fabs(r[12]);
        for (int i = 0; i < 3; i++) {
            err = fmax(err, fabs(r[9 + i] + ax[i]));
            for (int j = 0; j < 3; j++) err = fmax(err, fabs(Am[i][j] - kap * ((i == j ? 1.0 : 0.0) - ax[i] * ax[j])));
        }
        o[17] = (kap > 0.0 && err <= 1e-9 * (1.0 + kap)) ? kap : -1.0;
    }
    for (int i = 0; i < kRec; i++) rec64[(size_t)id * kRec + i] = o[i];
    // TX-local FP32 copy: positions shifted by TX, plane offsets adjusted
    double l[kRec];
    for (int i = 0; i < kRec; i++) l[i] = o[i];
    if (t == TP) {
        l[3] = o[3] - (o[0] * tx[0] + o[1] * tx[1] + o[2] * tx[2]);
        for (int i = 0; i < 3; i++) l[4 + i] = o[4 + i] - tx[i];
    } else {
        for (int i = 0; i < 3; i++) l[i] = o[i] - tx[i];
    }
    for (int i = 0; i < kRec; i++) rec32[(size_t)id * kRec + i] = (float)l[i];
}

// ------------------------------------------------------------------ workspace counters
__global__ void k_zero_i32(int *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ------------------------------------------------------------------ binning
__device__ inline bool finite3(const double *v) { return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]); }

// Order of a solve, or -1 if the solve is invalid (order, receiver or ids).
__device__ inline int valid_order(const BatchDev &b, int64_t i, int n_all)
{
    const int ord = b.order[i];
    bool bad = ord < 1 || ord > kMaxN;
    const int ri = b.rx_index[i];
    bad = bad || ri < 0 || ri >= b.n_rx;
    if (!bad) {
        bad = !finite3(b.rx + 3 * (size_t)ri);
        for (int k = 0; k < kMaxN; k++)
            if (k < ord) {
                const int id = b.prim[(size_t)k * b.n + i];
                bad = bad || id < 0 || id >= n_all;
            }
    }
    return bad ? -1 : ord;
}

// Binning by (order, sequence of primitive types): solves of one order are
// grouped, and within an order by the base-4 code of their type sequence, so
// the lanes of a wave mostly follow one type path (no divergence between
// reflection and diffraction code).  Key = kKeyBase[order] + code.
constexpr int kBinBlock = 256;
// solves per thread, their loads issued together (stress workload binning:
// 1.34 ms with two solves per thread each loaded as a chain of dependent
// loads; 1.11, 0.73 and 0.69 ms with the loads issued together and two,
// four and eight solves per thread; 0.77-0.80 ms with 16-32 solves per
// thread in chunks of eight, which halves or quarters the blocks' atomics
// on the key counters but loads the ids again after the atomics)
constexpr int kBinItems = 8;
constexpr int kBinPerBlock = kBinBlock * kBinItems;
constexpr int kNumKeys = 4 + 16 + 64 + 256 + 1024;
__device__ __constant__ int kKeyBase[kMaxN + 1] = {0, 0, 4, 20, 84, 340};

// A solve's order, receiver and ids as the binning reads them: every load
// is issued before any is used (the id rows beyond the order are the
// caller's memory as well), so a thread's loads are in flight together
// instead of one dependent round trip after another.  ord = -1 marks an
// invalid solve (the same test as valid_order).
struct SolveIds {
    int ord, ri, id[kMaxN];
};

__device__ inline void load_ids(const BatchDev &b, int64_t i, SolveIds &r)
{
    r.ord = b.order[i];
    r.ri = b.rx_index[i];
#pragma unroll
    for (int k = 0; k < kMaxN; k++) r.id[k] = b.prim[(size_t)k * b.n + i];
}

__device__ inline void check_ids(const BatchDev &b, int n_all, SolveIds &r)
{
    bool bad = r.ord < 1 || r.ord > kMaxN || r.ri < 0 || r.ri >= b.n_rx;
    if (!bad) {
        bad = !finite3(b.rx + 3 * (size_t)r.ri);
#pragma unroll
        for (int k = 0; k < kMaxN; k++)
            if (k < r.ord) bad = bad || r.id[k] < 0 || r.id[k] >= n_all;
    }
    if (bad) r.ord = -1;
}

__device__ inline int bin_key(const SolveIds &r, int a, int bb, int c)
{
    int code = 0, mul = 1;
#pragma unroll
    for (int k = 0; k < kMaxN; k++)
        if (k < r.ord) {
            code += prim_type(r.id[k], a, bb, c) * mul;
            mul *= 4;
        }
    return kKeyBase[r.ord] + code;
}

__global__ void __launch_bounds__(kBinBlock) k_bin_count(BatchDev b, OutDev out, int n_all, int n_pl, int n_pl_ln,
                                                          int n_pl_ln_q, int *__restrict__ key_cnt)
{
    __shared__ int loc[kNumKeys];
    for (int k = threadIdx.x; k < kNumKeys; k += kBinBlock) loc[k] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kBinPerBlock;
    SolveIds r[kBinItems];
#pragma unroll
    for (int j = 0; j < kBinItems; j++) {
        const int64_t i = base + (int64_t)j * kBinBlock + threadIdx.x;
        if (i < b.n) load_ids(b, i, r[j]);
    }
#pragma unroll
    for (int j = 0; j < kBinItems; j++) {
        const int64_t i = base + (int64_t)j * kBinBlock + threadIdx.x;
        if (i < b.n) check_ids(b, n_all, r[j]);
    }
#pragma unroll
    for (int j = 0; j < kBinItems; j++) {
        const int64_t i = base + (int64_t)j * kBinBlock + threadIdx.x;
        if (i >= b.n) break;
        if (r[j].ord < 0) {
            for (int q = 0; q < kRow; q++) out.x[(size_t)i * kRow + q] = 0.0;
            out.cost[i] = __builtin_huge_val();
            out.iters[i] = 0;
            out.status[i] = ST_BAD;
            if (out.stage)
                for (int q = 0; q < 4; q++) out.stage[(size_t)q * b.n + i] = 0;
        } else {
            // the later stages' iteration counts are zero: written here,
            // coalesced, so that the solver kernels store only what a path
            // produces (the solver writes a path's whole point row)
            if (out.stage)
                for (int q = 1; q < 4; q++) out.stage[(size_t)q * b.n + i] = 0;
            atomicAdd(&loc[bin_key(r[j], n_pl, n_pl_ln, n_pl_ln_q)], 1);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kNumKeys; k += kBinBlock)
        if (loc[k]) atomicAdd(&key_cnt[k], loc[k]);
}

// One block: exclusive scan of the key counts -> key offsets; per-order
// totals -> bin counts (the bins of the LM kernels are the orders).
// curved (or null): the start of each order's part of the list of the
// solves with a curved object ([5], then used as cursors by the scatter),
// and curved[25] receives the list's length (the counter slots of the
// solve's workspace are laid out so).
__global__ void __launch_bounds__(1024) k_bin_offsets(const int *__restrict__ key_cnt, int *__restrict__ key_off,
                                                       int *__restrict__ bin_cnt, int *__restrict__ curved)
{
    __shared__ int part[1024];
    __shared__ int offs[kNumKeys + 1];
    const int t = threadIdx.x;
    const int per = (kNumKeys + 1023) / 1024;
    const int lo = t * per, hi = min(lo + per, kNumKeys);
    int c[per], sum = 0;
#pragma unroll
    for (int q = 0; q < per; q++) {
        c[q] = (lo + q < hi) ? key_cnt[lo + q] : 0;
        sum += c[q];
    }
    part[t] = sum;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int v = (t >= d) ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = (t == 0) ? 0 : part[t - 1];
#pragma unroll
    for (int q = 0; q < per; q++)
        if (lo + q < hi) {
            key_off[lo + q] = run;
            offs[lo + q] = run;
            run += c[q];
        }
    if (t == 1023) offs[kNumKeys] = part[1023];
    __syncthreads();
    // per-order totals: the keys of one order are contiguous
    __shared__ int ccnt[kMaxN];
    if (t < kMaxN) {
        const int kb = kKeyBase[t + 1], ke = (t + 1 < kMaxN) ? kKeyBase[t + 2] : kNumKeys;
        bin_cnt[t] = offs[ke] - offs[kb];
        ccnt[t] = 0;
    }
    if (!curved) return;
    __syncthreads();
    // the solves with a curved object (a type digit of 2 or 3 in the key),
    // per order: each thread adds its own keys' counts
#pragma unroll
    for (int q = 0; q < per; q++) {
        const int k = lo + q;
        int o = 1;
        while (o < kMaxN && k >= kKeyBase[o + 1]) o++;
        if (k < hi && c[q] && ((k - kKeyBase[o]) & 0x2AA) != 0) atomicAdd(&ccnt[o - 1], c[q]);
    }
    __syncthreads();
    if (t == 0) {
        int run = 0;
        for (int o = 0; o < kMaxN; o++) {
            curved[o] = run;
            run += ccnt[o];
        }
        curved[25] = run;
    }
}

__device__ inline int bin_offset(const int *cnt, int k)  // k = order 1..5
{
    int off = 0;
    for (int j = 1; j < k; j++) off += cnt[j - 1];
    return off;
}

// Each solve's slot in bin order, and its receiver and primitive ids copied
// to that slot: the solver reads a wave's paths from consecutive slots
// (coalesced) instead of gathering them by solve id.  With `rows`, the
// solves whose list holds a paraboloid or a circle (a type digit of 2 or 3
// in the key) are also listed there, grouped by order (`curved`: each
// order's cursor, one atomic per block and order), so that the waves of the
// learned start's kernels hold one order each.
__global__ void __launch_bounds__(kBinBlock) k_bin_scatter(BatchDev b, int n_all, int n_pl, int n_pl_ln, int n_pl_ln_q,
                                                            const int *__restrict__ key_off,
                                                            int *__restrict__ key_cursor, int *__restrict__ perm,
                                                            int *__restrict__ slot_rx, int *__restrict__ slot_prim,
                                                            int *__restrict__ rows, int *__restrict__ curved)
{
    __shared__ int loc[kNumKeys];
    __shared__ int gbase[kNumKeys];
    __shared__ int ccount[kMaxN], cbase[kMaxN];
    for (int k = threadIdx.x; k < kNumKeys; k += kBinBlock) loc[k] = 0;
    if (threadIdx.x < kMaxN) ccount[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kBinPerBlock;
    int key[kBinItems], rank[kBinItems], crank[kBinItems];
    SolveIds r[kBinItems];
#pragma unroll
    for (int j = 0; j < kBinItems; j++) {
        const int64_t i = base + (int64_t)j * kBinBlock + threadIdx.x;
        r[j].ord = -1;
        if (i < b.n) load_ids(b, i, r[j]);
    }
#pragma unroll
    for (int j = 0; j < kBinItems; j++) {
        const int64_t i = base + (int64_t)j * kBinBlock + threadIdx.x;
        if (i < b.n) check_ids(b, n_all, r[j]);
    }
#pragma unroll
    for (int j = 0; j < kBinItems; j++) {
        const int ord = r[j].ord;
        key[j] = (ord > 0) ? bin_key(r[j], n_pl, n_pl_ln, n_pl_ln_q) : -1;
        rank[j] = (key[j] >= 0) ? atomicAdd(&loc[key[j]], 1) : 0;
        // base-4 type digits: 2 (quadric) and 3 (circle) have bit 1 set
        const bool cur = rows && key[j] >= 0 && ((key[j] - kKeyBase[ord > 0 ? ord : 1]) & 0x2AA) != 0;
        crank[j] = cur ? atomicAdd(&ccount[ord - 1], 1) : -1;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kNumKeys; k += kBinBlock)
        gbase[k] = loc[k] ? key_off[k] + atomicAdd(&key_cursor[k], loc[k]) : 0;
    if (rows && threadIdx.x < kMaxN)
        cbase[threadIdx.x] = ccount[threadIdx.x] ? atomicAdd(&curved[threadIdx.x], ccount[threadIdx.x]) : 0;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kBinItems; j++) {
        const int64_t i = base + (int64_t)j * kBinBlock + threadIdx.x;
        if (key[j] >= 0) {
            const int slot = gbase[key[j]] + rank[j];
            perm[slot] = (int)i;
            slot_rx[slot] = r[j].ri;
#pragma unroll
            for (int k = 0; k < kMaxN; k++)
                if (k < r[j].ord) slot_prim[(size_t)k * b.n + slot] = r[j].id[k];
        }
        if (crank[j] >= 0) rows[cbase[r[j].ord - 1] + crank[j]] = (int)i;
    }
}

// ------------------------------------------------------------------ init
// Uniform double in [0,1) from draw number c of SplitMix64 (Steele, Lea &
// Flood, OOPSLA 2014) started from state `seed`: the state after c+1
// golden-ratio increments, mixed, top 53 bits.
__device__ inline double splitmix_uniform(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + (c + 1u) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-53;
}

// Projection of a point onto an object (FP64 world): the straight-line start
// of each interaction is the projection of the point k/(N+1) of the way from
// TX to RX; the random start (Alg. 1) projects a point uniform in the scene
// box, draw 15 i + 3 k + axis for solve i.
__device__ inline void project(int t, const double *r, const double *P, double *X)
{
    if (t == TP) {
        const double f = r[0] * P[0] + r[1] * P[1] + r[2] * P[2] - r[3];
        for (int i = 0; i < 3; i++) X[i] = P[i] - f * r[i];
    } else if (t == TL) {
        const double s = (P[0] - r[0]) * r[3] + (P[1] - r[1]) * r[4] + (P[2] - r[2]) * r[5];
        for (int i = 0; i < 3; i++) X[i] = r[i] + s * r[3 + i];
    } else if (t == TQ) {
        // one Newton step towards f = 0 along grad f
        const double w[3] = {P[0] - r[0], P[1] - r[1], P[2] - r[2]};
        const double Aw0 = r[3] * w[0] + r[4] * w[1] + r[5] * w[2];
        const double Aw1 = r[4] * w[0] + r[6] * w[1] + r[7] * w[2];
        const double Aw2 = r[5] * w[0] + r[7] * w[1] + r[8] * w[2];
        const double f = w[0] * Aw0 + w[1] * Aw1 + w[2] * Aw2 + r[9] * w[0] + r[10] * w[1] + r[11] * w[2] + r[12];
        const double g[3] = {2.0 * Aw0 + r[9], 2.0 * Aw1 + r[10], 2.0 * Aw2 + r[11]};
        const double gg = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
        const double s = gg > 0.0 ? f / gg : 0.0;
        for (int i = 0; i < 3; i++) X[i] = P[i] - s * g[i];
    } else {
        const double d[3] = {P[0] - r[0], P[1] - r[1], P[2] - r[2]};
        const double h = d[0] * r[3] + d[1] * r[4] + d[2] * r[5];
        double w[3] = {d[0] - h * r[3], d[1] - h * r[4], d[2] - h * r[5]};
        double lw = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        if (!(lw > 0.0)) {
            double u2[3];
            across_dir(r + 3, w, u2);
            lw = 1.0;
        }
        for (int i = 0; i < 3; i++) X[i] = r[i] + r[6] * w[i] / lw;
    }
}

__device__ inline bool in_guard(const SceneDev &s, const double *X, int n)
{
    bool ok = true;
    for (int k = 0; k < n; k++)
        for (int i = 0; i < 3; i++) ok = ok && (X[3 * k + i] >= s.glo[i]) && (X[3 * k + i] <= s.ghi[i]);
    return ok;
}

// ------------------------------------------------------------------ learned start
// The network's points, projected onto their objects, replace the
// straight-line start of a path only when their FP64 cost is lower: the
// solver's own cost judges the prediction.  Writes the chosen start points
// into x0l (rows of the path; one thread per served path).
// Fraction along TX -> RX of the straight-line start of interaction k of N:
// k+1 over N+1, or, on a refracting facet (which the ray crosses), the
// point where the segment meets its plane when it does.
__device__ __forceinline__ double line_fraction(int ty, const double *r, const double *tx, const double *rx, int k,
                                                int N)
{
    double a = (double)(k + 1) / (double)(N + 1);
    if (ty == TP && r[16] > 0.0) {
        const double den = r[0] * (rx[0] - tx[0]) + r[1] * (rx[1] - tx[1]) + r[2] * (rx[2] - tx[2]);
        const double c = (den != 0.0) ? (r[3] - (r[0] * tx[0] + r[1] * tx[1] + r[2] * tx[2])) / den : -1.0;
        if (c > 0.0 && c < 1.0) a = c;
    }
    return a;
}

template <int N, bool REFR>
__device__ void choose_start(const SceneDev &s, const BatchDev &b, int64_t i, double *__restrict__ x0l, double gain)
{
    SceneT<double> s64;
    s64.rec = s.rec64;
    PathIn<double, N> q;
    const int ri = b.rx_index[i];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        s64.tx[c] = s.tx[c];
        s64.glo[c] = s.glo[c];
        s64.ghi[c] = s.ghi[c];
        q.rx[c] = b.rx[3 * (size_t)ri + c];
    }
    q.planar = false;
#pragma unroll
    for (int k = 0; k < N; k++) {
        q.id[k] = b.prim[(size_t)k * b.n + i];
        q.ty[k] = prim_type(q.id[k], s.n_pl, s.n_pl_ln, s.n_pl_ln_q);
    }
    double X0[3 * N], Xn[3 * N];
    bool okn = true;
#pragma unroll
    for (int k = 0; k < N; k++) {
        const double a = line_fraction(q.ty[k], s.rec64 + (size_t)q.id[k] * kRec, s.tx, q.rx, k, N);
        double P[3], Pn[3];
#pragma unroll
        for (int c = 0; c < 3; c++) {
            P[c] = s.tx[c] + a * (q.rx[c] - s.tx[c]);
            Pn[c] = x0l[(size_t)i * kRow + 3 * k + c];
            okn = okn && isfinite(Pn[c]);
        }
        const double *r = s.rec64 + (size_t)q.id[k] * kRec;
        project(q.ty[k], r, P, X0 + 3 * k);
        project(q.ty[k], r, okn ? Pn : P, Xn + 3 * k);
    }
    double c0 = 0.0, r0 = 0.0, c1 = 0.0, r1 = 0.0;
    const bool ok0 = eval_cost<double, N, REFR>(s64, q, X0, nullptr, c0, r0);
    const bool ok1 = okn && eval_cost<double, N, REFR>(s64, q, Xn, nullptr, c1, r1);
    const bool net = ok1 && (!ok0 || c1 < gain * c0);
#pragma unroll
    for (int j = 0; j < 3 * N; j++) x0l[(size_t)i * kRow + j] = net ? Xn[j] : X0[j];
}

template <bool REFR>
__global__ void __launch_bounds__(256) k_learned_choose(SceneDev s, BatchDev b, const int *__restrict__ rows,
                                                        const int *__restrict__ count, int all,
                                                        double *__restrict__ x0l, double gain)
{
    const int64_t m = all ? b.n : (int64_t)*count;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = all ? t : rows[t];
        switch (valid_order(b, i, s.n_all)) {
        case 1: choose_start<1, REFR>(s, b, i, x0l, gain); break;
        case 2: choose_start<2, REFR>(s, b, i, x0l, gain); break;
        case 3: choose_start<3, REFR>(s, b, i, x0l, gain); break;
        case 4: choose_start<4, REFR>(s, b, i, x0l, gain); break;
        case 5: choose_start<5, REFR>(s, b, i, x0l, gain); break;
        default: break;
        }
    }
}

// ------------------------------------------------------------------ LM lane state
template <typename T>
struct LMOpts {
    int max_iter, max_iter_planar, win, stat_win;
    T frac, tol_step, tol_res, tau_root, lambda0, stat_tol;
};

// State of one lane's path: the unknowns (D = 3N points, or 2N parameters
// in the parametric form) and the Levenberg-Marquardt scalars.
template <typename T, int N, int D = 3 * N>
struct Lane {
    T X[D];
    T lam, Cref, C, rinf;
    int it, stat;
    // The normal equations, gradient and cost of the current point, kept
    // after a rejected step: the point has not moved, so the next iteration
    // would rebuild the same values (only the damping changes).  FP32 and
    // orders 1-3, whose copies fit in registers beside the order-5 code (the
    // FP64 kernels already spill).
    static constexpr bool kKeep = N <= 3 && sizeof(T) == 4;
    static constexpr int kS = kKeep ? D * (D + 1) / 2 : 1;
    static constexpr int kM = kKeep ? D : 1;
    T A0[kS], g0[kM], C0, r0;
    bool keep;
};

// One Levenberg-Marquardt iteration on the cost of Eq. (12) with the
// rescaled rows; returns ST_RUNNING or the final status.  REFR: the scene
// has refracting facets (their rows are compiled in).
template <typename T, int N, bool REFR>
__device__ __forceinline__ int lm_step(const SceneT<T> &sc, const PathIn<T, N> &p, Lane<T, N> &L,
                                       const LMOpts<T> &o)
{
    constexpr int M = 3 * N;
    using LT = Lane<T, N>;
    L.it++;
    T A[Band<N>::SIZE], g[M], C, rinf;
    if (LT::kKeep && L.keep) {
#pragma unroll
        for (int i = 0; i < Band<N>::SIZE; i++) A[i] = L.A0[i % LT::kS];
#pragma unroll
        for (int i = 0; i < M; i++) g[i] = L.g0[i % LT::kM];
        C = L.C0;
        rinf = L.r0;
    } else {
        if (!assemble<T, N, REFR>(sc, p, L.X, A, g, C, rinf)) return ST_DEGEN;
        if constexpr (LT::kKeep) {
#pragma unroll
            for (int i = 0; i < Band<N>::SIZE; i++) L.A0[i] = A[i];
#pragma unroll
            for (int i = 0; i < M; i++) L.g0[i] = g[i];
            L.C0 = C;
            L.r0 = rinf;
        }
    }
    L.keep = false;
    L.C = C;
    L.rinf = rinf;
    T dmax = T(0);
#pragma unroll
    for (int i = 0; i < M; i++) dmax = fmax(dmax, A[Band<N>::at(i, i)]);
    if (L.it == 1) {
        L.lam = o.lambda0 * dmax;
        L.Cref = C;
    }
    if (rinf <= o.tol_res) return (L.rinf <= o.tau_root) ? ST_CONV : ST_LOCALMIN;
    if (o.win > 0 && L.it > 1 && (L.it - 1) % o.win == 0) {
        if (C > o.frac * L.Cref) return (L.rinf <= o.tau_root) ? ST_CONV : ST_LOCALMIN;
        L.Cref = C;
    }
    const T floor_d = T(1e-12) * dmax;
#pragma unroll
    for (int i = 0; i < M; i++) A[Band<N>::at(i, i)] += L.lam * fmax(A[Band<N>::at(i, i)], floor_d);
    if (!chol_band<T, N>(A)) {
        L.lam *= T(10);
        if (L.lam > T(1e12) * dmax) return ST_STALL;
        L.keep = LT::kKeep;
        return (L.it >= (p.planar ? o.max_iter_planar : o.max_iter)) ? ST_MAXIT : ST_RUNNING;
    }
#pragma unroll
    for (int i = 0; i < M; i++) g[i] = -g[i];
    const T pred = chol_solve_band<T, N>(A, g);  // g <- dx; pred = -g^T dx
    if (o.stat_win > 0 && p.planar) {
        // planes and straight edges: the descent has stalled when the damped
        // model predicts too small a decrease several iterations in a row
        L.stat = (pred < o.stat_tol * C) ? L.stat + 1 : 0;
        if (L.stat >= o.stat_win) return (L.rinf <= o.tau_root) ? ST_CONV : ST_LOCALMIN;
    }
    T xinf = T(0), dinf = T(0);
    bool guard = true;
#pragma unroll
    for (int k = 0; k < N; k++)
#pragma unroll
        for (int i = 0; i < 3; i++) {
            xinf = fmax(xinf, fabs(L.X[3 * k + i]));
            dinf = fmax(dinf, fabs(g[3 * k + i]));
            const T xt = L.X[3 * k + i] + g[3 * k + i];
            guard = guard && (xt >= sc.glo[i]) && (xt <= sc.ghi[i]);
        }
    const bool small = dinf <= o.tol_step * (T(1) + xinf);
    T Ct = T(0), rt = T(0);
    bool okt = guard && eval_cost<T, N, REFR>(sc, p, L.X, g, Ct, rt);
    if (okt && Ct < C) {
#pragma unroll
        for (int i = 0; i < M; i++) L.X[i] += g[i];
        L.C = Ct;
        L.rinf = rt;
        L.lam = fmax(L.lam / T(10), T(1e-15) * dmax);
        if (small) return (L.rinf <= o.tau_root) ? ST_CONV : ST_LOCALMIN;
    } else {
        if (small) return (L.rinf <= o.tau_root) ? ST_CONV : ST_LOCALMIN;
        L.lam *= T(10);
        if (L.lam > T(1e12) * dmax) return ST_STALL;
        L.keep = LT::kKeep;
    }
    return (L.it >= (p.planar ? o.max_iter_planar : o.max_iter)) ? ST_MAXIT : ST_RUNNING;
}

// One Levenberg-Marquardt iteration of the parametric form (Eq. (15)), with
// the same rules; the placeholder parameter of an edge is held fixed.
template <typename T, int N, bool REFR>
__device__ __forceinline__ int lm_step_param(const SceneT<T> &sc, const PathIn<T, N> &p, Lane<T, N, 2 * N> &L,
                                             const LMOpts<T> &o)
{
    constexpr int M = 2 * N;
    using LT = Lane<T, N, 2 * N>;
    L.it++;
    T A[Band<N, 2>::SIZE], g[M], C, rinf;
    if (LT::kKeep && L.keep) {
#pragma unroll
        for (int i = 0; i < Band<N, 2>::SIZE; i++) A[i] = L.A0[i % LT::kS];
#pragma unroll
        for (int i = 0; i < M; i++) g[i] = L.g0[i % LT::kM];
        C = L.C0;
        rinf = L.r0;
    } else {
        if (!assemble_param<T, N, REFR>(sc, p, L.X, A, g, C, rinf)) return ST_DEGEN;
        if constexpr (LT::kKeep) {
#pragma unroll
            for (int i = 0; i < Band<N, 2>::SIZE; i++) L.A0[i] = A[i];
#pragma unroll
            for (int i = 0; i < M; i++) L.g0[i] = g[i];
            L.C0 = C;
            L.r0 = rinf;
        }
    }
    L.keep = false;
    L.C = C;
    L.rinf = rinf;
    bool real[M];
#pragma unroll
    for (int k = 0; k < N; k++) {
        real[2 * k] = true;
        real[2 * k + 1] = p.ty[k] == TP || p.ty[k] == TQ;
    }
    T dmax = T(0);
#pragma unroll
    for (int i = 0; i < M; i++) dmax = real[i] ? fmax(dmax, A[Band<N, 2>::at(i, i)]) : dmax;
    if (L.it == 1) {
        L.lam = o.lambda0 * dmax;
        L.Cref = C;
    }
    if (rinf <= o.tol_res) return (L.rinf <= o.tau_root) ? ST_CONV : ST_LOCALMIN;
    if (o.win > 0 && L.it > 1 && (L.it - 1) % o.win == 0) {
        if (C > o.frac * L.Cref) return (L.rinf <= o.tau_root) ? ST_CONV : ST_LOCALMIN;
        L.Cref = C;
    }
    const T floor_d = T(1e-12) * dmax;
#pragma unroll
    for (int i = 0; i < M; i++) {
        const T a = A[Band<N, 2>::at(i, i)];
        A[Band<N, 2>::at(i, i)] = real[i] ? a + L.lam * fmax(a, floor_d) : T(1);
    }
    if (!chol_band<T, N, 2>(A)) {
        L.lam *= T(10);
        if (L.lam > T(1e12) * dmax) return ST_STALL;
        L.keep = LT::kKeep;
        return (L.it >= (p.planar ? o.max_iter_planar : o.max_iter)) ? ST_MAXIT : ST_RUNNING;
    }
#pragma unroll
    for (int i = 0; i < M; i++) g[i] = -g[i];
    const T pred = chol_solve_band<T, N, 2>(A, g);  // g <- dU (zero on the placeholders)
    if (o.stat_win > 0 && p.planar) {
        L.stat = (pred < o.stat_tol * C) ? L.stat + 1 : 0;
        if (L.stat >= o.stat_win) return (L.rinf <= o.tau_root) ? ST_CONV : ST_LOCALMIN;
    }
    T xinf = T(0), dinf = T(0);
#pragma unroll
    for (int i = 0; i < M; i++) {
        xinf = fmax(xinf, fabs(L.X[i]));
        dinf = fmax(dinf, fabs(g[i]));
    }
    const bool small = dinf <= o.tol_step * (T(1) + xinf);
    T Ct = T(0), rt = T(0);
    bool guard = true;
    bool okt = eval_cost_param<T, N, REFR>(sc, p, L.X, g, Ct, rt, guard) && guard;
    if (okt && Ct < C) {
#pragma unroll
        for (int i = 0; i < M; i++) L.X[i] += g[i];
        L.C = Ct;
        L.rinf = rt;
        L.lam = fmax(L.lam / T(10), T(1e-15) * dmax);
        if (small) return (L.rinf <= o.tau_root) ? ST_CONV : ST_LOCALMIN;
    } else {
        if (small) return (L.rinf <= o.tau_root) ? ST_CONV : ST_LOCALMIN;
        L.lam *= T(10);
        if (L.lam > T(1e12) * dmax) return ST_STALL;
        L.keep = LT::kKeep;
    }
    return (L.it >= (p.planar ? o.max_iter_planar : o.max_iter)) ? ST_MAXIT : ST_RUNNING;
}

// ------------------------------------------------------------------ persistent LM kernel
// Lane-refill loop for the bin of order N.  Each wave takes a chunk of the bin
// with one atomic, and hands the chunk's ids to its idle lanes; a lane whose
// path finishes is refilled at the next iteration, so lanes never wait for
// the slowest path of their wave.
template <int MODE> struct ModeT;
template <> struct ModeT<MODE_PLAIN64> { using T = double; };
template <> struct ModeT<MODE_FP32> { using T = float; };
template <> struct ModeT<MODE_FALLBACK64> { using T = double; };

// A plane reflection sends the ray back to the side it came from (the law
// negates the normal component of the direction), so at a root the points
// before and after it lie strictly on the same side of its plane.  When each
// of them is either fixed (TX, RX) or confined to an object that keeps one
// side of the plane everywhere (a plane or straight edge exactly parallel to
// it, off it by more than 1e-9 m), and the two sides differ, no root exists.
// Plain IEEE FP64 without contraction: an exactly parallel pair is found
// parallel whatever the scaling of its normals.
__device__ __forceinline__ bool const_side(const SceneDev &s, int id, int ty, const double *n, const double *o,
                                           double &side)
{
#pragma clang fp contract(off)
    const double *r = s.rec64 + (size_t)id * kRec;
    if (ty == TP) {
        // normals parallel: every point of the other plane is n.(o' - o) off
        if (n[1] * r[2] - n[2] * r[1] != 0.0 || n[2] * r[0] - n[0] * r[2] != 0.0 || n[0] * r[1] - n[1] * r[0] != 0.0)
            return false;
        side = n[0] * (r[4] - o[0]) + n[1] * (r[5] - o[1]) + n[2] * (r[6] - o[2]);
    } else if (ty == TL) {
        if (n[0] * r[3] + n[1] * r[4] + n[2] * r[5] != 0.0) return false;
        side = n[0] * (r[0] - o[0]) + n[1] * (r[1] - o[1]) + n[2] * (r[2] - o[2]);
    } else {
        return false;
    }
    return fabs(side) > 1e-9;
}

template <int N>
__device__ bool sides_forbid_root(const SceneDev &s, const int *id, const int *ty, const double *rx)
{
#pragma clang fp contract(off)
    bool forbid = false;
#pragma unroll
    for (int k = 0; k < N; k++) {
        if (ty[k] != TP) continue;
        const double *r = s.rec64 + (size_t)id[k] * kRec;
        if (r[16] > 0.0) continue;  // a refracting facet passes the ray to its other side
        const double n[3] = {r[0], r[1], r[2]}, o[3] = {r[4], r[5], r[6]};
        double a = 0.0, b = 0.0;
        bool ka = true, kb = true;
        if (k == 0) a = n[0] * (s.tx[0] - o[0]) + n[1] * (s.tx[1] - o[1]) + n[2] * (s.tx[2] - o[2]);
        else ka = const_side(s, id[k - 1], ty[k - 1], n, o, a);
        if (k == N - 1) b = n[0] * (rx[0] - o[0]) + n[1] * (rx[1] - o[1]) + n[2] * (rx[2] - o[2]);
        else kb = const_side(s, id[k + 1], ty[k + 1], n, o, b);
        forbid = forbid || (ka && kb && ((a < 0.0 && b > 0.0) || (a > 0.0 && b < 0.0)));
    }
    return forbid;
}

//
// Stragglers.  Iteration counts are bimodal (a root converges in a handful of
// iterations, a path without one creeps until the plateau test ends it), so
// once the bin's queue is empty a wave would idle most of its lanes while its
// slowest paths finish.  Instead, when no more than spill_t lanes are still
// busy, the wave parks their state (points, iteration count, damping,
// plateau reference) and leaves; a second launch of the same kernel
// (kp.resume) packs the parked paths densely and finishes them.  The same
// machine code runs every iteration of a path, from the exact state it was
// parked in, so the results are identical bit for bit.
// One iteration with the path's primitive types fixed at compile time (digit
// k of CODE, base 4: 0 plane, 1 straight edge), so that no per-type branch
// or select is left in the code.  Bins are type-homogeneous, so most waves
// hold one planar sequence and run one of these variants only.  Used by the
// parametric FP32 kernel: there it shortens an iteration (street canyon LM
// stage 0.550 -> 0.484 ms, room 0.157 -> 0.119 ms); the implicit kernel's
// larger variants made it slower (0.516 -> 0.556 ms).
template <typename T, int N, int FORM, int CODE>
__device__ __forceinline__ int lm_step_fixed(const SceneT<T> &sc, const PathIn<T, N> &p,
                                             Lane<T, N, FORM ? 2 * N : 3 * N> &L, const LMOpts<T> &o)
{
    PathIn<T, N> q = p;
#pragma unroll
    for (int k = 0; k < N; k++) q.ty[k] = (CODE >> (2 * k)) & 3;
    q.planar = true;  // planes and straight edges: no refracting facet
    if constexpr (FORM) return lm_step_param<T, N, false>(sc, q, L, o);
    else return lm_step<T, N, false>(sc, q, L, o);
}

// The fixed-type step for the planar sequence `code` of orders 1-3; -1 for
// any other sequence (the caller runs the generic step).
template <typename T, int N, int FORM>
__device__ __forceinline__ int lm_step_uniform(int code, const SceneT<T> &sc, const PathIn<T, N> &p,
                                               Lane<T, N, FORM ? 2 * N : 3 * N> &L, const LMOpts<T> &o)
{
#define MPT_FIXED(c) \
    case c: return lm_step_fixed<T, N, FORM, c>(sc, p, L, o);
    if constexpr (N == 1) {
        switch (code) { MPT_FIXED(0) MPT_FIXED(1) }
    } else if constexpr (N == 2) {
        switch (code) { MPT_FIXED(0) MPT_FIXED(1) MPT_FIXED(4) MPT_FIXED(5) }
    } else if constexpr (N == 3) {
        switch (code) {
            MPT_FIXED(0) MPT_FIXED(1) MPT_FIXED(4) MPT_FIXED(5) MPT_FIXED(16) MPT_FIXED(17) MPT_FIXED(20) MPT_FIXED(21)
        }
    }
#undef MPT_FIXED
    return -1;
}

// True when some point lies outside its object's finite extent by more
// than `margin` metres (rectangle sides, edge ends, paraboloid aperture; a
// circle is its own extent).  FP64 world points and records.
template <int N>
__device__ __forceinline__ bool outside_extent(const double *rec64, const int *id, const int *ty, const double *X,
                                               double margin)
{
    bool out = false;
#pragma unroll
    for (int k = 0; k < N; k++) {
        const double *r = rec64 + (size_t)id[k] * kRec;
        const double *x = X + 3 * k;
        if (ty[k] == TP) {
            const double e[3] = {x[0] - r[4], x[1] - r[5], x[2] - r[6]};
            const double la = sqrt(r[7] * r[7] + r[8] * r[8] + r[9] * r[9]);
            const double lb = sqrt(r[10] * r[10] + r[11] * r[11] + r[12] * r[12]);
            const double a = (e[0] * r[7] + e[1] * r[8] + e[2] * r[9]) / la;
            const double b = (e[0] * r[10] + e[1] * r[11] + e[2] * r[12]) / lb;
            out = out || a < -margin || a > la + margin || b < -margin || b > lb + margin;
        } else if (ty[k] == TL) {
            const double sp = (x[0] - r[0]) * r[3] + (x[1] - r[1]) * r[4] + (x[2] - r[2]) * r[5];
            out = out || sp < r[6] - margin || sp > r[7] + margin;
        } else if (ty[k] == TQ) {
            const double d[3] = {x[0] - r[0], x[1] - r[1], x[2] - r[2]};
            const double h = d[0] * r[13] + d[1] * r[14] + d[2] * r[15];
            const double w2 = (d[0] - h * r[13]) * (d[0] - h * r[13]) + (d[1] - h * r[14]) * (d[1] - h * r[14]) +
                              (d[2] - h * r[15]) * (d[2] - h * r[15]);
            out = out || w2 > (r[16] + margin) * (r[16] + margin);
        }
    }
    return out;
}

template <int MODE, int N, int FORM = 0, bool TYPED = false, bool REFR = false>
__device__ __forceinline__ void lm_bin(const KParams &kp, const typename ModeT<MODE>::T *__restrict__ srec)
{
    using T = typename ModeT<MODE>::T;
    constexpr int D = FORM ? 2 * N : 3 * N;  // unknowns: points, or parameters
    const int lane = __lane_id();
    const bool resume = kp.resume != 0;
    const int *cnt = resume ? kp.spill_cnt : (MODE == MODE_FALLBACK64) ? kp.fb_cnt : kp.bin_cnt;
    const int *list = resume ? kp.spill_list : (MODE == MODE_FALLBACK64) ? kp.fb_list : kp.perm;
    int *head = resume ? kp.spill_head + (N - 1) : kp.head + (MODE == MODE_FALLBACK64 ? 5 : 0) + (N - 1);
    const int count = cnt[N - 1];
    if (count == 0) return;
    const int off = bin_offset(kp.bin_cnt, N);
    const bool may_spill = !resume && MODE != MODE_FALLBACK64 && kp.spill_t > 0;

    SceneT<T> sc;
    sc.rec = srec;
    if (MODE == MODE_FP32) {
#pragma unroll
        for (int i = 0; i < 3; i++) {
            sc.tx[i] = T(0);
            sc.glo[i] = (T)(kp.s.glo[i] - kp.s.tx[i]);
            sc.ghi[i] = (T)(kp.s.ghi[i] - kp.s.tx[i]);
        }
    } else {
#pragma unroll
        for (int i = 0; i < 3; i++) {
            sc.tx[i] = (T)kp.s.tx[i];
            sc.glo[i] = (T)kp.s.glo[i];
            sc.ghi[i] = (T)kp.s.ghi[i];
        }
    }
    LMOpts<T> o;
    if (MODE == MODE_FP32) {
        o.max_iter = kp.o.max_iter32;
        o.max_iter_planar = kp.o.max_iter32_planar;
        o.tol_step = (T)kp.o.tol_step32;
        o.tol_res = (T)kp.o.tol_res32;
        o.tau_root = (T)kp.o.tau_root32;  // an FP32 point this close is taken for a root
    } else {
        o.max_iter = (MODE == MODE_FALLBACK64) ? kp.o.max_iter_fb : kp.o.max_iter;
        o.max_iter_planar = o.max_iter;
        o.tol_step = (T)kp.o.tol_step;
        o.tol_res = (T)kp.o.tol_res;
        o.tau_root = (T)kp.o.tau_root;
    }
    o.win = kp.o.plateau_win;
    o.frac = (T)kp.o.plateau_frac;
    o.lambda0 = (T)kp.o.lambda0;
    o.stat_win = (MODE == MODE_FALLBACK64) ? 0 : kp.o.stat_win;
    o.stat_tol = (T)kp.o.stat_tol;

    Lane<T, N, D> L;
    PathIn<T, N> p;
    int sid = -1;
    int it0 = 0;  // iteration count at the start of a resumed path
    bool active = false;
    int cbase = 0, cend = 0;  // wave-uniform chunk [cbase, cend) of the bin
    bool drained = false;
    constexpr int CH = 64;

    while (true) {
        // ---- refill idle lanes from the wave's chunk
        // (once enough lanes are idle: each refill stalls the wave on the
        // dependent loads of the new paths' inputs)
        uint64_t need = __ballot(!active);
        if (need && !drained && ((int)__popcll(need) >= kp.refill || need == ~0ull)) {
            if (cbase >= cend) {
                int b0 = 0;
                if (lane == 0) b0 = atomicAdd(head, CH);
                b0 = __shfl(b0, 0);
                cbase = b0;
                cend = min(b0 + CH, count);
                if (cbase >= count) drained = true;
            }
            if (!drained) {
                const int avail = cend - cbase;
                const int rank = (int)__popcll(need & ((1ull << lane) - 1ull));
                const int take = min((int)__popcll(need), avail);
                if (!active && rank < take) {
                    const int slot = off + cbase + rank;
                    sid = list[slot];
                    active = true;
                    // ---- start of one path
                    // the first pass reads the bin-ordered copies of the
                    // receiver and primitive ids (consecutive slots); the
                    // fallback and the straggler pass go by solve id
                    const bool binned = !resume && MODE != MODE_FALLBACK64;
                    const int *pid = binned ? kp.slot_prim + slot : kp.b.prim + sid;
                    double rx[3];
                    const int ri = binned ? kp.slot_rx[slot] : kp.b.rx_index[sid];
#pragma unroll
                    for (int i = 0; i < 3; i++) rx[i] = kp.b.rx[3 * (size_t)ri + i];
                    p.planar = true;
#pragma unroll
                    for (int k = 0; k < N; k++) {
                        p.id[k] = pid[(size_t)k * kp.b.n];
                        p.ty[k] = prim_type(p.id[k], kp.s.n_pl, kp.s.n_pl_ln, kp.s.n_pl_ln_q);
                        p.planar = p.planar && (p.ty[k] == TL ||
                                                (p.ty[k] == TP && kp.s.rec64[(size_t)p.id[k] * kRec + 16] <= 0.0));
                    }
                    const double sh[3] = {MODE == MODE_FP32 ? kp.s.tx[0] : 0.0, MODE == MODE_FP32 ? kp.s.tx[1] : 0.0,
                                          MODE == MODE_FP32 ? kp.s.tx[2] : 0.0};
#pragma unroll
                    for (int i = 0; i < 3; i++) p.rx[i] = (T)(rx[i] - sh[i]);
                    if (resume) {
                        // a parked path: its state exactly as it was left
#pragma unroll
                        for (int j = 0; j < D; j++) L.X[j] = (T)kp.out.x[(size_t)sid * kRow + j];
                        L.it = kp.out.iters[sid];
                        it0 = L.it;
                        L.lam = (T)kp.spill_f[sid];
                        L.Cref = (T)kp.spill_f[(size_t)kp.b.n + sid];
                        L.stat = (int)kp.spill_f[(size_t)2 * kp.b.n + sid];
                        L.keep = false;
                        L.C = T(__builtin_huge_val());
                        L.rinf = T(__builtin_huge_val());
                    } else {
                    bool ok = true, inside = true;
                    // the fallback restarts from the FP32 end point (already root-like)
                    const int init = (MODE == MODE_FALLBACK64) ? INIT_USER : kp.o.init;
                    // the learned start serves the paths with a curved object;
                    // planes and straight edges keep the straight-line start
                    bool use_net = (init == INIT_LEARNED_ALL);
                    if (init == INIT_LEARNED)
                        for (int k = 0; k < N; k++) use_net = use_net || p.ty[k] == TQ || p.ty[k] == TC;
                    const bool from_line = init == INIT_RANDOM || init == INIT_LINE || (init == INIT_LEARNED && !use_net);
                    const bool rnd = init == INIT_RANDOM;
                    // the fallback's FP32 end point, the caller's points, or
                    // the learned start chosen before the LM pass
                    const double *x0 = (MODE == MODE_FALLBACK64) ? kp.out.x
                                       : (init == INIT_USER)     ? kp.b.x0
                                                                 : kp.x0_learned;
                    // one interaction at a time (few FP64 values live beside
                    // the busy lanes' state): its start point, its parameters
                    // in the parametric form, the guard box test
#pragma unroll
                    for (int k = 0; k < N; k++) {
                        const double *r64 = kp.s.rec64 + (size_t)p.id[k] * kRec;
                        double Xk[3];
                        if (from_line) {
                            // the projection onto the object of a point on the
                            // TX -> RX segment, or of a random point of the scene box
                            const double a = line_fraction(p.ty[k], r64, kp.s.tx, rx, k, N);
                            double P[3];
#pragma unroll
                            for (int i = 0; i < 3; i++) {
                                if (rnd) {
                                    const double u = splitmix_uniform(kp.o.seed, 15u * (uint64_t)sid + 3u * k + i);
                                    P[i] = kp.s.lo[i] + u * (kp.s.hi[i] - kp.s.lo[i]);
                                } else {
                                    P[i] = kp.s.tx[i] + a * (rx[i] - kp.s.tx[i]);
                                }
                            }
                            project(p.ty[k], r64, P, Xk);
                        } else {
#pragma unroll
                            for (int i = 0; i < 3; i++) {
                                Xk[i] = x0[(size_t)sid * kRow + 3 * k + i];
                                ok = ok && isfinite(Xk[i]);
                            }
                        }
                        if constexpr (FORM) {
                            // the parameters of the start point; the path
                            // starts at X(U), which must lie in the guard box
                            double u2[2];
                            ok = param_of(p.ty[k], r64, Xk, u2) && ok;
                            if (p.ty[k] == TQ) {
                                // the start point lifted onto the paraboloid
                                double e1[3], e2[3];
                                across_dir(r64 + 13, e1, e2);
                                const double h = r64[17] * (u2[0] * u2[0] + u2[1] * u2[1]);
#pragma unroll
                                for (int i = 0; i < 3; i++) Xk[i] = r64[i] + u2[0] * e1[i] + u2[1] * e2[i] + h * r64[13 + i];
                            }
                            L.X[2 * k] = (T)u2[0];
                            L.X[2 * k + 1] = (T)u2[1];
                        } else {
#pragma unroll
                            for (int i = 0; i < 3; i++) L.X[3 * k + i] = (T)(Xk[i] - sh[i]);
                        }
#pragma unroll
                        for (int i = 0; i < 3; i++) inside = inside && (Xk[i] >= kp.s.glo[i]) && (Xk[i] <= kp.s.ghi[i]);
                    }
                    int st0 = !ok ? ST_BAD : !inside ? ST_DIVERGED : ST_RUNNING;
                    if (MODE != MODE_FALLBACK64 && st0 == ST_RUNNING && sides_forbid_root<N>(kp.s, p.id, p.ty, rx))
                        st0 = ST_LOCALMIN;
                    L.it = 0;
                    L.stat = 0;
                    L.keep = false;
                    L.lam = T(0);
                    L.C = T(__builtin_huge_val());
                    L.rinf = T(__builtin_huge_val());
                    L.Cref = L.C;
                    if (st0 != ST_RUNNING) {
                        // finished before the first iteration: the start
                        // points as the solver holds them (zeros for bad input)
                        double Xs[3 * N];
#pragma unroll
                        for (int k = 0; k < N; k++) {
                            if constexpr (FORM) {
                                T Xk[3], Tm[3][2];
                                param_map<T>(p.ty[k], sc.rec + (size_t)p.id[k] * kRec, L.X[2 * k], L.X[2 * k + 1], Xk,
                                             Tm);
#pragma unroll
                                for (int i = 0; i < 3; i++) Xs[3 * k + i] = (double)Xk[i] + sh[i];
                            } else {
#pragma unroll
                                for (int i = 0; i < 3; i++) Xs[3 * k + i] = (double)L.X[3 * k + i] + sh[i];
                            }
                        }
#pragma unroll
                        for (int j = 0; j < kRow; j++)
                            kp.out.x[(size_t)sid * kRow + j] = (j < 3 * N && st0 != ST_BAD) ? Xs[j < 3 * N ? j : 0] : 0.0;
                        kp.out.cost[sid] = __builtin_huge_val();
                        if (MODE != MODE_FALLBACK64) {
                            kp.out.iters[sid] = 0;
                            if (kp.out.stage) kp.out.stage[sid] = 0;
                        }
                        kp.out.status[sid] = (uint8_t)(st0 | (MODE == MODE_FALLBACK64 ? 0x80 : 0));
                        active = false;
                    }
                    }  // not RESUME
                }
                cbase += take;
            }
        }
        if (!__any(active)) {
            if (drained) break;
            continue;
        }
        // the bin is drained and few lanes are busy: park them (wave-uniform)
        const bool park = may_spill && drained && (int)__popcll(__ballot(active)) <= kp.spill_t;
        // ---- one iteration on every busy lane
        if (active) {
            int st = ST_PARKED;
            if (!park) {
                st = -1;
                if constexpr (TYPED && MODE == MODE_FP32 && FORM == 1 && N <= 3) {
                    if (p.planar) {
                        // every planar path takes its fixed-type step, whatever
                        // the other lanes of its wave hold, so that its result
                        // does not depend on the schedule
                        int code = 0;
#pragma unroll
                        for (int k = 0; k < N; k++) code |= p.ty[k] << (2 * k);
                        st = lm_step_uniform<T, N, FORM>(code, sc, p, L, o);
                    }
                }
                if (st == -1) {
                    if constexpr (FORM) st = lm_step_param<T, N, REFR>(sc, p, L, o);
                    else st = lm_step<T, N, REFR>(sc, p, L, o);
                }
            }
            if (st == ST_PARKED) {
                // ---- a parked path: its exact state, for the straggler launch
#pragma unroll
                for (int j = 0; j < D; j++) kp.out.x[(size_t)sid * kRow + j] = (double)L.X[j];
                kp.out.iters[sid] = L.it;
                kp.spill_f[sid] = (double)L.lam;
                kp.spill_f[(size_t)kp.b.n + sid] = (double)L.Cref;
                kp.spill_f[(size_t)2 * kp.b.n + sid] = (double)L.stat;
                kp.spill_list[off + atomicAdd(&kp.spill_cnt[N - 1], 1)] = sid;
                active = false;
            } else if (st != ST_RUNNING) {
                // ---- end of one path: write it (world frame)
                const double sh[3] = {MODE == MODE_FP32 ? kp.s.tx[0] : 0.0, MODE == MODE_FP32 ? kp.s.tx[1] : 0.0,
                                      MODE == MODE_FP32 ? kp.s.tx[2] : 0.0};
                double Xw[3 * N];
                if constexpr (FORM) {
                    // the points X(U) in the solver's frame, then world
#pragma unroll
                    for (int k = 0; k < N; k++) {
                        T Xk[3], Tm[3][2];
                        param_map<T>(p.ty[k], sc.rec + (size_t)p.id[k] * kRec, L.X[2 * k], L.X[2 * k + 1], Xk, Tm);
#pragma unroll
                        for (int i = 0; i < 3; i++) Xw[3 * k + i] = (double)Xk[i] + sh[i];
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < 3 * N; j++) Xw[j] = (double)L.X[j] + sh[j % 3];
                }
                // the whole row (one cache line): the points, then zeros
#pragma unroll
                for (int j = 0; j < kRow; j++) kp.out.x[(size_t)sid * kRow + j] = (j < 3 * N) ? Xw[j < 3 * N ? j : 0] : 0.0;
                kp.out.cost[sid] = (double)L.C;
                int it = L.it;
                if (MODE == MODE_FALLBACK64) it += kp.out.iters[sid];
                kp.out.iters[sid] = it;
                if (kp.out.stage) {
                    if (MODE == MODE_FALLBACK64) kp.out.stage[(size_t)2 * kp.b.n + sid] = L.it;
                    else kp.out.stage[sid] = L.it;
                    if (resume) kp.out.stage[(size_t)3 * kp.b.n + sid] = L.it - it0;
                }
                int code = st;
                if (MODE == MODE_FP32) {
                    // route: FP32 end points whose residual is below the gate
                    // look like roots and are polished in FP64; the others
                    // are final (no path).  FP64 re-solves the path from its
                    // FP32 end point on numerical trouble in FP32: a
                    // degenerate iterate, a path of planes and straight
                    // edges still far from a root at its iteration cap (such
                    // descents reach their unique root quickly, so the cap
                    // alone is no evidence that none exists), or - decided
                    // by the polish - a converged or stalled FP32 point that
                    // does not polish
                    // a path through a refracting facet has a unique root
                    // (the optical length is convex), so a descent that ends
                    // far from a root goes to the FP64 fallback as well
                    bool refr_path = false;
                    if constexpr (REFR) {
#pragma unroll
                        for (int k = 0; k < N; k++)
                            refr_path = refr_path || (p.ty[k] == TP && kp.s.rec64[(size_t)p.id[k] * kRec + 16] > 0.0);
                    }
                    // on such a path the gate is at least 30 times the FP32
                    // rounding level of its residual: a law row carries the
                    // rounding of its unit directions (eps32 |X| / shortest
                    // segment) times its scale (up to the longest segment),
                    // which reaches 1e-2 m on a thin glass pane far from TX
                    double gate = kp.o.polish_gate;
                    if (refr_path) {
                        const double rx_w[3] = {(double)p.rx[0] + sh[0], (double)p.rx[1] + sh[1],
                                                (double)p.rx[2] + sh[2]};
                        double xmax = 0.0, smin = __builtin_huge_val(), smax = 0.0;
#pragma unroll
                        for (int k = 0; k <= N; k++) {
                            double e2 = 0.0;
#pragma unroll
                            for (int i = 0; i < 3; i++) {
                                const double a = (k == 0) ? kp.s.tx[i] : Xw[3 * (k - 1) + i];
                                const double bq = (k == N) ? rx_w[i] : Xw[3 * k + i];
                                e2 += (bq - a) * (bq - a);
                                if (k < N) xmax = fmax(xmax, fabs(Xw[3 * k + i] - kp.s.tx[i]));
                            }
                            smin = fmin(smin, sqrt(e2));
                            smax = fmax(smax, sqrt(e2));
                        }
                        gate = fmax(gate, 30.0 * 6e-8 * (1.0 + xmax) * smax / fmax(smin, 1e-12));
                    }
                    const bool small_res = (double)L.rinf <= gate;
                    bool to_polish = small_res && (st == ST_CONV || st == ST_MAXIT || st == ST_LOCALMIN ||
                                                   st == ST_STALL);
                    const bool to_fb = (st == ST_DEGEN) || (st == ST_MAXIT && p.planar && !small_res) ||
                                       (refr_path && !small_res);
                    // a root-like end point far outside a finite extent: the
                    // polish and the fallback stay next to it (within a few
                    // times its residual), so the path cannot be accepted
                    if (to_polish && kp.o.extent_skip > 0.0 &&
                        outside_extent<N>(kp.s.rec64, p.id, p.ty, Xw, kp.o.extent_skip + 100.0 * (double)L.rinf)) {
                        to_polish = false;
                        code = ST_OUTSIDE;
                    }
                    if (to_polish) {
                        // listed for the polish after the LM passes (no
                        // atomic with a return value in the iteration loop)
                        const bool rootlike = (double)L.rinf <= kp.o.tau_root32;
                        code = (rootlike && (st == ST_CONV || st == ST_STALL)) ? ROUTE_POLISH_FB
                               : (st == ST_MAXIT)                             ? ROUTE_POLISH_MAXIT
                                                                              : ROUTE_POLISH_LOCALMIN;
                    } else if (to_fb && kp.o.fallback) {
                        const int q = atomicAdd(&kp.fb_cnt[N - 1], 1);
                        kp.fb_list[off + q] = sid;
                        code = ST_RUNNING;
                    }
                }
                if (MODE == MODE_FALLBACK64) code |= 0x80;
                kp.out.status[sid] = (uint8_t)code;
                active = false;
            }
        }
    }
}

// Register budget per lane: an order-N path keeps 3N points, the 3N x 3N
// band (93 entries at N = 5) and its factor in registers, so the occupancy
// target falls with the order and doubles from FP64 to FP32.
template <int MODE, int N, int FORM = 0> struct Occ { static constexpr int W = 1; };
template <> struct Occ<MODE_FP32, 1, 0> { static constexpr int W = 4; };
template <> struct Occ<MODE_FP32, 2, 0> { static constexpr int W = 3; };
template <> struct Occ<MODE_FP32, 3, 0> { static constexpr int W = 2; };
template <> struct Occ<MODE_PLAIN64, 1, 0> { static constexpr int W = 3; };
template <> struct Occ<MODE_PLAIN64, 2, 0> { static constexpr int W = 2; };
template <> struct Occ<MODE_FALLBACK64, 1, 0> { static constexpr int W = 3; };
template <> struct Occ<MODE_FALLBACK64, 2, 0> { static constexpr int W = 2; };
// the parametric form holds 2N unknowns and a band of 2 x 2 blocks
template <> struct Occ<MODE_FP32, 1, 1> { static constexpr int W = 3; };
template <> struct Occ<MODE_FP32, 2, 1> { static constexpr int W = 3; };
template <> struct Occ<MODE_FP32, 3, 1> { static constexpr int W = 2; };
template <> struct Occ<MODE_FP32, 4, 1> { static constexpr int W = 2; };
// Order 5 at two waves per SIMD spills 360 B per lane to scratch and still
// runs its LM launch 17% faster than at one wave without spills (stress
// workload: 36.1 -> 29.7 ms, bit-identical results): the second wave hides
// the first one's LDS and memory waits.  Orders 3 and 4 at one or three
// waves, order 5 at three, the implicit form's orders 4-5 and the FP64
// parametric orders 3-5 at two all ran slower.
template <> struct Occ<MODE_FP32, 5, 1> { static constexpr int W = 2; };
template <> struct Occ<MODE_PLAIN64, 1, 1> { static constexpr int W = 2; };
template <> struct Occ<MODE_PLAIN64, 2, 1> { static constexpr int W = 2; };

// The mixed-order kernel keeps the register budget of its largest order.
template <int MODE, int FORM> struct OccAll { static constexpr int W = 1; };

// Scene records staged in LDS by every block of a persistent launch (the
// whole scene: 651 primitives x 18 floats = 47 KB for the street canyon).
template <int MODE, bool LDS>
__device__ __forceinline__ const typename ModeT<MODE>::T *stage_scene(const KParams &kp)
{
    using T = typename ModeT<MODE>::T;
    const T *g = (MODE == MODE_FP32) ? (const T *)kp.s.rec32 : (const T *)kp.s.rec64;
    if (!LDS) return g;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *l = reinterpret_cast<T *>(smem_raw);
    const int total = kp.s.n_all * kRec;
    for (int i = threadIdx.x; i < total; i += blockDim.x) l[i] = g[i];
    __syncthreads();
    return l;
}

// One persistent launch over every order (register budget of order 5).
// FORM 0: the implicit form (points as unknowns); 1: the parametric form.
// REFR: the scene has refracting facets; their rows are compiled into this
// kernel only (a branch left in the other kernels slowed the stress
// workload's LM launches by 16% in the parametric and 7% in the implicit
// form, though no lane took it), so such scenes run this schedule.
template <int MODE, bool LDS, int FORM, bool REFR>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(OccAll<MODE, FORM>::W, OccAll<MODE, FORM>::W)))
k_lm(KParams kp)
{
    const int *cnt = kp.resume ? kp.spill_cnt : (MODE == MODE_FALLBACK64) ? kp.fb_cnt : kp.bin_cnt;
    if (cnt[0] + cnt[1] + cnt[2] + cnt[3] + cnt[4] == 0) return;  // nothing to solve: skip the staging
    const typename ModeT<MODE>::T *rec = stage_scene<MODE, LDS>(kp);
    // long paths first so that the short ones fill the tail
    lm_bin<MODE, 5, FORM, true, REFR>(kp, rec);
    lm_bin<MODE, 4, FORM, true, REFR>(kp, rec);
    lm_bin<MODE, 3, FORM, true, REFR>(kp, rec);
    lm_bin<MODE, 2, FORM, true, REFR>(kp, rec);
    lm_bin<MODE, 1, FORM, true, REFR>(kp, rec);
}

// One persistent launch over orders 3, 2, 1 with the register budget of
// order 3 (twice the waves per SIMD of the all-order kernel in FP32); the
// split schedule runs orders 4 and 5 beside it with their own launches.
template <int MODE, bool LDS, int FORM>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(Occ<MODE, 3, FORM>::W, Occ<MODE, 3, FORM>::W))) k_lm_low(KParams kp)
{
    const int *cnt = kp.resume ? kp.spill_cnt : (MODE == MODE_FALLBACK64) ? kp.fb_cnt : kp.bin_cnt;
    if (cnt[0] + cnt[1] + cnt[2] == 0) return;
    const typename ModeT<MODE>::T *rec = stage_scene<MODE, LDS>(kp);
    lm_bin<MODE, 3, FORM>(kp, rec);
    lm_bin<MODE, 2, FORM>(kp, rec);
    lm_bin<MODE, 1, FORM>(kp, rec);
}

// One persistent launch per order, each with its own register budget.
template <int MODE, int N, bool LDS, int FORM>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(Occ<MODE, N, FORM>::W, Occ<MODE, N, FORM>::W))) k_lm_one(KParams kp)
{
    if ((kp.resume ? kp.spill_cnt : (MODE == MODE_FALLBACK64) ? kp.fb_cnt : kp.bin_cnt)[N - 1] == 0) return;
    const typename ModeT<MODE>::T *rec = stage_scene<MODE, LDS>(kp);
    // fixed-type steps for the planar paths of orders 1-3 here as in the
    // mixed-order kernel (stress LM stage 22.0 -> 21.7 ms, bit-identical)
    lm_bin<MODE, N, FORM, (N <= 3)>(kp, rec);
}

// ------------------------------------------------------------------ polish
// Undamped FP64 Gauss-Newton from the FP32 end point (world frame).
template <int N, bool REFR>
__device__ void polish_bin(const KParams &kp)
{
    const int count = kp.pol_cnt[N - 1];
    if (count == 0) return;
    const int off = bin_offset(kp.bin_cnt, N);
    SceneT<double> sc;
    sc.rec = kp.s.rec64;
#pragma unroll
    for (int i = 0; i < 3; i++) { sc.tx[i] = kp.s.tx[i]; sc.glo[i] = kp.s.glo[i]; sc.ghi[i] = kp.s.ghi[i]; }
    constexpr int M = 3 * N;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < count; q += gridDim.x * blockDim.x) {
        const int sid = kp.pol_list[off + q];
        PathIn<double, N> p;
        const int ri = kp.b.rx_index[sid];
#pragma unroll
        for (int i = 0; i < 3; i++) p.rx[i] = kp.b.rx[3 * (size_t)ri + i];
#pragma unroll
        for (int k = 0; k < N; k++) {
            p.id[k] = kp.b.prim[(size_t)k * kp.b.n + sid];
            p.ty[k] = prim_type(p.id[k], kp.s.n_pl, kp.s.n_pl_ln, kp.s.n_pl_ln_q);
        }
        double X[M];
#pragma unroll
        for (int j = 0; j < M; j++) X[j] = kp.out.x[(size_t)sid * kRow + j];
        bool ok = true, small = false;
        int steps = 0;
        for (int ps = 0; ps < kp.o.polish_steps && ok && !small; ps++) {
            double A[Band<N>::SIZE], g[M], C, rinf;
            ok = assemble<double, N, REFR>(sc, p, X, A, g, C, rinf);
            if (!ok) break;
            steps++;
            if (rinf <= kp.o.tol_res) { small = true; break; }
            double dmax = 0.0;
#pragma unroll
            for (int i = 0; i < M; i++) dmax = fmax(dmax, A[Band<N>::at(i, i)]);
#pragma unroll
            for (int i = 0; i < M; i++) A[Band<N>::at(i, i)] += 1e-15 * dmax;
            ok = chol_band<double, N>(A);
            if (!ok) break;
#pragma unroll
            for (int i = 0; i < M; i++) g[i] = -g[i];
            chol_solve_band<double, N>(A, g);
            double xinf = 0.0, dinf = 0.0;
#pragma unroll
            for (int i = 0; i < M; i++) {
                xinf = fmax(xinf, fabs(X[i]));
                dinf = fmax(dinf, fabs(g[i]));
                X[i] += g[i];
            }
            small = dinf <= kp.o.tol_step * (1.0 + xinf);
        }
        double C = __builtin_huge_val(), rinf = __builtin_huge_val();
        if (ok) ok = eval_cost<double, N, REFR>(sc, p, X, nullptr, C, rinf) && in_guard(kp.s, X, N);
        const bool root = ok && rinf <= kp.o.tau_root;
        kp.out.iters[sid] += steps;
        if (kp.out.stage) kp.out.stage[(size_t)kp.b.n + sid] = steps;
        if (root) {
#pragma unroll
            for (int j = 0; j < M; j++) kp.out.x[(size_t)sid * kRow + j] = X[j];
            kp.out.cost[sid] = C;
            kp.out.status[sid] = ST_CONV;
        } else {
            const int route = kp.out.status[sid];
            if (route == ROUTE_POLISH_FB && kp.o.fallback) {
                const int qq = atomicAdd(&kp.fb_cnt[N - 1], 1);
                kp.fb_list[off + qq] = sid;
                kp.out.status[sid] = ST_RUNNING;
            } else {
                kp.out.status[sid] = (route == ROUTE_POLISH_MAXIT) ? ST_MAXIT : ST_LOCALMIN;
            }
        }
    }
}

// One kernel for every order: measured faster than one launch per order
// (back to back or concurrent), although order 5 sets its registers.
template <bool REFR>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) k_polish(KParams kp)
{
    polish_bin<5, REFR>(kp);
    polish_bin<4, REFR>(kp);
    polish_bin<3, REFR>(kp);
    polish_bin<2, REFR>(kp);
    polish_bin<1, REFR>(kp);
}

// ------------------------------------------------------------------ acceptance
// The acceptance test of Alg. 1 in FP64: converged, |R|_inf <= tau_res, every
// segment at least min_seg, every point inside its finite extent.
// Smallest |cos| between a reflection's incoming direction and the surface
// normal that acceptance allows.
constexpr double kGraze = 1e-9;

template <int N, bool REFR>
__device__ bool accept_path(const SceneDev &s, const double *rx, const int *id, const int *ty, const double *X,
                            double tau_res, double min_seg)
{
    SceneT<double> sc;
    sc.rec = s.rec64;
#pragma unroll
    for (int i = 0; i < 3; i++) { sc.tx[i] = s.tx[i]; sc.glo[i] = s.glo[i]; sc.ghi[i] = s.ghi[i]; }
    PathIn<double, N> p;
#pragma unroll
    for (int i = 0; i < 3; i++) p.rx[i] = rx[i];
#pragma unroll
    for (int k = 0; k < N; k++) { p.id[k] = id[k]; p.ty[k] = ty[k]; }
    double C, rinf;
    bool ok = eval_cost<double, N, REFR>(sc, p, X, nullptr, C, rinf) && (rinf <= tau_res);
#pragma unroll
    for (int k = 0; k <= N; k++) {
        const double *P = (k == 0) ? s.tx : X + 3 * (k - 1);
        const double *Q = (k == N) ? rx : X + 3 * k;
        const double d[3] = {Q[0] - P[0], Q[1] - P[1], Q[2] - P[2]};
        ok = ok && (sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) >= min_seg);
    }
    double medium = 0.0;  // index of the medium the ray travels in (0: not yet known)
#pragma unroll
    for (int k = 0; k < N; k++) {
        const double *r = s.rec64 + (size_t)id[k] * kRec;
        const double *x = X + 3 * k;
        const double d[3] = {x[0] - r[0], x[1] - r[1], x[2] - r[2]};
        if (ty[k] == TP) {
            const double e[3] = {x[0] - r[4], x[1] - r[5], x[2] - r[6]};
            const double a = e[0] * r[7] + e[1] * r[8] + e[2] * r[9];
            const double b = e[0] * r[10] + e[1] * r[11] + e[2] * r[12];
            const double la = r[7] * r[7] + r[8] * r[8] + r[9] * r[9];
            const double lb = r[10] * r[10] + r[11] * r[11] + r[12] * r[12];
            ok = ok && a >= 0.0 && a <= la && b >= 0.0 && b <= lb;
        } else if (ty[k] == TL) {
            const double sp = d[0] * r[3] + d[1] * r[4] + d[2] * r[5];
            ok = ok && sp >= r[6] && sp <= r[7];
        } else if (ty[k] == TQ) {
            const double h = d[0] * r[13] + d[1] * r[14] + d[2] * r[15];
            const double w[3] = {d[0] - h * r[13], d[1] - h * r[14], d[2] - h * r[15]};
            ok = ok && (w[0] * w[0] + w[1] * w[1] + w[2] * w[2] <= r[16] * r[16]);
        }
        if (ty[k] == TP || ty[k] == TQ) {
            // a grazing reflection is degenerate: the ray passes along the
            // surface unchanged and the point can slide along it
            const double *P = (k == 0) ? s.tx : X + 3 * (k - 1);
            const double v[3] = {x[0] - P[0], x[1] - P[1], x[2] - P[2]};
            double nr[3];
            if (ty[k] == TP) {
                nr[0] = r[0], nr[1] = r[1], nr[2] = r[2];
            } else {
                const double A[3][3] = {{r[3], r[4], r[5]}, {r[4], r[6], r[7]}, {r[5], r[7], r[8]}};
                for (int i = 0; i < 3; i++) nr[i] = 2.0 * (A[i][0] * d[0] + A[i][1] * d[1] + A[i][2] * d[2]) + r[9 + i];
            }
            const double vn = v[0] * nr[0] + v[1] * nr[1] + v[2] * nr[2];
            const double lv = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            const double ln = sqrt(nr[0] * nr[0] + nr[1] * nr[1] + nr[2] * nr[2]);
            ok = ok && (fabs(vn) >= kGraze * lv * ln);
            if (ty[k] == TP && r[16] > 0.0) {
                // a refracting facet passes the ray to its other side, and the
                // ray arrives in the medium the previous refracting facet of
                // the path sent it into
                const double *Q = (k == N - 1) ? rx : X + 3 * (k + 1);
                const double e[3] = {Q[0] - x[0], Q[1] - x[1], Q[2] - x[2]};
                const double en = e[0] * nr[0] + e[1] * nr[1] + e[2] * nr[2];
                ok = ok && (vn * en > 0.0);
                const double in = (vn < 0.0) ? r[16] : r[17], out = (vn < 0.0) ? r[17] : r[16];
                ok = ok && !(medium > 0.0 && in != medium);
                medium = out;
            }
        }
    }
    return ok;
}

// Pass 1: clear the flags and list the converged solves, the only ones the
// test can accept (a few percent of a batch), so that the FP64 test runs on
// full waves instead of one or two lanes of each.  A block covers
// 256 x kAccItems x kAccChunks solves and takes its part of the list with one
// device-wide atomic (one per wave contended on the counter and cost more
// than the test itself); each chunk's loads are issued together.
constexpr int kAccItems = 16;
constexpr int kAccChunks = 4;
__global__ void __launch_bounds__(256) k_accept_list(BatchDev b, const uint8_t *__restrict__ status,
                                                      uint8_t *__restrict__ acc, int *__restrict__ list,
                                                      int *__restrict__ cnt)
{
    __shared__ int bcount, bbase;
    if (threadIdx.x == 0) bcount = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * 256 * kAccItems * kAccChunks;
    const int lane = __lane_id();
    int r[kAccChunks][kAccItems];
    for (int c = 0; c < kAccChunks; c++) {
        int ord[kAccItems], st[kAccItems];
#pragma unroll
        for (int j = 0; j < kAccItems; j++) {
            const int64_t i = base + (int64_t)(c * kAccItems + j) * 256 + threadIdx.x;
            ord[j] = 0;
            st[j] = 0;
            if (i < b.n) {
                ord[j] = b.order[i];
                st[j] = status[i];
            }
        }
#pragma unroll
        for (int j = 0; j < kAccItems; j++) {
            const int64_t i = base + (int64_t)(c * kAccItems + j) * 256 + threadIdx.x;
            if (i < b.n) acc[i] = 0;
            const bool v = ord[j] >= 1 && ord[j] <= kMaxN && (st[j] & 0x7f) == ST_CONV;
            const uint64_t m = __ballot(v);
            int wb = 0;
            if (lane == 0 && m) wb = atomicAdd(&bcount, (int)__popcll(m));
            wb = __shfl(wb, 0);
            r[c][j] = v ? wb + (int)__popcll(m & ((1ull << lane) - 1ull)) : -1;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) bbase = bcount ? atomicAdd(cnt, bcount) : 0;
    __syncthreads();
    for (int c = 0; c < kAccChunks; c++)
#pragma unroll
        for (int j = 0; j < kAccItems; j++)
            if (r[c][j] >= 0) list[bbase + r[c][j]] = (int)(base + (int64_t)(c * kAccItems + j) * 256 + threadIdx.x);
}

// Pass 2: the test on the listed solves (grid-stride over the list).
template <bool REFR>
__global__ void __launch_bounds__(256) k_accept_eval(SceneDev s, BatchDev b, OutDevC in, double tau_res,
                                                      double min_seg, uint8_t *__restrict__ acc,
                                                      const int *__restrict__ list, const int *__restrict__ cnt)
{
    const int m = *cnt;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < m; t += gridDim.x * blockDim.x) {
        const int64_t i = list[t];
        const int ord = b.order[i];
        bool a = false;
        {
            const int ri = b.rx_index[i];
            double rx[3], X[3 * kMaxN];
            int id[kMaxN], ty[kMaxN];
            for (int j = 0; j < 3; j++) rx[j] = b.rx[3 * (size_t)ri + j];
            for (int j = 0; j < 3 * kMaxN; j++) X[j] = (j < 3 * ord) ? in.x[(size_t)i * kRow + j] : 0.0;
            bool okid = true;
            for (int k = 0; k < kMaxN; k++) {
                id[k] = (k < ord) ? b.prim[(size_t)k * b.n + i] : 0;
                okid = okid && id[k] >= 0 && id[k] < s.n_all;
                ty[k] = prim_type(id[k], s.n_pl, s.n_pl_ln, s.n_pl_ln_q);
            }
            if (okid) {
                switch (ord) {
                case 1: a = accept_path<1, REFR>(s, rx, id, ty, X, tau_res, min_seg); break;
                case 2: a = accept_path<2, REFR>(s, rx, id, ty, X, tau_res, min_seg); break;
                case 3: a = accept_path<3, REFR>(s, rx, id, ty, X, tau_res, min_seg); break;
                case 4: a = accept_path<4, REFR>(s, rx, id, ty, X, tau_res, min_seg); break;
                default: a = accept_path<5, REFR>(s, rx, id, ty, X, tau_res, min_seg); break;
                }
            }
        }
        acc[i] = a ? 1 : 0;
    }
}

// Pass 3: accepted solves per block of 256 (for the ordered compaction).
__global__ void __launch_bounds__(256) k_accept_count(const uint8_t *__restrict__ acc, int64_t n,
                                                       int *__restrict__ block_cnt)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool a = (i < n) && acc[i];
    __shared__ int wcnt[4];
    const uint64_t m = __ballot(a);
    if (__lane_id() == 0) wcnt[threadIdx.x >> 6] = (int)__popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); w++) t += wcnt[w];
        block_cnt[blockIdx.x] = t;
    }
}

// Exclusive scan of the per-block counts by one block; total -> *count.
__global__ void __launch_bounds__(1024) k_scan_blocks(int *__restrict__ block_cnt, int nblk, int *__restrict__ count)
{
    // wave w owns a contiguous segment and reads it 64 entries at a time
    // (coalesced, eight loads in flight per lane); the 16 segment totals
    // give each wave its starting offset
    constexpr int kU = 8;
    __shared__ int wtot[16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int seg = ((nblk + 15) / 16 + 64 * kU - 1) / (64 * kU) * (64 * kU);
    const int lo = min(w * seg, nblk), hi = min(lo + seg, nblk);
    int s = 0;
    for (int i0 = lo; i0 < hi; i0 += 64 * kU) {
        int v[kU];
#pragma unroll
        for (int u = 0; u < kU; u++) {
            const int i = i0 + 64 * u + lane;
            v[u] = (i < hi) ? block_cnt[i] : 0;
        }
#pragma unroll
        for (int u = 0; u < kU; u++) s += v[u];
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
    if (lane == 0) wtot[w] = s;
    __syncthreads();
    int run = 0;
    for (int j = 0; j < w; j++) run += wtot[j];
    for (int i0 = lo; i0 < hi; i0 += 64 * kU) {
        int v[kU];
#pragma unroll
        for (int u = 0; u < kU; u++) {
            const int i = i0 + 64 * u + lane;
            v[u] = (i < hi) ? block_cnt[i] : 0;
        }
#pragma unroll
        for (int u = 0; u < kU; u++) {
            int incl = v[u];
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int x = __shfl_up(incl, d);
                if (lane >= d) incl += x;
            }
            const int i = i0 + 64 * u + lane;
            if (i < hi) block_cnt[i] = run + incl - v[u];
            run += __shfl(incl, 63);
        }
    }
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int j = 0; j < 16; j++) tot += wtot[j];
        *count = tot;
    }
}

__global__ void __launch_bounds__(256) k_accept_scatter(const uint8_t *__restrict__ acc, int64_t n,
                                                         const int *__restrict__ block_off, int *__restrict__ idx)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool a = (i < n) && acc[i];
    __shared__ int wcnt[4];
    const uint64_t m = __ballot(a);
    const int w = threadIdx.x >> 6;
    if (__lane_id() == 0) wcnt[w] = (int)__popcll(m);
    __syncthreads();
    int base = block_off[blockIdx.x];
    for (int j = 0; j < w; j++) base += wcnt[j];
    if (a) idx[base + (int)__popcll(m & ((1ull << __lane_id()) - 1ull))] = (int)i;
}

// ------------------------------------------------------------------ host launchers
void launch_pack(const double *raw, const double *refr, const SceneDev &s, int n_pl, int n_ln, int n_q, int n_c,
                 hipStream_t st)
{
    const int n = n_pl + n_ln + n_q + n_c;
    if (n == 0) return;
    hipLaunchKernelGGL(k_pack, dim3((n + 127) / 128), dim3(128), 0, st, raw, refr, n_pl, n_ln, n_q, n_c, s.tx[0],
                       s.tx[1], s.tx[2], (double *)s.rec64, (float *)s.rec32);
}

void launch_zero(int *p, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_i32, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
}

int bin_key_count() { return kNumKeys; }

// keys: [3][kNumKeys] ints (counts, offsets, cursors), zeroed by the caller
void launch_bin(const BatchDev &b, const OutDev &out, const SceneDev &s, int *bin_cnt, int *keys, int *perm,
                int *slot_rx, int *slot_prim, int *rows, int *curved, hipStream_t st)
{
    if (b.n == 0) return;
    const unsigned g = (unsigned)((b.n + kBinPerBlock - 1) / kBinPerBlock);
    int *kcnt = keys, *koff = keys + kNumKeys, *kcur = keys + 2 * kNumKeys;
    hipLaunchKernelGGL(k_bin_count, dim3(g), dim3(kBinBlock), 0, st, b, out, s.n_all, s.n_pl, s.n_pl_ln, s.n_pl_ln_q,
                       kcnt);
    hipLaunchKernelGGL(k_bin_offsets, dim3(1), dim3(1024), 0, st, kcnt, koff, bin_cnt, rows ? curved : nullptr);
    hipLaunchKernelGGL(k_bin_scatter, dim3(g), dim3(kBinBlock), 0, st, b, s.n_all, s.n_pl, s.n_pl_ln, s.n_pl_ln_q,
                       koff, kcur, perm, slot_rx, slot_prim, rows, curved);
}

template <int MODE, bool LDS, int FORM>
static const void *lm_kernel_t(int order)
{
    switch (order) {
    case 0: return (const void *)k_lm<MODE, LDS, FORM, false>;
    case 1: return (const void *)k_lm_one<MODE, 1, LDS, FORM>;
    case 2: return (const void *)k_lm_one<MODE, 2, LDS, FORM>;
    case 3: return (const void *)k_lm_one<MODE, 3, LDS, FORM>;
    case 4: return (const void *)k_lm_one<MODE, 4, LDS, FORM>;
    case 5: return (const void *)k_lm_one<MODE, 5, LDS, FORM>;
    default: return (const void *)k_lm_low<MODE, LDS, FORM>;
    }
}

template <int MODE, bool LDS, int FORM>
static const void *lm_kernel_refr() { return (const void *)k_lm<MODE, LDS, FORM, true>; }

// order 0: the mixed-order kernel; 1..5: the per-order kernels; 6: the
// kernel of orders 1-3.  refr: the mixed-order kernel with the rows of
// refracting facets (order ignored).  The fallback runs one mixed-order
// launch in the solve's form (from the FP32 end point).
const void *lm_kernel(int mode, int order, bool lds, int form, bool refr)
{
    switch (mode) {
    case MODE_PLAIN64:
        if (refr)
            return form ? (lds ? lm_kernel_refr<MODE_PLAIN64, true, 1>() : lm_kernel_refr<MODE_PLAIN64, false, 1>())
                        : (lds ? lm_kernel_refr<MODE_PLAIN64, true, 0>() : lm_kernel_refr<MODE_PLAIN64, false, 0>());
        if (form) return lds ? lm_kernel_t<MODE_PLAIN64, true, 1>(order) : lm_kernel_t<MODE_PLAIN64, false, 1>(order);
        return lds ? lm_kernel_t<MODE_PLAIN64, true, 0>(order) : lm_kernel_t<MODE_PLAIN64, false, 0>(order);
    case MODE_FP32:
        if (refr)
            return form ? (lds ? lm_kernel_refr<MODE_FP32, true, 1>() : lm_kernel_refr<MODE_FP32, false, 1>())
                        : (lds ? lm_kernel_refr<MODE_FP32, true, 0>() : lm_kernel_refr<MODE_FP32, false, 0>());
        if (form) return lds ? lm_kernel_t<MODE_FP32, true, 1>(order) : lm_kernel_t<MODE_FP32, false, 1>(order);
        return lds ? lm_kernel_t<MODE_FP32, true, 0>(order) : lm_kernel_t<MODE_FP32, false, 0>(order);
    default:
        if (refr)
            return form ? (lds ? lm_kernel_refr<MODE_FALLBACK64, true, 1>() : lm_kernel_refr<MODE_FALLBACK64, false, 1>())
                        : (lds ? lm_kernel_refr<MODE_FALLBACK64, true, 0>()
                               : lm_kernel_refr<MODE_FALLBACK64, false, 0>());
        if (form) return lds ? (const void *)k_lm<MODE_FALLBACK64, true, 1, false>
                             : (const void *)k_lm<MODE_FALLBACK64, false, 1, false>;
        return lds ? (const void *)k_lm<MODE_FALLBACK64, true, 0, false>
                   : (const void *)k_lm<MODE_FALLBACK64, false, 0, false>;
    }
}

void launch_lm(int mode, int order, bool lds, int form, bool refr, size_t lds_bytes, const KParams &kp, int grid,
               int block, hipStream_t st)
{
    void *args[] = {(void *)&kp};
    hipLaunchKernel(lm_kernel(mode, order, lds, form, refr), dim3(grid), dim3(block), args, lds ? lds_bytes : 0, st);
}

const void *polish_kernel(bool refr) { return refr ? (const void *)k_polish<true> : (const void *)k_polish<false>; }

void launch_learned_choose(const SceneDev &s, const BatchDev &b, const int *rows, const int *count, bool all,
                           double *x0l, double gain, bool refr, hipStream_t st)
{
    if (b.n == 0) return;
    const unsigned g = (unsigned)std::min<int64_t>((b.n + 255) / 256, 2048);
    if (refr) hipLaunchKernelGGL(k_learned_choose<true>, dim3(g), dim3(256), 0, st, s, b, rows, count, all ? 1 : 0, x0l, gain);
    else hipLaunchKernelGGL(k_learned_choose<false>, dim3(g), dim3(256), 0, st, s, b, rows, count, all ? 1 : 0, x0l, gain);
}

// The polish list: the solves the FP32 passes routed to the polish, grouped
// by order at the bins' offsets.  Each block counts its solves per order in
// LDS and takes its slots with one global atomic per order, so that the
// counters see a few hundred atomics rather than one per wave.
// solves per thread: kPolChunks chunks of kPolListPer solves whose loads
// are issued together; large blocks, so that few blocks take slots with
// the device-wide atomics on the five per-order counters (one counter is
// served one atomic at a time: with 8 solves per thread the 8192 blocks'
// atomics took 0.29 ms on the stress workload)
constexpr int kPolListPer = 8;
constexpr int kPolChunks = 4;
__global__ void __launch_bounds__(256) k_polish_list(KParams kp)
{
    __shared__ int lcnt[kMaxN], lbase[kMaxN];
    const int64_t b0 = (int64_t)blockIdx.x * blockDim.x * kPolListPer * kPolChunks;
    if (threadIdx.x < kMaxN) lcnt[threadIdx.x] = 0;
    __syncthreads();
    // per solve: its order (0: not listed) | its rank among the block's
    // solves of that order << 3
    int os[kPolChunks][kPolListPer];
    for (int c = 0; c < kPolChunks; c++) {
        int ord[kPolListPer], st[kPolListPer];
        // every load of the chunk first (status and order), so that they
        // are in flight together
#pragma unroll
        for (int q = 0; q < kPolListPer; q++) {
            const int64_t i = b0 + (int64_t)(c * kPolListPer + q) * blockDim.x + threadIdx.x;
            st[q] = -1;
            ord[q] = 0;
            if (i < kp.b.n) {
                st[q] = kp.out.status[i];
                ord[q] = kp.b.order[i];
            }
        }
        for (int q = 0; q < kPolListPer; q++) {
            if (!(st[q] == ROUTE_POLISH_FB || st[q] == ROUTE_POLISH_MAXIT || st[q] == ROUTE_POLISH_LOCALMIN)) ord[q] = 0;
            int slot = 0;
            for (int o = 1; o <= kMaxN; o++) {
                const uint64_t m = __ballot(ord[q] == o);
                if (!m) continue;
                const int leader = (int)__builtin_ctzll(m);
                int base = 0;
                if (__lane_id() == leader) base = atomicAdd(&lcnt[o - 1], (int)__popcll(m));
                base = __shfl(base, leader);
                if (ord[q] == o) slot = base + (int)__popcll(m & ((1ull << __lane_id()) - 1ull));
            }
            os[c][q] = ord[q] | (slot << 3);
        }
    }
    __syncthreads();
    if (threadIdx.x < kMaxN)
        lbase[threadIdx.x] = lcnt[threadIdx.x] ? atomicAdd(&kp.pol_cnt[threadIdx.x], lcnt[threadIdx.x]) : 0;
    __syncthreads();
    for (int c = 0; c < kPolChunks; c++)
        for (int q = 0; q < kPolListPer; q++) {
            const int64_t i = b0 + (int64_t)(c * kPolListPer + q) * blockDim.x + threadIdx.x;
            const int o = os[c][q] & 7;
            if (o > 0) kp.pol_list[bin_offset(kp.bin_cnt, o) + lbase[o - 1] + (os[c][q] >> 3)] = (int)i;
        }
}

void launch_polish_list(const KParams &kp, hipStream_t st)
{
    if (kp.b.n == 0) return;
    const int64_t per_block = 256 * kPolListPer * kPolChunks;
    hipLaunchKernelGGL(k_polish_list, dim3((unsigned)((kp.b.n + per_block - 1) / per_block)), dim3(256), 0, st, kp);
}

void launch_polish(const KParams &kp, bool refr, int grid, int block, hipStream_t st)
{
    if (refr) hipLaunchKernelGGL(k_polish<true>, dim3(grid), dim3(block), 0, st, kp);
    else hipLaunchKernelGGL(k_polish<false>, dim3(grid), dim3(block), 0, st, kp);
}

// ------------------------------------------------------------------ physical validation
// block_cnt: nblk + 1 ints (the last one counts the listed solves); the
// converged solves are listed in idx, which the compaction then overwrites
void launch_accept(const SceneDev &s, const BatchDev &b, const OutDevC &in, double tau_res, double min_seg,
                   uint8_t *acc, int *idx, int *count, int *block_cnt, bool refr, hipStream_t st)
{
    const int nblk = (int)((b.n + 255) / 256);
    if (nblk == 0) {
        hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, count, 1);
        return;
    }
    int *lcnt = block_cnt + nblk;
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, lcnt, 1);
    const int64_t per_list_block = 256 * kAccItems * kAccChunks;
    hipLaunchKernelGGL(k_accept_list, dim3((unsigned)((b.n + per_list_block - 1) / per_list_block)), dim3(256), 0, st,
                       b, in.status, acc, idx, lcnt);
    const dim3 g(std::min(nblk, 2048));
    if (refr) hipLaunchKernelGGL(k_accept_eval<true>, g, dim3(256), 0, st, s, b, in, tau_res, min_seg, acc, idx, lcnt);
    else hipLaunchKernelGGL(k_accept_eval<false>, g, dim3(256), 0, st, s, b, in, tau_res, min_seg, acc, idx, lcnt);
    hipLaunchKernelGGL(k_accept_count, dim3(nblk), dim3(256), 0, st, acc, b.n, block_cnt);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, block_cnt, nblk, count);
    hipLaunchKernelGGL(k_accept_scatter, dim3(nblk), dim3(256), 0, st, acc, b.n, block_cnt, idx);
}

}  // namespace mpt
