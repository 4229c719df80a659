// Candidate generation of Alg. 1 on the GPU: the visibility matrix of the
// objects, the BS row and the UE columns of the adjacency matrix (Sec. II-C,
// Figs. 3-4), and the enumeration of every simple path BS -> objects -> UE
// of at most max_order objects as interaction lists.
//
//  k_samples        sample points of every object (mpt_geom.hpp)
//  k_vis_pairs      one wave per object pair i < j: lanes test sample pairs
//                   (sides / wedges, then every facet and patch staged in LDS)
//  k_vis_bs         one wave per object: its samples against BS
//  k_vis_rx         one wave per (receiver, object): its samples against RX
//  k_cand_count     one block per (receiver, first object): path counts per
//                   order from popcounts of the bit rows
//  k_scan_*         exclusive scan of the counts (receiver, order, first object)
//  k_cand_fill      one block per (receiver, first object): writes the paths in
//                   increasing object ids at the scanned offsets
#include "mpt_internal.hpp"
#include "mpt_geom.hpp"

namespace mpt {

__global__ void __launch_bounds__(256) k_fill_u32(uint32_t *__restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void __launch_bounds__(256) k_samples(SceneDev s, int k, double *__restrict__ samp, int *__restrict__ cnt)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= s.n_all) return;
    cnt[g] = obj_samples(s, g, k, samp + (size_t)g * sample_cap(k) * 3);
}

// Plane and quadric records staged in LDS (or read from HBM without).
struct Occluders {
    const double *prec, *qrec;
};

__device__ __forceinline__ Occluders stage_occluders(const SceneDev &s, double *srec, int lds)
{
    const int npl = s.n_pl, nq = s.n_pl_ln_q - s.n_pl_ln;
    if (lds) {
        for (int j = threadIdx.x; j < npl * kRec; j += blockDim.x) srec[j] = s.rec64[j];
        for (int j = threadIdx.x; j < nq * kRec; j += blockDim.x)
            srec[(size_t)npl * kRec + j] = s.rec64[(size_t)s.n_pl_ln * kRec + j];
        __syncthreads();
        return {srec, srec + (size_t)npl * kRec};
    }
    return {s.rec64, s.rec64 + (size_t)s.n_pl_ln * kRec};
}

// Pair index p of the strict upper triangle (row-major) -> (i, j), i < j.
__device__ __forceinline__ void pair_of(int64_t p, int n, int &i, int &j)
{
    // rows before i hold i n - i (i + 1) / 2 pairs; start from the real root
    // and correct by whole rows
    const double nn = (double)n - 0.5;
    int r = (int)(nn - sqrt(nn * nn - 2.0 * (double)p));
    if (r < 0) r = 0;
    if (r > n - 2) r = n - 2;
    auto before = [n](int64_t q) { return q * n - q * (q + 1) / 2; };
    while (r > 0 && before(r) > p) r--;
    while (r < n - 2 && before(r + 1) <= p) r++;
    i = r;
    j = (int)(p - before(r)) + r + 1;
}

__global__ void __launch_bounds__(256) k_vis_pairs(SceneDev s, int k, double min_seg, const double *__restrict__ samp,
                                                   const int *__restrict__ cnt, uint32_t *__restrict__ V, int W,
                                                   int lds)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const Occluders oc = stage_occluders(s, reinterpret_cast<double *>(smem_raw), lds);
    const int n = s.n_all, sc = sample_cap(k), lane = threadIdx.x & 63;
    const int64_t npairs = (int64_t)n * (n - 1) / 2;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t p = wave; p < npairs; p += nwave) {
        int i, j;
        pair_of(p, n, i, j);
        const int mi = cnt[i], mj = cnt[j], tot = mi * mj;
        const double *Si = samp + (size_t)i * sc * 3, *Sj = samp + (size_t)j * sc * 3;
        bool found = false;
        for (int t0 = 0; t0 < tot && !found; t0 += 64) {
            const int t = t0 + lane;
            bool vis = false;
            if (t < tot) {
                const double *P = Si + 3 * (t / mj), *Q = Sj + 3 * (t % mj);
                const double d[3] = {Q[0] - P[0], Q[1] - P[1], Q[2] - P[2]};
                const double e[3] = {P[0] - Q[0], P[1] - Q[1], P[2] - Q[2]};
                vis = leaves_obj(s, i, P, d) && leaves_obj(s, j, Q, e) &&
                      !seg_blocked(s, oc.prec, oc.qrec, P, Q, i, j, min_seg);
            }
            found = __any(vis);
        }
        if (found && lane == 0) {
            atomicOr(V + (size_t)i * W + (j >> 5), 1u << (j & 31));
            atomicOr(V + (size_t)j * W + (i >> 5), 1u << (i & 31));
        }
    }
}

__global__ void __launch_bounds__(256) k_vis_bs(SceneDev s, int k, double min_seg, const double *__restrict__ samp,
                                                const int *__restrict__ cnt, uint32_t *__restrict__ B, int lds)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const Occluders oc = stage_occluders(s, reinterpret_cast<double *>(smem_raw), lds);
    const int sc = sample_cap(k), lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t g = wave; g < s.n_all; g += nwave) {
        const int j = (int)g, m = cnt[j];
        const double *S = samp + (size_t)j * sc * 3;
        bool found = false;
        for (int t0 = 0; t0 < m && !found; t0 += 64) {
            const int t = t0 + lane;
            bool vis = false;
            if (t < m) {
                const double *Q = S + 3 * t;
                const double e[3] = {s.tx[0] - Q[0], s.tx[1] - Q[1], s.tx[2] - Q[2]};
                vis = leaves_obj(s, j, Q, e) && !seg_blocked(s, oc.prec, oc.qrec, s.tx, Q, -1, j, min_seg);
            }
            found = __any(vis);
        }
        if (found && lane == 0) atomicOr(B + (j >> 5), 1u << (j & 31));
    }
}

__global__ void __launch_bounds__(256) k_vis_rx(SceneDev s, int k, double min_seg, const double *__restrict__ samp,
                                                const int *__restrict__ cnt, const double *__restrict__ rx, int n_rx,
                                                uint32_t *__restrict__ U, uint8_t *__restrict__ los, int W, int lds)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const Occluders oc = stage_occluders(s, reinterpret_cast<double *>(smem_raw), lds);
    const int n = s.n_all, sc = sample_cap(k), lane = threadIdx.x & 63;
    // line of sight, one thread per receiver
    if (los)
        for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n_rx; r += (int64_t)gridDim.x * blockDim.x)
            los[r] = seg_blocked(s, oc.prec, oc.qrec, s.tx, rx + 3 * r, -1, -1, min_seg) ? 0 : 1;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t items = (int64_t)n_rx * n;
    for (int64_t it = wave; it < items; it += nwave) {
        const int r = (int)(it / n), j = (int)(it % n), m = cnt[j];
        const double *S = samp + (size_t)j * sc * 3, *R = rx + 3 * (size_t)r;
        bool found = false;
        for (int t0 = 0; t0 < m && !found; t0 += 64) {
            const int t = t0 + lane;
            bool vis = false;
            if (t < m) {
                const double *Q = S + 3 * t;
                const double d[3] = {R[0] - Q[0], R[1] - Q[1], R[2] - Q[2]};
                vis = leaves_obj(s, j, Q, d) && !seg_blocked(s, oc.prec, oc.qrec, Q, R, j, -1, min_seg);
            }
            found = __any(vis);
        }
        if (found && lane == 0) atomicOr(U + (size_t)r * W + (j >> 5), 1u << (j & 31));
    }
}

// ------------------------------------------------------------------ enumeration
// The graph: BS -> v iff B[v]; u -> v iff V[u][v] (an edge object u has no
// successor but UE when edges may only come last); v -> UE iff U[r][v].
struct CandGraph {
    const uint32_t *V, *B, *U;
    int n, W, n_pl, n_pl_ln, n_pl_ln_q, edge_last, maxo;
};

__device__ __forceinline__ bool is_edge(const CandGraph &G, int g)
{
    return (g >= G.n_pl && g < G.n_pl_ln) || g >= G.n_pl_ln_q;
}

__device__ __forceinline__ bool bit(const uint32_t *row, int v) { return (row[v >> 5] >> (v & 31)) & 1u; }

// The successors of u (none for an edge object when edges come last).
__device__ __forceinline__ const uint32_t *succ(const CandGraph &G, int u)
{
    return (G.edge_last && is_edge(G, u)) ? nullptr : G.V + (size_t)u * G.W;
}

// Depth-first walk, in increasing object ids and without recursion, of the
// simple paths that extend path[0..d0-1] to o objects, the last one seeing
// the receiver (row Ur).  Counts them, or writes them from position pos on.
template <bool WRITE>
__device__ int64_t walk_tail(const CandGraph &G, const uint32_t *Ur, int *path, int d0, int o, int r, int64_t pos,
                             int64_t cap, int32_t *rx_index, int32_t *order, int32_t *prim)
{
    const uint32_t *row[kMaxN];
    uint32_t m[kMaxN];
    int w[kMaxN];
    int64_t c = 0;
    int d = d0;
    row[d] = succ(G, path[d - 1]);
    if (!row[d]) return WRITE ? pos : 0;
    w[d] = 0;
    m[d] = row[d][0] & (d == o - 1 ? Ur[0] : ~0u);
    while (d >= d0) {
        while (m[d] == 0u && w[d] + 1 < G.W) {
            w[d]++;
            m[d] = row[d][w[d]] & (d == o - 1 ? Ur[w[d]] : ~0u);
        }
        if (m[d] == 0u) {  // this level is exhausted
            d--;
            continue;
        }
        const int v = (w[d] << 5) + (__ffs(m[d]) - 1);
        m[d] &= m[d] - 1u;
        bool seen = false;
        for (int q = 0; q < d; q++) seen = seen || path[q] == v;
        if (seen) continue;
        path[d] = v;
        if (d == o - 1) {
            if (WRITE) {
                rx_index[pos] = r;
                order[pos] = o;
                for (int q = 0; q < kMaxN; q++) prim[(size_t)q * cap + pos] = q < o ? path[q] : -1;
                pos++;
            } else {
                c++;
            }
            continue;
        }
        const uint32_t *nr = succ(G, v);
        if (!nr) continue;
        d++;
        row[d] = nr;
        w[d] = 0;
        m[d] = nr[0] & (d == o - 1 ? Ur[0] : ~0u);
    }
    return WRITE ? pos : c;
}

// Successors v2 of v1 in increasing order into an LDS list.
__device__ __forceinline__ int list_succ(const CandGraph &G, int v1, int *list)
{
    __shared__ int nlist;
    if (threadIdx.x == 0) nlist = 0;
    __syncthreads();
    const uint32_t *row = succ(G, v1);
    if (row && threadIdx.x == 0) {
        int c = 0;
        for (int w = 0; w < G.W; w++) {
            uint32_t m = row[w];
            while (m) {
                const int b = __ffs(m) - 1;
                m &= m - 1;
                list[c++] = (w << 5) + b;
            }
        }
        nlist = c;
    }
    __syncthreads();
    return nlist;
}

__device__ __forceinline__ int64_t block_sum_i64(int64_t v, int64_t *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const int64_t t = red[0];
    __syncthreads();
    return t;
}

// Inclusive scan over the block (Hillis-Steele in LDS).
__device__ __forceinline__ int64_t block_scan_i64(int64_t v, int64_t *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = 1; s < (int)blockDim.x; s <<= 1) {
        const int64_t a = (int)threadIdx.x >= s ? red[threadIdx.x - s] : 0;
        __syncthreads();
        red[threadIdx.x] += a;
        __syncthreads();
    }
    const int64_t t = red[threadIdx.x];
    __syncthreads();
    return t;
}

constexpr int kCandBlock = 256;
constexpr int kMaxObjCand = 4096;

__global__ void __launch_bounds__(kCandBlock) k_cand_count(CandGraph G, int n_rx, int64_t *__restrict__ cnt)
{
    __shared__ int list[kMaxObjCand];
    __shared__ int64_t red[kCandBlock];
    const int64_t items = (int64_t)n_rx * G.n;
    for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const int r = (int)(it / G.n), v1 = (int)(it % G.n);
        const uint32_t *Ur = G.U + (size_t)r * G.W;
        int64_t *out = cnt + (size_t)r * G.maxo * G.n + v1;
        if (!bit(G.B, v1)) {
            if (threadIdx.x == 0)
                for (int o = 1; o <= G.maxo; o++) out[(size_t)(o - 1) * G.n] = 0;
            continue;
        }
        const int nl = list_succ(G, v1, list);
        for (int o = 1; o <= G.maxo; o++) {
            int64_t c = 0;
            if (o == 1) {
                c = threadIdx.x == 0 ? (int64_t)bit(Ur, v1) : 0;
            } else {
                for (int e = threadIdx.x; e < nl; e += blockDim.x) {
                    const int v2 = list[e];
                    if (o == 2) {
                        c += bit(Ur, v2);
                    } else {
                        int path[kMaxN] = {v1, v2};
                        c += walk_tail<false>(G, Ur, path, 2, o, r, 0, 0, nullptr, nullptr, nullptr);
                    }
                }
            }
            c = block_sum_i64(c, red);
            if (threadIdx.x == 0) out[(size_t)(o - 1) * G.n] = c;
        }
    }
}

__global__ void __launch_bounds__(kCandBlock) k_cand_fill(CandGraph G, int n_rx, const int64_t *__restrict__ off,
                                                          int64_t cap, int32_t *__restrict__ rx_index,
                                                          int32_t *__restrict__ order, int32_t *__restrict__ prim)
{
    __shared__ int list[kMaxObjCand];
    __shared__ int64_t red[kCandBlock];
    const int64_t items = (int64_t)n_rx * G.n;
    for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const int r = (int)(it / G.n), v1 = (int)(it % G.n);
        if (!bit(G.B, v1)) continue;
        const uint32_t *Ur = G.U + (size_t)r * G.W;
        const int nl = list_succ(G, v1, list);
        for (int o = 1; o <= G.maxo; o++) {
            int64_t base = off[((size_t)r * G.maxo + (o - 1)) * G.n + v1];
            if (o == 1) {
                if (threadIdx.x == 0 && bit(Ur, v1)) {
                    rx_index[base] = r;
                    order[base] = 1;
                    for (int q = 0; q < kMaxN; q++) prim[(size_t)q * cap + base] = q < 1 ? v1 : -1;
                }
                continue;
            }
            // successors in increasing id, a chunk of blockDim at a time: each
            // thread's subtree count, scanned in list order, gives its offset
            for (int e0 = 0; e0 < nl; e0 += blockDim.x) {
                const int e = e0 + threadIdx.x;
                int64_t c = 0;
                int v2 = -1;
                if (e < nl) {
                    v2 = list[e];
                    if (o == 2) {
                        c = bit(Ur, v2);
                    } else {
                        int path[kMaxN] = {v1, v2};
                        c = walk_tail<false>(G, Ur, path, 2, o, r, 0, 0, nullptr, nullptr, nullptr);
                    }
                }
                const int64_t incl = block_scan_i64(c, red);
                const int64_t chunk = red[blockDim.x - 1];
                if (o == 3) {
                    // consecutive threads write consecutive paths: path q of
                    // the chunk belongs to the first successor whose inclusive
                    // count exceeds q, and is the rank-th object after it
                    const int ne = min((int)blockDim.x, nl - e0);
                    for (int64_t q = threadIdx.x; q < chunk; q += blockDim.x) {
                        int lo = 0, hi = ne - 1;
                        while (lo < hi) {
                            const int mid = (lo + hi) >> 1;
                            if (red[mid] > q) hi = mid;
                            else lo = mid + 1;
                        }
                        const int w2 = list[e0 + lo];
                        int64_t rank = q - (lo ? red[lo - 1] : 0);
                        const uint32_t *row2 = G.V + (size_t)w2 * G.W;
                        int v3 = -1;
                        for (int w = 0; w < G.W && v3 < 0; w++) {
                            uint32_t m = row2[w] & Ur[w];
                            if ((v1 >> 5) == w) m &= ~(1u << (v1 & 31));
                            const int pc = __popc(m);
                            if (rank < pc) {
                                for (int z = 0; z < (int)rank; z++) m &= m - 1u;
                                v3 = (w << 5) + (__ffs(m) - 1);
                            }
                            rank -= pc;
                        }
                        const int64_t pos = base + q;
                        rx_index[pos] = r;
                        order[pos] = 3;
                        prim[pos] = v1;
                        prim[(size_t)cap + pos] = w2;
                        prim[(size_t)2 * cap + pos] = v3;
                        prim[(size_t)3 * cap + pos] = -1;
                        prim[(size_t)4 * cap + pos] = -1;
                    }
                } else if (c > 0) {
                    int path[kMaxN] = {v1, v2};
                    const int64_t pos = base + incl - c;
                    if (o == 2) {
                        rx_index[pos] = r;
                        order[pos] = 2;
                        for (int q = 0; q < kMaxN; q++) prim[(size_t)q * cap + pos] = q < 2 ? path[q] : -1;
                    } else {
                        walk_tail<true>(G, Ur, path, 2, o, r, pos, cap, rx_index, order, prim);
                    }
                }
                __syncthreads();  // red is read above; the next chunk rewrites it
                base += chunk;
            }
        }
    }
}

// Exclusive scan of n int64 values in place: blocks of 1024 (4 per thread),
// their totals, then the offsets added back.
constexpr int kScanPer = 4;

__global__ void __launch_bounds__(256) k_scan_local(int64_t *__restrict__ a, int64_t n, int64_t *__restrict__ sums)
{
    __shared__ int64_t red[256];
    const int64_t b0 = (int64_t)blockIdx.x * 256 * kScanPer + (int64_t)threadIdx.x * kScanPer;
    int64_t v[kScanPer], t = 0;
    for (int q = 0; q < kScanPer; q++) {
        v[q] = (b0 + q < n) ? a[b0 + q] : 0;
        t += v[q];
    }
    const int64_t incl = block_scan_i64(t, red);
    int64_t run = incl - t;
    for (int q = 0; q < kScanPer; q++) {
        if (b0 + q < n) a[b0 + q] = run;
        run += v[q];
    }
    if (threadIdx.x == blockDim.x - 1) sums[blockIdx.x] = incl;
}

// One block: exclusive scan of the block totals (any count), and the grand
// total into sums[nb].
__global__ void __launch_bounds__(256) k_scan_sums(int64_t *__restrict__ sums, int64_t nb)
{
    __shared__ int64_t red[256];
    int64_t carry = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += blockDim.x) {
        const int64_t i = c0 + threadIdx.x;
        const int64_t v = i < nb ? sums[i] : 0;
        const int64_t incl = block_scan_i64(v, red);
        const int64_t chunk = red[blockDim.x - 1];
        __syncthreads();
        if (i < nb) sums[i] = carry + incl - v;
        carry += chunk;
    }
    if (threadIdx.x == 0) sums[nb] = carry;
}

__global__ void __launch_bounds__(256) k_scan_add(int64_t *__restrict__ a, int64_t n, const int64_t *__restrict__ sums)
{
    const int64_t b0 = (int64_t)blockIdx.x * 256 * kScanPer + (int64_t)threadIdx.x * kScanPer;
    const int64_t add = sums[blockIdx.x];
    for (int q = 0; q < kScanPer; q++)
        if (b0 + q < n) a[b0 + q] += add;
}

// ------------------------------------------------------------------ launchers
static size_t occluder_bytes(const SceneDev &s)
{
    return (size_t)(s.n_pl + (s.n_pl_ln_q - s.n_pl_ln)) * kRec * sizeof(double);
}

static int lds_choice(const void *kern, const SceneDev &s, size_t lds_max, size_t &bytes)
{
    bytes = occluder_bytes(s);
    const int lds = bytes <= lds_max && bytes <= 64 * 1024;
    if (lds) hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    else bytes = 0;
    return lds;
}

void launch_samples(const SceneDev &s, int k, double *samp, int *cnt, hipStream_t st)
{
    if (s.n_all == 0) return;
    hipLaunchKernelGGL(k_samples, dim3((s.n_all + 255) / 256), dim3(256), 0, st, s, k, samp, cnt);
}

void launch_visibility(const SceneDev &s, int k, double min_seg, const double *samp, const int *cnt, uint32_t *V,
                       uint32_t *B, int W, size_t lds_max, int cu, hipStream_t st)
{
    const int64_t nv = (int64_t)s.n_all * W;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<int64_t>((nv + 255) / 256 + 1, 4096)), dim3(256), 0, st, V,
                       nv);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, B, (int64_t)W);
    if (s.n_all == 0) return;
    size_t bytes;
    const int64_t npairs = (int64_t)s.n_all * (s.n_all - 1) / 2;
    if (npairs > 0) {
        const int lds = lds_choice((const void *)k_vis_pairs, s, lds_max, bytes);
        const unsigned g = (unsigned)std::min<int64_t>((npairs + 3) / 4, (int64_t)cu * 64);
        hipLaunchKernelGGL(k_vis_pairs, dim3(g), dim3(256), bytes, st, s, k, min_seg, samp, cnt, V, W, lds);
    }
    const int lds = lds_choice((const void *)k_vis_bs, s, lds_max, bytes);
    hipLaunchKernelGGL(k_vis_bs, dim3((s.n_all + 3) / 4), dim3(256), bytes, st, s, k, min_seg, samp, cnt, B, lds);
}

void launch_visibility_rx(const SceneDev &s, int k, double min_seg, const double *samp, const int *cnt,
                          const double *rx, int n_rx, uint32_t *U, uint8_t *los, int W, size_t lds_max, int cu,
                          hipStream_t st)
{
    const int64_t nu = (int64_t)n_rx * W;
    if (nu > 0)
        hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<int64_t>((nu + 255) / 256, 4096)), dim3(256), 0, st, U,
                           nu);
    if (n_rx == 0) return;
    size_t bytes;
    const int lds = lds_choice((const void *)k_vis_rx, s, lds_max, bytes);
    const int64_t items = (int64_t)n_rx * s.n_all;
    const unsigned g = (unsigned)std::max<int64_t>(std::min<int64_t>((items + 3) / 4, (int64_t)cu * 64),
                                                   (n_rx + 255) / 256);
    hipLaunchKernelGGL(k_vis_rx, dim3(g), dim3(256), bytes, st, s, k, min_seg, samp, cnt, rx, n_rx, U, los, W, lds);
}

static CandGraph graph_of(const SceneDev &s, const uint32_t *V, const uint32_t *B, const uint32_t *U, int W,
                          int maxo, int edge_last)
{
    CandGraph G;
    G.V = V;
    G.B = B;
    G.U = U;
    G.n = s.n_all;
    G.W = W;
    G.n_pl = s.n_pl;
    G.n_pl_ln = s.n_pl_ln;
    G.n_pl_ln_q = s.n_pl_ln_q;
    G.edge_last = edge_last;
    G.maxo = maxo;
    return G;
}

void launch_cand_count(const SceneDev &s, const uint32_t *V, const uint32_t *B, const uint32_t *U, int W, int n_rx,
                       int maxo, int edge_last, int64_t *cnt, int64_t *sums, int cu, hipStream_t st)
{
    const CandGraph G = graph_of(s, V, B, U, W, maxo, edge_last);
    const int64_t items = (int64_t)n_rx * s.n_all;
    hipLaunchKernelGGL(k_cand_count, dim3((unsigned)std::min<int64_t>(items, (int64_t)cu * 32)), dim3(kCandBlock), 0,
                       st, G, n_rx, cnt);
    // exclusive scan over (receiver, order, first object)
    const int64_t n = items * maxo;
    const int64_t nb = (n + 256 * kScanPer - 1) / (256 * kScanPer);
    hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(256), 0, st, cnt, n, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, st, sums, nb);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(256), 0, st, cnt, n, sums);
}

void launch_cand_fill(const SceneDev &s, const uint32_t *V, const uint32_t *B, const uint32_t *U, int W, int n_rx,
                      int maxo, int edge_last, const int64_t *off, int64_t cap, int32_t *rx_index, int32_t *order,
                      int32_t *prim, int cu, hipStream_t st)
{
    const CandGraph G = graph_of(s, V, B, U, W, maxo, edge_last);
    const int64_t items = (int64_t)n_rx * s.n_all;
    hipLaunchKernelGGL(k_cand_fill, dim3((unsigned)std::min<int64_t>(items, (int64_t)cu * 32)), dim3(kCandBlock), 0,
                       st, G, n_rx, off, cap, rx_index, order, prim);
}

}  // namespace mpt
