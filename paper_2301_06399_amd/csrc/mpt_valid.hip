// Physical validation of accepted paths on the GPU (mpt_visible): between
// interactions a ray travels in free space (Sec. II), so a kept path's
// segments may not cross another facet or paraboloid patch, and a segment at
// a wedged straight edge must leave it into free space.
//
//  k_vis_list   compacts the accepted solves into a list, clears visible[]
//  k_visible    one thread per accepted solve: every segment against every
//               facet and patch (staged in LDS) and the edges' wedges
#include "mpt_internal.hpp"
#include "mpt_geom.hpp"

namespace mpt {

__global__ void k_vis_zero(int *p) { if (threadIdx.x == 0) p[0] = 0; }

// The accepted solves, compacted (in no particular order) into list[1..],
// their count in list[0]; visible[] cleared for every solve.
__global__ void __launch_bounds__(256) k_vis_list(const uint8_t *__restrict__ acc, int64_t n, int *__restrict__ list,
                                                  uint8_t *__restrict__ vis)
{
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < n; i0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = i0 + threadIdx.x;
        const bool a = i < n && acc[i] != 0;
        if (i < n) vis[i] = 0;
        const uint64_t m = __ballot(a);
        if (!m) continue;
        const int leader = (int)__builtin_ctzll(m);
        int base = 0;
        if (__lane_id() == leader) base = atomicAdd(list, (int)__popcll(m));
        base = __shfl(base, leader);
        if (a) list[1 + base + (int)__popcll(m & ((1ull << __lane_id()) - 1ull))] = (int)i;
    }
}

// One thread per accepted solve of the list: visible[i] = 1 when no segment
// is blocked.  Plane and quadric records are staged in LDS when `lds` is set.
__global__ void __launch_bounds__(256) k_visible(SceneDev s, BatchDev b, OutDevC in, const int *__restrict__ list,
                                                 double min_seg, uint8_t *__restrict__ vis, int *__restrict__ count,
                                                 int lds)
{
#pragma clang fp contract(off)
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *srec = reinterpret_cast<double *>(smem_raw);
    const int npl = s.n_pl, nq = s.n_pl_ln_q - s.n_pl_ln;
    if (lds) {
        for (int j = threadIdx.x; j < npl * kRec; j += blockDim.x) srec[j] = s.rec64[j];
        for (int j = threadIdx.x; j < nq * kRec; j += blockDim.x)
            srec[(size_t)npl * kRec + j] = s.rec64[(size_t)s.n_pl_ln * kRec + j];
        __syncthreads();
    }
    const double *prec = lds ? srec : s.rec64;
    const double *qrec = lds ? srec + (size_t)npl * kRec : s.rec64 + (size_t)s.n_pl_ln * kRec;
    const int64_t na = list[0];
    for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x; t0 < na; t0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = t0 + threadIdx.x;
        bool ok = t < na;
        const int64_t i = ok ? list[1 + t] : 0;
        const int n = ok ? b.order[i] : 0;
        const double *rx = b.rx + 3 * (size_t)(ok ? b.rx_index[i] : 0);
        for (int k = 0; ok && k <= n; k++) {
            double P[3], Q[3], d[3];
            for (int c = 0; c < 3; c++) {
                P[c] = (k == 0) ? s.tx[c] : in.x[(size_t)i * kRow + 3 * (k - 1) + c];
                Q[c] = (k == n) ? rx[c] : in.x[(size_t)i * kRow + 3 * k + c];
                d[c] = Q[c] - P[c];
            }
            const int ip = (k == 0) ? -1 : b.prim[(size_t)(k - 1) * b.n + i];
            const int iq = (k == n) ? -1 : b.prim[(size_t)k * b.n + i];
            const double L = sqrt(vdot(d, d));
            if (!(L > 0.0)) { ok = false; break; }
            const double tmin = min_seg / L, tmax = 1.0 - tmin;
            for (int j = 0; ok && j < npl; j++)
                if (j != ip && j != iq && vis_plane(prec + (size_t)j * kRec, P, d, tmin, tmax)) ok = false;
            for (int j = 0; ok && j < nq; j++) {
                const int gid = s.n_pl_ln + j;
                if (gid != ip && gid != iq && vis_quadric(qrec + (size_t)j * kRec, P, d, tmin, tmax)) ok = false;
            }
            // the segment's ends on straight edges: both leave into free space
            if (ok && s.wedge && ip >= npl && ip < s.n_pl_ln && vis_wedge(s.wedge + 7 * (size_t)(ip - npl), P, Q))
                ok = false;
            if (ok && s.wedge && iq >= npl && iq < s.n_pl_ln && vis_wedge(s.wedge + 7 * (size_t)(iq - npl), Q, P))
                ok = false;
        }
        if (ok) vis[i] = 1;
        const uint64_t m = __ballot(ok);
        if (m && __lane_id() == __ffsll((unsigned long long)m) - 1) atomicAdd(count, (int)__popcll(m));
    }
}

void launch_visible(const SceneDev &s, const BatchDev &b, const OutDevC &in, const uint8_t *acc, double min_seg,
                    uint8_t *vis, int *count, int *list, size_t lds_max, int cu, hipStream_t st)
{
    hipLaunchKernelGGL(k_vis_zero, dim3(1), dim3(64), 0, st, count);
    if (b.n == 0) return;
    hipLaunchKernelGGL(k_vis_zero, dim3(1), dim3(64), 0, st, list);
    hipLaunchKernelGGL(k_vis_list, dim3((unsigned)std::min<int64_t>((b.n + 255) / 256, 8192)), dim3(256), 0, st, acc,
                       b.n, list, vis);
    const size_t bytes = (size_t)(s.n_pl + (s.n_pl_ln_q - s.n_pl_ln)) * kRec * sizeof(double);
    const int lds = bytes <= lds_max && bytes <= 64 * 1024;
    if (lds) hipFuncSetAttribute((const void *)k_visible, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    // the accepted count is on the device: enough blocks for a few per CU,
    // each looping over the list
    const unsigned g = (unsigned)std::min<int64_t>((b.n + 255) / 256, (int64_t)cu * 8);
    hipLaunchKernelGGL(k_visible, dim3(g), dim3(256), lds ? bytes : 0, st, s, b, in, list, min_seg, vis, count, lds);
}

}  // namespace mpt
