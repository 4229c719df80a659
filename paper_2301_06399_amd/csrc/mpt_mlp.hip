// Learned warm start: a small MLP that predicts the interaction points of a
// path from TX, RX and its objects (replacing the random guess of the
// paper's algorithm), trained on the GPU on solver outputs.
//
//   features (96) -> 256 -> 256 -> 256 -> 15, GELU (erf form) after the
//   hidden layers; BF16 weights and activations, FP32 accumulation on the
//   matrix cores (v_mfma_f32_32x32x16_bf16), FP32 master weights + Adam.
//
// Kernels: k_features (per path), k_gemm (LDS-tiled MFMA GEMM with bias /
// GELU / GELU' epilogues and split-K partials), k_reduce_splits, k_colsum
// (bias gradients), k_loss (masked MSE and its gradient), k_adam, k_decode.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>
#include <stdio.h>
#include <stdlib.h>
#include <string>
#include <vector>

#include "mpt_mlp.hpp"

namespace mpt {

constexpr int F_IN = 96, HID = 256, F_OUT = 15, F_OUTP = 16;
constexpr int SLOT = 17;  // per-interaction feature slot: one-hot 4, params 12, present 1

// ------------------------------------------------------------------ bf16
typedef uint16_t bf16;
// hardware round-to-nearest-even conversion (v_cvt_pk_bf16_f32 on gfx950)
__device__ __forceinline__ bf16 f2bf(float f) { return __builtin_bit_cast(bf16, (__bf16)f); }
__device__ __forceinline__ float bf2f(bf16 h) { return __uint_as_float((uint32_t)h << 16); }

// Inference copy of the three hidden-layer weight matrices in the order the
// fused kernel's waves read them as matrix-core A fragments: layer l (K
// inputs, S = K / 16 steps of 16) is a run of [4 unit blocks of 64][S steps]
// [2 halves of 32 units][64 lanes] fragments of 8 BF16, lane j holding unit
// 32 half + (j % 32) of its block, inputs 16 step + 8 (j / 32) .. +8.  One
// wave's fragment is 1 KB contiguous, so each load instruction reads whole
// cache lines (the [out][in] matrix gives each lane its own row).  Written
// wherever the BF16 weights are, from the same values.
constexpr size_t NFRAG = (size_t)HID * F_IN + 2 * (size_t)HID * HID;
__host__ __device__ constexpr long long frag_of(size_t i)
{
    // flat parameter layout: W1 [HID][F_IN], b1, W2 [HID][HID], b2, W3, b3, ...
    constexpr size_t w1 = 0, w2 = w1 + (size_t)HID * F_IN + HID, w3 = w2 + (size_t)HID * HID + HID;
    size_t off, K, base;
    if (i < w1 + (size_t)HID * F_IN) {
        off = i - w1, K = F_IN, base = 0;
    } else if (i >= w2 && i < w2 + (size_t)HID * HID) {
        off = i - w2, K = HID, base = (size_t)HID * F_IN;
    } else if (i >= w3 && i < w3 + (size_t)HID * HID) {
        off = i - w3, K = HID, base = (size_t)HID * F_IN + (size_t)HID * HID;
    } else {
        return -1;
    }
    const size_t u = off / K, k = off % K, S = K / 16;
    const size_t blk = u / 64, half = (u % 64) / 32, lane = u % 32 + 32 * ((k % 16) / 8);
    return (long long)(base + (((blk * S + k / 16) * 2 + half) * 64 + lane) * 8 + k % 8);
}

// GELU in its erf form, with erf from Abramowitz & Stegun 7.1.26 (Hastings'
// rational approximation, |error| <= 1.5e-7, far below BF16 resolution):
// erf(x) = 1 - t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-x^2),
// t = 1 / (1 + p x), x >= 0, odd extension.  One exponential serves both
// GELU(z) = z Phi(z) and GELU'(z) = Phi(z) + z phi(z).
__device__ __forceinline__ void gelu_both(float z, float &g, float &gd)
{
    const float x = fabsf(z) * 0.70710678118654752f;
    const float t = __builtin_amdgcn_rcpf(1.0f + 0.3275911f * x);
    const float poly =
        t * (0.254829592f + t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f + t * 1.061405429f))));
    const float e = __expf(-x * x);  // exp(-z^2/2)
    const float ea = 1.0f - poly * e;
    const float phi_c = 0.5f * (1.0f + (z < 0.0f ? -ea : ea));
    g = z * phi_c;
    gd = phi_c + z * e * 0.39894228040143268f;
}
__device__ __forceinline__ float gelu(float z)
{
    float g, gd;
    gelu_both(z, g, gd);
    return g;
}
__device__ __forceinline__ float gelu_d(float z)
{
    float g, gd;
    gelu_both(z, g, gd);
    return gd;
}

// ------------------------------------------------------------------ features
// Frame: origin TX, scale 1/L with L = |RX - TX|.  Per interaction slot k:
// one-hot type, then the object in the frame - plane: n, (d - n.TX)/L;
// straight edge: e, the edge point nearest TX; quadric: anchor, L A, b;
// circle: centre, normal, R/L - then a present bit.  Unused slots are zero.
// Frame of row i: its receiver and the scale L = |RX - TX| (1 when RX is
// missing or coincides with TX).
__device__ __forceinline__ double row_frame(const SceneDev &s, const BatchDev &b, int i, double rx[3])
{
    const int ri = b.rx_index[i];
    const bool ok_rx = ri >= 0 && ri < b.n_rx;
    for (int c = 0; c < 3; c++) rx[c] = ok_rx ? b.rx[3 * (size_t)ri + c] : 0.0;
    double L = sqrt((rx[0] - s.tx[0]) * (rx[0] - s.tx[0]) + (rx[1] - s.tx[1]) * (rx[1] - s.tx[1]) +
                    (rx[2] - s.tx[2]) * (rx[2] - s.tx[2]));
    if (!(L > 0.0) || !isfinite(L)) L = 1.0;
    return L;
}

// The SLOT features of interaction k of row i (zeros beyond its order or
// for an invalid id).
__device__ __forceinline__ void slot_features(const SceneDev &s, const BatchDev &b, int i, int k, int ord, double L,
                                              float f[SLOT])
{
#pragma unroll
    for (int j = 0; j < SLOT; j++) f[j] = 0.0f;
    if (k >= ord) return;
    const int id = b.prim[(size_t)k * b.n + i];
    if (id < 0 || id >= s.n_all) return;
    const double is = 1.0 / L;
    const int t = prim_type(id, s.n_pl, s.n_pl_ln, s.n_pl_ln_q);
    const double *q = s.rec64 + (size_t)id * kRec;
    float p[12];
#pragma unroll
    for (int j = 0; j < 12; j++) p[j] = 0.0f;
    if (t == TP) {
        for (int c = 0; c < 3; c++) p[c] = (float)q[c];
        p[3] = (float)((q[3] - (q[0] * s.tx[0] + q[1] * s.tx[1] + q[2] * s.tx[2])) * is);
    } else if (t == TL) {
        const double w = (s.tx[0] - q[0]) * q[3] + (s.tx[1] - q[1]) * q[4] + (s.tx[2] - q[2]) * q[5];
        for (int c = 0; c < 3; c++) {
            p[c] = (float)q[3 + c];
            p[3 + c] = (float)((q[c] + w * q[3 + c] - s.tx[c]) * is);
        }
    } else if (t == TQ) {
        for (int c = 0; c < 3; c++) p[c] = (float)((q[c] - s.tx[c]) * is);
        for (int c = 0; c < 6; c++) p[3 + c] = (float)(q[3 + c] * L);
        for (int c = 0; c < 3; c++) p[9 + c] = (float)q[9 + c];
    } else {
        for (int c = 0; c < 3; c++) {
            p[c] = (float)((q[c] - s.tx[c]) * is);
            p[3 + c] = (float)q[3 + c];
        }
        p[6] = (float)(q[6] * is);
    }
#pragma unroll
    for (int tt = 0; tt < 4; tt++) f[tt] = (t == tt) ? 1.0f : 0.0f;
#pragma unroll
    for (int j = 0; j < 12; j++) f[4 + j] = p[j];
    f[16] = 1.0f;
}

// Frame: origin TX, scale 1/L with L = |RX - TX|.  Per interaction slot k:
// one-hot type, then the object in the frame - plane: n, (d - n.TX)/L;
// straight edge: e, the edge point nearest TX; quadric: anchor, L A, b;
// circle: centre, normal, R/L - then a present bit.  Unused slots are zero.
__device__ __forceinline__ void row_features(const SceneDev &s, const BatchDev &b, int i, float f[F_IN], double &Lout)
{
#pragma unroll
    for (int j = 0; j < F_IN; j++) f[j] = 0.0f;
    const int ord = b.order[i];
    double rx[3];
    const double L = row_frame(s, b, i, rx);
    Lout = L;
    const double is = 1.0 / L;
    for (int c = 0; c < 3; c++) f[c] = (float)((rx[c] - s.tx[c]) * is);
#pragma unroll
    for (int k = 0; k < kMaxN; k++) {
        float g[SLOT];
        slot_features(s, b, i, k, ord, L, g);
#pragma unroll
        for (int j = 0; j < SLOT; j++) f[6 + SLOT * k + j] = g[j];
    }
}

__global__ void k_features(SceneDev s, BatchDev b, const int *__restrict__ rows, int nrows, float *__restrict__ fout,
                           bf16 *__restrict__ xout)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    const int i = rows ? rows[r] : r;
    float f[F_IN];
    double L;
    row_features(s, b, i, f, L);
#pragma unroll
    for (int j = 0; j < F_IN; j++) {
        const bf16 h = f2bf(f[j]);
        if (xout) xout[(size_t)r * F_IN + j] = h;
        if (fout) fout[(size_t)r * F_IN + j] = f[j];
    }
}

// ------------------------------------------------------------------ GEMM
// C[M x N] = A[M x K] B[K x N], BF16 operands, FP32 accumulation.
// A(m,k) = AT ? A[k*lda + m] : A[m*lda + k];  B(k,n) = BT ? B[n*ldb + k] : B[k*ldb + n].
// Block tile 64 x 64 x 32 staged in LDS; 4 waves, each one 32 x 32 MFMA tile.
// blockIdx.z splits K into chunks of kps (multiple of 32).
enum : int { EPI_BIAS_GELU = 0, EPI_BIAS = 1, EPI_DGELU = 2, EPI_F32 = 3 };

struct Epi {
    const float *bias;   // [N]
    float *zout;         // [M][ldc] pre-activation (EPI_BIAS_GELU, optional)
    bf16 *hout;          // [M][ldc] bf16 output (EPI_BIAS_GELU, EPI_DGELU)
    float *fout;         // [splits][M][ldc] fp32 output (EPI_BIAS, EPI_F32)
    const float *zin;    // [M][ldc] pre-activation to differentiate (EPI_DGELU)
    int ldc;
};

typedef float float16_t __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

constexpr int GT = 64, GK = 32, GPAD = 8;

template <bool AT, bool BT, int EPI>
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, const bf16 *__restrict__ A, int lda,
                                               const bf16 *__restrict__ B, int ldb, Epi e, int kps)
{
    __shared__ __align__(16) bf16 As[GT][GK + GPAD];
    __shared__ __align__(16) bf16 Bs[GT][GK + GPAD];  // [n][k]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int m0 = blockIdx.x * GT, n0 = blockIdx.y * GT;
    const int kb = blockIdx.z * kps, ke = min(K, kb + kps);
    const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
    float16_t acc;
#pragma unroll
    for (int v = 0; v < 16; v++) acc[v] = 0.0f;
    for (int k0 = kb; k0 < ke; k0 += GK) {
        // stage A: 64 x 32 (8 elements per thread)
#pragma unroll
        for (int j = 0; j < 8; j++) {
            int mm, kk;
            if (!AT) { mm = tid >> 2; kk = (tid & 3) * 8 + j; }
            else { kk = tid >> 3; mm = (tid & 7) * 8 + j; }
            const int gm = m0 + mm, gk = k0 + kk;
            bf16 v = 0;
            if (gm < M && gk < ke) v = AT ? A[(size_t)gk * lda + gm] : A[(size_t)gm * lda + gk];
            As[mm][kk] = v;
        }
#pragma unroll
        for (int j = 0; j < 8; j++) {
            int nn, kk;
            if (BT) { nn = tid >> 2; kk = (tid & 3) * 8 + j; }
            else { kk = tid >> 3; nn = (tid & 7) * 8 + j; }
            const int gn = n0 + nn, gk = k0 + kk;
            bf16 v = 0;
            if (gn < N && gk < ke) v = BT ? B[(size_t)gn * ldb + gk] : B[(size_t)gk * ldb + gn];
            Bs[nn][kk] = v;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < GK; ks += 16) {
            // A(i,k): lane = i + 32 (k / 8), element k % 8; B(k,j): lane = j + 32 (k / 8)
            const int kk = ks + 8 * (lane >> 5);
            const bf16x8_t a = *reinterpret_cast<const bf16x8_t *>(&As[wm + (lane & 31)][kk]);
            const bf16x8_t bb = *reinterpret_cast<const bf16x8_t *>(&Bs[wn + (lane & 31)][kk]);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bb, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    // D(i,j): lane = j + 32 ((i / 4) % 2), register (i % 4) + 4 (i / 8)
#pragma unroll
    for (int v = 0; v < 16; v++) {
        const int row = m0 + wm + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
        const int col = n0 + wn + (lane & 31);
        if (row >= M || col >= N) continue;
        const float x = acc[v];
        const size_t o = (size_t)row * e.ldc + col;
        if (EPI == EPI_BIAS_GELU) {
            const float z = x + e.bias[col];
            if (e.zout) e.zout[o] = z;
            e.hout[o] = f2bf(gelu(z));
        } else if (EPI == EPI_BIAS) {
            e.fout[o] = x + e.bias[col];
        } else if (EPI == EPI_DGELU) {
            e.hout[o] = f2bf(x * gelu_d(e.zin[o]));
        } else {
            e.fout[(size_t)blockIdx.z * M * e.ldc + o] = x;
        }
    }
}

// out[i] = sum over splits of part[s][i] (fixed order: deterministic)
__global__ void k_reduce_splits(const float *__restrict__ part, int splits, size_t n, float *__restrict__ out)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.0f;
    for (int q = 0; q < splits; q++) s += part[(size_t)q * n + i];
    out[i] = s;
}

// column sums of a [M][N] bf16 matrix (bias gradients), one block per column
__global__ void k_colsum(const bf16 *__restrict__ X, int M, int N, int ld, float *__restrict__ out)
{
    __shared__ float red[256];
    const int col = blockIdx.x;
    float s = 0.0f;
    for (int r = threadIdx.x; r < M; r += blockDim.x) s += bf2f(X[(size_t)r * ld + col]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) red[threadIdx.x] += red[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[col] = red[0];
}

// ------------------------------------------------------------------ FP32 check mode
// The same network in FP32 throughout (FP32 weights, features and
// activations, the erf GELU above, FP32 accumulation on the vector ALUs):
// a check of the backward pass's algebra without BF16 rounding.  Same
// operand conventions and epilogues as k_gemm, 64 x 64 block tiles, each
// thread 4 x 4 outputs, 16-deep K tiles in LDS.
struct EpiF {
    const float *bias;
    float *zout, *hout, *fout;
    const float *zin;
    int ldc;
};

template <bool AT, bool BT, int EPI>
__global__ void __launch_bounds__(256) k_gemm_f32(int M, int N, int K, const float *__restrict__ A, int lda,
                                                   const float *__restrict__ B, int ldb, EpiF e, int kps)
{
    __shared__ float As[16][64 + 1];  // [k][m]
    __shared__ float Bs[16][64 + 1];  // [k][n]
    const int tid = threadIdx.x, tm = tid & 15, tn = tid >> 4;
    const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
    const int kb = blockIdx.z * kps, ke = min(K, kb + kps);
    float acc[4][4] = {};
    for (int k0 = kb; k0 < ke; k0 += 16) {
        for (int q = tid; q < 16 * 64; q += 256) {
            const int kk = q >> 6, mm = q & 63, gk = k0 + kk;
            const int gm = m0 + mm, gn = n0 + mm;
            As[kk][mm] = (gm < M && gk < ke) ? (AT ? A[(size_t)gk * lda + gm] : A[(size_t)gm * lda + gk]) : 0.0f;
            Bs[kk][mm] = (gn < N && gk < ke) ? (BT ? B[(size_t)gn * ldb + gk] : B[(size_t)gk * ldb + gn]) : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; kk++)
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int j = 0; j < 4; j++) acc[i][j] = fmaf(As[kk][tm + 16 * i], Bs[kk][tn + 16 * j], acc[i][j]);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int row = m0 + tm + 16 * i, col = n0 + tn + 16 * j;
            if (row >= M || col >= N) continue;
            const float x = acc[i][j];
            const size_t o = (size_t)row * e.ldc + col;
            if (EPI == EPI_BIAS_GELU) {
                const float z = x + e.bias[col];
                e.zout[o] = z;
                e.hout[o] = gelu(z);
            } else if (EPI == EPI_BIAS) {
                e.fout[o] = x + e.bias[col];
            } else if (EPI == EPI_DGELU) {
                e.hout[o] = x * gelu_d(e.zin[o]);
            } else {
                e.fout[(size_t)blockIdx.z * M * e.ldc + o] = x;
            }
        }
}

__global__ void k_colsum_f32(const float *__restrict__ X, int M, int N, int ld, float *__restrict__ out)
{
    __shared__ float red[256];
    const int col = blockIdx.x;
    float s = 0.0f;
    for (int r = threadIdx.x; r < M; r += blockDim.x) s += X[(size_t)r * ld + col];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) red[threadIdx.x] += red[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[col] = red[0];
}

// ------------------------------------------------------------------ loss
// Masked mean squared error between the network's points Y (frame units) and
// the targets, over the coordinates of the first `order` points of the rows
// whose use flag is set.  dY = d loss / d Y (bf16, [nrows][16]).
__global__ void k_loss_partial(SceneDev s, BatchDev b, const int *__restrict__ rows, int nrows,
                               const float *__restrict__ Y, const double *__restrict__ target,
                               const uint8_t *__restrict__ use, float *__restrict__ diff, float *__restrict__ part,
                               int *__restrict__ cnt_part)
{
    __shared__ float red[256];
    __shared__ int redc[256];
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    float sum = 0.0f;
    int cnt = 0;
    if (r < nrows) {
        const int i = rows ? rows[r] : r;
        const int ord = b.order[i];
        const bool u = (!use || use[i]) && ord >= 1 && ord <= kMaxN;
        const int ri = b.rx_index[i];
        double L = 1.0;
        if (ri >= 0 && ri < b.n_rx) {
            double d2 = 0.0;
            for (int c = 0; c < 3; c++) {
                const double d = b.rx[3 * (size_t)ri + c] - s.tx[c];
                d2 += d * d;
            }
            if (d2 > 0.0 && isfinite(d2)) L = sqrt(d2);
        }
        for (int j = 0; j < F_OUTP; j++) {
            float dd = 0.0f;
            if (u && j < 3 * ord) {
                const double t = (target[(size_t)i * kRow + j] - s.tx[j % 3]) / L;
                dd = Y[(size_t)r * F_OUTP + j] - (float)t;
                if (!isfinite(dd)) dd = 0.0f;
                sum += dd * dd;
                cnt++;
            }
            diff[(size_t)r * F_OUTP + j] = dd;
        }
    }
    red[threadIdx.x] = sum;
    redc[threadIdx.x] = cnt;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) {
            red[threadIdx.x] += red[threadIdx.x + d];
            redc[threadIdx.x] += redc[threadIdx.x + d];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = red[0];
        cnt_part[blockIdx.x] = redc[0];
    }
}

// total loss and dY = 2 diff / count (bf16)
__global__ void k_loss_final(const float *__restrict__ part, const int *__restrict__ cnt_part, int nblk,
                             const float *__restrict__ diff, int nrows, bf16 *__restrict__ dY, float *__restrict__ loss,
                             float *__restrict__ dYf = nullptr)
{
    __shared__ float tot_s;
    __shared__ int tot_c;
    if (threadIdx.x == 0) {
        float t = 0.0f;
        int c = 0;
        for (int q = 0; q < nblk; q++) t += part[q], c += cnt_part[q];
        tot_s = t;
        tot_c = c;
        if (loss && blockIdx.x == 0) *loss = c ? t / c : 0.0f;
    }
    __syncthreads();
    // every block sums the few partials itself and scales its own slice
    const float sc = tot_c ? 2.0f / tot_c : 0.0f;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nrows * F_OUTP; i += gridDim.x * blockDim.x) {
        if (dY) dY[i] = f2bf(sc * diff[i]);
        if (dYf) dYf[i] = sc * diff[i];
    }
}

// ------------------------------------------------------------------ Adam
__global__ void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, bf16 *__restrict__ wb, bf16 *__restrict__ wf, int n, float lr,
                       float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wb) {
        const bf16 h = f2bf(wi);
        wb[i] = h;
        const long long j = frag_of((size_t)i);
        if (j >= 0) wf[j] = h;
    }
}

__global__ void k_to_bf16(const float *__restrict__ w, bf16 *__restrict__ wb, bf16 *__restrict__ wf, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bf16 h = f2bf(w[i]);
    wb[i] = h;
    const long long j = frag_of((size_t)i);
    if (j >= 0) wf[j] = h;
}

// ------------------------------------------------------------------ decode
// World points X_k = TX + L Y_k for the first `order` points (zero beyond).
__global__ void k_decode(SceneDev s, BatchDev b, int nrows, const float *__restrict__ Y, double *__restrict__ x)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    const int ord = b.order[i];
    const int ri = b.rx_index[i];
    double L = 1.0;
    if (ri >= 0 && ri < b.n_rx) {
        double d2 = 0.0;
        for (int c = 0; c < 3; c++) {
            const double d = b.rx[3 * (size_t)ri + c] - s.tx[c];
            d2 += d * d;
        }
        if (d2 > 0.0 && isfinite(d2)) L = sqrt(d2);
    }
    for (int j = 0; j < kRow; j++)
        x[(size_t)i * kRow + j] = (j < 3 * ord) ? s.tx[j % 3] + L * (double)Y[(size_t)i * F_OUTP + j] : 0.0;
}

// ------------------------------------------------------------------ fused inference
// One block = 64 paths and 4 waves: features -> three hidden layers ->
// output layer -> world points, activations in LDS (two buffers of
// 64 x 264 BF16, 76 KB with the GELU table), so two blocks share a CU and
// one block's feature gathers overlap the other's matrix work (128 paths
// and 8 waves in one block per CU took 7% longer).  Every layer is computed
// transposed, H^T = W X^T: the weights are the matrix cores' A operand
// (rows = output units), read from L2 as whole 1 KB fragments of the
// fragment-ordered copy a few steps ahead of the matrix cores (one row per
// lane, as the [out][in] matrix gives, made the layers a third slower), and
// the activations the B operand (8 consecutive BF16 of one path from LDS),
// so the accumulator holds 4 consecutive output units of one path per
// register group and the epilogue writes them to LDS with one 8-byte store.
// Wave w takes output units 64 (w % 4) .. +64 of paths 64 (w / 4) .. +64:
// 2 x 2 tiles of v_mfma_f32_32x32x16_bf16.  With two waves per SIMD one
// wave's matrix work overlaps the other's epilogue.
//
// GELU(z) = z Phi(z) with Phi read from a table in LDS: 1024 steps of 1/64
// on [-8, 8] (Phi and its forward difference; linear interpolation, error
// below 1e-5, under a tenth of a BF16 step; clamped ends give Phi = 0 and
// 1 to FP32 precision).  The table entries are Phi = erfc(-z/sqrt 2)/2 in
// FP32.
constexpr int IR = 64;                  // paths per block
// weight fragment steps loaded ahead of the matrix cores (1 and 2 ran 7%
// and 2% longer, 6 no faster, 8 leaves one wave per SIMD)
constexpr int PF = 4;
constexpr int ILD = HID + 8;            // LDS row stride in BF16 (132 dwords)
constexpr int TABN = 1024;
constexpr size_t OW1_ = 0, OB1_ = OW1_ + (size_t)HID * F_IN, OW2_ = OB1_ + HID, OB2_ = OW2_ + (size_t)HID * HID,
                 OW3_ = OB2_ + HID, OB3_ = OW3_ + (size_t)HID * HID, OW4_ = OB3_ + HID,
                 OB4_ = OW4_ + (size_t)F_OUTP * HID;
constexpr size_t INFER_LDS = (size_t)2 * IR * ILD * sizeof(bf16) + TABN * sizeof(float2) + IR * sizeof(double) +
                             IR * sizeof(int);

__device__ __forceinline__ float gelu_tab(const float2 *tab, float z)
{
    // u = 64 (z + 8), clamped to the table
    const float u = __builtin_amdgcn_fmed3f(fmaf(z, 64.0f, 512.0f), 0.0f, (float)TABN - 0.0009765625f);
    const int i = (int)u;
    const float f = u - (float)i;
    const float2 t = tab[i];
    return z * fmaf(t.y, f, t.x);
}

// out[path][unit] = GELU(in[path][0..K) W[unit]^T + bias[unit]) for this
// wave's 64 units and 64 paths; the next 16-deep weight fragments are
// loaded while the four MFMAs of the current ones run.
template <int K>
__device__ __forceinline__ void infer_layer(const bf16 *in, bf16 *out, const bf16 *__restrict__ Wf,
                                            const float *__restrict__ bias, const float2 *tab, int wave, int lane)
{
    static_assert(K % 16 == 0, "K must be a multiple of 16");
    const int u0 = 64 * (wave & 3), r0 = 64 * (wave >> 2);
    const int li = lane & 31, kq = 8 * (lane >> 5);
    float16_t acc[2][2];
#pragma unroll
    for (int mt = 0; mt < 2; mt++)
#pragma unroll
        for (int nt = 0; nt < 2; nt++)
#pragma unroll
            for (int v = 0; v < 16; v++) acc[mt][nt][v] = 0.0f;
    // this wave's fragments: unit block wave % 4, step t, half h at
    // wf[(2 t + h) 64]; each is read from L2 once per tile, so the loads run
    // PF steps ahead of the matrix cores (a ring of PF fragment pairs)
    constexpr int S = K / 16, D = PF < S ? PF : S;
    // the block offset is wave-uniform (scalar base), the lane offset the
    // only per-lane part of the address
    const int blk = __builtin_amdgcn_readfirstlane(wave & 3);
    const bf16x8_t *wf = reinterpret_cast<const bf16x8_t *>(Wf) + (size_t)blk * S * 2 * 64 + lane;
    const bf16 *ip0 = in + (r0 + li) * ILD + kq, *ip1 = in + (r0 + 32 + li) * ILD + kq;
    bf16x8_t a0[D], a1[D];
#pragma unroll
    for (int t = 0; t < D; t++) {
        a0[t] = wf[t * 128];
        a1[t] = wf[t * 128 + 64];
    }
#pragma unroll
    for (int t = 0; t < S; t++) {
        const bf16x8_t x0 = a0[t % D], x1 = a1[t % D];
        if (t + D < S) {
            a0[t % D] = wf[(t + D) * 128];
            a1[t % D] = wf[(t + D) * 128 + 64];
        }
        const bf16x8_t b0 = *reinterpret_cast<const bf16x8_t *>(ip0 + 16 * t);
        const bf16x8_t b1 = *reinterpret_cast<const bf16x8_t *>(ip1 + 16 * t);
        acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x1, b1, acc[1][1], 0, 0, 0);
        // keep each step's loads in their step: the scheduler would otherwise
        // issue all of a layer's fragment loads at once (128 VGPRs)
        __builtin_amdgcn_sched_barrier(0);
    }
    // D(i, j): unit i = 8 (v / 4) + 4 (lane / 32) + v % 4 of the tile, path j = lane % 32
#pragma unroll
    for (int mt = 0; mt < 2; mt++)
#pragma unroll
        for (int g = 0; g < 4; g++) {
            const int u = u0 + 32 * mt + 8 * g + 4 * (lane >> 5);
            const float4 bc = *reinterpret_cast<const float4 *>(bias + u);
#pragma unroll
            for (int nt = 0; nt < 2; nt++) {
                const float h0 = gelu_tab(tab, acc[mt][nt][4 * g + 0] + bc.x);
                const float h1 = gelu_tab(tab, acc[mt][nt][4 * g + 1] + bc.y);
                const float h2 = gelu_tab(tab, acc[mt][nt][4 * g + 2] + bc.z);
                const float h3 = gelu_tab(tab, acc[mt][nt][4 * g + 3] + bc.w);
                uint2 pk;
                pk.x = (uint32_t)f2bf(h0) | ((uint32_t)f2bf(h1) << 16);
                pk.y = (uint32_t)f2bf(h2) | ((uint32_t)f2bf(h3) << 16);
                *reinterpret_cast<uint2 *>(out + (r0 + 32 * nt + li) * ILD + u) = pk;
            }
        }
}

// rows (may be null): solve ids to predict, *count of them; else all b.n
__global__ void __launch_bounds__(256) k_mlp_fused(SceneDev s, BatchDev b, const int *__restrict__ rows,
                                                       const int *__restrict__ count, const bf16 *__restrict__ wb,
                                                       const bf16 *wf, const float *__restrict__ w,
                                                       double *__restrict__ x)
{
    extern __shared__ __align__(16) unsigned char smem[];
    bf16 *bufA = reinterpret_cast<bf16 *>(smem);
    bf16 *bufB = bufA + IR * ILD;
    float2 *tab = reinterpret_cast<float2 *>(bufB + IR * ILD);
    double *Ls = reinterpret_cast<double *>(tab + TABN);
    int *ids = reinterpret_cast<int *>(Ls + IR);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nrows = rows ? *count : (int)b.n;
    if ((int)blockIdx.x * IR >= nrows) return;  // block-uniform
    for (int i = tid; i < TABN; i += blockDim.x) {
        const float z0 = -8.0f + (float)i * (1.0f / 64.0f), z1 = z0 + (1.0f / 64.0f);
        const float p0 = 0.5f * erfcf(-z0 * 0.70710678118654752f), p1 = 0.5f * erfcf(-z1 * 0.70710678118654752f);
        tab[i] = make_float2(p0, p1 - p0);
    }
    // persistent: the block walks the 128-path tiles
    for (int row0 = blockIdx.x * IR; row0 < nrows; row0 += gridDim.x * IR) {
    {
        // features, four threads per path: thread q of a path writes slot q
        // (and thread 0 the receiver, slot 4 and the zero padding)
        const int pr = tid >> 2, q = tid & 3;
        const int r = row0 + pr;
        const int i = (r < nrows) ? (rows ? rows[r] : r) : -1;
        bf16 *dst = bufA + pr * ILD;
        double rx[3] = {0.0, 0.0, 0.0};
        const double L = (i >= 0) ? row_frame(s, b, i, rx) : 1.0;
        const int ord = (i >= 0) ? b.order[i] : 0;
        float g[SLOT];
        slot_features(s, b, i < 0 ? 0 : i, q, i < 0 ? 0 : ord, L, g);
        for (int j = 0; j < SLOT; j++) dst[6 + SLOT * q + j] = f2bf(g[j]);
        if (q == 0) {
            const double is = 1.0 / L;
            for (int c = 0; c < 3; c++) {
                dst[c] = f2bf(i >= 0 ? (float)((rx[c] - s.tx[c]) * is) : 0.0f);
                dst[3 + c] = f2bf(0.0f);
            }
            slot_features(s, b, i < 0 ? 0 : i, 4, i < 0 ? 0 : ord, L, g);
            for (int j = 0; j < SLOT; j++) dst[6 + SLOT * 4 + j] = f2bf(g[j]);
            for (int j = 6 + SLOT * kMaxN; j < F_IN; j++) dst[j] = f2bf(0.0f);
            Ls[pr] = L;
            ids[pr] = i;
        }
    }
    __syncthreads();
    infer_layer<F_IN>(bufA, bufB, wf, w + OB1_, tab, wave, lane);
    __syncthreads();
    infer_layer<HID>(bufB, bufA, wf + (size_t)HID * F_IN, w + OB2_, tab, wave, lane);
    __syncthreads();
    infer_layer<HID>(bufA, bufB, wf + (size_t)HID * F_IN + (size_t)HID * HID, w + OB3_, tab, wave, lane);
    __syncthreads();
    // output layer, transposed as well: units 0..15 (lanes 16..31 of the A
    // operand carry zero rows), waves 0 and 1 take 32 paths each
    if (wave < IR / 32) {
        float16_t acc;
#pragma unroll
        for (int v = 0; v < 16; v++) acc[v] = 0.0f;
        const int li = lane & 31, kq = 8 * (lane >> 5);
        const bf16 *wp = wb + OW4_ + (size_t)(li & 15) * HID + kq;
        const bf16 *ip = bufB + (32 * wave + li) * ILD + kq;
#pragma unroll 4
        for (int k0 = 0; k0 < HID; k0 += 16) {
            bf16x8_t a = *reinterpret_cast<const bf16x8_t *>(wp + k0);
            if (li >= F_OUTP) a = bf16x8_t{};
            const bf16x8_t bb = *reinterpret_cast<const bf16x8_t *>(ip + k0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bb, acc, 0, 0, 0);
        }
        const int r = 32 * wave + li;
        const int i = ids[r];
        if (i >= 0) {
            const int ord = b.order[i];
#pragma unroll
            for (int v = 0; v < 8; v++) {
                const int u = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                x[(size_t)i * kRow + u] = (u < 3 * ord) ? s.tx[u % 3] + Ls[r] * (double)(acc[v] + w[OB4_ + u]) : 0.0;
            }
        }
    }
    __syncthreads();  // the next tile's features overwrite bufA, ids and Ls
    }
}

// ------------------------------------------------------------------ state
// Parameter layout (FP32 master, one flat array): W1 [256][96], b1 [256],
// W2 [256][256], b2, W3 [256][256], b3, W4 [16][256] (row 15 unused, kept
// zero), b4 [16].  Weights are [out][in].
constexpr size_t OW1 = 0, OB1 = OW1 + (size_t)HID * F_IN, OW2 = OB1 + HID, OB2 = OW2 + (size_t)HID * HID,
                 OW3 = OB2 + HID, OB3 = OW3 + (size_t)HID * HID, OW4 = OB3 + HID, OB4 = OW4 + (size_t)F_OUTP * HID,
                 NPAR = OB4 + F_OUTP;

struct MlpState {
    float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
    bf16 *wb = nullptr;  // bf16 copy of the weights (same layout)
    bf16 *wf = nullptr;  // the hidden layers' bf16 weights in fragment order
    int64_t step = 0;
    uint64_t seed = 0;
    // activation workspace for up to cap rows
    size_t cap = 0;
    bf16 *X = nullptr, *H1 = nullptr, *H2 = nullptr, *H3 = nullptr, *dY = nullptr, *dA = nullptr, *dB = nullptr;
    float *Z1 = nullptr, *Z2 = nullptr, *Z3 = nullptr, *Y = nullptr, *diff = nullptr, *part = nullptr,
          *lpart = nullptr;
    int *lcnt = nullptr;
    size_t part_cap = 0;
    // FP32 check mode: features, activations and backward buffers in FP32
    size_t fcap = 0;
    float *Xf = nullptr, *H1f = nullptr, *H2f = nullptr, *H3f = nullptr, *dYf = nullptr, *dAf = nullptr,
          *dBf = nullptr;
};

bool mlp_ready(const MlpState *m) { return m != nullptr && m->w != nullptr; }

static void free_ws(MlpState *m)
{
    for (void *p : {(void *)m->X, (void *)m->H1, (void *)m->H2, (void *)m->H3, (void *)m->dY, (void *)m->dA,
                    (void *)m->dB, (void *)m->Z1, (void *)m->Z2, (void *)m->Z3, (void *)m->Y, (void *)m->diff,
                    (void *)m->lpart, (void *)m->lcnt})
        if (p) hipFree(p);
    m->X = m->H1 = m->H2 = m->H3 = m->dY = m->dA = m->dB = nullptr;
    m->Z1 = m->Z2 = m->Z3 = m->Y = m->diff = m->lpart = nullptr;
    m->lcnt = nullptr;
    m->cap = 0;
}

static void free_f32(MlpState *m)
{
    for (void *p : {(void *)m->Xf, (void *)m->H1f, (void *)m->H2f, (void *)m->H3f, (void *)m->dYf, (void *)m->dAf,
                    (void *)m->dBf})
        if (p) hipFree(p);
    m->Xf = m->H1f = m->H2f = m->H3f = m->dYf = m->dAf = m->dBf = nullptr;
    m->fcap = 0;
}

void mlp_free(MlpState *m)
{
    if (!m) return;
    free_ws(m);
    free_f32(m);
    hipFree(m->w);
    hipFree(m->m);
    hipFree(m->v);
    hipFree(m->g);
    hipFree(m->wb);
    hipFree(m->wf);
    hipFree(m->part);
    delete m;
}

static mpt_status ensure_ws(MlpState *m, size_t rows, bool train)
{
    if (rows <= m->cap && (!train || m->dY)) return MPT_OK;
    free_ws(m);
    size_t cap = rows < 1024 ? 1024 : rows;
    bool ok = true;
    auto A = [&](void **p, size_t bytes) { ok = ok && hipMalloc(p, bytes) == hipSuccess; };
    A((void **)&m->X, cap * F_IN * sizeof(bf16));
    A((void **)&m->H1, cap * HID * sizeof(bf16));
    A((void **)&m->H2, cap * HID * sizeof(bf16));
    A((void **)&m->H3, cap * HID * sizeof(bf16));
    A((void **)&m->Y, cap * F_OUTP * sizeof(float));
    if (train) {
        A((void **)&m->Z1, cap * HID * sizeof(float));
        A((void **)&m->Z2, cap * HID * sizeof(float));
        A((void **)&m->Z3, cap * HID * sizeof(float));
        A((void **)&m->dY, cap * F_OUTP * sizeof(bf16));
        A((void **)&m->dA, cap * HID * sizeof(bf16));
        A((void **)&m->dB, cap * HID * sizeof(bf16));
        A((void **)&m->diff, cap * F_OUTP * sizeof(float));
        A((void **)&m->lpart, ((cap + 255) / 256) * sizeof(float));
        A((void **)&m->lcnt, ((cap + 255) / 256) * sizeof(int));
    }
    if (!ok) {
        free_ws(m);
        return MPT_E_NOMEM;
    }
    m->cap = cap;
    return MPT_OK;
}

// host-side seeded initialisation (SplitMix64 -> uniform), Kaiming-uniform
// style bounds sqrt(6 / fan_in) for weights, zero biases
static uint64_t splitmix(uint64_t &x)
{
    uint64_t z = (x += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

static void init_host(std::vector<float> &w, uint64_t seed)
{
    w.assign(NPAR, 0.0f);
    uint64_t st = seed;
    auto uni = [&]() { return (float)((splitmix(st) >> 11) * (1.0 / 9007199254740992.0)) * 2.0f - 1.0f; };
    auto fill = [&](size_t off, int rows, int cols, int valid_rows) {
        const float bound = sqrtf(6.0f / (float)cols);
        for (int r = 0; r < rows; r++)
            for (int c = 0; c < cols; c++) w[off + (size_t)r * cols + c] = (r < valid_rows) ? bound * uni() : 0.0f;
    };
    fill(OW1, HID, F_IN, HID);
    fill(OW2, HID, HID, HID);
    fill(OW3, HID, HID, HID);
    fill(OW4, F_OUTP, HID, F_OUT);
    // the last layer starts small so that the first predictions sit near the
    // origin of the frame
    for (size_t i = OW4; i < OB4; i++) w[i] *= 0.1f;
}

static mpt_status alloc_params(MlpState *m)
{
    bool ok = hipMalloc((void **)&m->w, NPAR * 4) == hipSuccess && hipMalloc((void **)&m->m, NPAR * 4) == hipSuccess &&
              hipMalloc((void **)&m->v, NPAR * 4) == hipSuccess && hipMalloc((void **)&m->g, NPAR * 4) == hipSuccess &&
              hipMalloc((void **)&m->wb, NPAR * 2) == hipSuccess && hipMalloc((void **)&m->wf, NFRAG * 2) == hipSuccess;
    return ok ? MPT_OK : MPT_E_NOMEM;
}

mpt_status mlp_init(MlpState **pm, uint64_t seed, hipStream_t st)
{
    if (!*pm) *pm = new MlpState();
    MlpState *m = *pm;
    if (!m->w && alloc_params(m)) return MPT_E_NOMEM;
    std::vector<float> h;
    init_host(h, seed);
    std::vector<float> z(NPAR, 0.0f);
    if (hipMemcpyAsync(m->w, h.data(), NPAR * 4, hipMemcpyHostToDevice, st) != hipSuccess) return MPT_E_DEVICE;
    if (hipMemcpyAsync(m->m, z.data(), NPAR * 4, hipMemcpyHostToDevice, st) != hipSuccess) return MPT_E_DEVICE;
    if (hipMemcpyAsync(m->v, z.data(), NPAR * 4, hipMemcpyHostToDevice, st) != hipSuccess) return MPT_E_DEVICE;
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((NPAR + 255) / 256)), dim3(256), 0, st, m->w, m->wb, m->wf, (int)NPAR);
    if (hipStreamSynchronize(st) != hipSuccess) return MPT_E_DEVICE;
    m->step = 0;
    m->seed = seed;
    return MPT_OK;
}

// ------------------------------------------------------------------ launch helpers
template <bool AT, bool BT, int EPI>
static void gemm(int M, int N, int K, const bf16 *A, int lda, const bf16 *B, int ldb, const Epi &e, int splits,
                 hipStream_t st)
{
    int kps = (K + splits - 1) / splits;
    kps = ((kps + GK - 1) / GK) * GK;
    splits = (K + kps - 1) / kps;
    dim3 grid((M + GT - 1) / GT, (N + GT - 1) / GT, splits);
    hipLaunchKernelGGL((k_gemm<AT, BT, EPI>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, e, kps);
}

// forward over `nrows` rows already featurised in m->X; with train, keep Z
static void forward(MlpState *m, int nrows, bool train, hipStream_t st)
{
    Epi e{};
    e.ldc = HID;
    e.bias = m->w + OB1;
    e.zout = train ? m->Z1 : nullptr;
    e.hout = m->H1;
    gemm<false, true, EPI_BIAS_GELU>(nrows, HID, F_IN, m->X, F_IN, m->wb + OW1, F_IN, e, 1, st);
    e.bias = m->w + OB2;
    e.zout = train ? m->Z2 : nullptr;
    e.hout = m->H2;
    gemm<false, true, EPI_BIAS_GELU>(nrows, HID, HID, m->H1, HID, m->wb + OW2, HID, e, 1, st);
    e.bias = m->w + OB3;
    e.zout = train ? m->Z3 : nullptr;
    e.hout = m->H3;
    gemm<false, true, EPI_BIAS_GELU>(nrows, HID, HID, m->H2, HID, m->wb + OW3, HID, e, 1, st);
    Epi e4{};
    e4.ldc = F_OUTP;
    e4.bias = m->w + OB4;
    e4.fout = m->Y;
    gemm<false, true, EPI_BIAS>(nrows, F_OUTP, HID, m->H3, HID, m->wb + OW4, HID, e4, 1, st);
}

mpt_status mlp_predict_dev(MlpState *m, const SceneDev &s, const BatchDev &b, double *x_out, hipStream_t st,
                           const int *rows, const int *count)
{
    if (!mlp_ready(m)) return MPT_E_NO_MODEL;
    if (b.n == 0) return MPT_OK;
    static_assert(OW4_ == OW4 && OB4_ == OB4, "parameter layout");
    static_assert(frag_of(OW1) == 0 && frag_of(OW2) == (long long)HID * F_IN &&
                      frag_of(OW3) == (long long)(HID * F_IN + HID * HID) && frag_of(OB3 - 1) == (long long)NFRAG - 1,
                  "fragment layout: first and last weight of each layer");
    static_assert(frag_of(OB1) < 0 && frag_of(OB2) < 0 && frag_of(OB3) < 0 && frag_of(OW4) < 0,
                  "fragment layout: biases and the output layer are not in it");
    static_assert(frag_of(OW1 + 1) == 1 && frag_of(OW1 + 8) == 32 * 8 && frag_of(OW1 + F_IN) == 8 &&
                      frag_of(OW1 + 32 * F_IN) == 64 * 8 && frag_of(OW1 + 16) == 2 * 64 * 8 &&
                      frag_of(OW1 + 64 * F_IN) == (F_IN / 16) * 2 * 64 * 8,
                  "fragment layout: element, lane, half, step and unit-block strides");
    hipFuncSetAttribute((const void *)k_mlp_fused, hipFuncAttributeMaxDynamicSharedMemorySize, (int)INFER_LDS);
    // two resident blocks per CU (the LDS holds two), each walking tiles
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t tiles = (b.n + IR - 1) / IR;
    const unsigned g = (unsigned)(tiles < 2 * cus ? tiles : 2 * cus);
    hipLaunchKernelGGL(k_mlp_fused, dim3(g), dim3(256), INFER_LDS, st, s, b, rows, count, m->wb, m->wf, m->w, x_out);
    return hipGetLastError() == hipSuccess ? MPT_OK : MPT_E_DEVICE;
}

// Unfused forward through the GEMM kernels (the path training uses), kept
// as a check of the fused kernel.
mpt_status mlp_predict_unfused(MlpState *m, const SceneDev &s, const BatchDev &b, double *x_out, hipStream_t st)
{
    if (!mlp_ready(m)) return MPT_E_NO_MODEL;
    if (b.n == 0) return MPT_OK;
    const int64_t chunk = 1 << 20;
    if (ensure_ws(m, (size_t)(b.n < chunk ? b.n : chunk), false)) return MPT_E_NOMEM;
    for (int64_t c0 = 0; c0 < b.n; c0 += chunk) {
        const int nr = (int)((b.n - c0) < chunk ? (b.n - c0) : chunk);
        // a view of the batch starting at c0 (component-major arrays keep stride n)
        BatchDev v = b;
        v.rx_index = b.rx_index + c0;
        v.order = b.order + c0;
        v.prim = b.prim + c0;
        hipLaunchKernelGGL(k_features, dim3((nr + 127) / 128), dim3(128), 0, st, s, v, nullptr, nr, nullptr, m->X);
        forward(m, nr, false, st);
        hipLaunchKernelGGL(k_decode, dim3((nr + 255) / 256), dim3(256), 0, st, s, v, nr, m->Y, x_out + c0 * kRow);
    }
    return hipGetLastError() == hipSuccess ? MPT_OK : MPT_E_DEVICE;
}

// loss, gradient into m->g (no update); rows = minibatch ids (may be null)
static mpt_status grad_dev(MlpState *m, const SceneDev &s, const BatchDev &b, const int *rows, int nrows,
                           const double *target, const uint8_t *use, float *d_loss, hipStream_t st)
{
    if (ensure_ws(m, (size_t)nrows, true)) return MPT_E_NOMEM;
    hipLaunchKernelGGL(k_features, dim3((nrows + 127) / 128), dim3(128), 0, st, s, b, rows, nrows, nullptr, m->X);
    forward(m, nrows, true, st);
    const int nblk = (nrows + 255) / 256;
    hipLaunchKernelGGL(k_loss_partial, dim3(nblk), dim3(256), 0, st, s, b, rows, nrows, m->Y, target, use, m->diff,
                       m->lpart, m->lcnt);
    hipLaunchKernelGGL(k_loss_final, dim3(std::min(256, (nrows * F_OUTP + 255) / 256)), dim3(256), 0, st, m->lpart, m->lcnt, nblk, m->diff, nrows, m->dY,
                       d_loss);
    // split-K partial buffer for the weight gradients
    const int splits = nrows >= 4096 ? 16 : (nrows >= 1024 ? 4 : 1);
    const size_t need = (size_t)splits * HID * HID;
    if (m->part_cap < need) {
        if (m->part) hipFree(m->part);
        m->part = nullptr;
        if (hipMalloc((void **)&m->part, need * 4) != hipSuccess) return MPT_E_NOMEM;
        m->part_cap = need;
    }
    auto wgrad = [&](int Mo, int Ni, const bf16 *dZ, int ldz, const bf16 *Xin, int ldx, float *gout) {
        // dW[o][i] = sum_r dZ[r][o] X[r][i]: A = dZ^T (AT), B = X (row-major)
        Epi e{};
        e.ldc = Ni;
        e.fout = m->part;
        int kps = (nrows + splits - 1) / splits;
        kps = ((kps + GK - 1) / GK) * GK;
        const int sp = (nrows + kps - 1) / kps;
        gemm<true, false, EPI_F32>(Mo, Ni, nrows, dZ, ldz, Xin, ldx, e, splits, st);
        const size_t n = (size_t)Mo * Ni;
        hipLaunchKernelGGL(k_reduce_splits, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, m->part, sp, n, gout);
    };
    // layer 4: dW4, db4, dH3 = dY W4
    wgrad(F_OUTP, HID, m->dY, F_OUTP, m->H3, HID, m->g + OW4);
    hipLaunchKernelGGL(k_colsum, dim3(F_OUTP), dim3(256), 0, st, m->dY, nrows, F_OUTP, F_OUTP, m->g + OB4);
    Epi e{};
    e.ldc = HID;
    e.zin = m->Z3;
    e.hout = m->dA;  // dZ3
    gemm<false, false, EPI_DGELU>(nrows, HID, F_OUTP, m->dY, F_OUTP, m->wb + OW4, HID, e, 1, st);
    // layer 3
    wgrad(HID, HID, m->dA, HID, m->H2, HID, m->g + OW3);
    hipLaunchKernelGGL(k_colsum, dim3(HID), dim3(256), 0, st, m->dA, nrows, HID, HID, m->g + OB3);
    e.zin = m->Z2;
    e.hout = m->dB;  // dZ2
    gemm<false, false, EPI_DGELU>(nrows, HID, HID, m->dA, HID, m->wb + OW3, HID, e, 1, st);
    // layer 2
    wgrad(HID, HID, m->dB, HID, m->H1, HID, m->g + OW2);
    hipLaunchKernelGGL(k_colsum, dim3(HID), dim3(256), 0, st, m->dB, nrows, HID, HID, m->g + OB2);
    e.zin = m->Z1;
    e.hout = m->dA;  // dZ1
    gemm<false, false, EPI_DGELU>(nrows, HID, HID, m->dB, HID, m->wb + OW2, HID, e, 1, st);
    // layer 1
    wgrad(HID, F_IN, m->dA, HID, m->X, F_IN, m->g + OW1);
    hipLaunchKernelGGL(k_colsum, dim3(HID), dim3(256), 0, st, m->dA, nrows, HID, HID, m->g + OB1);
    return hipGetLastError() == hipSuccess ? MPT_OK : MPT_E_DEVICE;
}

template <bool AT, bool BT, int EPI>
static void gemm_f32(int M, int N, int K, const float *A, int lda, const float *B, int ldb, const EpiF &e, int splits,
                     hipStream_t st)
{
    int kps = (K + splits - 1) / splits;
    kps = ((kps + 15) / 16) * 16;
    splits = (K + kps - 1) / kps;
    dim3 grid((M + 63) / 64, (N + 63) / 64, splits);
    hipLaunchKernelGGL((k_gemm_f32<AT, BT, EPI>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, e, kps);
}

// Loss and gradient of the network run in FP32 throughout (the check mode).
mpt_status mlp_grad_f32_dev(MlpState *m, const SceneDev &s, const BatchDev &b, const int *rows, int nrows,
                            const double *target, const uint8_t *use, float *d_loss, float *d_grad, hipStream_t st)
{
    if (!mlp_ready(m)) return MPT_E_NO_MODEL;
    if (nrows <= 0) return MPT_E_INVALID_ARG;
    if (ensure_ws(m, (size_t)nrows, true)) return MPT_E_NOMEM;
    if ((size_t)nrows > m->fcap) {
        free_f32(m);
        const size_t cap = m->cap;
        bool ok = true;
        auto A = [&](float **p, size_t n) { ok = ok && hipMalloc((void **)p, n * sizeof(float)) == hipSuccess; };
        A(&m->Xf, cap * F_IN);
        A(&m->H1f, cap * HID);
        A(&m->H2f, cap * HID);
        A(&m->H3f, cap * HID);
        A(&m->dYf, cap * F_OUTP);
        A(&m->dAf, cap * HID);
        A(&m->dBf, cap * HID);
        if (!ok) {
            free_f32(m);
            return MPT_E_NOMEM;
        }
        m->fcap = cap;
    }
    const float *w = m->w;
    hipLaunchKernelGGL(k_features, dim3((nrows + 127) / 128), dim3(128), 0, st, s, b, rows, nrows, m->Xf, nullptr);
    EpiF e{};
    e.ldc = HID;
    e.bias = w + OB1, e.zout = m->Z1, e.hout = m->H1f;
    gemm_f32<false, true, EPI_BIAS_GELU>(nrows, HID, F_IN, m->Xf, F_IN, w + OW1, F_IN, e, 1, st);
    e.bias = w + OB2, e.zout = m->Z2, e.hout = m->H2f;
    gemm_f32<false, true, EPI_BIAS_GELU>(nrows, HID, HID, m->H1f, HID, w + OW2, HID, e, 1, st);
    e.bias = w + OB3, e.zout = m->Z3, e.hout = m->H3f;
    gemm_f32<false, true, EPI_BIAS_GELU>(nrows, HID, HID, m->H2f, HID, w + OW3, HID, e, 1, st);
    EpiF e4{};
    e4.ldc = F_OUTP;
    e4.bias = w + OB4, e4.fout = m->Y;
    gemm_f32<false, true, EPI_BIAS>(nrows, F_OUTP, HID, m->H3f, HID, w + OW4, HID, e4, 1, st);
    const int nblk = (nrows + 255) / 256;
    hipLaunchKernelGGL(k_loss_partial, dim3(nblk), dim3(256), 0, st, s, b, rows, nrows, m->Y, target, use, m->diff,
                       m->lpart, m->lcnt);
    hipLaunchKernelGGL(k_loss_final, dim3(std::min(256, (nrows * F_OUTP + 255) / 256)), dim3(256), 0, st, m->lpart,
                       m->lcnt, nblk, m->diff, nrows, (bf16 *)nullptr, d_loss, m->dYf);
    const int splits = nrows >= 4096 ? 16 : (nrows >= 1024 ? 4 : 1);
    const size_t need = (size_t)splits * HID * HID;
    if (m->part_cap < need) {
        if (m->part) hipFree(m->part);
        m->part = nullptr;
        if (hipMalloc((void **)&m->part, need * 4) != hipSuccess) return MPT_E_NOMEM;
        m->part_cap = need;
    }
    auto wgrad = [&](int Mo, int Ni, const float *dZ, int ldz, const float *Xin, int ldx, float *gout) {
        EpiF eg{};
        eg.ldc = Ni;
        eg.fout = m->part;
        int kps = (nrows + splits - 1) / splits;
        kps = ((kps + 15) / 16) * 16;
        const int sp = (nrows + kps - 1) / kps;
        gemm_f32<true, false, EPI_F32>(Mo, Ni, nrows, dZ, ldz, Xin, ldx, eg, splits, st);
        const size_t n = (size_t)Mo * Ni;
        hipLaunchKernelGGL(k_reduce_splits, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, m->part, sp, n, gout);
    };
    wgrad(F_OUTP, HID, m->dYf, F_OUTP, m->H3f, HID, m->g + OW4);
    hipLaunchKernelGGL(k_colsum_f32, dim3(F_OUTP), dim3(256), 0, st, m->dYf, nrows, F_OUTP, F_OUTP, m->g + OB4);
    EpiF ed{};
    ed.ldc = HID;
    ed.zin = m->Z3, ed.hout = m->dAf;
    gemm_f32<false, false, EPI_DGELU>(nrows, HID, F_OUTP, m->dYf, F_OUTP, w + OW4, HID, ed, 1, st);
    wgrad(HID, HID, m->dAf, HID, m->H2f, HID, m->g + OW3);
    hipLaunchKernelGGL(k_colsum_f32, dim3(HID), dim3(256), 0, st, m->dAf, nrows, HID, HID, m->g + OB3);
    ed.zin = m->Z2, ed.hout = m->dBf;
    gemm_f32<false, false, EPI_DGELU>(nrows, HID, HID, m->dAf, HID, w + OW3, HID, ed, 1, st);
    wgrad(HID, HID, m->dBf, HID, m->H1f, HID, m->g + OW2);
    hipLaunchKernelGGL(k_colsum_f32, dim3(HID), dim3(256), 0, st, m->dBf, nrows, HID, HID, m->g + OB2);
    ed.zin = m->Z1, ed.hout = m->dAf;
    gemm_f32<false, false, EPI_DGELU>(nrows, HID, HID, m->dBf, HID, w + OW2, HID, ed, 1, st);
    wgrad(HID, F_IN, m->dAf, HID, m->Xf, F_IN, m->g + OW1);
    hipLaunchKernelGGL(k_colsum_f32, dim3(HID), dim3(256), 0, st, m->dAf, nrows, HID, HID, m->g + OB1);
    if (hipGetLastError() != hipSuccess) return MPT_E_DEVICE;
    if (d_grad && hipMemcpyAsync(d_grad, m->g, NPAR * 4, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return MPT_E_DEVICE;
    return MPT_OK;
}

mpt_status mlp_grad_dev(MlpState *m, const SceneDev &s, const BatchDev &b, const int *rows, int nrows,
                        const double *target, const uint8_t *use, float *d_loss, float *d_grad, hipStream_t st)
{
    if (!mlp_ready(m)) return MPT_E_NO_MODEL;
    if (nrows <= 0) return MPT_E_INVALID_ARG;
    mpt_status r = grad_dev(m, s, b, rows, nrows, target, use, d_loss, st);
    if (r) return r;
    if (d_grad && hipMemcpyAsync(d_grad, m->g, NPAR * 4, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return MPT_E_DEVICE;
    return MPT_OK;
}

mpt_status mlp_train_step_dev(MlpState *m, const SceneDev &s, const BatchDev &b, const int *rows, int nrows,
                              const double *target, const uint8_t *use, float lr, float *d_loss, hipStream_t st)
{
    if (!mlp_ready(m)) return MPT_E_NO_MODEL;
    if (nrows <= 0) return MPT_E_INVALID_ARG;
    mpt_status r = grad_dev(m, s, b, rows, nrows, target, use, d_loss, st);
    if (r) return r;
    m->step++;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - powf(b1, (float)m->step), c2 = 1.0f - powf(b2, (float)m->step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((NPAR + 255) / 256)), dim3(256), 0, st, m->w, m->m, m->v, m->g, m->wb,
                       m->wf, (int)NPAR, lr, b1, b2, 1e-8f, c1, c2);
    return hipGetLastError() == hipSuccess ? MPT_OK : MPT_E_DEVICE;
}

mpt_status mlp_features_dev(const SceneDev &s, const BatchDev &b, float *fout, hipStream_t st)
{
    if (b.n == 0) return MPT_OK;
    hipLaunchKernelGGL(k_features, dim3((unsigned)((b.n + 127) / 128)), dim3(128), 0, st, s, b, nullptr, (int)b.n,
                       fout, nullptr);
    return hipGetLastError() == hipSuccess ? MPT_OK : MPT_E_DEVICE;
}

// ------------------------------------------------------------------ GEMM self-test entry
// C[M][N] (fp32) = A[M][K] B[K][N] with bf16 inputs given as fp32 (rounded
// here); layouts as the flags say.  Used by the tests of the MFMA tile code.
__global__ void k_f2bf_arr(const float *x, bf16 *y, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

mpt_status gemm_test_dev(int M, int N, int K, const float *A, int at, const float *B, int bt, float *C, int splits,
                         hipStream_t st)
{
    bf16 *Ab = nullptr, *Bb = nullptr;
    float *part = nullptr;
    const size_t na = (size_t)M * K, nb = (size_t)K * N;
    if (hipMalloc((void **)&Ab, na * 2) != hipSuccess || hipMalloc((void **)&Bb, nb * 2) != hipSuccess ||
        hipMalloc((void **)&part, (size_t)(splits < 1 ? 1 : splits) * M * N * 4) != hipSuccess) {
        hipFree(Ab), hipFree(Bb), hipFree(part);
        return MPT_E_NOMEM;
    }
    hipLaunchKernelGGL(k_f2bf_arr, dim3((unsigned)((na + 255) / 256)), dim3(256), 0, st, A, Ab, na);
    hipLaunchKernelGGL(k_f2bf_arr, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, B, Bb, nb);
    Epi e{};
    e.ldc = N;
    e.fout = part;
    const int lda = at ? M : K, ldb = bt ? K : N;
    int kps = (K + splits - 1) / splits;
    kps = ((kps + GK - 1) / GK) * GK;
    const int sp = (K + kps - 1) / kps;
    if (!at && !bt) gemm<false, false, EPI_F32>(M, N, K, Ab, lda, Bb, ldb, e, splits, st);
    else if (!at && bt) gemm<false, true, EPI_F32>(M, N, K, Ab, lda, Bb, ldb, e, splits, st);
    else if (at && !bt) gemm<true, false, EPI_F32>(M, N, K, Ab, lda, Bb, ldb, e, splits, st);
    else gemm<true, true, EPI_F32>(M, N, K, Ab, lda, Bb, ldb, e, splits, st);
    const size_t n = (size_t)M * N;
    hipLaunchKernelGGL(k_reduce_splits, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, part, sp, n, C);
    hipError_t err = hipStreamSynchronize(st);
    hipFree(Ab), hipFree(Bb), hipFree(part);
    return err == hipSuccess ? MPT_OK : MPT_E_DEVICE;
}

// ------------------------------------------------------------------ save / load
// Blob: "MPTMLP01", uint32 header length, JSON header, then FP32 arrays
// (weights, Adam first and second moments), each NPAR long.
mpt_status mlp_save(MlpState *m, void *blob, size_t *bytes, hipStream_t st)
{
    if (!mlp_ready(m)) return MPT_E_NO_MODEL;
    char hdr[512];
    const int hl = snprintf(hdr, sizeof hdr,
                            "{\"format\": \"mpt-mlp\", \"version\": 1, \"layers\": [%d, %d, %d, %d, %d], "
                            "\"out_padded\": %d, \"params\": %zu, \"dtype\": \"f32\", \"activation\": \"gelu-erf\", "
                            "\"step\": %lld, \"seed\": %llu, \"arrays\": [\"w\", \"adam_m\", \"adam_v\"]}",
                            F_IN, HID, HID, HID, F_OUT, F_OUTP, (size_t)NPAR, (long long)m->step,
                            (unsigned long long)m->seed);
    const size_t need = 8 + 4 + (size_t)hl + 3 * NPAR * 4;
    if (!blob) {
        *bytes = need;
        return MPT_OK;
    }
    if (*bytes < need) {
        *bytes = need;
        return MPT_E_INVALID_ARG;
    }
    unsigned char *p = (unsigned char *)blob;
    memcpy(p, "MPTMLP01", 8);
    const uint32_t h32 = (uint32_t)hl;
    memcpy(p + 8, &h32, 4);
    memcpy(p + 12, hdr, hl);
    unsigned char *d = p + 12 + hl;
    if (hipMemcpyAsync(d, m->w, NPAR * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(d + NPAR * 4, m->m, NPAR * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(d + 2 * NPAR * 4, m->v, NPAR * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return MPT_E_DEVICE;
    *bytes = need;
    return MPT_OK;
}

mpt_status mlp_load(MlpState **pm, const void *blob, size_t bytes, hipStream_t st)
{
    const unsigned char *p = (const unsigned char *)blob;
    if (bytes < 12 || memcmp(p, "MPTMLP01", 8) != 0) return MPT_E_INVALID_ARG;
    uint32_t hl;
    memcpy(&hl, p + 8, 4);
    if (bytes != 12 + (size_t)hl + 3 * NPAR * 4) return MPT_E_INVALID_ARG;
    std::string hdr((const char *)p + 12, hl);
    long long step = 0;
    unsigned long long seed = 0;
    const size_t ps = hdr.find("\"step\": "), pd = hdr.find("\"seed\": ");
    if (ps != std::string::npos) step = atoll(hdr.c_str() + ps + 8);
    if (pd != std::string::npos) seed = strtoull(hdr.c_str() + pd + 8, nullptr, 10);
    if (!*pm) *pm = new MlpState();
    MlpState *m = *pm;
    if (!m->w && alloc_params(m)) return MPT_E_NOMEM;
    const unsigned char *d = p + 12 + hl;
    if (hipMemcpyAsync(m->w, d, NPAR * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(m->m, d + NPAR * 4, NPAR * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(m->v, d + 2 * NPAR * 4, NPAR * 4, hipMemcpyHostToDevice, st) != hipSuccess)
        return MPT_E_DEVICE;
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((NPAR + 255) / 256)), dim3(256), 0, st, m->w, m->wb, m->wf, (int)NPAR);
    if (hipStreamSynchronize(st) != hipSuccess) return MPT_E_DEVICE;
    m->step = step;
    m->seed = seed;
    return MPT_OK;
}

size_t mlp_param_count() { return NPAR; }

}  // namespace mpt
