// Host side of the C ABI declared in include/mpt.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>
#include <string>
#include <vector>

#include "../../include/mpt.h"
#include "mpt_internal.hpp"
#include "mpt_mlp.hpp"

using namespace mpt;

struct mpt_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t own = nullptr;
    std::string err;
    int cu = 256;
    // scene
    double *raw = nullptr, *rec64 = nullptr;
    float *rec32 = nullptr;
    size_t scene_cap = 0, raw_cap = 0;
    SceneDev s{};
    bool has_scene = false;
    // workspace: counters | perm | polish lists | fallback lists
    int *ws = nullptr;
    size_t ws_cap = 0;  // solves
    int *blk = nullptr;
    size_t blk_cap = 0;
    double *x0l = nullptr;
    size_t x0l_cap = 0;
    hipEvent_t ev[5] = {};
    bool timed = false;
    MlpState *mlp = nullptr;
};

static const int kCounters = 32;  // bin_cnt 0..4, cursor 5..9, head 10..19, pol_cnt 20..24, fb_cnt 25..29

static mpt_status fail(mpt_ctx *c, mpt_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return st;
}

#define HIPCHK(c, call)                                                                             \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess) return fail((c), MPT_E_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

static mpt_status ensure(mpt_ctx *c, void **p, size_t *cap, size_t need, size_t elem)
{
    if (need <= *cap && *p) return MPT_OK;
    if (*p) hipFree(*p);
    *p = nullptr;
    *cap = 0;
    if (need == 0) need = 1;
    if (hipMalloc(p, need * elem) != hipSuccess) {
        *p = nullptr;
        return fail(c, MPT_E_NOMEM, "device allocation of %zu bytes failed", need * elem);
    }
    *cap = need;
    return MPT_OK;
}

extern "C" {

mpt_status mpt_create(int device, void *hip_stream, mpt_ctx **out)
{
    if (!out) return MPT_E_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return MPT_E_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return MPT_E_DEVICE;
    mpt_ctx *c = new mpt_ctx();
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->cu = prop.multiProcessorCount;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return MPT_E_DEVICE;
        }
        c->stream = c->own;
    }
    for (auto &e : c->ev) hipEventCreate(&e);
    *out = c;
    return MPT_OK;
}

mpt_status mpt_destroy(mpt_ctx *c)
{
    if (!c) return MPT_E_INVALID_ARG;
    hipSetDevice(c->device);
    hipStreamSynchronize(c->stream);
    hipFree(c->raw);
    hipFree(c->rec64);
    hipFree(c->rec32);
    hipFree(c->ws);
    hipFree(c->blk);
    hipFree(c->x0l);
    mlp_free(c->mlp);
    for (auto &e : c->ev) hipEventDestroy(e);
    if (c->own) hipStreamDestroy(c->own);
    delete c;
    return MPT_OK;
}

const char *mpt_last_error(const mpt_ctx *c) { return c ? c->err.c_str() : "null context"; }

mpt_status mpt_set_stream(mpt_ctx *c, void *hip_stream)
{
    if (!c) return MPT_E_INVALID_ARG;
    c->stream = hip_stream ? (hipStream_t)hip_stream : c->own;
    if (!c->stream) {
        if (hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking) != hipSuccess)
            return fail(c, MPT_E_DEVICE, "stream creation failed");
        c->stream = c->own;
    }
    return MPT_OK;
}

mpt_status mpt_synchronize(mpt_ctx *c)
{
    if (!c) return MPT_E_INVALID_ARG;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return MPT_OK;
}

static bool finite_all(const double *p, size_t n)
{
    for (size_t i = 0; i < n; i++)
        if (!isfinite(p[i])) return false;
    return true;
}

static bool unit3(const double *v) { return fabs(sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) - 1.0) <= 1e-9; }

mpt_status mpt_scene_upload(mpt_ctx *c, const mpt_scene_desc *d)
{
    if (!c || !d) return fail(c, MPT_E_INVALID_ARG, "null argument");
    const int np = d->n_planes, nl = d->n_lines, nq = d->n_quadrics, nc = d->n_circles;
    if (np < 0 || nl < 0 || nq < 0 || nc < 0) return fail(c, MPT_E_INVALID_ARG, "negative primitive count");
    if ((np && !d->planes) || (nl && !d->lines) || (nq && !d->quadrics) || (nc && !d->circles))
        return fail(c, MPT_E_INVALID_ARG, "null primitive array");
    if (!finite_all(d->tx, 3) || !finite_all(d->aabb_lo, 3) || !finite_all(d->aabb_hi, 3))
        return fail(c, MPT_E_INVALID_ARG, "non-finite TX or scene box");
    for (int i = 0; i < 3; i++)
        if (!(d->aabb_hi[i] >= d->aabb_lo[i])) return fail(c, MPT_E_INVALID_ARG, "scene box hi < lo");
    if (!finite_all(d->planes, (size_t)np * 13) || !finite_all(d->lines, (size_t)nl * 8) ||
        !finite_all(d->quadrics, (size_t)nq * 17) || !finite_all(d->circles, (size_t)nc * 7))
        return fail(c, MPT_E_INVALID_ARG, "non-finite primitive value");
    for (int i = 0; i < np; i++)
        if (!unit3(d->planes + 13 * (size_t)i)) return fail(c, MPT_E_INVALID_ARG, "plane %d: normal not unit", i);
    for (int i = 0; i < nl; i++)
        if (!unit3(d->lines + 8 * (size_t)i + 3)) return fail(c, MPT_E_INVALID_ARG, "line %d: direction not unit", i);
    for (int i = 0; i < nq; i++)
        if (!unit3(d->quadrics + 17 * (size_t)i + 13)) return fail(c, MPT_E_INVALID_ARG, "quadric %d: axis not unit", i);
    for (int i = 0; i < nc; i++) {
        if (!unit3(d->circles + 7 * (size_t)i + 3)) return fail(c, MPT_E_INVALID_ARG, "circle %d: normal not unit", i);
        if (!(d->circles[7 * (size_t)i + 6] > 0)) return fail(c, MPT_E_INVALID_ARG, "circle %d: radius <= 0", i);
    }
    const size_t n_all = (size_t)np + nl + nq + nc;
    const size_t raw_n = (size_t)np * 13 + (size_t)nl * 8 + (size_t)nq * 17 + (size_t)nc * 7;
    hipSetDevice(c->device);
    mpt_status st;
    if ((st = ensure(c, (void **)&c->raw, &c->raw_cap, raw_n, sizeof(double)))) return st;
    size_t cap64 = c->scene_cap, cap32 = c->scene_cap;
    if ((st = ensure(c, (void **)&c->rec64, &cap64, n_all * kRec, sizeof(double)))) return st;
    if ((st = ensure(c, (void **)&c->rec32, &cap32, n_all * kRec, sizeof(float)))) return st;
    c->scene_cap = cap64 < cap32 ? cap64 : cap32;
    std::vector<double> host(raw_n ? raw_n : 1);
    size_t o = 0;
    memcpy(host.data() + o, d->planes, (size_t)np * 13 * 8), o += (size_t)np * 13;
    memcpy(host.data() + o, d->lines, (size_t)nl * 8 * 8), o += (size_t)nl * 8;
    memcpy(host.data() + o, d->quadrics, (size_t)nq * 17 * 8), o += (size_t)nq * 17;
    memcpy(host.data() + o, d->circles, (size_t)nc * 7 * 8), o += (size_t)nc * 7;
    HIPCHK(c, hipMemcpyAsync(c->raw, host.data(), raw_n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    SceneDev s{};
    s.rec64 = c->rec64;
    s.rec32 = c->rec32;
    s.n_pl = np;
    s.n_pl_ln = np + nl;
    s.n_pl_ln_q = np + nl + nq;
    s.n_all = (int)n_all;
    for (int i = 0; i < 3; i++) {
        s.tx[i] = d->tx[i];
        const double ctr = 0.5 * (d->aabb_lo[i] + d->aabb_hi[i]);
        const double h = 10.0 * 0.5 * (d->aabb_hi[i] - d->aabb_lo[i]) + 1.0;
        s.glo[i] = ctr - h;
        s.ghi[i] = ctr + h;
    }
    launch_pack(c->raw, s, np, nl, nq, nc, c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->s = s;
    c->has_scene = true;
    return MPT_OK;
}

void mpt_default_opts(mpt_solve_opts *o)
{
    if (!o) return;
    memset(o, 0, sizeof *o);
    o->precision = MPT_FP32_POLISH64;
    o->init = MPT_INIT_LINE;
    o->max_iter = 200;
    o->max_iter32 = 100;
    o->polish_steps = 5;
    o->fallback = MPT_FALLBACK_GPU_FP64;
    o->plateau_win = 10;
    o->sched = MPT_SCHED_PERSISTENT;
    o->block = 0;
    o->grid = 0;
    o->plateau_frac = 0.999;
    o->tol_step = 1e-12;
    o->tol_res = 1e-13;
    o->tau_root = 1e-9;
    o->lambda0 = 1e-3;
    o->tol_step32 = 1e-6;
    o->tol_res32 = 1e-5;
    o->polish_gate = 1e-2;
}

static mpt_status batch_dev(mpt_ctx *c, const mpt_batch_desc *b, BatchDev &bd)
{
    if (!b) return fail(c, MPT_E_INVALID_ARG, "null batch");
    if (b->n < 0) return fail(c, MPT_E_INVALID_ARG, "negative batch size");
    if (b->n > 0 && (!b->rx || !b->rx_index || !b->order || !b->prim || b->n_rx < 1))
        return fail(c, MPT_E_INVALID_ARG, "null batch array or n_rx < 1");
    if (b->n > (int64_t)0x7fffffff) return fail(c, MPT_E_INVALID_ARG, "batch larger than 2^31-1 solves");
    bd.n = b->n;
    bd.n_rx = b->n_rx;
    bd.rx = b->rx;
    bd.rx_index = b->rx_index;
    bd.order = b->order;
    bd.prim = b->prim;
    bd.x0 = b->x0;
    return MPT_OK;
}

// Blocks of a persistent launch: as many as can be resident at once.
static int resident_grid(mpt_ctx *c, const void *kern, int block, int64_t n)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, 0) != hipSuccess || per_cu < 1) per_cu = 1;
    int64_t g = (int64_t)per_cu * c->cu;
    const int64_t need = (n + block - 1) / block;
    if (need < g) g = need;
    return (int)(g < 1 ? 1 : g);
}

mpt_status mpt_solve_batch(mpt_ctx *c, const mpt_batch_desc *b, const mpt_solve_opts *opts, const mpt_solve_out *out)
{
    if (!c) return MPT_E_INVALID_ARG;
    if (!opts || !out) return fail(c, MPT_E_INVALID_ARG, "null options or outputs");
    if (!c->has_scene) return fail(c, MPT_E_NO_SCENE, "no scene uploaded");
    BatchDev bd;
    mpt_status st = batch_dev(c, b, bd);
    if (st) return st;
    if (b->n > 0 && (!out->x || !out->cost || !out->iters || !out->status))
        return fail(c, MPT_E_INVALID_ARG, "null output array");
    if (opts->precision != MPT_FP64_PLAIN && opts->precision != MPT_FP32_POLISH64)
        return fail(c, MPT_E_UNSUPPORTED, "precision %d", opts->precision);
    if (opts->init < MPT_INIT_LINE || opts->init > MPT_INIT_LEARNED)
        return fail(c, MPT_E_UNSUPPORTED, "init %d", opts->init);
    if (opts->init == MPT_INIT_USER && b->n > 0 && !b->x0) return fail(c, MPT_E_INVALID_ARG, "user start without x0");
    if (opts->init == MPT_INIT_LEARNED && !mlp_ready(c->mlp))
        return fail(c, MPT_E_NO_MODEL, "learned start requested but no network initialised");
    if (opts->max_iter < 0 || opts->max_iter32 < 0 || opts->polish_steps < 0 || opts->plateau_win < 0)
        return fail(c, MPT_E_INVALID_ARG, "negative iteration option");
    if (opts->block != 0 && (opts->block % 64 != 0 || opts->block > 256 || opts->block < 64))
        return fail(c, MPT_E_INVALID_ARG, "block must be 64, 128, 192 or 256");
    hipSetDevice(c->device);
    const int64_t n = b->n;
    if ((st = ensure(c, (void **)&c->ws, &c->ws_cap, kCounters + 3 * (size_t)(n > 0 ? n : 1), sizeof(int)))) return st;
    if (opts->init == MPT_INIT_LEARNED && (st = ensure(c, (void **)&c->x0l, &c->x0l_cap, 15 * (size_t)n, sizeof(double))))
        return st;
    int *ctr = c->ws;
    KParams kp{};
    kp.s = c->s;
    kp.b = bd;
    kp.out = OutDev{out->x, out->cost, out->iters, out->status};
    kp.o.init = opts->init;
    kp.o.max_iter = opts->max_iter;
    kp.o.max_iter32 = opts->max_iter32;
    kp.o.polish_steps = opts->polish_steps;
    kp.o.fallback = opts->fallback;
    kp.o.plateau_win = opts->plateau_win;
    kp.o.plateau_frac = opts->plateau_frac;
    kp.o.tol_step = opts->tol_step;
    kp.o.tol_res = opts->tol_res;
    kp.o.tau_root = opts->tau_root;
    kp.o.lambda0 = opts->lambda0;
    kp.o.tol_step32 = opts->tol_step32;
    kp.o.tol_res32 = opts->tol_res32;
    kp.o.polish_gate = opts->polish_gate;
    kp.x0_learned = c->x0l;
    kp.bin_cnt = ctr + 0;
    kp.head = ctr + 10;
    kp.pol_cnt = ctr + 20;
    kp.fb_cnt = ctr + 25;
    kp.perm = ctr + kCounters;
    kp.pol_list = ctr + kCounters + n;
    kp.fb_list = ctr + kCounters + 2 * n;

    hipStream_t s = c->stream;
    hipEventRecord(c->ev[0], s);
    launch_zero(ctr, kCounters, s);
    launch_bin(bd, kp.out, c->s.n_all, ctr + 0, ctr + 5, (int *)kp.perm, s);
    hipEventRecord(c->ev[1], s);
    if (opts->init == MPT_INIT_LEARNED && n > 0) {
        if ((st = mlp_predict_dev(c->mlp, c->s, bd, c->x0l, s))) return fail(c, st, "network forward failed");
    }
    hipEventRecord(c->ev[2], s);
    const int block = opts->block ? opts->block : 256;
    const int mode = (opts->precision == MPT_FP64_PLAIN) ? MODE_PLAIN64 : MODE_FP32;
    auto run_lm = [&](int md) {
        if (opts->sched == MPT_SCHED_PERSISTENT) {
            const void *k = lm_kernel(md, 0);
            const int g = opts->grid ? opts->grid : resident_grid(c, k, block, n);
            launch_lm(md, 0, kp, g, block, s);
        } else {
            for (int ord = MPT_MAX_ORDER; ord >= 1; ord--) {
                const void *k = lm_kernel(md, ord);
                const int g = opts->grid ? opts->grid : resident_grid(c, k, block, n);
                launch_lm(md, ord, kp, g, block, s);
            }
        }
    };
    if (n > 0) {
        run_lm(mode);
        if (mode == MODE_FP32) {
            const int g = resident_grid(c, polish_kernel(), 256, n);
            launch_polish(kp, g, 256, s);
        }
    }
    hipEventRecord(c->ev[3], s);
    if (n > 0 && mode == MODE_FP32 && opts->fallback) run_lm(MODE_FALLBACK64);
    hipEventRecord(c->ev[4], s);
    c->timed = true;
    HIPCHK(c, hipGetLastError());
    return MPT_OK;
}

mpt_status mpt_last_timings(mpt_ctx *c, float ms[4])
{
    if (!c || !ms) return MPT_E_INVALID_ARG;
    if (!c->timed) return fail(c, MPT_E_INVALID_ARG, "no solve recorded");
    HIPCHK(c, hipEventSynchronize(c->ev[4]));
    for (int i = 0; i < 4; i++) HIPCHK(c, hipEventElapsedTime(&ms[i], c->ev[i], c->ev[i + 1]));
    return MPT_OK;
}

mpt_status mpt_accept(mpt_ctx *c, const mpt_batch_desc *b, const mpt_solve_out *in, double tau_res, double min_seg,
                      uint8_t *accept, int32_t *accepted_idx, int32_t *d_count, int64_t *h_count)
{
    if (!c) return MPT_E_INVALID_ARG;
    if (!c->has_scene) return fail(c, MPT_E_NO_SCENE, "no scene uploaded");
    BatchDev bd;
    mpt_status st = batch_dev(c, b, bd);
    if (st) return st;
    if (!in || !d_count || (b->n > 0 && (!in->x || !in->status || !accept || !accepted_idx)))
        return fail(c, MPT_E_INVALID_ARG, "null accept argument");
    if (!(tau_res >= 0) || !(min_seg >= 0)) return fail(c, MPT_E_INVALID_ARG, "negative threshold");
    hipSetDevice(c->device);
    const size_t nblk = (size_t)((b->n + 255) / 256);
    if ((st = ensure(c, (void **)&c->blk, &c->blk_cap, nblk ? nblk : 1, sizeof(int)))) return st;
    OutDevC ic{in->x, in->cost, in->iters, in->status};
    launch_accept(c->s, bd, ic, tau_res, min_seg, accept, accepted_idx, d_count, c->blk, c->stream);
    HIPCHK(c, hipGetLastError());
    if (h_count) {
        int32_t v = 0;
        HIPCHK(c, hipMemcpyAsync(&v, d_count, sizeof v, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        *h_count = v;
    }
    return MPT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- network entry points
extern "C" {

mpt_status mpt_mlp_init(mpt_ctx *c, uint64_t seed)
{
    if (!c) return MPT_E_INVALID_ARG;
    hipSetDevice(c->device);
    mpt_status st = mlp_init(&c->mlp, seed, c->stream);
    return st ? fail(c, st, "network initialisation failed") : MPT_OK;
}

mpt_status mpt_mlp_train_step(mpt_ctx *c, const mpt_batch_desc *b, const double *target_x, const uint8_t *use,
                              float lr, float *d_loss)
{
    if (!c) return MPT_E_INVALID_ARG;
    if (!c->has_scene) return fail(c, MPT_E_NO_SCENE, "no scene uploaded");
    if (!mlp_ready(c->mlp)) return fail(c, MPT_E_NO_MODEL, "no network initialised");
    BatchDev bd;
    mpt_status st = batch_dev(c, b, bd);
    if (st) return st;
    if (b->n > 0 && !target_x) return fail(c, MPT_E_INVALID_ARG, "null targets");
    if (!(lr >= 0.0f)) return fail(c, MPT_E_INVALID_ARG, "negative learning rate");
    hipSetDevice(c->device);
    st = mlp_train_step_dev(c->mlp, c->s, bd, target_x, use, lr, d_loss, c->stream);
    return st ? fail(c, st, "training step failed") : MPT_OK;
}

mpt_status mpt_mlp_predict(mpt_ctx *c, const mpt_batch_desc *b, double *x_out)
{
    if (!c) return MPT_E_INVALID_ARG;
    if (!c->has_scene) return fail(c, MPT_E_NO_SCENE, "no scene uploaded");
    if (!mlp_ready(c->mlp)) return fail(c, MPT_E_NO_MODEL, "no network initialised");
    BatchDev bd;
    mpt_status st = batch_dev(c, b, bd);
    if (st) return st;
    if (b->n > 0 && !x_out) return fail(c, MPT_E_INVALID_ARG, "null output");
    hipSetDevice(c->device);
    st = mlp_predict_dev(c->mlp, c->s, bd, x_out, c->stream);
    return st ? fail(c, st, "network forward failed") : MPT_OK;
}

mpt_status mpt_mlp_save(mpt_ctx *c, void *blob, size_t *bytes)
{
    if (!c || !bytes) return MPT_E_INVALID_ARG;
    if (!mlp_ready(c->mlp)) return fail(c, MPT_E_NO_MODEL, "no network initialised");
    hipSetDevice(c->device);
    mpt_status st = mlp_save(c->mlp, blob, bytes, c->stream);
    return st ? fail(c, st, "network save failed (buffer too small?)") : MPT_OK;
}

mpt_status mpt_mlp_load(mpt_ctx *c, const void *blob, size_t bytes)
{
    if (!c || !blob) return MPT_E_INVALID_ARG;
    hipSetDevice(c->device);
    mpt_status st = mlp_load(&c->mlp, blob, bytes, c->stream);
    return st ? fail(c, st, "network load failed (bad blob)") : MPT_OK;
}

}  // extern "C"
