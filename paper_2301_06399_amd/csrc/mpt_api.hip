// Host side of the C ABI declared in include/mpt.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdlib.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>
#include <string>
#include <vector>
#include <algorithm>
#include <mutex>

#include "../../include/mpt.h"
#include "mpt_internal.hpp"
#include "mpt_mlp.hpp"
#include "mpt_flops.hpp"

static_assert(mpt::kRow == MPT_ROW, "point row width");

using namespace mpt;

struct mpt_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t own = nullptr;
    std::string err;
    int cu = 256;
    size_t lds_max = 65536;  // dynamic LDS a block may use
    // scene
    double *raw = nullptr, *rec64 = nullptr, *wd = nullptr, *sd = nullptr, *rfd = nullptr;
    float *rec32 = nullptr;
    size_t scene_cap = 0, raw_cap = 0, wd_cap = 0, sd_cap = 0, rfd_cap = 0;
    // candidate generation: sample points, their counts, path counts / offsets
    double *samp = nullptr;
    int *scnt = nullptr;
    int64_t *ccnt = nullptr, *csum = nullptr;
    size_t samp_cap = 0, scnt_cap = 0, ccnt_cap = 0, csum_cap = 0;
    // physical validation: count and list of the accepted solves
    int *vlist = nullptr;
    size_t vlist_cap = 0;
    SceneDev s{};
    bool has_scene = false;
    bool curved = false;     // the scene has paraboloids or circles
    bool refr = false;       // some facet of the scene refracts
    bool param_ok = true;    // every quadric is a paraboloid of revolution
    uint64_t scene_hash = 0; // FNV-1a of the uploaded records and TX: the tuning key
    // workspace: counters | perm | polish lists | fallback lists
    int *ws = nullptr;
    size_t ws_cap = 0;  // solves
    int *blk = nullptr;
    size_t blk_cap = 0;
    double *x0l = nullptr;
    size_t x0l_cap = 0;
    double *spf = nullptr;  // parked stragglers: damping, plateau reference, stall count [3][n]
    size_t spf_cap = 0;
    int *scratch = nullptr;  // this device's copy of the allocation-free solve's scratch (device address)
    std::string scratch_err;
    hipEvent_t ev[7] = {};
    hipStream_t aux[MPT_MAX_ORDER] = {};  // per-order launches run concurrently
    hipEvent_t fork = nullptr, join[MPT_MAX_ORDER] = {};
    hipEvent_t kev[MPT_MAX_ORDER][2] = {};  // per-order kernel start / end of the first LM pass
    bool kev_valid = false;
    bool timed = false;
    bool timing = true;  // record the stage events in mpt_solve_batch
    int32_t last_launch[5] = {};  // sched, block, gdiv, spill, form of the last solve
    bool launched = false;
    MlpState *mlp = nullptr;
    // autotuned launch choices: key (precision, form run, size class, scene
    // hash) -> (schedule, block, grid divisor, straggler threshold)
    struct Tune { int prec, form, nbucket; uint64_t scene; int sched, block, gdiv, spill; float ms; };
    std::vector<Tune> tune;
    bool tune_loaded = false;
    // captured graph of the last solve (replayed while the key matches)
    hipStream_t cap = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<unsigned char> gkey;
};

// bin_cnt 0..4, curved-row cursors 5..9, head 10..19, pol_cnt 20..24, fb_cnt 25..29, curved rows 30, then
// 3 x 1364 key counters, then spill_cnt 0..4 and spill_head 5..9
static const int kKeyCounters = 3 * 1364;
static const int kSpillCounters = 32 + kKeyCounters;
static const int kCounters = kSpillCounters + 16;

// Scratch of the allocation-free solve (mpt_solve_batch_noalloc): the
// counters, the perm / polish / fallback lists and the bin-ordered receiver
// and primitive ids of at most MPT_NOALLOC_MAX_SOLVES solves (37.8 MB).  Every GPU the library runs on
// holds its own copy until the process ends, and every such call on that
// GPU shares it.  In host code `scratch` names a host-side stand-in: its
// device address comes from hipGetSymbolAddress, once per device, when a
// context is created there (scratch_setup).
static const size_t kScratchInts = (size_t)kCounters + 9 * (size_t)MPT_NOALLOC_MAX_SOLVES;
static __device__ __align__(256) int scratch[kScratchInts];
static const int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static int *g_scratch_dev[kMaxDevices];

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

// The device address of this device's scratch, looked up once per device
// with that device current; a failure is kept and reported by the
// allocation-free solve (the other entry points do not use the scratch).
static void scratch_setup(mpt_ctx *c)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (c->device >= kMaxDevices) {
        c->scratch_err = "device index beyond the scratch table";
        return;
    }
    if (!g_scratch_dev[c->device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            c->scratch_err = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
            return;
        }
        g_scratch_dev[c->device] = (int *)p;
    }
    c->scratch = g_scratch_dev[c->device];
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
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        c->cu = prop.multiProcessorCount;
        // leave room for the static LDS of the kernels
        const size_t per_cu = prop.maxSharedMemoryPerMultiProcessor;
        if (per_cu > 4096) c->lds_max = per_cu - 4096;
    }
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
    for (int i = 0; i < MPT_MAX_ORDER; i++) {
        hipStreamCreateWithFlags(&c->aux[i], hipStreamNonBlocking);
        hipEventCreateWithFlags(&c->join[i], hipEventDisableTiming);
    }
    hipEventCreateWithFlags(&c->fork, hipEventDisableTiming);
    for (int i = 0; i < MPT_MAX_ORDER; i++)
        for (int j = 0; j < 2; j++) hipEventCreate(&c->kev[i][j]);
    scratch_setup(c);
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
    hipFree(c->wd);
    hipFree(c->sd);
    hipFree(c->rfd);
    hipFree(c->samp);
    hipFree(c->scnt);
    hipFree(c->ccnt);
    hipFree(c->csum);
    hipFree(c->vlist);
    hipFree(c->ws);
    hipFree(c->blk);
    hipFree(c->x0l);
    hipFree(c->spf);
    mlp_free(c->mlp);
    for (auto &e : c->ev) hipEventDestroy(e);
    for (int i = 0; i < MPT_MAX_ORDER; i++) {
        if (c->aux[i]) hipStreamSynchronize(c->aux[i]), hipStreamDestroy(c->aux[i]);
        if (c->join[i]) hipEventDestroy(c->join[i]);
    }
    if (c->fork) hipEventDestroy(c->fork);
    for (int i = 0; i < MPT_MAX_ORDER; i++)
        for (int j = 0; j < 2; j++)
            if (c->kev[i][j]) hipEventDestroy(c->kev[i][j]);
    if (c->gexec) hipGraphExecDestroy(c->gexec);
    if (c->cap) hipStreamDestroy(c->cap);
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
    if (d->wedges) {
        if (!finite_all(d->wedges, (size_t)nl * 7)) return fail(c, MPT_E_INVALID_ARG, "non-finite wedge value");
        for (int i = 0; i < nl; i++) {
            const double *w = d->wedges + 7 * (size_t)i;
            if (w[6] != 0.0 && w[6] != 1.0 && w[6] != 2.0)
                return fail(c, MPT_E_INVALID_ARG, "wedge %d: kind is not 0, 1 or 2", i);
            if (w[6] != 0.0 && !(unit3(w) && unit3(w + 3)))
                return fail(c, MPT_E_INVALID_ARG, "wedge %d: face normal not unit", i);
        }
    }
    if (d->sides)
        for (int i = 0; i < np; i++)
            if (d->sides[i] != -1.0 && d->sides[i] != 0.0 && d->sides[i] != 1.0)
                return fail(c, MPT_E_INVALID_ARG, "plane %d: side is not -1, 0 or 1", i);
    if (d->refraction)
        for (int i = 0; i < np; i++) {
            const double a = d->refraction[2 * (size_t)i], b = d->refraction[2 * (size_t)i + 1];
            if (!((a == 0.0 && b == 0.0) || (a > 0.0 && b > 0.0 && isfinite(a) && isfinite(b))))
                return fail(c, MPT_E_INVALID_ARG, "plane %d: refractive indices must be both positive or both 0", i);
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
    const bool wedges = d->wedges && nl > 0;
    if (wedges) {
        if ((st = ensure(c, (void **)&c->wd, &c->wd_cap, (size_t)nl * 7, sizeof(double)))) return st;
        HIPCHK(c, hipMemcpyAsync(c->wd, d->wedges, (size_t)nl * 7 * sizeof(double), hipMemcpyHostToDevice,
                                 c->stream));
    }
    const bool sides = d->sides && np > 0;
    if (sides) {
        if ((st = ensure(c, (void **)&c->sd, &c->sd_cap, (size_t)np, sizeof(double)))) return st;
        HIPCHK(c, hipMemcpyAsync(c->sd, d->sides, (size_t)np * sizeof(double), hipMemcpyHostToDevice, c->stream));
    }
    SceneDev s{};
    s.wedge = wedges ? c->wd : nullptr;
    s.side = sides ? c->sd : nullptr;
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
        s.lo[i] = d->aabb_lo[i];
        s.hi[i] = d->aabb_hi[i];
    }
    const bool refr = d->refraction && np > 0;
    if (refr) {
        if ((st = ensure(c, (void **)&c->rfd, &c->rfd_cap, (size_t)np * 2, sizeof(double)))) return st;
        HIPCHK(c, hipMemcpyAsync(c->rfd, d->refraction, (size_t)np * 2 * sizeof(double), hipMemcpyHostToDevice,
                                 c->stream));
    }
    launch_pack(c->raw, refr ? c->rfd : nullptr, s, np, nl, nq, nc, c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->s = s;
    c->has_scene = true;
    // FNV-1a over the counts, TX, box and records: launch choices tuned on
    // one scene are kept apart from another's
    uint64_t h = 0xcbf29ce484222325ull;
    auto mix = [&h](const void *p, size_t bytes) {
        const unsigned char *q = (const unsigned char *)p;
        for (size_t i = 0; i < bytes; i++) h = (h ^ q[i]) * 0x100000001b3ull;
    };
    const int32_t counts[4] = {np, nl, nq, nc};
    mix(counts, sizeof counts);
    mix(d->tx, 3 * sizeof(double));
    mix(d->aabb_lo, 3 * sizeof(double));
    mix(d->aabb_hi, 3 * sizeof(double));
    mix(host.data(), raw_n * sizeof(double));
    if (refr) mix(d->refraction, (size_t)np * 2 * sizeof(double));
    c->scene_hash = h;
    c->curved = (nq + nc) > 0;
    c->refr = false;
    if (refr)
        for (int i = 0; i < np && !c->refr; i++) c->refr = d->refraction[2 * (size_t)i] > 0.0;
    c->param_ok = true;
    for (int i = 0; i < nq; i++) {
        // the parametric form needs A = k (I - ax ax^T), b = -ax, c = 0
        const double *q = d->quadrics + 17 * (size_t)i, *ax = q + 13;
        const double kap = 0.5 * (q[3] + q[6] + q[8]);
        const double Am[3][3] = {{q[3], q[4], q[5]}, {q[4], q[6], q[7]}, {q[5], q[7], q[8]}};
        double err = fabs(q[12]);
        for (int a = 0; a < 3; a++) {
            err = fmax(err, fabs(q[9 + a] + ax[a]));
            for (int b = 0; b < 3; b++) err = fmax(err, fabs(Am[a][b] - kap * ((a == b ? 1.0 : 0.0) - ax[a] * ax[b])));
        }
        c->param_ok = c->param_ok && kap > 0.0 && err <= 1e-9 * (1.0 + kap);
    }
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
    o->max_iter32_planar = 80;
    o->polish_steps = 5;
    o->fallback = MPT_FALLBACK_GPU_FP64;
    o->plateau_win = 10;
    o->sched = MPT_SCHED_AUTO;
    o->block = 0;
    o->grid = 0;
    o->graph = 0;
    o->max_iter_fb = 50;
    o->plateau_frac = 0.999;
    o->tol_step = 1e-12;
    o->tol_res = 1e-13;
    o->tau_root = 1e-9;
    o->lambda0 = 1e-3;
    o->tol_step32 = 1e-6;
    o->tol_res32 = 1e-5;
    o->tau_root32 = 1e-4;
    o->polish_gate = 1e-2;
    o->seed = 0;
    o->spill = -1;
    o->form = MPT_FORM_IMPLICIT;
    o->stat_tol = 0.02;
    o->stat_win = 4;
    o->refill = 16;
    o->extent_skip = 0.05;
    o->learned_gain = 1.0;
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
static int resident_grid(mpt_ctx *c, const void *kern, int block, int64_t n, size_t lds = 0)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int64_t g = (int64_t)per_cu * c->cu;
    const int64_t need = (n + block - 1) / block;
    if (need < g) g = need;
    return (int)(g < 1 ? 1 : g);
}

}  // extern "C"

// ---------------------------------------------------------------- launch choices
// Default launch choices before (or without) tuning, from back-to-back
// measurements on MI355X: one mixed-order launch of 256 threads per block
// (the short orders fill the tail of the long ones); no straggler launch
// (it pays on long curved chains, which the tuner finds).
static void default_choice(int prec, int &sched, int &block, int &gdiv, int &spill)
{
    (void)prec;
    gdiv = 1;
    spill = 0;
    sched = MPT_SCHED_PERSISTENT;
    block = 256;
}

static int nbucket(int64_t n)
{
    int b = 0;
    while ((int64_t(1) << (b + 1)) <= n) b++;
    return b;
}

static void tune_load(mpt_ctx *c)
{
    if (c->tune_loaded) return;
    c->tune_loaded = true;
    const char *path = getenv("MPT_AUTOTUNE_CACHE");
    if (!path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    // one entry per line: prec form nbucket scene-hash sched block gdiv spill ms
    mpt_ctx::Tune t;
    unsigned long long h = 0;
    while (fscanf(f, "%d %d %d %llx %d %d %d %d %f", &t.prec, &t.form, &t.nbucket, &h, &t.sched, &t.block, &t.gdiv,
                  &t.spill, &t.ms) == 9) {
        t.scene = (uint64_t)h;
        c->tune.push_back(t);
    }
    fclose(f);
}

static void tune_save(mpt_ctx *c)
{
    const char *path = getenv("MPT_AUTOTUNE_CACHE");
    if (!path) return;
    FILE *f = fopen(path, "w");
    if (!f) return;
    for (auto &t : c->tune)
        fprintf(f, "%d %d %d %llx %d %d %d %d %.6f\n", t.prec, t.form, t.nbucket, (unsigned long long)t.scene, t.sched,
                t.block, t.gdiv, t.spill, t.ms);
    fclose(f);
}

// The form a solve runs in: MPT_FORM_AUTO takes the parametric form
// whenever every object of the scene has a parametric expression (every
// quadric is a paraboloid of revolution), else the implicit one.  It is a
// property of the scene, never a timing choice.
static int auto_form(const mpt_ctx *c)
{
    return c->param_ok ? MPT_FORM_PARAMETRIC : MPT_FORM_IMPLICIT;
}

static int resolved_form(const mpt_ctx *c, const mpt_solve_opts *o)
{
    return (o->form == MPT_FORM_AUTO) ? auto_form(c) : o->form;
}

static void choose(mpt_ctx *c, const mpt_solve_opts *o, int64_t n, int &sched, int &block, int &gdiv, int &spill,
                   int &form, bool load = true)
{
    default_choice(o->precision, sched, block, gdiv, spill);
    form = resolved_form(c, o);
    if (load) tune_load(c);
    for (auto &t : c->tune)
        if (t.prec == o->precision && t.form == form && t.nbucket == nbucket(n) && t.scene == c->scene_hash) {
            sched = t.sched;
            block = t.block;
            gdiv = t.gdiv;
            spill = t.spill;
        }
    if (o->sched != MPT_SCHED_AUTO) sched = o->sched;
    if (o->block) block = o->block;
    if (o->spill >= 0) spill = o->spill;
    // the rows of refracting facets are compiled into the mixed-order
    // kernel only
    if (c->refr) sched = MPT_SCHED_PERSISTENT, gdiv = 1;
}

static mpt_status check_opts(mpt_ctx *c, const mpt_batch_desc *b, const mpt_solve_opts *opts, const mpt_solve_out *out)
{
    if (!opts || !out) return fail(c, MPT_E_INVALID_ARG, "null options or outputs");
    if (!c->has_scene) return fail(c, MPT_E_NO_SCENE, "no scene uploaded");
    BatchDev bd;
    mpt_status st = batch_dev(c, b, bd);
    if (st) return st;
    if (b->n > 0 && (!out->x || !out->cost || !out->iters || !out->status))
        return fail(c, MPT_E_INVALID_ARG, "null output array");
    if (opts->precision != MPT_FP64_PLAIN && opts->precision != MPT_FP32_POLISH64)
        return fail(c, MPT_E_UNSUPPORTED, "precision %d", opts->precision);
    if (opts->init < MPT_INIT_LINE || opts->init > MPT_INIT_RANDOM)
        return fail(c, MPT_E_UNSUPPORTED, "init %d", opts->init);
    if (opts->init == MPT_INIT_USER && b->n > 0 && !b->x0) return fail(c, MPT_E_INVALID_ARG, "user start without x0");
    if ((opts->init == MPT_INIT_LEARNED || opts->init == MPT_INIT_LEARNED_ALL) && !mlp_ready(c->mlp))
        return fail(c, MPT_E_NO_MODEL, "learned start requested but no network initialised");
    if (opts->max_iter < 0 || opts->max_iter32 < 0 || opts->max_iter_fb < 0 || opts->polish_steps < 0 ||
        opts->plateau_win < 0)
        return fail(c, MPT_E_INVALID_ARG, "negative iteration option");
    if (opts->max_iter32_planar < 1 || opts->max_iter32_planar > opts->max_iter32)
        return fail(c, MPT_E_INVALID_ARG, "max_iter32_planar must be 1..max_iter32");
    if (opts->block != 0 && (opts->block % 64 != 0 || opts->block > 256 || opts->block < 64))
        return fail(c, MPT_E_INVALID_ARG, "block must be 64, 128, 192 or 256");
    if (opts->sched < MPT_SCHED_PER_ORDER || opts->sched > MPT_SCHED_SPLIT)
        return fail(c, MPT_E_UNSUPPORTED, "sched %d", opts->sched);
    if (opts->grid < 0) return fail(c, MPT_E_INVALID_ARG, "negative grid");
    if (opts->spill < -1 || opts->spill > 64) return fail(c, MPT_E_INVALID_ARG, "spill must be -1..64");
    if (opts->stat_win < 0 || !(opts->stat_tol >= 0.0)) return fail(c, MPT_E_INVALID_ARG, "bad stall test options");
    if (!(opts->extent_skip >= 0.0) || !isfinite(opts->extent_skip))
        return fail(c, MPT_E_INVALID_ARG, "extent_skip must be finite and >= 0");
    if (!(opts->learned_gain > 0.0) || !isfinite(opts->learned_gain))
        return fail(c, MPT_E_INVALID_ARG, "learned_gain must be finite and > 0");
    if (opts->form != MPT_FORM_IMPLICIT && opts->form != MPT_FORM_PARAMETRIC && opts->form != MPT_FORM_AUTO)
        return fail(c, MPT_E_UNSUPPORTED, "form %d", opts->form);
    return MPT_OK;
}

// Work buffers of a solve of n paths (sized before any graph capture).
static mpt_status size_buffers(mpt_ctx *c, int64_t n, bool learned)
{
    const size_t m = (size_t)(n > 0 ? n : 1);
    mpt_status st;
    if ((st = ensure(c, (void **)&c->ws, &c->ws_cap, kCounters + 10 * m, sizeof(int)))) return st;
    if ((st = ensure(c, (void **)&c->spf, &c->spf_cap, 3 * m, sizeof(double)))) return st;
    if (learned && (st = ensure(c, (void **)&c->x0l, &c->x0l_cap, MPT_ROW * m, sizeof(double)))) return st;
    return MPT_OK;
}

// Workspace of one solve: counters and lists (int32), parked straggler
// state and network start points (FP64; null when unused).
struct Work {
    int *ws;
    double *spf, *x0l;
};

// Enqueue the whole solve on stream s (no host synchronisation).  With
// `timed`, HIP events mark the stage boundaries (not inside graph capture).
// The workspace is the context's own (sized here) unless `w` brings one.
static mpt_status enqueue_solve(mpt_ctx *c, const mpt_batch_desc *b, const mpt_solve_opts *opts,
                                const mpt_solve_out *out, hipStream_t s, bool timed, int sched, int block,
                                int gdiv, int spill, int form_used, const Work *w = nullptr)
{
    BatchDev bd;
    mpt_status st = batch_dev(c, b, bd);
    if (st) return st;
    const int64_t n = b->n;
    const bool learned = opts->init == MPT_INIT_LEARNED || opts->init == MPT_INIT_LEARNED_ALL;
    if (c->refr) sched = MPT_SCHED_PERSISTENT, gdiv = 1;  // the only kernel with refracting rows
    Work own{nullptr, nullptr, nullptr};
    if (!w) {
        if ((st = size_buffers(c, n, learned))) return st;
        own = Work{c->ws, c->spf, c->x0l};
        w = &own;
    }
    if ((learned && !w->x0l) || (spill > 0 && !w->spf)) return fail(c, MPT_E_INVALID_ARG, "workspace too small");
    if (!timed) c->timed = c->kev_valid = false;  // no stale stage timings
    int *ctr = w->ws;
    KParams kp{};
    kp.s = c->s;
    kp.b = bd;
    kp.out = OutDev{out->x, out->cost, out->iters, out->status, out->stage_iters};
    kp.o.init = opts->init;
    kp.o.max_iter = opts->max_iter;
    kp.o.max_iter32 = opts->max_iter32;
    kp.o.max_iter32_planar = opts->max_iter32_planar;
    kp.o.max_iter_fb = opts->max_iter_fb;
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
    kp.o.tau_root32 = opts->tau_root32;
    kp.o.polish_gate = opts->polish_gate;
    kp.o.seed = opts->seed;
    kp.o.stat_tol = opts->stat_tol;
    kp.o.stat_win = opts->stat_win;
    kp.o.extent_skip = opts->extent_skip;
    kp.x0_learned = w->x0l;
    kp.bin_cnt = ctr + 0;
    kp.head = ctr + 10;
    kp.pol_cnt = ctr + 20;
    kp.fb_cnt = ctr + 25;
    kp.perm = ctr + kCounters;
    kp.pol_list = ctr + kCounters + n;
    kp.fb_list = ctr + kCounters + 2 * n;
    kp.slot_rx = ctr + kCounters + 3 * n;
    kp.slot_prim = ctr + kCounters + 4 * n;
    kp.spill_t = spill;
    kp.refill = opts->refill > 1 ? (opts->refill < 64 ? opts->refill : 64) : 1;
    kp.spill_cnt = ctr + kSpillCounters;
    kp.spill_head = ctr + kSpillCounters + 5;
    kp.spill_list = w->spf ? ctr + kCounters + 9 * n : nullptr;
    kp.spill_f = w->spf;

    // the network serves the paths with a curved object: none without
    // paraboloids and circles in the scene
    const bool net = learned && n > 0 && (opts->init == MPT_INIT_LEARNED_ALL || c->s.n_pl_ln < c->s.n_all);
    // with MPT_INIT_LEARNED the binning lists the paths with a curved object
    // (in the polish list, free until the FP32 pass), grouped by order:
    // per-order cursors in counters 5..9, the length in counter 30
    int *rows = (net && opts->init == MPT_INIT_LEARNED) ? (int *)kp.pol_list : nullptr, *rows_cnt = ctr + 30;
    if (timed) hipEventRecord(c->ev[0], s);
    launch_zero(ctr, kCounters, s);
    launch_bin(bd, kp.out, c->s, ctr + 0, ctr + 32, (int *)kp.perm, (int *)kp.slot_rx, (int *)kp.slot_prim, rows,
               ctr + 5, s);
    if (timed) hipEventRecord(c->ev[1], s);
    if (net) {
        if (opts->init == MPT_INIT_LEARNED) {
            st = mlp_predict_dev(c->mlp, c->s, bd, w->x0l, s, rows, rows_cnt);
            if (!st) launch_learned_choose(c->s, bd, rows, rows_cnt, false, w->x0l, opts->learned_gain, c->refr, s);
        } else {
            st = mlp_predict_dev(c->mlp, c->s, bd, w->x0l, s);
            if (!st) launch_learned_choose(c->s, bd, nullptr, nullptr, true, w->x0l, opts->learned_gain, c->refr, s);
        }
        if (st) return fail(c, st, "network forward failed");
    }
    if (timed) hipEventRecord(c->ev[2], s);
    const int mode = (opts->precision == MPT_FP64_PLAIN) ? MODE_PLAIN64 : MODE_FP32;
    auto run_lm = [&](int md, int sch, int blk, bool first) {
        // stage the scene in LDS when it fits
        const size_t rec_bytes = (size_t)c->s.n_all * kRec * (md == MODE_FP32 ? sizeof(float) : sizeof(double));
        const bool lds = rec_bytes <= c->lds_max;
        auto go = [&](int ord, hipStream_t where) {
            const int form = form_used;
            const void *k = lm_kernel(md, ord, lds, form, c->refr);
            if (lds) hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)rec_bytes);
            int g = opts->grid;
            if (!g) {
                // all resident blocks, divided by gdiv for the concurrent
                // per-order launches (fewer waves per SIMD in their tails)
                g = resident_grid(c, k, blk, n, lds ? rec_bytes : 0);
                if (first && gdiv > 1) g = (g + gdiv - 1) / gdiv;
            }
            launch_lm(md, ord, lds, form, c->refr, rec_bytes, kp, g, blk, where);
        };
        if (sch == MPT_SCHED_PERSISTENT) {
            go(0, s);
        } else if (sch == MPT_SCHED_SPLIT) {
            // orders 1-3 in one launch on s, orders 4 and 5 beside it
            hipEventRecord(c->fork, s);
            for (int ord = MPT_MAX_ORDER; ord >= 4; ord--) {
                hipStreamWaitEvent(c->aux[ord - 1], c->fork, 0);
                go(ord, c->aux[ord - 1]);
                hipEventRecord(c->join[ord - 1], c->aux[ord - 1]);
            }
            go(6, s);
            for (int ord = 4; ord <= MPT_MAX_ORDER; ord++) hipStreamWaitEvent(s, c->join[ord - 1], 0);
        } else {
            // one launch per order, each on its own stream (fork / join on
            // the stream s): the waves of a later order fill the CUs an
            // earlier order's drained bin leaves idle
            hipEventRecord(c->fork, s);
            for (int ord = MPT_MAX_ORDER; ord >= 1; ord--) {
                hipStreamWaitEvent(c->aux[ord - 1], c->fork, 0);
                if (timed && first) hipEventRecord(c->kev[ord - 1][0], c->aux[ord - 1]);
                go(ord, c->aux[ord - 1]);
                if (timed && first) hipEventRecord(c->kev[ord - 1][1], c->aux[ord - 1]);
                hipEventRecord(c->join[ord - 1], c->aux[ord - 1]);
            }
            for (int ord = 1; ord <= MPT_MAX_ORDER; ord++) hipStreamWaitEvent(s, c->join[ord - 1], 0);
        }
    };
    if (timed) c->kev_valid = (n > 0) && sched == MPT_SCHED_PER_ORDER;
    if (n > 0) run_lm(mode, sched, block, true);
    if (timed) hipEventRecord(c->ev[3], s);
    if (n > 0 && spill > 0) {
        // the parked stragglers: the same kernels, launched again to resume
        kp.resume = 1;
        run_lm(mode, sched, block, false);
        kp.resume = 0;
    }
    if (timed) hipEventRecord(c->ev[4], s);
    if (n > 0 && mode == MODE_FP32) {
        launch_polish_list(kp, s);
        launch_polish(kp, c->refr, resident_grid(c, polish_kernel(c->refr), 256, n), 256, s);
    }
    if (timed) hipEventRecord(c->ev[5], s);
    // the fallback handles a handful of paths: one mixed-order launch
    if (n > 0 && mode == MODE_FP32 && opts->fallback) run_lm(MODE_FALLBACK64, MPT_SCHED_PERSISTENT, 256, false);
    if (timed) hipEventRecord(c->ev[6], s);
    if (timed) c->timed = true;
    HIPCHK(c, hipGetLastError());
    return MPT_OK;
}

static std::vector<unsigned char> graph_key(const mpt_batch_desc *b, const mpt_solve_opts *o, const mpt_solve_out *out,
                                            int sched, int block, int gdiv, int spill, int form, const SceneDev &s)
{
    std::vector<unsigned char> k(sizeof *b + sizeof *o + sizeof *out + 5 * sizeof(int) + sizeof s);
    unsigned char *p = k.data();
    memcpy(p, b, sizeof *b), p += sizeof *b;
    memcpy(p, o, sizeof *o), p += sizeof *o;
    memcpy(p, out, sizeof *out), p += sizeof *out;
    memcpy(p, &sched, sizeof sched), p += sizeof sched;
    memcpy(p, &block, sizeof block), p += sizeof block;
    memcpy(p, &gdiv, sizeof gdiv), p += sizeof gdiv;
    memcpy(p, &spill, sizeof spill), p += sizeof spill;
    memcpy(p, &form, sizeof form), p += sizeof form;
    memcpy(p, &s, sizeof s);
    return k;
}

extern "C" {

mpt_status mpt_solve_batch(mpt_ctx *c, const mpt_batch_desc *b, const mpt_solve_opts *opts, const mpt_solve_out *out)
{
    if (!c) return MPT_E_INVALID_ARG;
    mpt_status st = check_opts(c, b, opts, out);
    if (st) return st;
    hipSetDevice(c->device);
    int sched, block, gdiv, spill, form;
    choose(c, opts, b->n, sched, block, gdiv, spill, form);
    const int32_t chosen[5] = {sched, block, gdiv, spill, form};
    memcpy(c->last_launch, chosen, sizeof chosen);
    c->launched = true;
    if (!opts->graph) return enqueue_solve(c, b, opts, out, c->stream, c->timing, sched, block, gdiv, spill, form);

    // graph mode: capture once per (batch, options, outputs, scene) and replay
    std::vector<unsigned char> key = graph_key(b, opts, out, sched, block, gdiv, spill, form, c->s);
    if (!c->gexec || key != c->gkey) {
        if (c->gexec) hipGraphExecDestroy(c->gexec), c->gexec = nullptr;
        if (!c->cap) HIPCHK(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
        // buffers are sized before capture: no allocation inside it
        const bool learned = opts->init == MPT_INIT_LEARNED || opts->init == MPT_INIT_LEARNED_ALL;
        if ((st = size_buffers(c, b->n, learned))) return st;
        HIPCHK(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
        st = enqueue_solve(c, b, opts, out, c->cap, false, sched, block, gdiv, spill, form);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c->cap, &g);
        if (st) {
            if (g) hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return fail(c, MPT_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e != hipSuccess) return fail(c, MPT_E_DEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
        c->gkey = key;
    }
    c->timed = c->kev_valid = false;  // a replay records no stage events
    HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
    return MPT_OK;
}

mpt_status mpt_solve_batch_noalloc(mpt_ctx *c, const mpt_batch_desc *b, const mpt_solve_opts *opts,
                                   const mpt_solve_out *out)
{
    if (!c) return MPT_E_INVALID_ARG;
    mpt_status st = check_opts(c, b, opts, out);
    if (st) return st;
    if (!c->scratch) return fail(c, MPT_E_DEVICE, "no scratch on this device: %s", c->scratch_err.c_str());
    if (b->n > MPT_NOALLOC_MAX_SOLVES)
        return fail(c, MPT_E_INVALID_ARG, "%lld solves exceed the allocation-free limit of %d", (long long)b->n,
                    (int)MPT_NOALLOC_MAX_SOLVES);
    if (opts->init == MPT_INIT_LEARNED || opts->init == MPT_INIT_LEARNED_ALL)
        return fail(c, MPT_E_UNSUPPORTED, "the learned start needs the context's workspace");
    if (opts->graph) return fail(c, MPT_E_UNSUPPORTED, "graph mode instantiates a graph (allocates)");
    hipSetDevice(c->device);
    // the tuned choices already in memory (no cache file is read); no
    // straggler launch, whose parked state needs the context's workspace
    int sched, block, gdiv, spill, form;
    choose(c, opts, b->n, sched, block, gdiv, spill, form, false);
    spill = 0;
    const int32_t chosen[5] = {sched, block, gdiv, spill, form};
    memcpy(c->last_launch, chosen, sizeof chosen);
    c->launched = true;
    const Work w{c->scratch, nullptr, nullptr};
    return enqueue_solve(c, b, opts, out, c->stream, c->timing, sched, block, gdiv, spill, form, &w);
}

mpt_status mpt_autotune(mpt_ctx *c, const mpt_batch_desc *b, const mpt_solve_opts *opts, const mpt_solve_out *out,
                        int32_t *best_sched, int32_t *best_block, float *best_ms, int32_t *best_gdiv,
                        int32_t *best_spill, int32_t *best_form)
{
    if (!c) return MPT_E_INVALID_ARG;
    mpt_status st = check_opts(c, b, opts, out);
    if (st) return st;
    hipSetDevice(c->device);
    tune_load(c);
    // candidates: schedule x block size x grid divisor (per-order only) x
    // straggler threshold, in the form the options resolve to (the form is
    // never a timing choice: the forms can accept different paths)
    std::vector<int> forms = {resolved_form(c, opts)};
    struct Cand { int sched, block, gdiv, spill, form; };
    std::vector<Cand> cands;
    for (int fm : forms) {
        for (int sp : {0, 8, 16, 32})
            for (int blk : {128, 256}) cands.push_back({MPT_SCHED_PERSISTENT, blk, 1, sp, fm});
        if (c->refr) continue;  // refracting facets: the mixed-order kernel only
        for (int sp : {0, 16})
            for (int blk : {64, 128, 256})
                for (int gd : {1, 2}) cands.push_back({MPT_SCHED_PER_ORDER, blk, gd, sp, fm});
        for (int sp : {0, 16})
            for (int blk : {128, 256}) cands.push_back({MPT_SCHED_SPLIT, blk, 1, sp, fm});
    }
    float best = 1e30f;
    Cand bc = cands[0];
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return fail(c, MPT_E_DEVICE, "event creation failed");
    }
    for (const Cand &cd : cands) {
        // whole solves back to back, as a caller runs them: after one
        // warm-up solve, three groups of runs (four each, two when a solve
        // takes more than 20 ms), each timed from its first launch to its
        // last; the median group mean counts
        if ((st = enqueue_solve(c, b, opts, out, c->stream, false, cd.sched, cd.block, cd.gdiv, cd.spill, cd.form)))
            break;
        hipEventRecord(e0, c->stream);
        if ((st = enqueue_solve(c, b, opts, out, c->stream, false, cd.sched, cd.block, cd.gdiv, cd.spill, cd.form)))
            break;
        hipEventRecord(e1, c->stream);
        if (hipEventSynchronize(e1) != hipSuccess) { st = fail(c, MPT_E_DEVICE, "tuning run failed"); break; }
        float one = 0.0f;
        hipEventElapsedTime(&one, e0, e1);
        const int per = one > 20.0f ? 2 : 4;
        float t[3];
        for (int g = 0; g < 3 && !st; g++) {
            hipEventRecord(e0, c->stream);
            for (int r = 0; r < per && !st; r++)
                st = enqueue_solve(c, b, opts, out, c->stream, false, cd.sched, cd.block, cd.gdiv, cd.spill, cd.form);
            hipEventRecord(e1, c->stream);
            if (!st && hipEventSynchronize(e1) != hipSuccess) st = fail(c, MPT_E_DEVICE, "tuning run failed");
            float ms = 0.0f;
            hipEventElapsedTime(&ms, e0, e1);
            t[g] = ms / per;
        }
        if (st) break;
        std::sort(t, t + 3);
        if (t[1] < best) best = t[1], bc = cd;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st) return st;
    bool found = false;
    for (auto &t : c->tune)
        if (t.prec == opts->precision && t.form == bc.form && t.nbucket == nbucket(b->n) && t.scene == c->scene_hash)
            t.sched = bc.sched, t.block = bc.block, t.gdiv = bc.gdiv, t.spill = bc.spill, t.ms = best, found = true;
    if (!found)
        c->tune.push_back({opts->precision, bc.form, nbucket(b->n), c->scene_hash, bc.sched, bc.block, bc.gdiv,
                           bc.spill, best});
    tune_save(c);
    if (best_sched) *best_sched = bc.sched;
    if (best_block) *best_block = bc.block;
    if (best_ms) *best_ms = best;
    if (best_gdiv) *best_gdiv = bc.gdiv;
    if (best_spill) *best_spill = bc.spill;
    if (best_form) *best_form = bc.form;
    return MPT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- FLOP count
template <int N>
static void count_one(const int32_t *types, int64_t out[4], bool param, int64_t *asm_flops = nullptr)
{
    // a small synthetic scene: one record per interaction with generic
    // (non-zero, non-special) values, so no operation is skipped by accident;
    // planes are mirrors (the rows of a refracting facet are not counted)
    uint64_t st = 0x9e3779b97f4a7c15ull;
    auto rnd = [&]() {
        st = st * 6364136223846793005ull + 1442695040888963407ull;
        return 0.25 + 0.5 * (double)((st >> 11) & ((1ull << 53) - 1)) / (double)(1ull << 53);
    };
    Cnt rec[N * kRec];
    int np = 0, nl = 0, nq = 0;
    for (int k = 0; k < N; k++) {
        if (types[k] == MPT_PLANE) np++;
        else if (types[k] == MPT_LINE) nl++;
        else if (types[k] == MPT_QUADRIC) nq++;
    }
    PathIn<Cnt, N> p;
    p.planar = false;
    int next[4] = {0, np, np + nl, np + nl + nq};
    for (int k = 0; k < N; k++) {
        const int id = next[types[k]]++;
        p.id[k] = id;
        p.ty[k] = types[k];
        for (int i = 0; i < kRec; i++) rec[id * kRec + i] = Cnt(rnd());
    }
    SceneT<Cnt> sc;
    sc.rec = rec;
    for (int i = 0; i < 3; i++) {
        sc.tx[i] = Cnt(rnd());
        sc.glo[i] = Cnt(-1e9);
        sc.ghi[i] = Cnt(1e9);
        p.rx[i] = Cnt(rnd() + 5.0);
    }
    Cnt X[3 * N], A[Band<N>::SIZE], g[3 * N], C, rinf;
    for (int i = 0; i < 3 * N; i++) X[i] = Cnt(rnd() + i);
    constexpr int M = 3 * N;
    // one LM iteration
    tally() = FlopTally();
    assemble<Cnt, N, false>(sc, p, X, A, g, C, rinf);
    if (asm_flops && !param) *asm_flops = tally().flops();
    Cnt lam(rnd()), dmax(rnd());
    for (int i = 0; i < M; i++) A[Band<N>::at(i, i)] += lam * fmax(A[Band<N>::at(i, i)], Cnt(1e-12) * dmax);
    chol_band<Cnt, N>(A);
    chol_solve_band<Cnt, N>(A, g);
    Cnt Ct, rt;
    eval_cost<Cnt, N, false>(sc, p, X, g, Ct, rt);
    for (int i = 0; i < M; i++) X[i] += g[i];
    out[0] = tally().flops();
    out[3] = tally().sqrt + tally().div;
    // one polish step
    tally() = FlopTally();
    assemble<Cnt, N, false>(sc, p, X, A, g, C, rinf);
    chol_band<Cnt, N>(A);
    chol_solve_band<Cnt, N>(A, g);
    for (int i = 0; i < M; i++) X[i] += g[i];
    out[1] = tally().flops();
    // one residual evaluation
    tally() = FlopTally();
    eval_cost<Cnt, N, false>(sc, p, X, nullptr, C, rinf);
    out[2] = tally().flops();
    if (!param) return;
    // the parametric form: one iteration over the 2N parameters (the polish
    // stays implicit); an edge's placeholder parameter costs nothing
    Cnt U[2 * N], Ap[Band<N, 2>::SIZE], gp[2 * N];
    for (int k = 0; k < N; k++) {
        U[2 * k] = Cnt(rnd());
        U[2 * k + 1] = (types[k] == MPT_PLANE || types[k] == MPT_QUADRIC) ? Cnt(rnd()) : Cnt(0.0);
    }
    tally() = FlopTally();
    assemble_param<Cnt, N, false>(sc, p, U, Ap, gp, C, rinf);
    if (asm_flops) *asm_flops = tally().flops();
    for (int i = 0; i < 2 * N; i++) {
        const bool real = (i % 2 == 0) || types[i / 2] == MPT_PLANE || types[i / 2] == MPT_QUADRIC;
        Cnt &d = Ap[Band<N, 2>::at(i, i)];
        d = real ? d + lam * fmax(d, Cnt(1e-12) * dmax) : Cnt(1.0);
    }
    chol_band<Cnt, N, 2>(Ap);
    chol_solve_band<Cnt, N, 2>(Ap, gp);
    bool guard;
    eval_cost_param<Cnt, N, false>(sc, p, U, gp, Ct, rt, guard);
    out[0] = tally().flops();
    out[3] = tally().sqrt + tally().div;
    tally() = FlopTally();
    eval_cost_param<Cnt, N, false>(sc, p, U, nullptr, C, rinf, guard);
    out[2] = tally().flops();
}

extern "C" mpt_status mpt_flops_per_iter(int order, const int32_t *types, int32_t form, int64_t out[4])
{
    if (!types || !out || order < 1 || order > MPT_MAX_ORDER) return MPT_E_INVALID_ARG;
    if (form != MPT_FORM_IMPLICIT && form != MPT_FORM_PARAMETRIC) return MPT_E_INVALID_ARG;
    for (int k = 0; k < order; k++)
        if (types[k] < MPT_PLANE || types[k] > MPT_CIRCLE) return MPT_E_INVALID_ARG;
    const bool param = form == MPT_FORM_PARAMETRIC;
    switch (order) {
    case 1: count_one<1>(types, out, param); break;
    case 2: count_one<2>(types, out, param); break;
    case 3: count_one<3>(types, out, param); break;
    case 4: count_one<4>(types, out, param); break;
    default: count_one<5>(types, out, param); break;
    }
    return MPT_OK;
}

extern "C" mpt_status mpt_flops_assembly(int order, const int32_t *types, int32_t form, int64_t *out)
{
    if (!types || !out || order < 1 || order > MPT_MAX_ORDER) return MPT_E_INVALID_ARG;
    if (form != MPT_FORM_IMPLICIT && form != MPT_FORM_PARAMETRIC) return MPT_E_INVALID_ARG;
    for (int k = 0; k < order; k++)
        if (types[k] < MPT_PLANE || types[k] > MPT_CIRCLE) return MPT_E_INVALID_ARG;
    const bool param = form == MPT_FORM_PARAMETRIC;
    int64_t all[4];
    switch (order) {
    case 1: count_one<1>(types, all, param, out); break;
    case 2: count_one<2>(types, all, param, out); break;
    case 3: count_one<3>(types, all, param, out); break;
    case 4: count_one<4>(types, all, param, out); break;
    default: count_one<5>(types, all, param, out); break;
    }
    return MPT_OK;
}

extern "C" {

mpt_status mpt_last_timings(mpt_ctx *c, float ms[6])
{
    if (!c || !ms) return MPT_E_INVALID_ARG;
    if (!c->timed) return fail(c, MPT_E_INVALID_ARG, "no solve recorded");
    HIPCHK(c, hipEventSynchronize(c->ev[6]));
    for (int i = 0; i < 6; i++) HIPCHK(c, hipEventElapsedTime(&ms[i], c->ev[i], c->ev[i + 1]));
    return MPT_OK;
}

mpt_status mpt_set_timing(mpt_ctx *c, int32_t on)
{
    if (!c) return MPT_E_INVALID_ARG;
    c->timing = on != 0;
    return MPT_OK;
}

mpt_status mpt_last_launch(mpt_ctx *c, int32_t out[5])
{
    if (!c || !out) return MPT_E_INVALID_ARG;
    if (!c->launched) return fail(c, MPT_E_INVALID_ARG, "no solve recorded");
    memcpy(out, c->last_launch, sizeof c->last_launch);
    return MPT_OK;
}

mpt_status mpt_last_lm_timings(mpt_ctx *c, float ms[5])
{
    if (!c || !ms) return MPT_E_INVALID_ARG;
    if (!c->timed || !c->kev_valid) return fail(c, MPT_E_INVALID_ARG, "no per-order solve recorded");
    HIPCHK(c, hipEventSynchronize(c->ev[6]));
    for (int i = 0; i < MPT_MAX_ORDER; i++) HIPCHK(c, hipEventElapsedTime(&ms[i], c->kev[i][0], c->kev[i][1]));
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
    if ((st = ensure(c, (void **)&c->blk, &c->blk_cap, nblk + 1, sizeof(int)))) return st;
    OutDevC ic{in->x, in->cost, in->iters, in->status};
    launch_accept(c->s, bd, ic, tau_res, min_seg, accept, accepted_idx, d_count, c->blk, c->refr, c->stream);
    HIPCHK(c, hipGetLastError());
    if (h_count) {
        int32_t v = 0;
        HIPCHK(c, hipMemcpyAsync(&v, d_count, sizeof v, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        *h_count = v;
    }
    return MPT_OK;
}

mpt_status mpt_visible(mpt_ctx *c, const mpt_batch_desc *b, const mpt_solve_out *in, const uint8_t *accept,
                       double min_seg, uint8_t *visible, int32_t *d_count, int64_t *h_count)
{
    if (!c) return MPT_E_INVALID_ARG;
    if (!c->has_scene) return fail(c, MPT_E_NO_SCENE, "no scene uploaded");
    BatchDev bd;
    mpt_status st = batch_dev(c, b, bd);
    if (st) return st;
    if (!in || !d_count || (b->n > 0 && (!in->x || !accept || !visible)))
        return fail(c, MPT_E_INVALID_ARG, "null visibility argument");
    if (!(min_seg >= 0)) return fail(c, MPT_E_INVALID_ARG, "negative segment margin");
    hipSetDevice(c->device);
    OutDevC ic{in->x, in->cost, in->iters, in->status};
    if ((st = ensure(c, (void **)&c->vlist, &c->vlist_cap, (size_t)b->n + 1, sizeof(int)))) return st;
    launch_visible(c->s, bd, ic, accept, min_seg, visible, d_count, c->vlist, c->lds_max, c->cu, c->stream);
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
                              const int32_t *rows, int32_t n_rows, float lr, float *d_loss)
{
    if (!c) return MPT_E_INVALID_ARG;
    if (!c->has_scene) return fail(c, MPT_E_NO_SCENE, "no scene uploaded");
    if (!mlp_ready(c->mlp)) return fail(c, MPT_E_NO_MODEL, "no network initialised");
    BatchDev bd;
    mpt_status st = batch_dev(c, b, bd);
    if (st) return st;
    if (b->n > 0 && !target_x) return fail(c, MPT_E_INVALID_ARG, "null targets");
    if (!(lr >= 0.0f)) return fail(c, MPT_E_INVALID_ARG, "negative learning rate");
    const int nr = rows ? n_rows : (int)b->n;
    if (nr <= 0 || (rows && (int64_t)n_rows > b->n)) return fail(c, MPT_E_INVALID_ARG, "bad row count");
    hipSetDevice(c->device);
    st = mlp_train_step_dev(c->mlp, c->s, bd, rows, nr, target_x, use, lr, d_loss, c->stream);
    return st ? fail(c, st, "training step failed") : MPT_OK;
}

static mpt_status mlp_grad_common(mpt_ctx *c, const mpt_batch_desc *b, const double *target_x, const uint8_t *use,
                                  const int32_t *rows, int32_t n_rows, float *d_loss, float *d_grad, bool fp32)
{
    if (!c) return MPT_E_INVALID_ARG;
    if (!c->has_scene) return fail(c, MPT_E_NO_SCENE, "no scene uploaded");
    if (!mlp_ready(c->mlp)) return fail(c, MPT_E_NO_MODEL, "no network initialised");
    BatchDev bd;
    mpt_status st = batch_dev(c, b, bd);
    if (st) return st;
    if (b->n > 0 && !target_x) return fail(c, MPT_E_INVALID_ARG, "null targets");
    const int nr = rows ? n_rows : (int)b->n;
    if (nr <= 0 || (rows && (int64_t)n_rows > b->n)) return fail(c, MPT_E_INVALID_ARG, "bad row count");
    hipSetDevice(c->device);
    st = fp32 ? mlp_grad_f32_dev(c->mlp, c->s, bd, rows, nr, target_x, use, d_loss, d_grad, c->stream)
              : mlp_grad_dev(c->mlp, c->s, bd, rows, nr, target_x, use, d_loss, d_grad, c->stream);
    return st ? fail(c, st, "gradient failed") : MPT_OK;
}

mpt_status mpt_mlp_grad(mpt_ctx *c, const mpt_batch_desc *b, const double *target_x, const uint8_t *use,
                        const int32_t *rows, int32_t n_rows, float *d_loss, float *d_grad)
{
    return mlp_grad_common(c, b, target_x, use, rows, n_rows, d_loss, d_grad, false);
}

mpt_status mpt_mlp_grad_fp32(mpt_ctx *c, const mpt_batch_desc *b, const double *target_x, const uint8_t *use,
                             const int32_t *rows, int32_t n_rows, float *d_loss, float *d_grad)
{
    return mlp_grad_common(c, b, target_x, use, rows, n_rows, d_loss, d_grad, true);
}

mpt_status mpt_mlp_features(mpt_ctx *c, const mpt_batch_desc *b, float *d_feat)
{
    if (!c) return MPT_E_INVALID_ARG;
    if (!c->has_scene) return fail(c, MPT_E_NO_SCENE, "no scene uploaded");
    BatchDev bd;
    mpt_status st = batch_dev(c, b, bd);
    if (st) return st;
    if (b->n > 0 && !d_feat) return fail(c, MPT_E_INVALID_ARG, "null output");
    hipSetDevice(c->device);
    st = mlp_features_dev(c->s, bd, d_feat, c->stream);
    return st ? fail(c, st, "features failed") : MPT_OK;
}

mpt_status mpt_mlp_param_count(size_t *count)
{
    if (!count) return MPT_E_INVALID_ARG;
    *count = mlp_param_count();
    return MPT_OK;
}

mpt_status mpt_gemm_bf16_check(mpt_ctx *c, int32_t M, int32_t N, int32_t K, const float *A, int32_t a_trans,
                               const float *B, int32_t b_trans, float *C, int32_t splits)
{
    if (!c) return MPT_E_INVALID_ARG;
    if (M < 1 || N < 1 || K < 1 || splits < 1 || !A || !B || !C) return fail(c, MPT_E_INVALID_ARG, "bad GEMM args");
    hipSetDevice(c->device);
    mpt_status st = gemm_test_dev(M, N, K, A, a_trans, B, b_trans, C, splits, c->stream);
    return st ? fail(c, st, "GEMM check failed") : MPT_OK;
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

mpt_status mpt_mlp_predict_unfused(mpt_ctx *c, const mpt_batch_desc *b, double *x_out)
{
    if (!c) return MPT_E_INVALID_ARG;
    if (!c->has_scene) return fail(c, MPT_E_NO_SCENE, "no scene uploaded");
    if (!mlp_ready(c->mlp)) return fail(c, MPT_E_NO_MODEL, "no network initialised");
    BatchDev bd;
    mpt_status st = batch_dev(c, b, bd);
    if (st) return st;
    if (b->n > 0 && !x_out) return fail(c, MPT_E_INVALID_ARG, "null output");
    hipSetDevice(c->device);
    st = mlp_predict_unfused(c->mlp, c->s, bd, x_out, c->stream);
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

static mpt_status cand_samples(mpt_ctx *c, int k)
{
    mpt_status st;
    const size_t n = (size_t)c->s.n_all;
    if ((st = ensure(c, (void **)&c->samp, &c->samp_cap, n * (size_t)(k * k + 2 * k) * 3, sizeof(double)))) return st;
    if ((st = ensure(c, (void **)&c->scnt, &c->scnt_cap, n, sizeof(int)))) return st;
    launch_samples(c->s, k, c->samp, c->scnt, c->stream);
    return MPT_OK;
}

static mpt_status cand_check(mpt_ctx *c, int k, double min_seg)
{
    if (!c) return MPT_E_INVALID_ARG;
    if (!c->has_scene) return fail(c, MPT_E_NO_SCENE, "no scene uploaded");
    if (k < 1 || k > 16) return fail(c, MPT_E_INVALID_ARG, "samples per side %d outside 1..16", k);
    if (!(min_seg >= 0)) return fail(c, MPT_E_INVALID_ARG, "negative segment margin");
    if (c->s.n_all > 4096) return fail(c, MPT_E_UNSUPPORTED, "more than 4096 objects");
    return MPT_OK;
}

mpt_status mpt_visibility(mpt_ctx *c, int32_t k, double min_seg, uint32_t *vis, uint32_t *bs)
{
    mpt_status st = cand_check(c, k, min_seg);
    if (st) return st;
    if (!vis || !bs) return fail(c, MPT_E_INVALID_ARG, "null visibility output");
    hipSetDevice(c->device);
    if ((st = cand_samples(c, k))) return st;
    const int W = (c->s.n_all + 31) / 32;
    launch_visibility(c->s, k, min_seg, c->samp, c->scnt, vis, bs, W, c->lds_max, c->cu, c->stream);
    HIPCHK(c, hipGetLastError());
    return MPT_OK;
}

mpt_status mpt_visibility_rx(mpt_ctx *c, const double *rx, int32_t n_rx, int32_t k, double min_seg, uint32_t *ue,
                             uint8_t *los)
{
    mpt_status st = cand_check(c, k, min_seg);
    if (st) return st;
    if (n_rx < 0) return fail(c, MPT_E_INVALID_ARG, "negative receiver count");
    if (n_rx > 0 && (!rx || !ue)) return fail(c, MPT_E_INVALID_ARG, "null receiver argument");
    hipSetDevice(c->device);
    if ((st = cand_samples(c, k))) return st;
    const int W = (c->s.n_all + 31) / 32;
    launch_visibility_rx(c->s, k, min_seg, c->samp, c->scnt, rx, n_rx, ue, los, W, c->lds_max, c->cu, c->stream);
    HIPCHK(c, hipGetLastError());
    return MPT_OK;
}

mpt_status mpt_candidates(mpt_ctx *c, const uint32_t *vis, const uint32_t *bs, const uint32_t *ue, int32_t n_rx,
                          int32_t max_order, int32_t edge_last, int64_t cap, int32_t *rx_index, int32_t *order,
                          int32_t *prim, int64_t *h_total)
{
    mpt_status st = cand_check(c, 1, 0.0);
    if (st) return st;
    if (!h_total) return fail(c, MPT_E_INVALID_ARG, "null total");
    *h_total = 0;
    if (max_order < 1 || max_order > MPT_MAX_ORDER) return fail(c, MPT_E_INVALID_ARG, "max_order outside 1..5");
    if (n_rx < 0 || cap < 0) return fail(c, MPT_E_INVALID_ARG, "negative receiver count or capacity");
    if (n_rx > 0 && (!vis || !bs || !ue)) return fail(c, MPT_E_INVALID_ARG, "null visibility input");
    if (cap > 0 && (!rx_index || !order || !prim)) return fail(c, MPT_E_INVALID_ARG, "null candidate output");
    const int64_t n = (int64_t)n_rx * c->s.n_all * max_order;
    if (n == 0) return MPT_OK;
    hipSetDevice(c->device);
    const int W = (c->s.n_all + 31) / 32;
    const int64_t nb = (n + 1023) / 1024;
    if ((st = ensure(c, (void **)&c->ccnt, &c->ccnt_cap, (size_t)n, sizeof(int64_t)))) return st;
    if ((st = ensure(c, (void **)&c->csum, &c->csum_cap, (size_t)nb + 1, sizeof(int64_t)))) return st;
    launch_cand_count(c->s, vis, bs, ue, W, n_rx, max_order, edge_last ? 1 : 0, c->ccnt, c->csum, c->cu, c->stream);
    HIPCHK(c, hipGetLastError());
    int64_t total = 0;
    HIPCHK(c, hipMemcpyAsync(&total, c->csum + nb, sizeof total, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *h_total = total;
    if (cap == 0 || total == 0) return MPT_OK;
    if (cap < total) return fail(c, MPT_E_CAPACITY, "%lld candidates do not fit in %lld", (long long)total,
                                 (long long)cap);
    launch_cand_fill(c->s, vis, bs, ue, W, n_rx, max_order, edge_last ? 1 : 0, c->ccnt, cap, rx_index, order, prim,
                     c->cu, c->stream);
    HIPCHK(c, hipGetLastError());
    return MPT_OK;
}

}  // extern "C"
