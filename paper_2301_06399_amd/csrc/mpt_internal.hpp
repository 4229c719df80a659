// Internal interfaces shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "mpt_device.hpp"

namespace mpt {

enum : int { MODE_PLAIN64 = 0, MODE_FP32 = 1, MODE_FALLBACK64 = 2 };
enum : int { INIT_LINE = 0, INIT_USER = 1, INIT_LEARNED = 2, INIT_LEARNED_ALL = 3, INIT_RANDOM = 4 };
// transient status codes between the FP32 pass and the polish
enum : int { ROUTE_POLISH_FB = 254, ROUTE_POLISH_MAXIT = 253, ROUTE_POLISH_LOCALMIN = 252 };

// Scene as the kernels see it (device pointers).
struct SceneDev {
    const double *rec64;  // [n_all][kRec] world frame
    const float *rec32;   // [n_all][kRec] TX-local frame
    int n_pl, n_pl_ln, n_pl_ln_q, n_all;
    double tx[3];
    double glo[3], ghi[3];  // guard box
    double lo[3], hi[3];    // scene box (random starts)
    const double *wedge;    // [n_pl_ln - n_pl][7] wedges of the straight edges, or null
    const double *side;     // [n_pl] free side of each facet (+1, -1, 0), or null
};

struct BatchDev {
    int64_t n;
    int n_rx;
    const double *rx;
    const int *rx_index;
    const int *order;
    const int *prim;
    const double *x0;
};

struct OutDev {
    double *x;
    double *cost;
    int *iters;
    uint8_t *status;
    int *stage;  // [3][n] or null
};

struct OutDevC {
    const double *x;
    const double *cost;
    const int *iters;
    const uint8_t *status;
};

struct OptsDev {
    int init, max_iter, max_iter32, max_iter32_planar, max_iter_fb, polish_steps, fallback, plateau_win;
    double plateau_frac, tol_step, tol_res, tau_root, lambda0, tol_step32, tol_res32, tau_root32, polish_gate;
    uint64_t seed;
    double stat_tol;
    int stat_win;
    double extent_skip;  // FP32 end points this far (m) outside a finite extent skip the polish (<= 0: off)
};

// Everything a solver kernel needs, passed by value.
struct KParams {
    SceneDev s;
    BatchDev b;
    OutDev out;
    OptsDev o;
    const double *x0_learned;  // [n][kRow] network start points (world)
    const int *bin_cnt;        // [5] solves per order
    const int *perm;           // [n] solve ids grouped by order (bin order)
    const int *slot_rx;        // [n] receiver of each bin slot
    const int *slot_prim;      // [5][n] primitive ids of each bin slot
    int *head;                 // [10] work counters: bins, fallback lists
    int *pol_cnt;              // [5]
    int *pol_list;             // [n] polish lists (bin-relative slots)
    int *fb_cnt;               // [5]
    int *fb_list;              // [n] fallback lists (bin-relative slots)
    int spill_t;               // park a drained bin's busy lanes when at most this many (0: never)
    int refill;                // a wave takes new paths once at least this many lanes are idle
    int resume;                // 1: this launch finishes the parked paths
    int *spill_cnt;            // [5] parked paths per order
    int *spill_head;           // [5] work counters of the straggler pass
    int *spill_list;           // [n] parked paths (bin-relative slots)
    double *spill_f;           // [2][n] damping and plateau reference of a parked path
};

void launch_pack(const double *raw, const double *refr, const SceneDev &s, int n_pl, int n_ln, int n_q, int n_c,
                 hipStream_t st);
void launch_zero(int *p, int n, hipStream_t st);
int bin_key_count();
// rows (or null): the list of the solves with a paraboloid or a circle,
// grouped by order; curved: [5] per-order cursors, and curved[25] receives
// the list's length
void launch_bin(const BatchDev &b, const OutDev &out, const SceneDev &s, int *bin_cnt, int *keys, int *perm,
                int *slot_rx, int *slot_prim, int *rows, int *curved, hipStream_t st);
const void *lm_kernel(int mode, int order, bool lds, int form, bool refr);
void launch_lm(int mode, int order, bool lds, int form, bool refr, size_t lds_bytes, const KParams &kp, int grid,
               int block, hipStream_t st);
const void *polish_kernel(bool refr);
void launch_learned_choose(const SceneDev &s, const BatchDev &b, const int *rows, const int *count, bool all,
                           double *x0l, double gain, bool refr, hipStream_t st);
void launch_polish(const KParams &kp, bool refr, int grid, int block, hipStream_t st);
void launch_polish_list(const KParams &kp, hipStream_t st);
void launch_samples(const SceneDev &s, int k, double *samp, int *cnt, hipStream_t st);
void launch_visibility(const SceneDev &s, int k, double min_seg, const double *samp, const int *cnt, uint32_t *V,
                       uint32_t *B, int W, size_t lds_max, int cu, hipStream_t st);
void launch_visibility_rx(const SceneDev &s, int k, double min_seg, const double *samp, const int *cnt,
                          const double *rx, int n_rx, uint32_t *U, uint8_t *los, int W, size_t lds_max, int cu,
                          hipStream_t st);
void launch_cand_count(const SceneDev &s, const uint32_t *V, const uint32_t *B, const uint32_t *U, int W, int n_rx,
                       int maxo, int edge_last, int64_t *cnt, int64_t *sums, int cu, hipStream_t st);
void launch_cand_fill(const SceneDev &s, const uint32_t *V, const uint32_t *B, const uint32_t *U, int W, int n_rx,
                      int maxo, int edge_last, const int64_t *off, int64_t cap, int32_t *rx_index, int32_t *order,
                      int32_t *prim, int cu, hipStream_t st);
void launch_visible(const SceneDev &s, const BatchDev &b, const OutDevC &in, const uint8_t *acc, double min_seg,
                    uint8_t *vis, int *count, int *list, size_t lds_max, int cu, hipStream_t st);
void launch_accept(const SceneDev &s, const BatchDev &b, const OutDevC &in, double tau_res, double min_seg,
                   uint8_t *acc, int *idx, int *count, int *block_cnt, bool refr, hipStream_t st);

}  // namespace mpt
