// Learned warm start: network state and its device entry points.
#pragma once
#include <stddef.h>
#include <stdint.h>
#include "../../include/mpt.h"
#include "mpt_internal.hpp"

namespace mpt {

struct MlpState;

bool mlp_ready(const MlpState *m);
void mlp_free(MlpState *m);
mpt_status mlp_init(MlpState **m, uint64_t seed, hipStream_t st);
mpt_status mlp_predict_dev(MlpState *m, const SceneDev &s, const BatchDev &b, double *x_out, hipStream_t st,
                           const int *rows = nullptr, const int *count = nullptr);
mpt_status mlp_predict_unfused(MlpState *m, const SceneDev &s, const BatchDev &b, double *x_out, hipStream_t st);
mpt_status mlp_train_step_dev(MlpState *m, const SceneDev &s, const BatchDev &b, const int *rows, int nrows,
                              const double *target, const uint8_t *use, float lr, float *d_loss, hipStream_t st);
mpt_status mlp_grad_dev(MlpState *m, const SceneDev &s, const BatchDev &b, const int *rows, int nrows,
                        const double *target, const uint8_t *use, float *d_loss, float *d_grad, hipStream_t st);
mpt_status mlp_grad_f32_dev(MlpState *m, const SceneDev &s, const BatchDev &b, const int *rows, int nrows,
                            const double *target, const uint8_t *use, float *d_loss, float *d_grad, hipStream_t st);
mpt_status mlp_features_dev(const SceneDev &s, const BatchDev &b, float *fout, hipStream_t st);
mpt_status gemm_test_dev(int M, int N, int K, const float *A, int at, const float *B, int bt, float *C, int splits,
                         hipStream_t st);
size_t mlp_param_count();
mpt_status mlp_save(MlpState *m, void *blob, size_t *bytes, hipStream_t st);
mpt_status mlp_load(MlpState **m, const void *blob, size_t bytes, hipStream_t st);

}  // namespace mpt
