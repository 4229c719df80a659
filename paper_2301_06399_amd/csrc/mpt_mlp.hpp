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
mpt_status mlp_predict_dev(MlpState *m, const SceneDev &s, const BatchDev &b, double *x_out, hipStream_t st);
mpt_status mlp_train_step_dev(MlpState *m, const SceneDev &s, const BatchDev &b, const double *target_x,
                              const uint8_t *use, float lr, float *d_loss, hipStream_t st);
mpt_status mlp_save(MlpState *m, void *blob, size_t *bytes, hipStream_t st);
mpt_status mlp_load(MlpState **m, const void *blob, size_t bytes, hipStream_t st);

}  // namespace mpt
