// Learned warm start (placeholder until the network kernels land).
#include "mpt_mlp.hpp"

namespace mpt {

struct MlpState {
    int dummy;
};

bool mlp_ready(const MlpState *m) { return m != nullptr; }
void mlp_free(MlpState *m) { delete m; }
mpt_status mlp_init(MlpState **, uint64_t, hipStream_t) { return MPT_E_UNSUPPORTED; }
mpt_status mlp_predict_dev(MlpState *, const SceneDev &, const BatchDev &, double *, hipStream_t) { return MPT_E_UNSUPPORTED; }
mpt_status mlp_train_step_dev(MlpState *, const SceneDev &, const BatchDev &, const double *, const uint8_t *, float,
                              float *, hipStream_t)
{
    return MPT_E_UNSUPPORTED;
}
mpt_status mlp_save(MlpState *, void *, size_t *, hipStream_t) { return MPT_E_UNSUPPORTED; }
mpt_status mlp_load(MlpState **, const void *, size_t, hipStream_t) { return MPT_E_UNSUPPORTED; }

}  // namespace mpt
