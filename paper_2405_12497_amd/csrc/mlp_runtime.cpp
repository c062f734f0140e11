// Learned per-query nprobe (placeholder until the MLP kernels land).
#include "rbq_runtime.hpp"

namespace rbq {
rbq_status learned_nprobe(rbq_index*, const float*, int64_t, int, int64_t, hipStream_t,
                          const int32_t** out) {
  *out = nullptr;
  return RBQ_OK;
}
}  // namespace rbq

extern "C" {
rbq_status rbq_nprobe_features(rbq_index*, const float*, int64_t, int64_t, float*, void*) { return RBQ_EUNSUPPORTED; }
rbq_status rbq_nprobe_model_train(rbq_index*, const float*, const int32_t*, int64_t, const rbq_train_cfg*, float*, void*) { return RBQ_EUNSUPPORTED; }
rbq_status rbq_nprobe_model_set(rbq_index*, const float*, float) { return RBQ_EUNSUPPORTED; }
rbq_status rbq_nprobe_model_get(const rbq_index*, float*, float*) { return RBQ_EUNSUPPORTED; }
rbq_status rbq_nprobe_predict(rbq_index*, const float*, int64_t, int32_t*, float*, void*) { return RBQ_EUNSUPPORTED; }
rbq_status rbq_mlp_loss_grad(const float*, const int32_t*, int64_t, const float*, float*, float*, void*) { return RBQ_EUNSUPPORTED; }
rbq_status rbq_autotune(rbq_index*, const float*, int64_t, int32_t, int32_t, void*) { return RBQ_EUNSUPPORTED; }
}
