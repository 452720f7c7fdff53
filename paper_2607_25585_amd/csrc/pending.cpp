// Entry points whose implementation lands in later files of this library.
#include "ftlm_internal.hpp"

using namespace ftlm;

extern "C" {

int ftlm_mlp_workspace_size(int32_t, size_t *) { set_error("not available"); return FTLM_EINVAL; }
int ftlm_mlp_forward(const ftlm_mlp_weights *, int32_t, const float *, float *, void *, size_t,
                     void *) { set_error("not available"); return FTLM_EINVAL; }
int ftlm_mlp_backward(const ftlm_mlp_weights *, int32_t, const float *, float *, float *const[4],
                      float *const[4], void *, size_t, void *) { set_error("not available"); return FTLM_EINVAL; }
int ftlm_adam_step(int64_t, float *, const float *, float *, float *, uint16_t *, float, float,
                   float, float, int32_t, void *) { set_error("not available"); return FTLM_EINVAL; }
}
