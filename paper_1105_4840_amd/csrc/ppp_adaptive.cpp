// Entry points of include/ppp.h not built yet in this library version.
#include "ppp.h"
extern "C" {
ppp_status ppp_mlp_forward(const float *, const float *, int32_t, float *, float *, void *) { return PPP_E_UNSUPPORTED; }
ppp_status ppp_mlp_grad(const float *, const float *, const float *, const float *, const float *, const float *, int32_t,
                        float *, float *, void *) { return PPP_E_UNSUPPORTED; }
ppp_status ppp_mlp_adam(float *, const float *, float *, float *, float, int32_t, void *) { return PPP_E_UNSUPPORTED; }
ppp_status ppp_adaptive_workspace_size(const ppp_problem *, const ppp_adaptive *, size_t *) { return PPP_E_UNSUPPORTED; }
ppp_status ppp_adaptive_run(const ppp_problem *, const ppp_adaptive *, void *, size_t, void *, double *, int32_t *,
                            int64_t *, ppp_result *) { return PPP_E_UNSUPPORTED; }
}
