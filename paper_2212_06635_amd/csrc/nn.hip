// Learned gauge-covariant preconditioner (entry points; kernels land next).
#include "tmx_ctx.h"

using namespace tmx;

extern "C" {

void tmx_pc_free(tmx_ctx *c) { (void)c; }

int tmx_fgcr_solve_internal(tmx_ctx *c, SpinorPtr, SpinorPtr, const tmx_solver_cfg *, tmx_info *)
{
    return set_err(c, TMX_EINVAL, "FGCR with the learned preconditioner is not available yet");
}

int tmx_pc_num_params(const tmx_ctx *c, size_t *n)
{
    (void)c;
    (void)n;
    return TMX_EINVAL;
}
int tmx_pc_set_weights(tmx_ctx *c, const float *, size_t) { return set_err(c, TMX_EINVAL, "not available yet"); }
int tmx_pc_get_weights(tmx_ctx *c, float *, size_t) { return set_err(c, TMX_EINVAL, "not available yet"); }
int tmx_pc_apply(tmx_ctx *c, double *, const double *, int) { return set_err(c, TMX_EINVAL, "not available yet"); }
int tmx_pc_train(tmx_ctx *c, const double *, const double *, int, const tmx_train_cfg *, float *)
{
    return set_err(c, TMX_EINVAL, "not available yet");
}

}  // extern "C"
