// Learned preconditioner (placeholder until the network kernels land).
#include "internal.hpp"

int mlp_precond_ready(lobpcg_ctx *ctx) {
    if (!ctx->mlp) return set_err(ctx, LOBPCG_EINVAL, "no MLP attached to this context");
    return LOBPCG_OK;
}

int launch_mlp_precond(lobpcg_ctx *ctx, const void *R, const double *theta, void *W, int k, hipStream_t s) {
    (void)R; (void)theta; (void)W; (void)k; (void)s;
    return set_err(ctx, LOBPCG_EUNSUPPORTED, "MLP preconditioner not built");
}
