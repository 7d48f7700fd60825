// md_extras.cpp -- per-context subsystems that are optional for the plain step.
#include "md_ctx.h"

namespace md {

void destroy_extras(md_ctx *ctx) { (void)ctx; }

void invalidate_layout_users(md_ctx *ctx) { (void)ctx; }

md_status surrogate_step(md_ctx *ctx, const md_state *, const float *, int, float *, int, int, int64_t,
                         hipStream_t) {
    ctx->err = "md_step: surrogate weights not loaded";
    return MD_E_UNSUPPORTED;
}

}  // namespace md
