// md_extras.cpp -- teardown hooks for the per-context subsystems.
#include "md_ctx.h"

namespace md {

void destroy_extras(md_ctx *ctx) { free_surrogate(ctx); }

void invalidate_layout_users(md_ctx *ctx) { (void)ctx; }

}  // namespace md
