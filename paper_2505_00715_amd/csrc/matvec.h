// Entry points of the compressed (3D-ACA) products, used by the API dispatcher
// and by the solver.
#pragma once
#include "internal.h"

namespace gcq {
// mode GCQ_PER_FREQUENCY or GCQ_WEIGHTED_SUM; X, Y in the caller's layout
int run_compressed(gcq_context* ctx, int mode, int precision, const void* X, void* Y);
}  // namespace gcq
