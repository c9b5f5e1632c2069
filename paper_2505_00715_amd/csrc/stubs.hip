// Entry points not implemented yet: they return GCQ_ERR_UNSUPPORTED.
#include "internal.h"
using namespace gcq;
extern "C" {
GCQ_API int gcq_solve(gcq_context*, const void*, void*, double, int32_t, int32_t, int32_t, gcq_solve_stats*) { return fail(GCQ_ERR_UNSUPPORTED, "not implemented"); }
GCQ_API int gcq_rank_features(gcq_context*, const int32_t*, int32_t, float*) { return fail(GCQ_ERR_UNSUPPORTED, "not implemented"); }
GCQ_API int gcq_rank_model_train(gcq_context*, const float*, const float*, int64_t, const gcq_train_cfg*, gcq_train_stats*) { return fail(GCQ_ERR_UNSUPPORTED, "not implemented"); }
GCQ_API int gcq_rank_model_grad(gcq_context*, const float*, const float*, int64_t, float*, float*) { return fail(GCQ_ERR_UNSUPPORTED, "not implemented"); }
GCQ_API int gcq_rank_model_predict(gcq_context*, const float*, int64_t, float*) { return fail(GCQ_ERR_UNSUPPORTED, "not implemented"); }
GCQ_API int gcq_rank_model_get(gcq_context*, float*, float*, float*) { return fail(GCQ_ERR_UNSUPPORTED, "not implemented"); }
GCQ_API int gcq_rank_model_set(gcq_context*, const float*, const float*, const float*) { return fail(GCQ_ERR_UNSUPPORTED, "not implemented"); }
}
