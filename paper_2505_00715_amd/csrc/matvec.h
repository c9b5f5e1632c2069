// Entry points of the compressed (3D-ACA) products, used by the API dispatcher
// and by the solver.
#pragma once
#include "internal.h"

namespace gcq {
// mode GCQ_PER_FREQUENCY or GCQ_WEIGHTED_SUM; X, Y in the caller's layout
int run_compressed(gcq_context* ctx, int mode, int precision, const void* X, void* Y);
// the per-frequency product split for capture: buffers and tables first, then
// its kernels on a stream (no allocation, no host transfer)
int prepare_perfreq(gcq_context* ctx, int precision);
// tile_mask (device, one int per 32-column frequency tile, may be NULL): tiles
// whose entry is 0 may be skipped, their output columns left undefined (the
// split-bf16 product skips them; the others compute every column)
void enqueue_perfreq_any(gcq_context* ctx, hipStream_t s, int precision, const void* X, void* Y,
                         const int* tile_mask = nullptr);
// split-bf16 per-frequency product (matvec_bf16.hip): the operator's bf16
// copy (once per operator), the size of the product's buffers (ctx->F.pxy),
// and the product's kernels on a stream (capturable: no allocation)
int bf16_setup(gcq_context* ctx);
size_t bf16_buffer_bytes(gcq_context* ctx);
void enqueue_perfreq_bf16(gcq_context* ctx, hipStream_t st, const void* X, void* Y,
                          const int* tile_mask = nullptr);
}  // namespace gcq
