// Host-side interface of the contraction kernels (internal).
#pragma once

#include "common.h"

namespace cgh {

constexpr int kTileM = 128;  // output tile rows
constexpr int kTileN = 128;  // output tile columns (complex)
constexpr int kTileK = 16;   // K tile

struct GemmShape {
    int ny, nx, layers, levels, split_k;
    int precision;       // cgh_precision of both contractions
    size_t t_layer;      // complex elements of T per layer
    size_t flags_layer;  // flag bytes per layer
};

hipError_t launch_reduce_partial(const GemmShape& sh, const float2* partial, float2* out,
                                 int accumulate, hipStream_t s);

hipError_t launch_backward(const GemmShape& sh, const float2* grad_h, const float* lut_x,
                               const float* lut_y, float2* q, float* gcoef, hipStream_t s);

}  // namespace cgh
