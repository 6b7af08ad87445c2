// Split-K reduction of partial holograms: out (+)= sum over the splits.
#include "common.h"

namespace cgh {

namespace {

__global__ __launch_bounds__(256) void reduce_partial_kernel(const float2* __restrict__ partial,
                                                             int split, size_t n, int accumulate,
                                                             float2* __restrict__ out) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) {
        float2 v = accumulate ? out[i] : make_float2(0.f, 0.f);
        for (int s = 0; s < split; ++s) {
            const float2 p = partial[(size_t)s * n + i];
            v.x += p.x;
            v.y += p.y;
        }
        out[i] = v;
    }
}

}  // namespace

hipError_t launch_reduce_partial(int ny, int nx, int split, const float2* partial, float2* out,
                                 int accumulate, hipStream_t s) {
    if (split <= 1) return hipSuccess;
    const size_t n = (size_t)ny * nx;
    size_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(reduce_partial_kernel, dim3((unsigned)blocks), dim3(256), 0, s, partial,
                       split, n, accumulate, out);
    return hipGetLastError();
}

}  // namespace cgh
