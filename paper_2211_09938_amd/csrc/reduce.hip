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

// Two complex values per lane (16-byte loads and stores: n even, partial and out 16-byte
// aligned): the same sums as reduce_partial_kernel.
__global__ __launch_bounds__(256) void reduce_partial2_kernel(const float4* __restrict__ partial,
                                                              int split, size_t n2, int accumulate,
                                                              float4* __restrict__ out) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n2; i += stride) {
        float4 v = accumulate ? out[i] : make_float4(0.f, 0.f, 0.f, 0.f);
        for (int s = 0; s < split; ++s) {
            const float4 p = partial[(size_t)s * n2 + i];
            v.x += p.x;
            v.y += p.y;
            v.z += p.z;
            v.w += p.w;
        }
        out[i] = v;
    }
}

// Largest |x[i]| over n floats into *word (float bits, atomicMax; cleared by the
// caller).  Every lane reaches the reductions (no early exit); one atomic per
// workgroup, few workgroups: atomics on one address serialise (one per wave of a
// 1024-workgroup grid had cost 49 us for 8 MB).
__global__ __launch_bounds__(256) void absmax_kernel(const float* __restrict__ x, size_t n,
                                                     unsigned long long* __restrict__ word) {
    __shared__ float s_max[4];
    float m = 0.f;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t n4 = (reinterpret_cast<uintptr_t>(x) & 15) == 0 ? n / 4 : 0;
    const float4* x4 = reinterpret_cast<const float4*>(x);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
        const float4 v = x4[i];
        m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
    }
    for (size_t i = 4 * n4 + (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        m = fmaxf(m, fabsf(x[i]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if (__lane_id() == 0) s_max[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        m = fmaxf(fmaxf(s_max[0], s_max[1]), fmaxf(s_max[2], s_max[3]));
        if (m > 0.f) atomicMax(word, (unsigned long long)__float_as_uint(m));
    }
}

}  // namespace

hipError_t launch_absmax(const float* x, size_t n, unsigned long long* word, hipStream_t s) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n / 4 + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 256) blocks = 256;
    hipLaunchKernelGGL(absmax_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, n, word);
    return hipGetLastError();
}

hipError_t launch_reduce_partial(int ny, int nx, int split, const float2* partial, float2* out,
                                 int accumulate, hipStream_t s) {
    if (split <= 1) return hipSuccess;
    const size_t n = (size_t)ny * nx;
    if (n % 2 == 0 && ((reinterpret_cast<uintptr_t>(partial) | reinterpret_cast<uintptr_t>(out)) & 15) == 0) {
        const size_t n2 = n / 2;
        size_t blocks = (n2 + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        hipLaunchKernelGGL(reduce_partial2_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                           reinterpret_cast<const float4*>(partial), split, n2, accumulate,
                           reinterpret_cast<float4*>(out));
        return hipGetLastError();
    }
    size_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(reduce_partial_kernel, dim3((unsigned)blocks), dim3(256), 0, s, partial,
                       split, n, accumulate, out);
    return hipGetLastError();
}

}  // namespace cgh
