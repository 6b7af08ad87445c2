// Matrix-core throughput probe (diagnostics, not part of the hologram path).
//
// Each wave runs a register-resident loop of MFMAs on eight independent
// accumulator sets, with no memory traffic inside the loop, so the launch
// measures what the matrix cores of this chip sustain under dense load: the
// attainable rate against which the contractions' roofline fractions can be
// read beside the published peak.  Operands are either pseudo-random bit
// patterns that change from one MFMA to the next (four A and four B operand
// sets in rotation, as a contraction's operands do) or all zeros; the power a
// matrix core draws depends on how many operand bits toggle, so the two show
// whether a power limit, rather than the issue rate, sets the attainable rate.
#include "common.h"

namespace cgh {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kChains = 8;  // independent accumulators per wave
constexpr int kSets = 4;    // operand sets in rotation

// splitmix-style hash: a fixed pseudo-random word per (lane, set, word)
__device__ __forceinline__ unsigned hash32(unsigned x) {
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

// A pair of random 16-bit floats of magnitude in [0.5, 2) with random signs and
// mantissas: random sign, mantissa and lowest exponent bit over exponent 2^-1.
__device__ __forceinline__ unsigned rand_pair16(unsigned h, bool bf16) {
    // bf16: sign 1, exponent 8, mantissa 7; f16: sign 1, exponent 5, mantissa 10
    const unsigned mant = bf16 ? 0x007F007FU : 0x03FF03FFU;
    const unsigned sign = 0x80008000U;
    const unsigned expo = bf16 ? 0x3F003F00U : 0x38003800U;  // 2^-1; the random low exponent bit gives [0.5, 2)
    const unsigned e1 = bf16 ? 0x00800080U : 0x04000400U;
    return (h & (mant | sign | e1)) | expo;
}

template <int KIND>
__global__ __launch_bounds__(256) void mfma_peak_kernel(int iters, int zero, float* __restrict__ sink) {
    const unsigned gid = blockIdx.x * 256u + threadIdx.x;
    floatx16 acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[c][r] = 0.f;

    if constexpr (KIND == 0) {
        float a[kSets], b[kSets];
#pragma unroll
        for (int t = 0; t < kSets; ++t) {
            const unsigned ha = hash32(gid * 8u + t), hb = hash32(gid * 8u + 4u + t);
            // magnitude in [0.5, 2), random sign and mantissa
            a[t] = zero ? 0.f : __uint_as_float((ha & 0x807FFFFFU) | 0x3F000000U | (ha & 0x00800000U));
            b[t] = zero ? 0.f : __uint_as_float((hb & 0x807FFFFFU) | 0x3F000000U | (hb & 0x00800000U));
        }
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int t = 0; t < kSets; ++t)
#pragma unroll
                for (int c = 0; c < kChains; ++c)
                    acc[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[t], b[(t + c) & (kSets - 1)],
                                                                  acc[c], 0, 0, 0);
        }
    } else {
        u32x4 a[kSets], b[kSets];
#pragma unroll
        for (int t = 0; t < kSets; ++t)
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const unsigned ha = hash32(gid * 32u + t * 4u + w);
                const unsigned hb = hash32(gid * 32u + 16u + t * 4u + w);
                a[t][w] = zero ? 0u : rand_pair16(ha, KIND == 1);
                b[t][w] = zero ? 0u : rand_pair16(hb, KIND == 1);
            }
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int t = 0; t < kSets; ++t)
#pragma unroll
                for (int c = 0; c < kChains; ++c) {
                    const u32x4 x = a[t], y = b[(t + c) & (kSets - 1)];
                    if constexpr (KIND == 1)
                        acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            __builtin_bit_cast(bf16x8, x), __builtin_bit_cast(bf16x8, y), acc[c], 0,
                            0, 0);
                    else
                        acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                            __builtin_bit_cast(halfx8, x), __builtin_bit_cast(halfx8, y), acc[c], 0,
                            0, 0);
                }
        }
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < kChains; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) s += acc[c][r];
    sink[gid] = s;  // keeps every MFMA live
}

}  // namespace

double mfma_peak_flops(int kind, int blocks, int iters) {
    const double per = kind == 0 ? 2.0 * 32 * 32 * 2 : 2.0 * 32 * 32 * 16;
    return per * (double)blocks * 4.0 * (double)iters * kSets * kChains;
}

hipError_t launch_mfma_peak(int kind, int zero, int blocks, int iters, float* sink, hipStream_t s) {
    if (kind == 0)
        hipLaunchKernelGGL(mfma_peak_kernel<0>, dim3(blocks), dim3(256), 0, s, iters, zero, sink);
    else if (kind == 1)
        hipLaunchKernelGGL(mfma_peak_kernel<1>, dim3(blocks), dim3(256), 0, s, iters, zero, sink);
    else
        hipLaunchKernelGGL(mfma_peak_kernel<2>, dim3(blocks), dim3(256), 0, s, iters, zero, sink);
    return hipGetLastError();
}

}  // namespace cgh
