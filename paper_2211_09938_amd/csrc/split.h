// Rounding helpers for the split-precision operand forms: v = hi + lo with
// hi = round_to_nearest_even_16bit(v) and lo = round_to_nearest_even_16bit(v - hi).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace cgh {

__device__ __forceinline__ uint16_t bf16_bits_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_bits_to_float(uint16_t b) {
    return __uint_as_float(((uint32_t)b) << 16);
}
__device__ __forceinline__ uint16_t f16_bits_rne(float f) {
    _Float16 h = (_Float16)f;  // round to nearest even
    return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float f16_bits_to_float(uint16_t b) {
    return (float)__builtin_bit_cast(_Float16, b);
}

template <int P>
__device__ __forceinline__ void split16(float v, uint16_t& hi, uint16_t& lo) {
    if constexpr (P == P_BF16) {
        hi = bf16_bits_rne(v);
        lo = bf16_bits_rne(v - bf16_bits_to_float(hi));
    } else {
        hi = f16_bits_rne(v);
        lo = f16_bits_rne(v - f16_bits_to_float(hi));
    }
}

// Store one complex / real operand element into planar operand storage:
// FP32 planes (re, im) or split planes (re_hi, re_lo, im_hi, im_lo) / (hi, lo),
// plane stride ps elements.
template <int P>
__device__ __forceinline__ void put_c(void* base, size_t ps, size_t off, float re, float im) {
    if constexpr (P == P_FP32) {
        float* b = static_cast<float*>(base);
        b[off] = re;
        b[ps + off] = im;
    } else {
        uint16_t* b = static_cast<uint16_t*>(base);
        uint16_t h, l;
        split16<P>(re, h, l);
        b[off] = h;
        b[ps + off] = l;
        split16<P>(im, h, l);
        b[2 * ps + off] = h;
        b[3 * ps + off] = l;
    }
}

// Real value -> planes (FP32: one plane; split: hi, lo).
template <int P>
__device__ __forceinline__ void put_r(void* base, size_t ps, size_t off, float v) {
    if constexpr (P == P_FP32) {
        static_cast<float*>(base)[off] = v;
    } else {
        uint16_t* b = static_cast<uint16_t*>(base);
        uint16_t h, l;
        split16<P>(v, h, l);
        b[off] = h;
        b[ps + off] = l;
    }
}

// Four consecutive complex / real elements (off a multiple of 4, 16-byte
// aligned planes): one vector store per plane.
template <int P>
__device__ __forceinline__ void put_c4(void* base, size_t ps, size_t off, const float* re,
                                      const float* im) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    if constexpr (P == P_FP32) {
        float* b = static_cast<float*>(base);
        *reinterpret_cast<f4*>(b + off) = f4{re[0], re[1], re[2], re[3]};
        *reinterpret_cast<f4*>(b + ps + off) = f4{im[0], im[1], im[2], im[3]};
    } else {
        uint16_t* b = static_cast<uint16_t*>(base);
        unsigned rh[4], rl[4], ih[4], il[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint16_t h, l;
            split16<P>(re[q], h, l);
            rh[q] = h;
            rl[q] = l;
            split16<P>(im[q], h, l);
            ih[q] = h;
            il[q] = l;
        }
        *reinterpret_cast<u2*>(b + off) = u2{rh[0] | (rh[1] << 16), rh[2] | (rh[3] << 16)};
        *reinterpret_cast<u2*>(b + ps + off) = u2{rl[0] | (rl[1] << 16), rl[2] | (rl[3] << 16)};
        *reinterpret_cast<u2*>(b + 2 * ps + off) = u2{ih[0] | (ih[1] << 16), ih[2] | (ih[3] << 16)};
        *reinterpret_cast<u2*>(b + 3 * ps + off) = u2{il[0] | (il[1] << 16), il[2] | (il[3] << 16)};
    }
}

template <int P>
__device__ __forceinline__ void put_r4(void* base, size_t ps, size_t off, const float* v) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    if constexpr (P == P_FP32) {
        *reinterpret_cast<f4*>(static_cast<float*>(base) + off) = f4{v[0], v[1], v[2], v[3]};
    } else {
        uint16_t* b = static_cast<uint16_t*>(base);
        unsigned h4[4], l4[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint16_t h, l;
            split16<P>(v[q], h, l);
            h4[q] = h;
            l4[q] = l;
        }
        *reinterpret_cast<u2*>(b + off) = u2{h4[0] | (h4[1] << 16), h4[2] | (h4[3] << 16)};
        *reinterpret_cast<u2*>(b + ps + off) = u2{l4[0] | (l4[1] << 16), l4[2] | (l4[3] << 16)};
    }
}

}  // namespace cgh
