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

// Store one real value in the representation of precision P.
template <int P>
__device__ __forceinline__ void store_val(void* hi, void* lo, size_t i, float v) {
    if constexpr (P == P_FP32) {
        static_cast<float*>(hi)[i] = v;
    } else {
        uint16_t h, l;
        split16<P>(v, h, l);
        static_cast<uint16_t*>(hi)[i] = h;
        static_cast<uint16_t*>(lo)[i] = l;
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

}  // namespace cgh
