// Device-side helpers shared by the SFOC / Fast-NCC kernels (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define SFOC_DEV __device__ __forceinline__

// Load a launch-table entry (read-only for the whole launch) through the
// constant address space.  Pointers loaded that way are known to address
// global memory, so accesses through them stay global loads and stores with
// scalar bases instead of flat ones.  The host pass never runs this.
template <class T>
SFOC_DEV T load_table(const T* p, int i) {
#if defined(__HIP_DEVICE_COMPILE__)
    return ((const __attribute__((address_space(4))) T*)p)[i];
#else
    return p[i];
#endif
}

// Reflect-101 index (mirror without repeating the edge), periodic for any i.
SFOC_DEV int reflect101(int i, int n) {
    if (n == 1) return 0;
    const int p = 2 * (n - 1);
    int j = i % p;
    if (j < 0) j += p;
    return j > n - 1 ? p - j : j;
}

// float -> bfloat16 bits, round to nearest even; NaN stays NaN.
SFOC_DEV uint16_t f32_to_bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
SFOC_DEV float bf16_bits_to_f32(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

SFOC_DEV uint16_t f32_to_f16_bits(float f) {
    _Float16 h = (_Float16)f;               // v_cvt_f16_f32, round to nearest even
    return __builtin_bit_cast(uint16_t, h);
}
SFOC_DEV float f16_bits_to_f32(uint16_t b) { return (float)__builtin_bit_cast(_Float16, b); }

// Load one descriptor element of type dt (0 f32, 1 bf16, 2 f16).
SFOC_DEV float load_desc(const void* base, int64_t idx, int dt) {
    if (dt == 0) return ((const float*)base)[idx];
    const uint16_t b = ((const uint16_t*)base)[idx];
    return dt == 1 ? bf16_bits_to_f32(b) : f16_bits_to_f32(b);
}
