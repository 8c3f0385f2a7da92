// q10_blend.h -- the integer bilinear blend of packed u8 pixels shared by the
// u8 warp chain and the remap chain.
#pragma once
#include "dev_common.h"

namespace miaug {

// Bilinear blend of four packed pixels of C bytes with Q10 weights, rounded
// half to even per channel (2^20 is the product of the weights' scales): the
// row sums t = a0 (1024 - ax) + a1 ax take one byte permute (the two bytes into
// 16-bit lanes) and one packed 16-bit dot product, exact in int32; then
// t0 (1024 - ay) + t1 ay with 24-bit multiplies.  wx = q10_pair(ax).  Bytes of
// the taps above C are ignored; those of the result are 0.
typedef short q10_short2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t q10_pair(int ax) { return (uint32_t)(kFOne - ax) | (uint32_t)ax << 16; }
template <int C>
__device__ __forceinline__ uint32_t blend_q10(uint32_t p00, uint32_t p01, uint32_t p10, uint32_t p11, uint32_t wx,
                                              int ay) {
    const q10_short2 w = __builtin_bit_cast(q10_short2, wx);
    uint32_t out = 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const uint32_t sel = (uint32_t)c | 0x0c00u | (uint32_t)(4 + c) << 16 | 0x0c000000u;
        const uint32_t t0 = (uint32_t)__builtin_amdgcn_sdot2(
            __builtin_bit_cast(q10_short2, __builtin_amdgcn_perm(p01, p00, sel)), w, 0, false);
        const uint32_t t1 = (uint32_t)__builtin_amdgcn_sdot2(
            __builtin_bit_cast(q10_short2, __builtin_amdgcn_perm(p11, p10, sel)), w, 0, false);
        const uint32_t acc = umad24(t0, (uint32_t)(kFOne - ay), umad24(t1, (uint32_t)ay, 0u));
        out |= ((acc + 0x7FFFFu + ((acc >> 20) & 1u)) >> 20) << (8 * c);
    }
    return out;
}

}  // namespace miaug
