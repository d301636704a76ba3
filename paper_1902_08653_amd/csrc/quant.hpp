// quant.hpp -- low-precision codes shared by the mixed-precision kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cdm {

// BF16 code of a real value: round to FP32 (nearest even), then keep the top 16
// bits with round-to-nearest-even on the dropped half.
__device__ __forceinline__ uint16_t bf16_code(double v) {
    const float f = (float)v;
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    uint32_t q = u >> 16;
    const uint32_t rem = u & 0xffffu;
    if (rem > 0x8000u || (rem == 0x8000u && (q & 1u))) q += 1u;
    return (uint16_t)q;
}

}  // namespace cdm
