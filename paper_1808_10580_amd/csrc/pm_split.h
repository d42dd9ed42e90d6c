// pm_split.h -- FP16 hi + lo pairs of FP32 values for the split matrix-core
// products (pm_mx.hip, pm_hk.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pm {

// FP16 pairs of two values: hi = (f16(v0), f16(v1)), one packed conversion
// rounding to nearest even, and lo = (f16(v0 - hi0), f16(v1 - hi1)), each half
// written in place by a mixed-precision FMA (v * 1 - hi is exact in the FMA,
// so lo is the correctly rounded remainder).
__device__ __forceinline__ void split_pair(float v0, float v1, uint32_t &hi, uint32_t &lo)
{
    typedef float f32x2_t __attribute__((ext_vector_type(2)));
    typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));
    const uint32_t h = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){v0, v1}, f16x2_t));
    uint32_t l;
    asm("v_fma_mixlo_f16 %0, %1, 1.0, -%2 op_sel_hi:[0,0,1]" : "=v"(l) : "v"(v0), "v"(h));
    asm("v_fma_mixhi_f16 %0, %1, 1.0, -%2 op_sel:[0,0,1] op_sel_hi:[0,0,1]" : "+v"(l) : "v"(v1), "v"(h));
    hi = h;
    lo = l;
}

}  // namespace pm
