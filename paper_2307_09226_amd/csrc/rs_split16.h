// Binary32 phasor primitives of the split-FP16 matrix-core form: the
// binary64 -> binary32 mod-1 reduction, the hi/lo fp16 split and the pinned
// binary32 rotation.  Shared by rs_mfma.hip and the primitive tests.
#pragma once
#include <hip/hip_runtime.h>

typedef _Float16 rs_half2v __attribute__((ext_vector_type(2)));

// frac in binary64 (v_fract_f64: v - floor(v), held below 1), then binary32
__device__ __forceinline__ float rs_frac32(double v) { return (float)__builtin_amdgcn_fract(v); }

// hi = rne16(x) for a pair, packed in one register (v_cvt_pk_f16_f32)
__device__ __forceinline__ rs_half2v rs_hi2(float x, float y) { return rs_half2v{(_Float16)x, (_Float16)y}; }

// Pins a binary32 value: the empty asm statement hides how it was produced,
// so the compiler cannot fuse a later fp16 conversion with the multiply-add
// that produced it (that would round the exact result once, to fp16).  Every
// code path then yields the same bits for the same phasor, which keeps a
// cube independent of how its steps were split over launches.
__device__ __forceinline__ void rs_pin(float &u, float &w) { asm("" : "+v"(u), "+v"(w)); }

// lo = rne16(x - hi): x - hi is exact in fp32, so the mixed-precision
// multiply-add -hi * 1 + x rounded once to fp16 gives it, one instruction per
// component (v_fma_mixlo_f16 writes bits 15:0, v_fma_mixhi_f16 bits 31:16;
// op_sel_hi marks the fp16 source, op_sel picks its half).  (Widening hi with
// v_cvt_f32_f16 and subtracting in binary32 gives the same bits but measured
// slower in the matrix-core kernel.)
__device__ __forceinline__ rs_half2v rs_lo2(float x, float y, rs_half2v h)
{
    const unsigned hb = __builtin_bit_cast(unsigned, h);
    unsigned r;
    asm("v_fma_mixlo_f16 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(hb), "v"(x));
    asm("v_fma_mixhi_f16 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "+v"(r) : "v"(hb), "v"(y));
    return __builtin_bit_cast(rs_half2v, r);
}

// (x, y) -> (-y, x): a packed fp16 pair times j.  One packed multiply by
// 1.0 with the halves swapped (op_sel picks the high half for the low result,
// op_sel_hi the low half for the high one) and the low result negated.
// Multiplying by 1.0 and negating are exact, so applied to the split of
// (x, y) it gives the split of (-y, x): rne16(-y) = -rne16(y) and
// rne16(-y - rne16(-y)) = -rne16(y - rne16(y)), bit for bit except that a
// zero lo half may come out as -0 where the direct split gives +0 (no sum
// of products changes with the sign of a zero term).
__device__ __forceinline__ rs_half2v rs_jmul(rs_half2v v)
{
    unsigned r;
    asm("v_pk_mul_f16 %0, %1, 1.0 op_sel:[1,0] op_sel_hi:[0,0] neg_lo:[1,0]"
        : "=v"(r) : "v"(__builtin_bit_cast(unsigned, v)));
    return __builtin_bit_cast(rs_half2v, r);
}

__device__ __forceinline__ unsigned rs_bits(rs_half2v v) { return __builtin_bit_cast(unsigned, v); }

// (u + j w) * (rx + j ry) in binary32
__device__ __forceinline__ void rs_rot(float &u, float &w, float rx, float ry)
{
    float un = __builtin_fmaf(u, rx, -(w * ry));
    w = __builtin_fmaf(u, ry, w * rx);
    u = un;
    rs_pin(u, w);
}
