// Device helpers shared by the stencil kernels: 2-element vectors, buffer
// loads, the LDS-only barrier and the reciprocal-based quotient.
#pragma once

#include "mgp_kernels.hpp"

namespace mgp {

template <typename T>
struct Vec2;
template <>
struct Vec2<double> {
    using type = double2;
};
template <>
struct Vec2<float> {
    using type = float2;
};

// LDS-only barrier: waits for this wave's LDS operations, then synchronises the
// workgroup.  Outstanding global loads stay in flight (a full __syncthreads
// would drain them).
__device__ inline void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Quotient n/d from the hardware reciprocal.  FP32: n * rcp(d), about 1 ulp
// and not refined: the FP32 division is that of the smoother of the mixed
// V-cycle, whose rounding the FP64 defect correction around it removes.  FP64:
// the reciprocal estimate is refined by two Newton-Raphson steps for 1/d,
// r <- r + r (1 - d r), and the quotient by one residual correction,
// q <- q + r (n - d q), each with a fused multiply-add: the iteration of
// P. Markstein, "Computation of elementary functions on the IBM RISC System/6000
// processor", IBM J. Res. Develop. 34(1), 1990; within 1 ulp of the correctly
// rounded quotient.  d > 0 here.
__device__ __forceinline__ float quot(float n, float d) { return n * __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double quot(double n, double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    r = fma(fma(-d, r, 1.0), r, r);
    const double q = n * r;
    return fma(fma(-d, q, n), r, q);
}

// Buffer loads: a loop-invariant resource per array (base, size in bytes), a
// wave-uniform byte offset of the z-plane and a 32-bit lane byte offset.  A
// lane offset at or beyond the resource size reads 0, so kOutside masks one
// lane and a resource of size 0 masks a whole plane, without any per-load
// vector instruction.  Every array of a level must stay below 2^31 bytes.
constexpr unsigned kOutside = 0x80000000u;
constexpr int kBufWord3 = 0x00020000;  // raw 32-bit data format, no swizzle

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kBufWord3);
}
__device__ __forceinline__ float bload(float*, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ double bload(double*, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

template <typename T>
__device__ __forceinline__ typename Vec2<T>::type bload2(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ float2 bload2<float>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ double2 bload2<double>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
template <typename T>
__device__ __forceinline__ T bload1(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    return bload((T*)nullptr, r, voff, soff);
}

// Vector stores through a buffer resource (32-bit lane offset, plane offset in
// an SGPR): no 64-bit per-lane address is kept live for the output arrays.
__device__ __forceinline__ void bstore1f(__amdgpu_buffer_rsrc_t r, float v, unsigned voff, unsigned soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}
__device__ __forceinline__ void bstore2(__amdgpu_buffer_rsrc_t r, float2 v, unsigned voff, unsigned soff)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r, voff,
                                          soff, 0);
}
__device__ __forceinline__ void bstore2(__amdgpu_buffer_rsrc_t r, double2 v, unsigned voff, unsigned soff)
{
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, v), r,
                                           voff, soff, 0);
}

}  // namespace mgp
