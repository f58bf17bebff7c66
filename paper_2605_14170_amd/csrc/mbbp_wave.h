// Wave-level helpers shared by the HIP kernels of the MBBP-LD library (gfx950,
// wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mbbp {

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ long long uniform_i64(long long v) {
    unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v & 0xffffffffu));
    unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)((unsigned long long)v >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ int wave_max_i32(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_min_i32(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ long long wave_sum_i64(long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ float wave_sum_f32(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ uint32_t fbits(float x) { return __float_as_uint(x); }
__device__ __forceinline__ float bitsf(uint32_t x) { return __uint_as_float(x); }

typedef __attribute__((address_space(3))) float lds_f32;
typedef __attribute__((address_space(3))) unsigned char lds_u8;
typedef __attribute__((address_space(3))) uint64_t lds_u64;
typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) f32x2 lds_f32x2;

__device__ __forceinline__ lds_f32 *lds_ptr_f32(uint32_t byte_addr) { return (lds_f32 *)(size_t)byte_addr; }
__device__ __forceinline__ lds_u8 *lds_ptr_u8(uint32_t byte_addr) { return (lds_u8 *)(size_t)byte_addr; }
__device__ __forceinline__ lds_u64 *lds_ptr_u64(uint32_t byte_addr) { return (lds_u64 *)(size_t)byte_addr; }
__device__ __forceinline__ lds_u32 *lds_ptr_u32(uint32_t byte_addr) { return (lds_u32 *)(size_t)byte_addr; }
__device__ __forceinline__ lds_f32x2 *lds_ptr_f32x2(uint32_t byte_addr) { return (lds_f32x2 *)(size_t)byte_addr; }

}  // namespace mbbp
