// Storage types of f in the block pool and their conversions.
//   VL_F64 : double
//   VL_F32 : float, round to nearest even from FP64
//   VL_BF16: bfloat16 (upper half of an IEEE float), round to nearest even
//            from FP64 (bf16_rne_f64): FP64 -> FP32 to nearest, with the FP32
//            word moved one unit toward the FP64 value where it landed exactly
//            on a BF16 midpoint without being the value, then BF16 to nearest
//            even.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "../../include/vlasov.h"

namespace vl {

__host__ __device__ inline uint32_t f32_bits(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

__host__ __device__ inline float bits_f32(uint32_t u)
{
    float f;
    memcpy(&f, &u, 4);
    return f;
}

__host__ __device__ inline uint16_t f32_to_bf16_rne(float f)
{
    uint32_t u = f32_bits(f);
    if ((u & 0x7f800000u) == 0x7f800000u) {  // inf / nan
        uint16_t h = (uint16_t)(u >> 16);
        if (u & 0x007fffffu) h |= 0x40;
        return h;
    }
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

__host__ __device__ inline float bf16_to_f32(uint16_t h)
{
    return bits_f32(((uint32_t)h) << 16);
}

// FP64 -> BF16, round to nearest even, for finite values.  FP64 -> FP32 (to
// nearest) can only change the BF16 rounding where it lands exactly on a BF16
// midpoint (low half 0x8000) without being the value itself; there the FP32
// word is moved one unit toward the value, so the midpoint no longer ties.
__host__ __device__ inline uint16_t bf16_rne_f64(double d)
{
    const float t = (float)d;
    uint32_t u = f32_bits(t);
    const double back = (double)t;
    const bool tie = (u & 0xFFFFu) == 0x8000u && back != d;
    const uint32_t step = (fabs(d) > fabs(back)) ? 1u : 0xFFFFFFFFu;
    u += tie ? step : 0u;
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <int ST>
struct Storage;

template <>
struct Storage<VL_F64> {
    using T = double;
    using Word = unsigned long long;
    static constexpr int WORDS_PER_BLOCK = 64;
    static constexpr int BYTES = 8;
    __device__ static double load(const void *pool, int64_t i) { return ((const double *)pool)[i]; }
    __device__ static void store(void *pool, int64_t i, double v) { ((double *)pool)[i] = v; }
    __device__ static double round(double v) { return v; }
    __device__ static double widen(double v) { return v; }
};

template <>
struct Storage<VL_F32> {
    using T = float;
    using Word = uint32_t;
    static constexpr int WORDS_PER_BLOCK = 64;
    static constexpr int BYTES = 4;
    __device__ static double load(const void *pool, int64_t i) { return (double)((const float *)pool)[i]; }
    __device__ static float loadf(const void *pool, int64_t i) { return ((const float *)pool)[i]; }
    __device__ static void store(void *pool, int64_t i, double v) { ((float *)pool)[i] = (float)v; }
    // value actually stored for v (as FP64)
    __device__ static double round(double v) { return (double)(float)v; }
    __device__ static double widen(float v) { return (double)v; }
};

template <>
struct Storage<VL_BF16> {
    using T = uint16_t;
    using Word = uint32_t;
    static constexpr int WORDS_PER_BLOCK = 32;
    static constexpr int BYTES = 2;
    __device__ static double load(const void *pool, int64_t i)
    {
        return (double)bf16_to_f32(((const uint16_t *)pool)[i]);
    }
    __device__ static float loadf(const void *pool, int64_t i) { return bf16_to_f32(((const uint16_t *)pool)[i]); }
    __device__ static uint16_t encode(double v) { return bf16_rne_f64(v); }
    __device__ static void store(void *pool, int64_t i, double v) { ((uint16_t *)pool)[i] = encode(v); }
    __device__ static double round(double v) { return (double)bf16_to_f32(encode(v)); }
    __device__ static double widen(uint16_t v) { return (double)bf16_to_f32(v); }
};

inline int storage_bytes(int st) { return st == VL_F64 ? 8 : st == VL_F32 ? 4 : 2; }

// One block (64 values of one cell) of the pool as a buffer resource: the
// block's address is formed in scalar registers and each lane's value is at
// byte offset lane * bytes, so no vector instruction computes addresses.
// Offsets past the block (none occur) would read zero and drop stores.
typedef unsigned int vl_u32x2 __attribute__((ext_vector_type(2)));
constexpr int RSRC_WORD3 = 0x00020000;  // untyped 32-bit buffer access on this architecture

template <int ST>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t block_rsrc(void *pool, uint32_t slot)
{
    constexpr int NB = 64 * Storage<ST>::BYTES;
    return __builtin_amdgcn_make_buffer_rsrc((char *)pool + (uint64_t)slot * NB, (short)0, NB, RSRC_WORD3);
}

// a lane's value of a block: double for FP64 storage, else float
template <int ST>
__device__ __forceinline__ auto block_load(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    if constexpr (ST == VL_F64)
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    else if constexpr (ST == VL_F32)
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    else
        return bf16_to_f32(__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0));
}

// a lane's raw storage word of a block (BF16 bits not yet widened)
template <int ST>
__device__ __forceinline__ typename Storage<ST>::T block_load_raw(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    if constexpr (ST == VL_BF16)
        return __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
    else
        return block_load<ST>(r, off);
}

__device__ __forceinline__ void block_store(__amdgpu_buffer_rsrc_t r, uint32_t off, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(vl_u32x2, v), r, off, 0, 0);
}
__device__ __forceinline__ void block_store(__amdgpu_buffer_rsrc_t r, uint32_t off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, 0);
}
__device__ __forceinline__ void block_store(__amdgpu_buffer_rsrc_t r, uint32_t off, uint16_t v)
{
    __builtin_amdgcn_raw_buffer_store_b16(v, r, off, 0, 0);
}

}  // namespace vl
