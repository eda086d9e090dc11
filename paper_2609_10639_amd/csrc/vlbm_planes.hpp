// Wavefront shuffles and buffer addressing of the population arrays, shared by
// the marching kernels of the VLBM library.  Not part of the public ABI.
#pragma once

#include "vlbm_common.hpp"

namespace vlbm {

template <typename T>
__device__ __forceinline__ T shfl(T v, int src)
{
    return __shfl(v, src, 64);
}

// Neighbour moves across the wavefront through DPP, a VALU operand modifier
// (no LDS crossbar round trip): wave_shr:1 gives lane i the value of lane i-1,
// wave_shl:1 the value of lane i+1.  A lane with no source lane (lane 0,
// respectively lane 63) keeps its own value.  Every lane of the wavefront must
// be active.
constexpr int kDppWaveShr1 = 0x138, kDppWaveShl1 = 0x130;

template <int CTRL>
__device__ __forceinline__ int dpp_move(int v)
{
    return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v)
{
    return __builtin_bit_cast(float, dpp_move<CTRL>(__builtin_bit_cast(int, v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v)
{
    typedef int i2 __attribute__((ext_vector_type(2)));
    i2 h = __builtin_bit_cast(i2, v);
    h.x = dpp_move<CTRL>(h.x);
    h.y = dpp_move<CTRL>(h.y);
    return __builtin_bit_cast(double, h);
}

// value of the left (x-1) neighbour lane; `keep` (a clamped edge) takes the own value
template <typename T>
__device__ __forceinline__ T from_left(T v, bool keep)
{
    const T n = dpp_move<kDppWaveShr1>(v);
    return keep ? v : n;
}
// value of the right (x+1) neighbour lane; `keep` takes the own value
template <typename T>
__device__ __forceinline__ T from_right(T v, bool keep)
{
    const T n = dpp_move<kDppWaveShl1>(v);
    return keep ? v : n;
}

// Buffer addressing of the population arrays: one resource per group of four
// planes (base in SGPRs), the plane offset within the group in the scalar
// offset and the cell's byte offset as the only per-lane operand, so that no
// per-lane 64-bit address arithmetic is spent on the 32 loads and stores of a row.
struct Planes {
    __amdgpu_buffer_rsrc_t rs[4];
    unsigned plane_bytes;
};

template <typename S>
__device__ __forceinline__ Planes make_planes(const S* base, unsigned plane)
{
    Planes p;
#pragma unroll
    for (int g = 0; g < 4; ++g)
        p.rs[g] = __builtin_amdgcn_make_buffer_rsrc((void*)(base + (size_t)4 * g * plane), (short)0, (int)0xffffffff,
                                                    0x00020000);
    p.plane_bytes = plane * (unsigned)sizeof(S);
    return p;
}

__device__ __forceinline__ double bload(const Planes& p, int j, unsigned off, double)
{
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    const u2 v = __builtin_amdgcn_raw_buffer_load_b64(p.rs[j >> 2], off, (j & 3) * p.plane_bytes, 0);
    return __builtin_bit_cast(double, v);
}
__device__ __forceinline__ float bload(const Planes& p, int j, unsigned off, float)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(p.rs[j >> 2], off, (j & 3) * p.plane_bytes, 0));
}
__device__ __forceinline__ void bstore(const Planes& p, int j, unsigned off, double v)
{
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), p.rs[j >> 2], off, (j & 3) * p.plane_bytes, 0);
}
__device__ __forceinline__ void bstore(const Planes& p, int j, unsigned off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), p.rs[j >> 2], off, (j & 3) * p.plane_bytes, 0);
}

}  // namespace vlbm
