// pc_block.h -- wavefront (64 lanes) and workgroup scans and reductions for
// the gfx950 kernels.  Every workgroup size used is a multiple of 64.
#pragma once

#include "pc_device.h"

__device__ __forceinline__ uint32_t pc_lane() { return __lane_id(); }

// A value the whole wavefront holds alike, moved to scalar registers (the
// compiler then keeps loads through it scalar and out of vector registers).
__device__ __forceinline__ uint32_t pc_uniform(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ uint64_t pc_uniform64(uint64_t v)
{
    return ((uint64_t)pc_uniform((uint32_t)(v >> 32)) << 32) | pc_uniform((uint32_t)v);
}
template <typename P> __device__ __forceinline__ P *pc_uniform_ptr(P *p)
{
    return (P *)pc_uniform64((uint64_t)p);
}

// 32-bit wavefront sum and inclusive scan with DPP lane moves (gfx9 row
// operations), no LDS traffic.  Every lane must be active.
#define PC_DPP(v, ctrl, rm) ((uint32_t)__builtin_amdgcn_update_dpp(0, (int)(v), ctrl, rm, 0xF, false))

// sum of v over the wavefront, returned (uniform) in every lane
__device__ __forceinline__ uint32_t pc_wave_sum_u32(uint32_t v)
{
    v += PC_DPP(v, 0xB1, 0xF);  // quad_perm [1,0,3,2]
    v += PC_DPP(v, 0x4E, 0xF);  // quad_perm [2,3,0,1]
    v += PC_DPP(v, 0x141, 0xF); // row_half_mirror
    v += PC_DPP(v, 0x140, 0xF); // row_mirror: every lane holds its row's sum
    return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) +
           __builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48);
}

// inclusive prefix sum across the wavefront
__device__ __forceinline__ uint32_t pc_wave_incl_scan_u32(uint32_t v)
{
    v += PC_DPP(v, 0x111, 0xF); // row_shr:1
    v += PC_DPP(v, 0x112, 0xF); // row_shr:2
    v += PC_DPP(v, 0x114, 0xF); // row_shr:4
    v += PC_DPP(v, 0x118, 0xF); // row_shr:8  -> inclusive within rows of 16
    v += PC_DPP(v, 0x142, 0xA); // row_bcast:15 into rows 1 and 3
    v += PC_DPP(v, 0x143, 0xC); // row_bcast:31 into rows 2 and 3
    return v;
}

// Inclusive prefix sum across the 64 lanes of a wavefront.
template <typename T> __device__ __forceinline__ T pc_wave_incl_scan(T v)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T o = __shfl_up(v, d, 64);
        if ((int)pc_lane() >= d)
            v += o;
    }
    return v;
}

template <typename T> __device__ __forceinline__ T pc_wave_sum(T v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1)
        v += __shfl_xor(v, d, 64);
    return v;
}

// 128-bit wave sum via two 64-bit halves (carry handled exactly).
__device__ __forceinline__ pc_s128 pc_wave_sum128(pc_s128 v)
{
    uint64_t lo = (uint64_t)v;
    int64_t hi = (int64_t)(v >> 64);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        uint64_t olo = __shfl_xor(lo, d, 64);
        int64_t ohi = __shfl_xor(hi, d, 64);
        uint64_t nlo = lo + olo;
        hi = hi + ohi + (nlo < lo ? 1 : 0);
        lo = nlo;
    }
    return ((pc_s128)hi << 64) | (pc_s128)lo;
}

// Exclusive prefix sum over a workgroup of NT threads; returns this thread's
// exclusive prefix and writes the workgroup total to *total.  scratch holds
// NT/64 elements.  Contains two barriers; every thread must call it.
template <int NT, typename T>
__device__ __forceinline__ T pc_block_excl_scan(T v, T *scratch, T *total)
{
    constexpr int NW = NT / 64;
    const int w = threadIdx.x >> 6;
    T inc;
    if constexpr (sizeof(T) == 4)
        inc = (T)pc_wave_incl_scan_u32((uint32_t)v);
    else
        inc = pc_wave_incl_scan(v);
    if (pc_lane() == 63)
        scratch[w] = inc;
    __syncthreads();
    T wsum = 0, all = 0;
#pragma unroll
    for (int i = 0; i < NW; i++) {
        T s = scratch[i];
        if (i < w)
            wsum += s;
        all += s;
    }
    *total = all;
    __syncthreads();
    return wsum + inc - v;
}

// Workgroup sum; every thread receives the total.  scratch holds NT/64 elements.
template <int NT, typename T> __device__ __forceinline__ T pc_block_sum(T v, T *scratch)
{
    constexpr int NW = NT / 64;
    if constexpr (sizeof(T) == 4)
        v = (T)pc_wave_sum_u32((uint32_t)v);
    else
        v = pc_wave_sum(v);
    if (pc_lane() == 0)
        scratch[threadIdx.x >> 6] = v;
    __syncthreads();
    T all = 0;
#pragma unroll
    for (int i = 0; i < NW; i++)
        all += scratch[i];
    __syncthreads();
    return all;
}

template <int NT> __device__ __forceinline__ pc_s128 pc_block_sum128(pc_s128 v, pc_s128 *scratch)
{
    constexpr int NW = NT / 64;
    v = pc_wave_sum128(v);
    if (pc_lane() == 0)
        scratch[threadIdx.x >> 6] = v;
    __syncthreads();
    pc_s128 all = 0;
#pragma unroll
    for (int i = 0; i < NW; i++)
        all += scratch[i];
    __syncthreads();
    return all;
}

// *dst += v for a signed 128-bit accumulator in device memory, from any number
// of threads: the low words are added atomically, and each adder carries its
// own overflow into the high word, so the total is exact in any order.
__device__ __forceinline__ void pc_atomic_add128(pc_s128 *dst, pc_s128 v)
{
    unsigned long long *w = reinterpret_cast<unsigned long long *>(dst);
    const unsigned long long lo = (unsigned long long)(uint64_t)v;
    const unsigned long long hi = (unsigned long long)(uint64_t)(v >> 64);
    const unsigned long long old = atomicAdd(&w[0], lo);
    const unsigned long long carry = old + lo < old ? 1ull : 0ull;
    if (hi + carry)
        atomicAdd(&w[1], hi + carry);
}
