// vi_device.h -- device helpers shared by the build and render kernels of libvi.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vi {

// Raw hardware transcendentals (v_exp_f32 / v_log_f32): 2^x and log2(x).
__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }

__device__ __forceinline__ int clampi(int x, int lo, int hi) { return min(max(x, lo), hi); }
__device__ __forceinline__ float clampf01(float x) { return fminf(fmaxf(x, 0.0f), 1.0f); }

// One voxel, normalised and clamped to [0,1] before interpolation.
template <typename VT>
__device__ __forceinline__ float voxel_norm(const VT* __restrict__ v, uint32_t idx, float scale);

template <>
__device__ __forceinline__ float voxel_norm<uint8_t>(const uint8_t* __restrict__ v, uint32_t idx, float scale)
{
    return clampf01((float)v[idx] * scale);
}
template <>
__device__ __forceinline__ float voxel_norm<uint16_t>(const uint16_t* __restrict__ v, uint32_t idx, float scale)
{
    return clampf01((float)v[idx] * scale);
}
template <>
__device__ __forceinline__ float voxel_norm<__half>(const __half* __restrict__ v, uint32_t idx, float scale)
{
    return clampf01(__half2float(v[idx]) * scale);
}
template <>
__device__ __forceinline__ float voxel_norm<float>(const float* __restrict__ v, uint32_t idx, float scale)
{
    return clampf01(v[idx] * scale);
}

// Trilinear sample at offset-voxel coordinates h = g - M (g = p*N - 1/2),
// clamp to edge.  M is an integer so floor/fraction are taken on h exactly.
template <typename VT>
__device__ __forceinline__ float sample_volume(const VT* __restrict__ vol, int N, int M, float scale, float hx,
                                               float hy, float hz)
{
    float fx = floorf(hx), fy = floorf(hy), fz = floorf(hz);
    float wx = hx - fx, wy = hy - fy, wz = hz - fz;
    int x0 = (int)fx + M, y0 = (int)fy + M, z0 = (int)fz + M;
    int xa = clampi(x0, 0, N - 1), xb = clampi(x0 + 1, 0, N - 1);
    int ya = clampi(y0, 0, N - 1), yb = clampi(y0 + 1, 0, N - 1);
    int za = clampi(z0, 0, N - 1), zb = clampi(z0 + 1, 0, N - 1);
    uint32_t Nu = (uint32_t)N;
    uint32_t raa = ((uint32_t)za * Nu + (uint32_t)ya) * Nu;
    uint32_t rab = ((uint32_t)za * Nu + (uint32_t)yb) * Nu;
    uint32_t rba = ((uint32_t)zb * Nu + (uint32_t)ya) * Nu;
    uint32_t rbb = ((uint32_t)zb * Nu + (uint32_t)yb) * Nu;
    float v000 = voxel_norm(vol, raa + xa, scale), v001 = voxel_norm(vol, raa + xb, scale);
    float v010 = voxel_norm(vol, rab + xa, scale), v011 = voxel_norm(vol, rab + xb, scale);
    float v100 = voxel_norm(vol, rba + xa, scale), v101 = voxel_norm(vol, rba + xb, scale);
    float v110 = voxel_norm(vol, rbb + xa, scale), v111 = voxel_norm(vol, rbb + xb, scale);
    float c00 = fmaf(wx, v001 - v000, v000), c01 = fmaf(wx, v011 - v010, v010);
    float c10 = fmaf(wx, v101 - v100, v100), c11 = fmaf(wx, v111 - v110, v110);
    float c0 = fmaf(wy, c01 - c00, c00), c1 = fmaf(wy, c11 - c10, c10);
    return fmaf(wz, c1 - c0, c0);
}

// Round a float to bfloat16 (nearest even), finite inputs.
__device__ __forceinline__ uint16_t f32_to_bf16(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Tile index with the workgroups of each XCD given a contiguous range of
// tiles: workgroups are dealt round-robin to the 8 XCDs, so block b runs on
// XCD b % 8; mapping it to tile (b % 8) * per + b / 8 keeps neighbouring
// tiles in one XCD's L2.
__device__ __forceinline__ uint32_t xcd_swizzle(uint32_t b, uint32_t nblocks)
{
    const uint32_t X = 8;
    uint32_t per = nblocks / X, rem = nblocks % X;
    uint32_t x = b % X, q = b / X;
    // XCDs 0..rem-1 own per+1 tiles, the rest own per
    return x * per + min(x, rem) + q;
}

}  // namespace vi
