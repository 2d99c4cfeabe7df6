// vi_device.h -- device helpers shared by the build and render kernels of libvi.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vi.h"
#include "vi_internal.h"

namespace vi {

// Raw hardware transcendentals (v_exp_f32 / v_log_f32): 2^x and log2(x).
__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }

__device__ __forceinline__ int clampi(int x, int lo, int hi) { return min(max(x, lo), hi); }

// Knuth's two-sum: s = fl(a + b) and the exact error e = (a + b) - s, for
// the float pairs below.  The error term holds only for separately rounded
// operations, so contraction of products and sums into FMAs is off here.
__device__ __forceinline__ float two_sum(float a, float b, float* e)
{
#pragma clang fp contract(off)
    const float s = a + b, t = s - a;
    *e = (a - (s - t)) + (b - t);
    return s;
}
__device__ __forceinline__ float clampf01(float x) { return fminf(fmaxf(x, 0.0f), 1.0f); }

// Float pairs: a value held as hi + lo with |lo| <= ulp(hi) / 2, about 48
// significant bits from FP32 operations alone (Dekker's product via FMA,
// Knuth's two-sum).  The per-ray set-up of the render uses them where a
// single float would misplace a ray entering the cube ~10^3 voxels from the
// eye by ~10^-4 voxel.  Contraction stays off: every error term assumes
// separately rounded operations.
struct F2 {
    float hi, lo;
};
__device__ __forceinline__ F2 f2(float a) { return F2{a, 0.0f}; }
__device__ __forceinline__ F2 f2_fast(float a, float b)  // |a| >= |b|
{
#pragma clang fp contract(off)
    const float s = a + b;
    return F2{s, b - (s - a)};
}
__device__ __forceinline__ F2 f2_add(F2 a, F2 b)
{
#pragma clang fp contract(off)
    float e;
    const float s = two_sum(a.hi, b.hi, &e);
    return f2_fast(s, e + (a.lo + b.lo));
}
__device__ __forceinline__ F2 f2_neg(F2 a) { return F2{-a.hi, -a.lo}; }
__device__ __forceinline__ F2 f2_sub(F2 a, F2 b) { return f2_add(a, f2_neg(b)); }
__device__ __forceinline__ F2 f2_mul(F2 a, F2 b)
{
#pragma clang fp contract(off)
    const float p = a.hi * b.hi;
    const float e = fmaf(a.hi, b.hi, -p) + (a.hi * b.lo + a.lo * b.hi);
    return f2_fast(p, e);
}
// a / b: a quotient from the hardware reciprocal, corrected once by the
// pair residual a - q b (the reciprocal's error enters squared)
__device__ __forceinline__ F2 f2_div(F2 a, F2 b)
{
#pragma clang fp contract(off)
    const float r = __builtin_amdgcn_rcpf(b.hi);
    const float q = a.hi * r;
    const F2 e = f2_sub(a, f2_mul(f2(q), b));  // a - q b
    const float q2 = e.hi * r;
    const F2 e2 = f2_sub(e, f2_mul(f2(q2), b));
    return f2_add(f2_fast(q, q2), f2(e2.hi * r));
}
// 1 / sqrt(a), a > 0: the hardware estimate and one Newton step on the pair
__device__ __forceinline__ F2 f2_rsqrt(F2 a)
{
#pragma clang fp contract(off)
    const float r = __builtin_amdgcn_rsqf(a.hi);
    const F2 y = f2_mul(f2_mul(a, f2(r)), f2(r));           // a r^2, about 1
    const F2 h = f2_sub(f2(1.5f), f2_mul(f2(0.5f), y));      // (3 - a r^2) / 2
    return f2_mul(f2(r), h);
}
__device__ __forceinline__ bool f2_lt(F2 a, F2 b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }
__device__ __forceinline__ F2 f2_max(F2 a, F2 b) { return f2_lt(a, b) ? b : a; }
__device__ __forceinline__ F2 f2_min(F2 a, F2 b) { return f2_lt(a, b) ? a : b; }
__device__ __forceinline__ F2 f2_dot3(const F2* a, const F2* b)
{
    return f2_add(f2_add(f2_mul(a[0], b[0]), f2_mul(a[1], b[1])), f2_mul(a[2], b[2]));
}

// One voxel, normalised and clamped to [0,1] before interpolation.
// Element idx of an array below 4 GiB, addressed with a 32-bit byte offset
// (the load then takes the base from scalar registers: no 64-bit address
// arithmetic per load).  Stacks and one copy of a volume's voxels are
// refused at 4 GiB and above; the quad layout, four copies, is not (it keeps
// 64-bit addressing).
template <typename T>
__device__ __forceinline__ T ld32(const void* __restrict__ base, uint32_t idx)
{
    return *(const T*)((const char*)base + idx * (uint32_t)sizeof(T));
}

template <typename VT>
__device__ __forceinline__ float voxel_norm(const VT* __restrict__ v, uint32_t idx, float scale);

template <>
__device__ __forceinline__ float voxel_norm<uint8_t>(const uint8_t* __restrict__ v, uint32_t idx, float scale)
{
    return clampf01((float)ld32<uint8_t>(v, idx) * scale);
}
template <>
__device__ __forceinline__ float voxel_norm<uint16_t>(const uint16_t* __restrict__ v, uint32_t idx, float scale)
{
    return clampf01((float)ld32<uint16_t>(v, idx) * scale);
}
template <>
__device__ __forceinline__ float voxel_norm<__half>(const __half* __restrict__ v, uint32_t idx, float scale)
{
    return clampf01(__half2float(ld32<__half>(v, idx)) * scale);
}
template <>
__device__ __forceinline__ float voxel_norm<float>(const float* __restrict__ v, uint32_t idx, float scale)
{
    return clampf01(ld32<float>(v, idx) * scale);
}

// Element offsets of the two volume layouts, separable per axis so the
// eight corners of a trilinear footprint cost six offset evaluations:
//   linear : (z*N + y)*N + x
//   brick4 : 4x4x4 bricks (one 128-byte line at 16 bits), bricks in z,y,x
//            order: ((z/4)*nb*nb + (y/4)*nb + x/4)*64 + (z%4)*16 + (y%4)*4 + x%4
struct VolIndex {
    uint32_t sx, sy, sz;  // linear: 1, N, N*N     brick4: unused, nb*64, nb*nb*64
};
template <int LAYOUT>
__device__ __forceinline__ uint32_t vol_ox(const VolIndex& I, int x)
{
    if (LAYOUT != VI_LAYOUT_LINEAR) return ((uint32_t)x >> 2) * 64u + ((uint32_t)x & 3u);
    return (uint32_t)x;
}
// (Products in 24-bit multiplies, full rate where a 32-bit multiply is
// quarter rate: a volume below 4 GiB has N < 2^11, so the coordinates and
// the strides N, N^2, (N/4)*64 and (N/4)^2*64 all stay below 2^24.)
template <int LAYOUT>
__device__ __forceinline__ uint32_t vol_oy(const VolIndex& I, int y)
{
    if (LAYOUT != VI_LAYOUT_LINEAR) return __umul24((uint32_t)y >> 2, I.sy) + ((uint32_t)y & 3u) * 4u;
    return __umul24((uint32_t)y, I.sy);
}
template <int LAYOUT>
__device__ __forceinline__ uint32_t vol_oz(const VolIndex& I, int z)
{
    if (LAYOUT != VI_LAYOUT_LINEAR) return __umul24((uint32_t)z >> 2, I.sz) + ((uint32_t)z & 3u) * 16u;
    return __umul24((uint32_t)z, I.sz);
}

// The four normalised values of quad slot `q` (VI_LAYOUT_QUAD4): one load
// of 4 elements, each converted exactly as voxel_norm converts it.
template <typename VT>
__device__ __forceinline__ float4 quad_norm(const VT* __restrict__ v, uint32_t q, float scale);
template <>
__device__ __forceinline__ float4 quad_norm<uint8_t>(const uint8_t* __restrict__ v, uint32_t q, float scale)
{
    const uint32_t w = ((const uint32_t*)v)[q];
    return make_float4(clampf01((float)(w & 0xffu) * scale), clampf01((float)((w >> 8) & 0xffu) * scale),
                       clampf01((float)((w >> 16) & 0xffu) * scale), clampf01((float)(w >> 24) * scale));
}
template <>
__device__ __forceinline__ float4 quad_norm<uint16_t>(const uint16_t* __restrict__ v, uint32_t q, float scale)
{
    const uint2 w = ((const uint2*)v)[q];
    return make_float4(clampf01((float)(w.x & 0xffffu) * scale), clampf01((float)(w.x >> 16) * scale),
                       clampf01((float)(w.y & 0xffffu) * scale), clampf01((float)(w.y >> 16) * scale));
}
template <>
__device__ __forceinline__ float4 quad_norm<__half>(const __half* __restrict__ v, uint32_t q, float scale)
{
    const uint2 w = ((const uint2*)v)[q];
    return make_float4(clampf01(__half2float(__ushort_as_half((unsigned short)(w.x & 0xffffu))) * scale),
                       clampf01(__half2float(__ushort_as_half((unsigned short)(w.x >> 16))) * scale),
                       clampf01(__half2float(__ushort_as_half((unsigned short)(w.y & 0xffffu))) * scale),
                       clampf01(__half2float(__ushort_as_half((unsigned short)(w.y >> 16))) * scale));
}
template <>
__device__ __forceinline__ float4 quad_norm<float>(const float* __restrict__ v, uint32_t q, float scale)
{
    const float4 w = ((const float4*)v)[q];
    return make_float4(clampf01(w.x * scale), clampf01(w.y * scale), clampf01(w.z * scale), clampf01(w.w * scale));
}

// A trilinear footprint split into its loads and its arithmetic, so that a
// caller can issue the loads of several footprints before it needs any of
// them.  RawFoot holds the raw elements (eight voxels, or the two quad slots
// at z and z+1); foot_value converts and interpolates them exactly as
// sample_volume does.
template <typename VT> struct QuadRaw { using T = uint2; };           // 16-bit voxels
template <> struct QuadRaw<uint8_t> { using T = uint32_t; };
template <> struct QuadRaw<float> { using T = float4; };
template <typename VT, int LAYOUT> struct RawFoot { VT v[8]; };
template <typename VT> struct RawFoot<VT, VI_LAYOUT_QUAD4> { typename QuadRaw<VT>::T a, b; };

__device__ __forceinline__ float norm1(uint8_t x, float scale) { return clampf01((float)x * scale); }
__device__ __forceinline__ float norm1(uint16_t x, float scale) { return clampf01((float)x * scale); }
__device__ __forceinline__ float norm1(__half x, float scale) { return clampf01(__half2float(x) * scale); }
__device__ __forceinline__ float norm1(float x, float scale) { return clampf01(x * scale); }

__device__ __forceinline__ float4 quad_decode(uint32_t w, float scale, uint8_t)
{
    return make_float4(clampf01((float)(w & 0xffu) * scale), clampf01((float)((w >> 8) & 0xffu) * scale),
                       clampf01((float)((w >> 16) & 0xffu) * scale), clampf01((float)(w >> 24) * scale));
}
__device__ __forceinline__ float4 quad_decode(uint2 w, float scale, uint16_t)
{
    return make_float4(clampf01((float)(w.x & 0xffffu) * scale), clampf01((float)(w.x >> 16) * scale),
                       clampf01((float)(w.y & 0xffffu) * scale), clampf01((float)(w.y >> 16) * scale));
}
__device__ __forceinline__ float4 quad_decode(uint2 w, float scale, __half)
{
    return make_float4(clampf01(__half2float(__ushort_as_half((unsigned short)(w.x & 0xffffu))) * scale),
                       clampf01(__half2float(__ushort_as_half((unsigned short)(w.x >> 16))) * scale),
                       clampf01(__half2float(__ushort_as_half((unsigned short)(w.y & 0xffffu))) * scale),
                       clampf01(__half2float(__ushort_as_half((unsigned short)(w.y >> 16))) * scale));
}
__device__ __forceinline__ float4 quad_decode(float4 w, float scale, float)
{
    return make_float4(clampf01(w.x * scale), clampf01(w.y * scale), clampf01(w.z * scale), clampf01(w.w * scale));
}

// Issue the loads of the footprint whose lower corner is voxel (x0, y0, z0)
// (before clamping to the volume); a quad footprint below the first voxel in
// x or y takes a zero weight there (both of its corners clamp to voxel 0).
template <typename VT, int LAYOUT>
__device__ __forceinline__ void foot_load_g(RawFoot<VT, LAYOUT>& r, float& wx, float& wy, const VT* __restrict__ vol,
                                            const VolIndex& I, int N, int x0, int y0, int z0)
{
    const uint32_t za = vol_oz<LAYOUT>(I, clampi(z0, 0, N - 1)), zb = vol_oz<LAYOUT>(I, clampi(z0 + 1, 0, N - 1));
    if constexpr (LAYOUT == VI_LAYOUT_QUAD4) {
        using Q = typename QuadRaw<VT>::T;
        const uint32_t xy = vol_ox<LAYOUT>(I, clampi(x0, 0, N - 1)) + vol_oy<LAYOUT>(I, clampi(y0, 0, N - 1));
        // (a quad volume holds four copies of the voxels and may pass 4 GiB:
        // 64-bit addressing)
        r.a = ((const Q*)vol)[za + xy];
        r.b = ((const Q*)vol)[zb + xy];
        if (x0 < 0) wx = 0.0f;
        if (y0 < 0) wy = 0.0f;
    } else {
        const uint32_t xa = vol_ox<LAYOUT>(I, clampi(x0, 0, N - 1)), xb = vol_ox<LAYOUT>(I, clampi(x0 + 1, 0, N - 1));
        const uint32_t ya = vol_oy<LAYOUT>(I, clampi(y0, 0, N - 1)), yb = vol_oy<LAYOUT>(I, clampi(y0 + 1, 0, N - 1));
        r.v[0] = ld32<VT>(vol, za + ya + xa);
        r.v[1] = ld32<VT>(vol, za + ya + xb);
        r.v[2] = ld32<VT>(vol, za + yb + xa);
        r.v[3] = ld32<VT>(vol, za + yb + xb);
        r.v[4] = ld32<VT>(vol, zb + ya + xa);
        r.v[5] = ld32<VT>(vol, zb + ya + xb);
        r.v[6] = ld32<VT>(vol, zb + yb + xa);
        r.v[7] = ld32<VT>(vol, zb + yb + xb);
    }
}

template <typename VT, int LAYOUT>
__device__ __forceinline__ float foot_value(const RawFoot<VT, LAYOUT>& r, float wx, float wy, float wz, float scale)
{
    float4 a, b;
    if constexpr (LAYOUT == VI_LAYOUT_QUAD4) {
        a = quad_decode(r.a, scale, VT());
        b = quad_decode(r.b, scale, VT());
    } else {
        a = make_float4(norm1(r.v[0], scale), norm1(r.v[1], scale), norm1(r.v[2], scale), norm1(r.v[3], scale));
        b = make_float4(norm1(r.v[4], scale), norm1(r.v[5], scale), norm1(r.v[6], scale), norm1(r.v[7], scale));
    }
    const float c00 = fmaf(wx, a.y - a.x, a.x), c01 = fmaf(wx, a.w - a.z, a.z);
    const float c10 = fmaf(wx, b.y - b.x, b.x), c11 = fmaf(wx, b.w - b.z, b.z);
    const float c0 = fmaf(wy, c01 - c00, c00), c1 = fmaf(wy, c11 - c10, c10);
    return fmaf(wz, c1 - c0, c0);
}

// Trilinear sample at offset-voxel coordinates h = g - M (g = p*N - 1/2),
// clamp to edge.  M is an integer so floor/fraction are taken on h exactly.
template <typename VT, int LAYOUT>
__device__ __forceinline__ float sample_volume(const VT* __restrict__ vol, const VolIndex& I, int N, int M,
                                               float scale, float hx, float hy, float hz)
{
    float fx = floorf(hx), fy = floorf(hy), fz = floorf(hz);
    float wx = hx - fx, wy = hy - fy, wz = hz - fz;
    int x0 = (int)fx + M, y0 = (int)fy + M, z0 = (int)fz + M;
    if (LAYOUT == VI_LAYOUT_QUAD4) {
        // the slot of the clamped lower corner holds the x/y neighbours,
        // themselves clamped; below the first voxel both x (or y) corners
        // clamp to voxel 0, which a zero weight reproduces exactly
        const uint32_t xy = vol_ox<LAYOUT>(I, clampi(x0, 0, N - 1)) + vol_oy<LAYOUT>(I, clampi(y0, 0, N - 1));
        const float4 a = quad_norm(vol, vol_oz<LAYOUT>(I, clampi(z0, 0, N - 1)) + xy, scale);
        const float4 b = quad_norm(vol, vol_oz<LAYOUT>(I, clampi(z0 + 1, 0, N - 1)) + xy, scale);
        if (x0 < 0) wx = 0.0f;
        if (y0 < 0) wy = 0.0f;
        const float c00 = fmaf(wx, a.y - a.x, a.x), c01 = fmaf(wx, a.w - a.z, a.z);
        const float c10 = fmaf(wx, b.y - b.x, b.x), c11 = fmaf(wx, b.w - b.z, b.z);
        const float c0 = fmaf(wy, c01 - c00, c00), c1 = fmaf(wy, c11 - c10, c10);
        return fmaf(wz, c1 - c0, c0);
    }
    const uint32_t xa = vol_ox<LAYOUT>(I, clampi(x0, 0, N - 1)), xb = vol_ox<LAYOUT>(I, clampi(x0 + 1, 0, N - 1));
    const uint32_t ya = vol_oy<LAYOUT>(I, clampi(y0, 0, N - 1)), yb = vol_oy<LAYOUT>(I, clampi(y0 + 1, 0, N - 1));
    const uint32_t za = vol_oz<LAYOUT>(I, clampi(z0, 0, N - 1)), zb = vol_oz<LAYOUT>(I, clampi(z0 + 1, 0, N - 1));
    const uint32_t raa = za + ya, rab = za + yb, rba = zb + ya, rbb = zb + yb;
    float v000 = voxel_norm(vol, raa + xa, scale), v001 = voxel_norm(vol, raa + xb, scale);
    float v010 = voxel_norm(vol, rab + xa, scale), v011 = voxel_norm(vol, rab + xb, scale);
    float v100 = voxel_norm(vol, rba + xa, scale), v101 = voxel_norm(vol, rba + xb, scale);
    float v110 = voxel_norm(vol, rbb + xa, scale), v111 = voxel_norm(vol, rbb + xb, scale);
    float c00 = fmaf(wx, v001 - v000, v000), c01 = fmaf(wx, v011 - v010, v010);
    float c10 = fmaf(wx, v101 - v100, v100), c11 = fmaf(wx, v111 - v110, v110);
    float c0 = fmaf(wy, c01 - c00, c00), c1 = fmaf(wy, c11 - c10, c10);
    return fmaf(wz, c1 - c0, c0);
}

// Stack layout: every layer is stored as 8 x 4 texel tiles (one 128-byte
// line in float), tiles row-major; a layer holds R8 x R4 texels (res rounded
// up to 8 along i and to 4 along j):
//   offset(k, j, i) = k*layer + ((j/4)*(R8/8) + i/8)*32 + (j%4)*8 + i%8
__device__ __forceinline__ uint32_t stack_oi(int i) { return ((uint32_t)i >> 3) * 32u + ((uint32_t)i & 7u); }
__device__ __forceinline__ uint32_t stack_oj(int j, uint32_t row_tiles32)
{
    return ((uint32_t)j >> 2) * row_tiles32 + ((uint32_t)j & 3u) * 8u;
}

// Empty-space test.  s_next[e] = first transfer-function entry >= e with
// non-zero opacity (K if none), built in LDS per workgroup.  A cell is empty
// when no entry a value in [min, max] can interpolate between -- widened by
// one entry on each side for rounding -- has opacity.
__device__ __forceinline__ void build_next_opaque(int* s_next, const float* tf, int K)
{
    for (int e = threadIdx.x; e < K; e += blockDim.x) {
        int j = e;
        while (j < K && !(tf[4 * j + 3] > 0.0f)) ++j;
        s_next[e] = j;
    }
}
__device__ __forceinline__ bool cell_empty(const float2 m, const int* s_next, float Km1, int K)
{
    const int lo = max((int)(m.x * Km1) - 1, 0);
    const int hi = min((int)(m.y * Km1) + 2, K - 1);
    return s_next[lo] > hi;
}
// Whether cell c may hold opacity: its occupancy bit (the LDS copy
// `s_bits`), or the map entry against the transfer function.
__device__ __forceinline__ bool cell_occupied(const OccMap& o, const uint32_t* s_bits, uint32_t c,
                                              const int* s_next, float Km1, int K)
{
    if (o.bits) return (s_bits[c >> 5] >> (c & 31u)) & 1u;
    return !cell_empty(o.mm[c], s_next, Km1, K);
}
__device__ __forceinline__ bool occupancy_bit(const uint32_t* s_bits, uint32_t c)
{
    return (s_bits[c >> 5] >> (c & 31u)) & 1u;
}
// Stage the occupancy bits in LDS (call before the workgroup's barrier).
__device__ __forceinline__ void stage_occupancy(const OccMap& o, uint32_t* s_bits)
{
    if (o.bits)
        for (uint32_t w = threadIdx.x; w < o.words + o.swords; w += blockDim.x) s_bits[w] = o.bits[w];
}

// Cell index of a trilinear footprint whose lower corner is voxel (x0,y0,z0)
// (before clamping).
__device__ __forceinline__ uint32_t cell_of(int x0, int y0, int z0, int N, int shift, uint32_t nc)
{
    const uint32_t cx = (uint32_t)clampi(x0, 0, N - 1) >> shift;
    const uint32_t cy = (uint32_t)clampi(y0, 0, N - 1) >> shift;
    const uint32_t cz = (uint32_t)clampi(z0, 0, N - 1) >> shift;
    return (cz * nc + cy) * nc + cx;
}

// Round a float to bfloat16 (nearest even), finite inputs.
__device__ __forceinline__ uint16_t f32_to_bf16(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Workgroups are dealt round-robin to the 8 XCDs (block b runs on XCD b % 8),
// each with its own L2.  The tile grid is cut into super-tiles of 4 x 4 tiles;
// super-tile s belongs to XCD s % 8, and the XCD's blocks walk its
// super-tiles tile by tile.  Neighbouring tiles thus share an L2 while the
// work of every region of the image (or light square) is spread over all
// XCDs -- a contiguous band per XCD would leave the XCDs of empty bands idle.
constexpr uint32_t kXcds = 8, kSuper = 4;
__host__ __device__ inline uint32_t supertile_grid(uint32_t tiles_x, uint32_t tiles_y)
{
    const uint32_t sx = (tiles_x + kSuper - 1) / kSuper, sy = (tiles_y + kSuper - 1) / kSuper;
    return (sx * sy + kXcds - 1) / kXcds * kXcds * kSuper * kSuper;
}
// Returns false for padding blocks.
__device__ __forceinline__ bool supertile_of(uint32_t b, uint32_t tiles_x, uint32_t tiles_y, uint32_t* tx,
                                             uint32_t* ty)
{
    const uint32_t sx = (tiles_x + kSuper - 1) / kSuper, sy = (tiles_y + kSuper - 1) / kSuper;
    const uint32_t x = b % kXcds, q = b / kXcds;
    const uint32_t st = x + kXcds * (q / (kSuper * kSuper)), t = q % (kSuper * kSuper);
    if (st >= sx * sy) return false;
    *tx = (st % sx) * kSuper + t % kSuper;
    *ty = (st / sx) * kSuper + t / kSuper;
    return *tx < tiles_x && *ty < tiles_y;
}
// A list of n tiles: groups of 16 consecutive entries dealt round-robin to the
// XCDs.  Returns false for padding blocks; grid = list_grid(n).
__host__ __device__ inline uint32_t list_grid(uint32_t n) { return (n + 127) / 128 * 128; }
__device__ __forceinline__ bool list_of(uint32_t b, uint32_t n, uint32_t* idx)
{
    const uint32_t G = 16, x = b % kXcds, q = b / kXcds;
    *idx = ((q / G) * kXcds + x) * G + q % G;
    return *idx < n;
}

}  // namespace vi
