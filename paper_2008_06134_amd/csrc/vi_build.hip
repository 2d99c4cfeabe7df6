// vi_build.hip -- light-space attenuation build (section 3.2.1, Alg. 1).
//
// One lane owns one texel column of the light square and scans the n slabs
// from the light (Eq. 8 ordering): per slab it samples the volume at the slab
// midpoint, looks up the transfer-function opacity, corrects it to the slab
// thickness (extinction form, Eq. 6) and multiplies the running
// transmittance by (1 - alpha) -- Eq. 4 applied to opacity.  Every layer is
// written as soon as it is known, so the pass is a single streaming sweep:
// the volume is read through the caches and the stack is written once,
// coalesced along the texel row.
//
// Workgroup = 16 x 16 texels (4 waves of 16 x 4) for the tiled stack: at
// every slab a wave stores two whole 8 x 4 texel tiles, i.e. two full
// 128-byte lines; 64 x 4 texels (a wave per 64-texel row run) for the row
// stack.  The alpha column of the transfer function sits in LDS.
#include "vi_device.h"
#include "vi_internal.h"

namespace vi {

// Block of texel columns per workgroup: 16 x 16 (waves of 16 x 4) for the
// tiled layout, whose 8 x 4 tiles a wave then writes whole; 64 x 4 (waves of
// one 64-texel row segment) for the row layout, so every slab store of a
// wave is one contiguous 256-byte run.
#ifndef VI_BUILD_ROW_RUN
#define VI_BUILD_ROW_RUN 64
#endif
template <int SL> struct BuildBlock { static constexpr int X = 16, Y = 16, WX = 16; };
template <> struct BuildBlock<VI_STACK_ROWS> {
    static constexpr int WX = VI_BUILD_ROW_RUN;       // texels of a row per wave
    static constexpr int X = WX, Y = 4 * (64 / WX);
};

// Row layout: a lane stores its own texel and, on the edge of the grid, the
// fully transmitting border texels next to it (the corners by the corner
// lanes).
// stack stores: streamed past the caches (the render reads the stack long
// after the build has moved on)
template <typename ET>
__device__ __forceinline__ void put(ET* p, ET v)
{
#ifdef VI_BUILD_NT
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}

template <typename ET>
__device__ __forceinline__ void put_rows(ET* __restrict__ out, const BuildParams& P, int k, int i, int j, ET v,
                                         ET one)
{
    const int r = P.res;
    // texel (i, j) of this layer at row j+1, column rorg+i
    ET* L = out + (size_t)k * P.rlayer + P.rorg;
    const uint32_t row = (uint32_t)(j + 1) * P.rpitch, last = (uint32_t)(r + 1) * P.rpitch;
    put(L + row + i, v);
    const bool lo_i = i == 0, hi_i = i == r - 1, lo_j = j == 0, hi_j = j == r - 1;
    if (lo_i) L[row - 1] = one;
    if (hi_i) L[row + r] = one;
    if (lo_j) L[i] = one;
    if (hi_j) L[last + i] = one;
    if (lo_i && lo_j) L[-1] = one;
    if (hi_i && lo_j) L[r] = one;
    if (lo_i && hi_j) L[last - 1] = one;
    if (hi_i && hi_j) L[last + r] = one;
}

template <typename VT, int LAYOUT, int OUT_DTYPE, int SL>
__global__ __launch_bounds__(256) void build_kernel(BuildParams P)
{
    extern __shared__ float s_alpha[];  // K alphas, then K next-opaque indices
    int* s_next = (int*)(s_alpha + P.K);
    for (int t = threadIdx.x; t < P.K; t += blockDim.x) s_alpha[t] = P.tf[4 * t + 3];
    if (P.occ.mm) build_next_opaque(s_next, P.tf, P.K);
    __syncthreads();

    constexpr int BX = BuildBlock<SL>::X, BY = BuildBlock<SL>::Y;
    const uint32_t tiles_x = (P.res + BX - 1) / BX, tiles_y = (P.res + BY - 1) / BY;
    uint32_t tx, ty;
    if (!supertile_of(blockIdx.x, tiles_x, tiles_y, &tx, &ty)) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int WX = BuildBlock<SL>::WX, WY = 64 / WX;  // wave footprint
    const int i = (int)tx * BX + lane % WX;
    const int j = (int)ty * BY + wave * WY + lane / WX;
    if (i >= P.res || j >= P.res) return;

    // column base (slab 0 midpoint) in offset-voxel coordinates, in double
    const float hx0 = (float)(P.B0[0] + i * P.BU[0] + j * P.BV[0]);
    const float hy0 = (float)(P.B0[1] + i * P.BU[1] + j * P.BV[1]);
    const float hz0 = (float)(P.B0[2] + i * P.BU[2] + j * P.BV[2]);

    const VT* __restrict__ vol = (const VT*)P.vol;
    const VolIndex VI_ = {1u, P.vsy, P.vsz};
    const float Km1 = (float)(P.K - 1);
    const size_t layer = P.layer;
    const size_t col = stack_oj(j, P.row_tiles32) + stack_oi(i);
    float T = 1.0f;     // transmittance (F32 form)
    float tau = 0.0f;   // optical depth (BF16 form)
    const float ln2 = 0.69314718055994531f;
    uint32_t last_cell = 0xffffffffu;
    bool cell_is_empty = false;

#ifdef VI_BUILD_UNROLL
#pragma unroll VI_BUILD_UNROLL
#endif
    for (int k = 0; k < P.n; ++k) {
        const float kf = (float)k;
        const float hx = fmaf(kf, P.AL[0], hx0);
        const float hy = fmaf(kf, P.AL[1], hy0);
        const float hz = fmaf(kf, P.AL[2], hz0);
        // log2 of the slab's (1 - alpha)/e, 0 outside the cube (empty)
        float l2 = 0.0f;
        bool fetch = hx >= P.lo && hx <= P.hi && hy >= P.lo && hy <= P.hi && hz >= P.lo && hz <= P.hi;
        if (fetch && P.occ.mm) {
            // empty-space map: a zero-opacity cell leaves T unchanged exactly
            const uint32_t c = cell_of((int)floorf(hx) + P.M, (int)floorf(hy) + P.M, (int)floorf(hz) + P.M, P.N,
                                       P.occ.shift, P.occ.nc);
            if (c != last_cell) {
                last_cell = c;
                cell_is_empty = cell_empty(P.occ.mm[c], s_next, Km1, P.K);
            }
            fetch = !cell_is_empty;
        }
        if (fetch) {
            const float v = sample_volume<VT, LAYOUT>(vol, VI_, P.N, P.M, P.scale, hx, hy, hz);
            const float x = v * Km1;
            const int e0 = min((int)x, P.K - 2);
            const float w = x - (float)e0;
            const float a = fmaf(w, s_alpha[e0 + 1] - s_alpha[e0], s_alpha[e0]);
            l2 = fast_log2(fmaxf(1.0f - a, 0.0f));  // -inf for a = 1
        }
        if (OUT_DTYPE == VI_F32) {
            // (1 - alpha(ds)) = (1 - a)^(ds / dref) = 2^(e log2(1 - a))
            float f = fast_exp2(P.e * l2);
            // section 4 compensation: times (1 + alpha)^m, at most 1
            if (P.darken > 0.0f) f = fminf(f * fast_exp2(P.darken * fast_log2(2.0f - f)), 1.0f);
            T *= f;
            if (SL == VI_STACK_ROWS) {
                put_rows((float*)P.out, P, k, i, j, T, 1.0f);
            } else {
                put((float*)P.out + (size_t)k * layer + col, T);
            }
        } else {
            // sigma * ds = -e ln(1 - a), capped at 64 per slab; the
            // compensation subtracts m ln(1 + alpha), floored at 0
            float dtau = -P.e * ln2 * l2;
            if (P.darken > 0.0f) dtau = fmaxf(dtau - P.darken * ln2 * fast_log2(2.0f - fast_exp2(P.e * l2)), 0.0f);
            tau += fminf(dtau, 64.0f);
            if (SL == VI_STACK_ROWS) {
                put_rows((uint16_t*)P.out, P, k, i, j, f32_to_bf16(tau), (uint16_t)0);
            } else {
                put((uint16_t*)P.out + (size_t)k * layer + col, f32_to_bf16(tau));
            }
        }
    }
}

template <typename VT, int LAYOUT>
static hipError_t launch_build_t(const BuildParams& p, hipStream_t s)
{
    const bool rows = p.out_layout == VI_STACK_ROWS;
    const uint32_t bx = rows ? BuildBlock<VI_STACK_ROWS>::X : BuildBlock<VI_STACK_TILED>::X;
    const uint32_t by = rows ? BuildBlock<VI_STACK_ROWS>::Y : BuildBlock<VI_STACK_TILED>::Y;
    dim3 grid(supertile_grid(((uint32_t)p.res + bx - 1) / bx, ((uint32_t)p.res + by - 1) / by)), block(256);
    const size_t lds = (sizeof(float) + sizeof(int)) * (size_t)p.K;
    if (p.out_dtype == VI_F32) {
        if (rows) hipLaunchKernelGGL((build_kernel<VT, LAYOUT, VI_F32, VI_STACK_ROWS>), grid, block, lds, s, p);
        else hipLaunchKernelGGL((build_kernel<VT, LAYOUT, VI_F32, VI_STACK_TILED>), grid, block, lds, s, p);
    } else {
        if (rows) hipLaunchKernelGGL((build_kernel<VT, LAYOUT, VI_BF16, VI_STACK_ROWS>), grid, block, lds, s, p);
        else hipLaunchKernelGGL((build_kernel<VT, LAYOUT, VI_BF16, VI_STACK_TILED>), grid, block, lds, s, p);
    }
    return hipGetLastError();
}

template <typename VT>
static hipError_t launch_build_l(const BuildParams& p, hipStream_t s)
{
    return p.vol_layout == VI_LAYOUT_BRICK4 ? launch_build_t<VT, VI_LAYOUT_BRICK4>(p, s)
                                            : launch_build_t<VT, VI_LAYOUT_LINEAR>(p, s);
}

hipError_t launch_build(const BuildParams& p, hipStream_t s)
{
    switch (p.vol_dtype) {
    case VI_U8: return launch_build_l<uint8_t>(p, s);
    case VI_U16: return launch_build_l<uint16_t>(p, s);
    case VI_F16: return launch_build_l<__half>(p, s);
    default: return launch_build_l<float>(p, s);
    }
}

}  // namespace vi
