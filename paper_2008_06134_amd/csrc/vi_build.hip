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

// Block of texel columns per workgroup.  Tiled layout: 16 x 16, waves of
// 16 x 4 columns, so that at every slab a wave stores two whole 8 x 4 tiles
// (two full 128-byte lines).  Row layout: one 512-texel row run, each wave
// 128 texels with two adjacent columns per lane -- the lane's two slab
// products are independent (twice the work in flight) and leave as one
// 8-byte store, a wave's store being one 512-byte run of the row.
template <int SL> struct BuildBlock {
    static constexpr int CPL = 1, WX = 16, X = 16, Y = 16;  // columns per lane, wave width, block
};
template <> struct BuildBlock<VI_STACK_ROWS> {
    static constexpr int CPL = 2, WX = 128, X = 512, Y = 1;
};

typedef float f32x2_a4 __attribute__((ext_vector_type(2), aligned(4)));
constexpr int kStage = 8;  // slabs whose layers a wave stages in LDS before storing them

// Row layout: the texels of the one-texel border around the grid are the
// same in every layer (fully transmitting: T = 1, optical depth 0), so a
// separate small kernel writes them and the slab loop stores only its own
// texel.  One lane per border texel and layer: rows -1 and res (res+2 texels
// each), then columns -1 and res of rows 0..res-1.
template <typename ET>
__global__ __launch_bounds__(256) void border_kernel(ET* __restrict__ out, int n, int res, uint32_t rlayer,
                                                     uint32_t rpitch, uint32_t rorg, ET one)
{
    const uint32_t per_layer = 2u * (uint32_t)(res + 2) + 2u * (uint32_t)res;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)per_layer * (size_t)n) return;
    const uint32_t k = (uint32_t)(t / per_layer), q = (uint32_t)(t % per_layer);
    int row, col;  // grid texel coordinates in [-1, res]
    if (q < 2u * (uint32_t)(res + 2)) {
        row = q < (uint32_t)(res + 2) ? -1 : res;
        col = (int)(q % (uint32_t)(res + 2)) - 1;
    } else {
        const uint32_t r = q - 2u * (uint32_t)(res + 2);
        row = (int)(r >> 1);
        col = (r & 1u) ? res : -1;
    }
    out[(size_t)k * rlayer + (uint32_t)(row + 1) * rpitch + rorg + col] = one;
}

template <typename VT, int LAYOUT, int OUT_DTYPE, int SL, bool DARKEN>
__global__ __launch_bounds__(256) void build_kernel(BuildParams P)
{
    extern __shared__ float s_alpha[];  // K alphas, K next-opaque indices, then the waves' store stages
    int* s_next = (int*)(s_alpha + P.K);
    for (int t = threadIdx.x; t < P.K; t += blockDim.x) s_alpha[t] = P.tf[4 * t + 3];
    if (P.occ.mm) build_next_opaque(s_next, P.tf, P.K);
    __syncthreads();

    constexpr int BX = BuildBlock<SL>::X, BY = BuildBlock<SL>::Y, CPL = BuildBlock<SL>::CPL;
    const uint32_t tiles_x = (P.res + BX - 1) / BX, tiles_y = (P.res + BY - 1) / BY;
    uint32_t tx, ty;
    if (!supertile_of(blockIdx.x, tiles_x, tiles_y, &tx, &ty)) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // wave footprint WX x WY texels (CPL adjacent columns per lane); the
    // block's waves are laid out along x first
    constexpr int WX = BuildBlock<SL>::WX, LX = WX / CPL, WY = 64 / LX, NWX = BX / WX;
    const int i = (int)tx * BX + (wave % NWX) * WX + (lane % LX) * CPL;  // first column of the lane
    const int j = (int)ty * BY + (wave / NWX) * WY + lane / LX;
    if (i >= P.res || j >= P.res) return;
    const bool second = CPL == 2 && i + 1 < P.res;  // the lane's second column exists

    // column bases (slab 0 midpoint) in offset-voxel coordinates, in double
    float hx0[CPL], hy0[CPL], hz0[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        hx0[c] = (float)(P.B0[0] + (i + c) * P.BU[0] + j * P.BV[0]);
        hy0[c] = (float)(P.B0[1] + (i + c) * P.BU[1] + j * P.BV[1]);
        hz0[c] = (float)(P.B0[2] + (i + c) * P.BU[2] + j * P.BV[2]);
    }

    const VT* __restrict__ vol = (const VT*)P.vol;
    const VolIndex VI_ = {1u, P.vsy, P.vsz};
    const float Km1 = (float)(P.K - 1);
    // the lane's first texel in layer 0, and the layer stride (elements)
    const size_t layer = SL == VI_STACK_ROWS ? (size_t)P.rlayer : (size_t)P.layer;
    size_t at = SL == VI_STACK_ROWS ? (size_t)(j + 1) * P.rpitch + P.rorg + i
                                    : (size_t)(stack_oj(j, P.row_tiles32) + stack_oi(i));
    float T[CPL], tau[CPL];  // transmittance (F32 form) / optical depth (BF16 form)
    uint32_t last_cell[CPL];
    bool cell_is_empty[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        T[c] = 1.0f;
        tau[c] = 0.0f;
        last_cell[c] = 0xffffffffu;
        cell_is_empty[c] = false;
    }
    const float ln2 = 0.69314718055994531f;
    // The layers computed over kStage slabs wait in LDS (this wave's own
    // slots) and leave together: on this GPU a wait for a load also waits
    // for every store issued before it, so a store per slab would hold each
    // volume or map fetch of the next slab behind it.
    float* s_stage = (float*)(s_next + P.K) + (size_t)wave * kStage * CPL * 64;

    for (int k0 = 0; k0 < P.n; k0 += kStage) {
        const int m = min(kStage, P.n - k0);
        for (int kk = 0; kk < m; ++kk) {
            const float kf = (float)(k0 + kk);
            // The lane's columns are fetched together under wave-uniform
            // branches (a divergent branch per column would serialise their
            // memory round trips): map entries where a lane enters a new
            // cell, then the trilinear footprints of every column whenever
            // any lane of the wave has a slab with opacity.
            float hx[CPL], hy[CPL], hz[CPL], l2[CPL];
            bool fetch[CPL], enter[CPL];
            uint32_t cell[CPL];
            bool any_enter = false;
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                hx[c] = fmaf(kf, P.AL[0], hx0[c]);
                hy[c] = fmaf(kf, P.AL[1], hy0[c]);
                hz[c] = fmaf(kf, P.AL[2], hz0[c]);
                l2[c] = 0.0f;  // log2 of the slab's (1 - alpha)/e: 0 outside the cube or in empty cells
                fetch[c] = (hx[c] >= P.lo) & (hx[c] <= P.hi) & (hy[c] >= P.lo) & (hy[c] <= P.hi) &
                           (hz[c] >= P.lo) & (hz[c] <= P.hi);
                cell[c] = cell_of((int)floorf(hx[c]) + P.M, (int)floorf(hy[c]) + P.M, (int)floorf(hz[c]) + P.M,
                                  P.N, P.occ.shift, P.occ.nc);
                enter[c] = P.occ.mm && fetch[c] && cell[c] != last_cell[c];
                any_enter |= enter[c];
            }
            if (__ballot(any_enter)) {
                float2 mm[CPL];
#pragma unroll
                for (int c = 0; c < CPL; ++c)
                    if (enter[c]) mm[c] = P.occ.mm[cell[c]];
#pragma unroll
                for (int c = 0; c < CPL; ++c)
                    if (enter[c]) {
                        last_cell[c] = cell[c];
                        cell_is_empty[c] = cell_empty(mm[c], s_next, Km1, P.K);
                    }
            }
            bool any_fetch = false;
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                // an empty-space cell leaves T unchanged exactly
                fetch[c] = fetch[c] && !(P.occ.mm && cell_is_empty[c]);
                any_fetch |= fetch[c];
            }
            if (__ballot(any_fetch)) {
                float v[CPL];
#pragma unroll
                for (int c = 0; c < CPL; ++c)  // clamped addresses: safe for every lane
                    v[c] = sample_volume<VT, LAYOUT>(vol, VI_, P.N, P.M, P.scale, hx[c], hy[c], hz[c]);
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    const float x = v[c] * Km1;
                    const int e0 = min((int)x, P.K - 2);
                    const float w = x - (float)e0;
                    const float a = fmaf(w, s_alpha[e0 + 1] - s_alpha[e0], s_alpha[e0]);
                    if (fetch[c]) l2[c] = fast_log2(fmaxf(1.0f - a, 0.0f));  // -inf for a = 1
                }
            }
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                float out;
                if (OUT_DTYPE == VI_F32) {
                    // (1 - alpha(ds)) = (1 - a)^(ds / dref) = 2^(e log2(1 - a))
                    float f = fast_exp2(P.e * l2[c]);
                    // section 4 compensation: times (1 + alpha)^m, at most 1
                    if (DARKEN) f = fminf(f * fast_exp2(P.darken * fast_log2(2.0f - f)), 1.0f);
                    T[c] *= f;
                    out = T[c];
                } else {
                    // sigma * ds = -e ln(1 - a), capped at 64 per slab; the
                    // compensation subtracts m ln(1 + alpha), floored at 0
                    float dtau = -P.e * ln2 * l2[c];
                    if (DARKEN)
                        dtau = fmaxf(dtau - P.darken * ln2 * fast_log2(2.0f - fast_exp2(P.e * l2[c])), 0.0f);
                    tau[c] += fminf(dtau, 64.0f);
                    out = tau[c];
                }
                s_stage[(kk * CPL + c) * 64 + lane] = out;
            }
        }
        // the chunk's layers, one store per slab (both columns of the lane in one)
        for (int kk = 0; kk < m; ++kk, at += layer) {
            const float v0 = s_stage[(kk * CPL) * 64 + lane];
            const float v1 = s_stage[(kk * CPL + CPL - 1) * 64 + lane];
            if (OUT_DTYPE == VI_F32) {
                float* o = (float*)P.out + at;
                if (CPL == 2 && second) {
                    f32x2_a4 v;
                    v.x = v0;
                    v.y = v1;
                    *(f32x2_a4*)o = v;
                } else {
                    o[0] = v0;
                }
            } else {
                uint16_t* o = (uint16_t*)P.out + at;
                o[0] = f32_to_bf16(v0);
                if (CPL == 2 && second) o[1] = f32_to_bf16(v1);
            }
        }
    }
}

template <typename VT, int LAYOUT, int SL, bool DARKEN>
static void launch_build_k(const BuildParams& p, dim3 grid, size_t lds, hipStream_t s)
{
    if (p.out_dtype == VI_F32)
        hipLaunchKernelGGL((build_kernel<VT, LAYOUT, VI_F32, SL, DARKEN>), grid, dim3(256), lds, s, p);
    else
        hipLaunchKernelGGL((build_kernel<VT, LAYOUT, VI_BF16, SL, DARKEN>), grid, dim3(256), lds, s, p);
}

template <typename VT, int LAYOUT>
static hipError_t launch_build_t(const BuildParams& p, hipStream_t s)
{
    const bool rows = p.out_layout == VI_STACK_ROWS;
    const uint32_t bx = rows ? BuildBlock<VI_STACK_ROWS>::X : BuildBlock<VI_STACK_TILED>::X;
    const uint32_t by = rows ? BuildBlock<VI_STACK_ROWS>::Y : BuildBlock<VI_STACK_TILED>::Y;
    const dim3 grid(supertile_grid(((uint32_t)p.res + bx - 1) / bx, ((uint32_t)p.res + by - 1) / by));
    const size_t cpl = rows ? BuildBlock<VI_STACK_ROWS>::CPL : BuildBlock<VI_STACK_TILED>::CPL;
    const size_t lds = (sizeof(float) + sizeof(int)) * (size_t)p.K + sizeof(float) * 4 * kStage * cpl * 64;
    const bool dk = p.darken > 0.0f;
    if (rows) {
        if (dk) launch_build_k<VT, LAYOUT, VI_STACK_ROWS, true>(p, grid, lds, s);
        else launch_build_k<VT, LAYOUT, VI_STACK_ROWS, false>(p, grid, lds, s);
        // the border, the same in every layer
        const size_t nb = (2u * (size_t)(p.res + 2) + 2u * (size_t)p.res) * (size_t)p.n;
        const dim3 bgrid((uint32_t)((nb + 255) / 256));
        if (p.out_dtype == VI_F32)
            hipLaunchKernelGGL((border_kernel<float>), bgrid, dim3(256), 0, s, (float*)p.out, p.n, p.res, p.rlayer,
                               p.rpitch, p.rorg, 1.0f);
        else
            hipLaunchKernelGGL((border_kernel<uint16_t>), bgrid, dim3(256), 0, s, (uint16_t*)p.out, p.n, p.res,
                               p.rlayer, p.rpitch, p.rorg, (uint16_t)0);
    } else {
        if (dk) launch_build_k<VT, LAYOUT, VI_STACK_TILED, true>(p, grid, lds, s);
        else launch_build_k<VT, LAYOUT, VI_STACK_TILED, false>(p, grid, lds, s);
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
