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
#include <algorithm>

#include "vi_device.h"
#include "vi_internal.h"

namespace vi {

// Block of texel columns per workgroup: 16 x 16 (waves of 16 x 4) for the
// tiled layout, whose 8 x 4 tiles a wave then writes whole; 64 x 4 (waves of
// one 64-texel row segment) for the row layout, so every slab store of a
// wave is one contiguous 256-byte run.
template <int SL> struct BuildBlock { static constexpr int X = 16, Y = 16, WX = 16; };
template <> struct BuildBlock<VI_STACK_ROWS> {
    static constexpr int WX = 64, X = 64, Y = 4;  // a wave: one 64-texel row run
};

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

// slabs per batch of the build loop
#ifndef VI_BUILD_BATCH
#define VI_BUILD_BATCH 4
#endif
constexpr int kBatch = VI_BUILD_BATCH;

template <typename VT, int LAYOUT, int OUT_DTYPE, int SL, bool DARKEN>
__device__ __forceinline__ void build_columns(const BuildParams& P)
{
    extern __shared__ float s_alpha[];  // K alphas, K next-opaque indices, then the occupancy bits
    int* s_next = (int*)(s_alpha + P.K);
    uint32_t* s_bits = (uint32_t*)(s_next + P.K);
    for (int t = threadIdx.x; t < P.K; t += blockDim.x) s_alpha[t] = P.tf[4 * t + 3];
    build_next_opaque(s_next, P.tf, P.K);  // read by every batch (unused without a map)
    stage_occupancy(P.occ, s_bits);
    __syncthreads();

    constexpr int BX = BuildBlock<SL>::X, BY = BuildBlock<SL>::Y;
    const uint32_t tiles_x = (P.res + BX - 1) / BX, tiles_y = (P.res + BY - 1) / BY;
    uint32_t tx, ty;
    if (!supertile_of(blockIdx.x, tiles_x, tiles_y, &tx, &ty)) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // wave footprint WX x WY; the block's waves are laid out along x first
    constexpr int WX = BuildBlock<SL>::WX, WY = 64 / WX, NWX = BX / WX;
    const int i = (int)tx * BX + (wave % NWX) * WX + lane % WX;
    const int j = (int)ty * BY + (wave / NWX) * WY + lane / WX;
    if (i >= P.res || j >= P.res) return;

    // column base (slab 0 midpoint) in offset-voxel coordinates, in double
    const float hx0 = (float)(P.B0[0] + i * P.BU[0] + j * P.BV[0]);
    const float hy0 = (float)(P.B0[1] + i * P.BU[1] + j * P.BV[1]);
    const float hz0 = (float)(P.B0[2] + i * P.BU[2] + j * P.BV[2]);
    // step per slab, and the slab exponent (its length in voxels); a point
    // light's column is its own ray from the light
    float alx = P.AL[0], aly = P.AL[1], alz = P.AL[2], e = P.e;
    if (P.point) {
        const double ax = P.AL0[0] + i * P.ALU[0] + j * P.ALV[0];
        const double ay = P.AL0[1] + i * P.ALU[1] + j * P.ALV[1];
        const double az = P.AL0[2] + i * P.ALU[2] + j * P.ALV[2];
        alx = (float)ax;
        aly = (float)ay;
        alz = (float)az;
        e = (float)sqrt(ax * ax + ay * ay + az * az);
    }

    const VT* __restrict__ vol = (const VT*)P.vol;
    const VolIndex VI_ = {1u, P.vsy, P.vsz};
    const float Km1 = (float)(P.K - 1);
    // this column's texel in layer 0, and the layer stride (elements)
    const size_t layer = SL == VI_STACK_ROWS ? (size_t)P.rlayer : (size_t)P.layer;
    size_t at = SL == VI_STACK_ROWS ? (size_t)(j + 1) * P.rpitch + P.rorg + i
                                    : (size_t)(stack_oj(j, P.row_tiles32) + stack_oi(i));
    float T = 1.0f;     // transmittance (F32 form)
    float tau = 0.0f;   // optical depth (BF16 form)
    const float ln2 = 0.69314718055994531f;
    uint32_t last_cell = 0xffffffffu;
    bool cell_is_empty = false;
    const bool use_map = P.occ.mm != nullptr;
    const bool use_bits = P.occ.bits != nullptr;  // verdicts from the occupancy bits, no map loads

    // The slabs go in batches of kBatch: first every slab's position and the
    // map entries of newly entered cells (loaded together), then the
    // empty-space verdicts, then the volume loads of all slabs that need one,
    // and only then the arithmetic, the running product and the stores -- so
    // a column waits on one round trip per batch instead of one per slab.
    // Each slab's arithmetic is the same as one at a time.
    for (int k0 = 0; k0 < P.n; k0 += kBatch) {
        float hx[kBatch], hy[kBatch], hz[kBatch];
        bool fetch[kBatch];
        uint32_t cell[kBatch];
        float2 mm[kBatch];
        uint32_t cur = last_cell;  // cell of the latest slab inside the cube
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const float kf = (float)(k0 + u);
            hx[u] = fmaf(kf, alx, hx0);
            hy[u] = fmaf(kf, aly, hy0);
            hz[u] = fmaf(kf, alz, hz0);
            fetch[u] = (k0 + u < P.n) & (hx[u] >= P.lo) & (hx[u] <= P.hi) & (hy[u] >= P.lo) & (hy[u] <= P.hi) &
                       (hz[u] >= P.lo) & (hz[u] <= P.hi);
            cell[u] = 0xffffffffu;
            mm[u] = make_float2(0.0f, 0.0f);
            if (fetch[u] && use_map) {
                cell[u] = cell_of((int)floorf(hx[u]) + P.M, (int)floorf(hy[u]) + P.M, (int)floorf(hz[u]) + P.M, P.N,
                                  P.occ.shift, P.occ.nc);
                if (cell[u] != cur) {
                    if (!use_bits) mm[u] = P.occ.mm[cell[u]];  // a newly entered cell
                    cur = cell[u];
                }
            }
        }
        // Empty-space verdicts: a zero-opacity cell leaves T unchanged
        // exactly.  Every entry's verdict is taken, on every path and with
        // selects rather than branches (entries not loaded hold zeros and
        // their verdicts are not used; without a map none is), so no map
        // load is left in flight behind the volume loads below.  The cell
        // sequence is the one above, so an entry is loaded wherever its
        // verdict is used.
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            // Both verdicts are taken and one is selected (slabs outside the
            // cube, and runs without bits, read word 0 of the bits: always
            // allocated, unused then)
            const uint32_t cq = (cell[u] == 0xffffffffu || !use_bits) ? 0u : cell[u];
            const bool empty_bit = !occupancy_bit(s_bits, cq);
            const bool empty_map = cell_empty(mm[u], s_next, Km1, P.K);
            const bool empty = use_bits ? empty_bit : empty_map;
            const bool entered = use_map && fetch[u] && cell[u] != last_cell;
            cell_is_empty = entered ? empty : cell_is_empty;
            last_cell = entered ? cell[u] : last_cell;
            fetch[u] = fetch[u] && !cell_is_empty;
        }
        RawFoot<VT, LAYOUT> raw[kBatch];
        float wx[kBatch], wy[kBatch], wz[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u)
            if (fetch[u]) foot_load<VT, LAYOUT>(raw[u], wx[u], wy[u], wz[u], vol, VI_, P.N, P.M, hx[u], hy[u], hz[u]);
#pragma unroll
        for (int u = 0; u < kBatch; ++u, at += layer) {
            if (k0 + u >= P.n) break;
            // log2 of the slab's (1 - alpha)/e, 0 outside the cube or in empty cells
            float l2 = 0.0f;
            if (fetch[u]) {
                const float v = foot_value<VT, LAYOUT>(raw[u], wx[u], wy[u], wz[u], P.scale);
                const float x = v * Km1;
                const int e0 = min((int)x, P.K - 2);
                const float w = x - (float)e0;
                const float a = fmaf(w, s_alpha[e0 + 1] - s_alpha[e0], s_alpha[e0]);
                l2 = fast_log2(fmaxf(1.0f - a, 0.0f));  // -inf for a = 1
            }
            if (OUT_DTYPE == VI_F32) {
                // (1 - alpha(ds)) = (1 - a)^(ds / dref) = 2^(e log2(1 - a))
                float f = fast_exp2(e * l2);
                // section 4 compensation: times (1 + alpha)^m, at most 1
                if (DARKEN) f = fminf(f * fast_exp2(P.darken * fast_log2(2.0f - f)), 1.0f);
                T *= f;
                ((float*)P.out)[at] = T;
            } else {
                // sigma * ds = -e ln(1 - a), capped at 64 per slab; the
                // compensation subtracts m ln(1 + alpha), floored at 0
                float dtau = -e * ln2 * l2;
                if (DARKEN) dtau = fmaxf(dtau - P.darken * ln2 * fast_log2(2.0f - fast_exp2(e * l2)), 0.0f);
                tau += fminf(dtau, 64.0f);
                ((uint16_t*)P.out)[at] = f32_to_bf16(tau);
            }
        }
    }
}

// The kernel.  With the quad layout of 8- and 16-bit voxels a batch's
// footprints take few registers, and five resident waves per SIMD (at most
// 96 VGPRs, no spills) measured faster than the compiler's choice of four;
// the other cases (eight voxels per footprint, 32-bit quads, the
// compensation) keep the compiler's budget.
template <typename VT, int LAYOUT, int OUT_DTYPE, int SL, bool DARKEN>
__global__ __launch_bounds__(256) void build_kernel(BuildParams P)
{
    build_columns<VT, LAYOUT, OUT_DTYPE, SL, DARKEN>(P);
}
#ifndef VI_BUILD_QUAD_WAVES
#define VI_BUILD_QUAD_WAVES 5
#endif
template <typename VT, int OUT_DTYPE, int SL, bool DARKEN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(VI_BUILD_QUAD_WAVES))) void build_kernel_quads(
    BuildParams P)
{
    build_columns<VT, VI_LAYOUT_QUAD4, OUT_DTYPE, SL, DARKEN>(P);
}

template <typename VT, int LAYOUT, int SL, bool DARKEN>
static void launch_build_k(const BuildParams& p, dim3 grid, size_t lds, hipStream_t s)
{
    constexpr bool kFive = LAYOUT == VI_LAYOUT_QUAD4 && sizeof(VT) <= 2 && !DARKEN;
    if (p.out_dtype == VI_F32)
        if constexpr (kFive)
            hipLaunchKernelGGL((build_kernel_quads<VT, VI_F32, SL, DARKEN>), grid, dim3(256), lds, s, p);
        else
            hipLaunchKernelGGL((build_kernel<VT, LAYOUT, VI_F32, SL, DARKEN>), grid, dim3(256), lds, s, p);
    else if constexpr (kFive)
        hipLaunchKernelGGL((build_kernel_quads<VT, VI_BF16, SL, DARKEN>), grid, dim3(256), lds, s, p);
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
    // (at least one word of bits, which the slab loop reads even without them)
    const size_t lds = (sizeof(float) + sizeof(int)) * (size_t)p.K + sizeof(uint32_t) * std::max(p.occ.words, 1u);
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
    if (p.vol_layout == VI_LAYOUT_QUAD4) return launch_build_t<VT, VI_LAYOUT_QUAD4>(p, s);
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
