// vi_build.hip -- light-space attenuation build (section 3.2.1, Alg. 1).
//
// Every texel column of the light square is scanned over the n slabs from
// the light (Eq. 8 ordering): per slab the volume is sampled at the slab
// midpoint, the transfer-function opacity is looked up and corrected to the
// slab thickness (extinction form, Eq. 6), and the running transmittance is
// multiplied by (1 - alpha) -- Eq. 4 applied to opacity.  Every layer is
// written as soon as it is known, so the pass is one streaming sweep: the
// volume is read through the caches and the stack is written once.
//
// Mapping: one workgroup per run of NT * C texels of one stack row, lane l
// owning columns l, l + NT, ..., l + NT (C - 1) of the run.  At every slab a
// workgroup stores its run as one contiguous stretch of the layer (4 KiB for
// a 1024-texel row); many short runs spread over the layer (64 x 4 texel
// tiles per workgroup) measured at half that write rate.  For a fixed c the
// 64 lanes of a wave hold 64 neighbouring columns, so each volume gather of
// a wave stays compact.
//
// Per column the slabs whose midpoints lie in the cube form one interval
// [k_in, k_out], found once by exact integer division; a wave stores the
// unattenuated layers in front of its columns' union of intervals and the
// final transmittance behind it without touching the volume, and runs the
// full per-slab work (fetch, transfer function, Eq. 6 correction, product)
// only inside.  Empty-space verdicts come from the occupancy bits in LDS
// (without bits every slab in the cube is fetched).
//
// Slab-midpoint positions are fixed-point numbers (h * 2^40 in an int64, h
// the offset-voxel coordinate), so stepping from slab to slab is an exact
// integer add and the voxel index and trilinear weight are exact bit fields
// of the position: no rounding accumulates over the 512 slabs, and a float
// would resolve |h| ~ N/2 only to 2^-16 voxel.
#include <algorithm>

#include "vi_device.h"
#include "vi_internal.h"

namespace vi {

// Row layout: the texels of the two-texel border around the grid are the
// same in every layer, and so is the whole leading layer -1 (fully
// transmitting: T = 1, optical depth 0), so a separate small kernel writes
// the border rings of layers -1 .. n-1 and the slab loop stores only its own
// texels (layer -1 included).  One lane per border texel and layer: rows -2,
// -1, res, res+1 (res+4 texels each), then columns -2, -1, res, res+1 of rows
// 0..res-1.
template <typename ET>
__global__ __launch_bounds__(256) void border_kernel(ET* __restrict__ out, int n, int res, uint32_t rlayer,
                                                     uint32_t rpitch, uint32_t rorg, ET one)
{
    const uint32_t W = (uint32_t)res + 4u, per_layer = 4u * W + 4u * (uint32_t)res;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)per_layer * ((size_t)n + 1u)) return;
    const int k = (int)(t / per_layer) - 1;
    const uint32_t q = (uint32_t)(t % per_layer);
    int row, col;  // grid texel coordinates in [-2, res+1]
    if (q < 4u * W) {
        const uint32_t r = q / W;  // 0, 1, 2, 3 -> rows -2, -1, res, res+1
        row = r < 2u ? (int)r - 2 : res + (int)r - 2;
        col = (int)(q % W) - 2;
    } else {
        const uint32_t r = q - 4u * W, c = r & 3u;
        row = (int)(r >> 2);
        col = c < 2u ? (int)c - 2 : res + (int)c - 2;
    }
    out[(int64_t)rorg + (int64_t)k * rlayer + (int64_t)row * rpitch + col] = one;
}

// Workgroup b -> (row, run): rows are dealt to the 8 XCDs in groups of 4
// consecutive rows (neighbouring rows sample the same voxels and share an
// L2), the groups of an XCD spread over the whole light square.
constexpr uint32_t kRowGroup = 4;
__device__ __forceinline__ bool row_run_of(uint32_t b, uint32_t rows, uint32_t runs, uint32_t* row, uint32_t* run)
{
    const uint32_t x = b % kXcds, q = b / kXcds;  // XCD, index within it
    const uint32_t unit = q / runs, r = q % runs;
    const uint32_t grp = unit / kRowGroup, within = unit % kRowGroup;
    *row = (grp * kXcds + x) * kRowGroup + within;
    *run = r;
    return *row < rows;
}
inline uint32_t row_run_grid(uint32_t rows, uint32_t runs)
{
    const uint32_t groups = (rows + kRowGroup - 1) / kRowGroup;
    return (groups + kXcds - 1) / kXcds * kRowGroup * runs * kXcds;
}

// Q40 positions: floor(h) and the trilinear weight h - floor(h) (its top 24
// bits, exact in a float).
__device__ __forceinline__ int q_floor(int64_t H) { return (int)(H >> kQBits); }
__device__ __forceinline__ float q_frac(int64_t H)
{
    return (float)((uint32_t)((uint64_t)H >> (kQBits - 24)) & 0xFFFFFFu) * (1.0f / 16777216.0f);
}
__device__ __forceinline__ float q_to_float(int64_t H) { return (float)H * (1.0f / 1099511627776.0f); }

// (NT, C, B): threads per workgroup, columns per lane, slabs per batch;
// a lane's C columns are NT apart (CONSEC = 0: each store instruction of a
// wave covers 64 neighbouring texels) or adjacent (CONSEC = 1: one
// C-element store per lane)
#ifndef VI_BUILD_NT
#define VI_BUILD_NT 1024
#endif
#ifndef VI_BUILD_C
#define VI_BUILD_C 1
#endif
#ifndef VI_BUILD_BATCH
#define VI_BUILD_BATCH 2
#endif
#ifndef VI_BUILD_CONSEC
#define VI_BUILD_CONSEC 0
#endif
constexpr int kBuildNT = VI_BUILD_NT, kBuildC = VI_BUILD_C, kBuildB = VI_BUILD_BATCH;
constexpr bool kBuildConsec = VI_BUILD_CONSEC != 0;

// The slabs of a column whose midpoints lie in the cube: k in [k_in, k_out]
// (empty when k_in > k_out), exactly as the per-slab test lo <= h_k <= hi
// on all three axes decides it: per axis a half-line or interval of k from
// an exact integer division of Q40 values.
__device__ __forceinline__ int64_t floor_div(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
    return q;
}
__device__ __forceinline__ int64_t ceil_div(int64_t a, int64_t b) { return -floor_div(-a, b); }
__device__ __forceinline__ void slab_range(const int64_t H[3], const int64_t A[3], int n, int64_t lo, int64_t hi,
                                           int* k_in, int* k_out)
{
    int64_t kl = 0, kh = n - 1;
    for (int a = 0; a < 3; ++a) {
        if (A[a] == 0) {
            if (H[a] < lo || H[a] > hi) kl = n;  // never inside along this axis
        } else if (A[a] > 0) {
            kl = max(kl, ceil_div(lo - H[a], A[a]));
            kh = min(kh, floor_div(hi - H[a], A[a]));
        } else {
            kl = max(kl, ceil_div(hi - H[a], A[a]));
            kh = min(kh, floor_div(lo - H[a], A[a]));
        }
    }
    if (kl > kh) {
        *k_in = n;
        *k_out = -1;
    } else {
        *k_in = (int)kl;
        *k_out = (int)kh;
    }
}

__device__ __forceinline__ int wave_min(int v)
{
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off));
    return v;
}
__device__ __forceinline__ int wave_max(int v)
{
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
    return v;
}

// One stack texel: transmittance (F32), optical depth in base-2 units
// -log2 T (BF16), or the transmittance 2^-tau of the float optical depth
// rounded to half precision (F16).
// (The stack is below 4 GiB: byte offsets in 32 bits, so a store takes the
// stack's base from scalar registers.)
template <int OUT_DTYPE>
__device__ __forceinline__ void put_texel(void* out, uint32_t at, float T, float tau)
{
    if (OUT_DTYPE == VI_F32) *(float*)((char*)out + (at << 2)) = T;
    else if (OUT_DTYPE == VI_BF16) *(uint16_t*)((char*)out + (at << 1)) = f32_to_bf16(tau);
    else *(__half*)((char*)out + (at << 1)) = __float2half_rn(fast_exp2(-tau));
}

template <typename VT, int LAYOUT, int OUT_DTYPE, int SL, bool PT>
__device__ __forceinline__ void build_run(const BuildParams& P)
{
    constexpr int NT = kBuildNT, C = kBuildC, B = kBuildB;
    constexpr int CS = kBuildConsec ? 1 : NT;  // stride between a lane's columns
    extern __shared__ float s_alpha[];  // K alphas, then the occupancy bits
    uint32_t* s_bits = (uint32_t*)(s_alpha + P.K);
    for (int t = threadIdx.x; t < P.K; t += blockDim.x) s_alpha[t] = P.tf[4 * t + 3];
    // Empty-space verdicts come from the occupancy bits in LDS; without them
    // one set bit stands for "every cell may hold opacity" (cell index 0).
    const bool use_bits = P.occ.bits != nullptr;
    if (use_bits) stage_occupancy(P.occ, s_bits);
    else if (threadIdx.x == 0) s_bits[0] = 1u;
    const int cshift = use_bits ? P.occ.shift : 30;
    const uint32_t cnc = use_bits ? P.occ.nc : 1u;
    __syncthreads();

    const uint32_t runs = ((uint32_t)P.res + NT * C - 1) / (NT * C);
    uint32_t row, run;
    if (!row_run_of(blockIdx.x, (uint32_t)P.res, runs, &row, &run)) return;
    const int j = (int)row;
    const int i0 = (int)(run * NT * C) + (kBuildConsec ? C * (int)threadIdx.x : (int)threadIdx.x);

    // per column: the slab-0 midpoint and (point light) the step, in Q40;
    // the slabs inside the cube; the texel's element in layer 0
    int64_t Hx[C], Hy[C], Hz[C];
    int64_t Ax[PT ? C : 1], Ay[PT ? C : 1], Az[PT ? C : 1];
    float ex[PT ? C : 1];
    int kin[C], kout[C];
    uint32_t at[C];
    int kmin = P.n, kmax = -1;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int i = i0 + CS * c;
        const int q = PT ? c : 0;
        Hx[c] = P.B0q[0] + (int64_t)i * P.BUq[0] + (int64_t)j * P.BVq[0];
        Hy[c] = P.B0q[1] + (int64_t)i * P.BUq[1] + (int64_t)j * P.BVq[1];
        Hz[c] = P.B0q[2] + (int64_t)i * P.BUq[2] + (int64_t)j * P.BVq[2];
        if constexpr (PT) {
            Ax[c] = P.ALq[0] + (int64_t)i * P.ALUq[0] + (int64_t)j * P.ALVq[0];
            Ay[c] = P.ALq[1] + (int64_t)i * P.ALUq[1] + (int64_t)j * P.ALVq[1];
            Az[c] = P.ALq[2] + (int64_t)i * P.ALUq[2] + (int64_t)j * P.ALVq[2];
            const float ax = q_to_float(Ax[c]), ay = q_to_float(Ay[c]), az = q_to_float(Az[c]);
            ex[c] = sqrtf(fmaf(ax, ax, fmaf(ay, ay, az * az)));  // the step's length, voxels
        } else if (c == 0) {
            Ax[0] = P.ALq[0], Ay[0] = P.ALq[1], Az[0] = P.ALq[2];
            ex[0] = P.e;
        }
        if (i < P.res) {
            const int64_t H3[3] = {Hx[c], Hy[c], Hz[c]}, A3[3] = {Ax[q], Ay[q], Az[q]};
            slab_range(H3, A3, P.n, P.loq, P.hiq, &kin[c], &kout[c]);
        } else {
            kin[c] = P.n;  // not a column of the grid: no slab, no store
            kout[c] = -1;
        }
        kmin = min(kmin, kin[c]);
        kmax = max(kmax, kout[c]);
        at[c] = SL == VI_STACK_ROWS ? P.rorg + (uint32_t)j * P.rpitch + (uint32_t)i
                                    : stack_oj(j, P.row_tiles32) + stack_oi(i);
    }
    bool col[C];
#pragma unroll
    for (int c = 0; c < C; ++c) col[c] = i0 + CS * c < P.res;
    // the wave's slabs with any midpoint in the cube: [kmin, kmax]
    kmin = __builtin_amdgcn_readfirstlane(wave_min(kmin));
    kmax = __builtin_amdgcn_readfirstlane(wave_max(kmax));
    const uint32_t layer = SL == VI_STACK_ROWS ? P.rlayer : P.layer;
    // row layout: the leading layer -1 (face 0) transmits fully
    if (SL == VI_STACK_ROWS)
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (col[c]) put_texel<OUT_DTYPE>(P.out, at[c] - layer, 1.0f, 0.0f);

    // slabs in front of the cube: the light arrives unattenuated
    {
        const int k1 = min(kmin, P.n);
        for (int k = 0; k < k1; ++k)
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if (col[c]) put_texel<OUT_DTYPE>(P.out, at[c], 1.0f, 0.0f);
                at[c] += layer;
            }
    }

    const VT* __restrict__ vol = (const VT*)P.vol;
    const VolIndex VI_ = {1u, P.vsy, P.vsz};
    const float Km1 = (float)(P.K - 1);
    float T[C], tau[C];  // transmittance (F32 form), optical depth (BF16 form)
#pragma unroll
    for (int c = 0; c < C; ++c) {
        T[c] = 1.0f, tau[c] = 0.0f;
        // positions at the first slab of the wave's range
        const int q = PT ? c : 0;
        const int k0 = kmin < P.n ? kmin : 0;
        Hx[c] += (int64_t)k0 * Ax[q];
        Hy[c] += (int64_t)k0 * Ay[q];
        Hz[c] += (int64_t)k0 * Az[q];
    }
    // the section 4 compensation (1 + alpha)^m; m = 0 leaves every factor
    // unchanged exactly (f * 2^0 = f, min(f, 1) = f)
    const bool darken = P.darken > 0.0f;

    // The wave's range in batches of B slabs for all C columns: positions and
    // empty-space verdicts, then every volume load of the batch, and only then
    // the arithmetic and the stores -- one wait per batch, with C * B
    // footprints in flight.
    for (int k0 = kmin; k0 <= kmax; k0 += B) {
        bool fetch[C][B];
        int gx[C][B], gy[C][B], gz[C][B];
        float wx[C][B], wy[C][B], wz[C][B];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int q = PT ? c : 0;
#pragma unroll
            for (int u = 0; u < B; ++u) {
                // slab k0 + u: H0 + (k0 + u) A, exact
                const int64_t hx = Hx[c] + (int64_t)u * Ax[q], hy = Hy[c] + (int64_t)u * Ay[q],
                              hz = Hz[c] + (int64_t)u * Az[q];
                const int k = k0 + u;
                gx[c][u] = q_floor(hx) + P.M;
                gy[c][u] = q_floor(hy) + P.M;
                gz[c][u] = q_floor(hz) + P.M;
                wx[c][u] = q_frac(hx);
                wy[c][u] = q_frac(hy);
                wz[c][u] = q_frac(hz);
                const uint32_t cell = cell_of(gx[c][u], gy[c][u], gz[c][u], P.N, cshift, cnc);
                // a zero-opacity cell leaves T unchanged exactly
                fetch[c][u] = k >= kin[c] && k <= kout[c] && occupancy_bit(s_bits, cell);
            }
            Hx[c] += (int64_t)B * Ax[q];
            Hy[c] += (int64_t)B * Ay[q];
            Hz[c] += (int64_t)B * Az[q];
        }
        RawFoot<VT, LAYOUT> raw[C][B];
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int u = 0; u < B; ++u)
                if (fetch[c][u])
                    foot_load_g<VT, LAYOUT>(raw[c][u], wx[c][u], wy[c][u], vol, VI_, P.N, gx[c][u], gy[c][u],
                                            gz[c][u]);
#pragma unroll
        for (int u = 0; u < B; ++u) {
            if (k0 + u > kmax) break;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if (fetch[c][u]) {
                    const float v = foot_value<VT, LAYOUT>(raw[c][u], wx[c][u], wy[c][u], wz[c][u], P.scale);
                    const float x = v * Km1;
                    const int e0 = min((int)x, P.K - 2);
                    const float w = x - (float)e0;
                    // the table's opacity clamped to [0, 1], as the render clamps it
                    const float a = clampf01(fmaf(w, s_alpha[e0 + 1] - s_alpha[e0], s_alpha[e0]));
                    const float l2 = fast_log2(1.0f - a);  // -inf for a = 1
                    const float e = ex[PT ? c : 0];
                    if (OUT_DTYPE == VI_F32) {
                        // (1 - alpha(ds)) = (1 - a)^(ds / dref) = 2^(e log2(1 - a))
                        float f = fast_exp2(e * l2);
                        // section 4 compensation: times (1 + alpha)^m, at most 1
                        if (darken) f = fminf(f * fast_exp2(P.darken * fast_log2(2.0f - f)), 1.0f);
                        T[c] *= f;
                    } else {
                        // optical depth in base-2 units: sigma ds / ln 2 =
                        // -e log2(1 - a), capped at 64 / ln 2 per slab (a factor
                        // e^-64); the compensation subtracts m log2(1 + alpha),
                        // floored at 0
                        float dtau = -e * l2;
                        if (darken) dtau = fmaxf(dtau - P.darken * fast_log2(2.0f - fast_exp2(e * l2)), 0.0f);
                        tau[c] += fminf(dtau, 92.332482616893656f);
                    }
                }
                if (col[c]) put_texel<OUT_DTYPE>(P.out, at[c], T[c], tau[c]);
                at[c] += layer;
            }
        }
    }

    // slabs behind the cube: the transmittance stays as it left the cube
    for (int k = max(kmax + 1, kmin < P.n ? kmin : P.n); k < P.n; ++k)
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if (col[c]) put_texel<OUT_DTYPE>(P.out, at[c], T[c], tau[c]);
            at[c] += layer;
        }
}

template <typename VT, int LAYOUT, int OUT_DTYPE, int SL, bool PT>
__global__ __launch_bounds__(kBuildNT) void build_kernel(BuildParams P)
{
    build_run<VT, LAYOUT, OUT_DTYPE, SL, PT>(P);
}

template <typename VT, int LAYOUT, int SL, bool PT>
static void launch_build_k(const BuildParams& p, dim3 grid, size_t lds, hipStream_t s)
{
    if (p.out_dtype == VI_F32)
        hipLaunchKernelGGL((build_kernel<VT, LAYOUT, VI_F32, SL, PT>), grid, dim3(kBuildNT), lds, s, p);
    else if (p.out_dtype == VI_BF16)
        hipLaunchKernelGGL((build_kernel<VT, LAYOUT, VI_BF16, SL, PT>), grid, dim3(kBuildNT), lds, s, p);
    else if constexpr (SL == VI_STACK_ROWS)
        hipLaunchKernelGGL((build_kernel<VT, LAYOUT, VI_F16, SL, PT>), grid, dim3(kBuildNT), lds, s, p);
}

template <typename VT, int LAYOUT>
static hipError_t launch_build_t(const BuildParams& p, hipStream_t s)
{
    const uint32_t runs = ((uint32_t)p.res + kBuildNT * kBuildC - 1) / (kBuildNT * kBuildC);
    const dim3 grid(row_run_grid((uint32_t)p.res, runs));
    // (at least one word of bits: without them word 0 says "occupied")
    const size_t lds = sizeof(float) * (size_t)p.K + sizeof(uint32_t) * std::max(p.occ.words + p.occ.swords, 1u);
    if (p.out_layout == VI_STACK_ROWS) {
        if (p.point) launch_build_k<VT, LAYOUT, VI_STACK_ROWS, true>(p, grid, lds, s);
        else launch_build_k<VT, LAYOUT, VI_STACK_ROWS, false>(p, grid, lds, s);
        // the border, the same in every layer
        const size_t nb = (4u * (size_t)(p.res + 4) + 4u * (size_t)p.res) * ((size_t)p.n + 1u);
        const dim3 bgrid((uint32_t)((nb + 255) / 256));
        if (p.out_dtype == VI_F32)
            hipLaunchKernelGGL((border_kernel<float>), bgrid, dim3(256), 0, s, (float*)p.out, p.n, p.res, p.rlayer,
                               p.rpitch, p.rorg, 1.0f);
        else  // bfloat16 optical depth 0, or half-precision transmittance 1
            hipLaunchKernelGGL((border_kernel<uint16_t>), bgrid, dim3(256), 0, s, (uint16_t*)p.out, p.n, p.res,
                               p.rlayer, p.rpitch, p.rorg, (uint16_t)(p.out_dtype == VI_F16 ? 0x3c00u : 0u));
    } else {
        if (p.point) launch_build_k<VT, LAYOUT, VI_STACK_TILED, true>(p, grid, lds, s);
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
