// vi_layout.hip -- volume layout conversion: linear raw[z][y][x] -> 4x4x4
// bricks (one 64-element brick = one 128-byte line at 16 bits), or the quad
// layout (brick order, every slot holding its voxel's 2x2 x/y neighbourhood).  One thread
// per destination element, so the stores are fully coalesced; each run of
// four source elements along x is contiguous.  A bit-exact copy: results
// computed from the bricked volume equal those from the linear one.
#include "vi_device.h"
#include "vi_internal.h"

namespace vi {

template <typename T>
__global__ __launch_bounds__(256) void to_bricks_kernel(const T* __restrict__ src, T* __restrict__ dst, int N,
                                                        uint32_t nb, uint64_t total)
{
    const uint64_t idx = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    if (idx >= total) return;
    const uint32_t b = (uint32_t)(idx >> 6), w = (uint32_t)(idx & 63u);
    const uint32_t bx = b % nb, by = (b / nb) % nb, bz = b / (nb * nb);
    const int x = (int)(bx * 4u + (w & 3u)), y = (int)(by * 4u + ((w >> 2) & 3u)), z = (int)(bz * 4u + (w >> 4));
    T v = T(0);
    if (x < N && y < N && z < N) v = src[((size_t)z * N + y) * N + x];
    dst[idx] = v;
}

template <typename T>
static hipError_t launch_t(const void* src, void* dst, int N, hipStream_t s)
{
    const uint32_t NP = round_up((uint32_t)N, 4u), nb = NP / 4u;
    const uint64_t total = (uint64_t)NP * NP * NP;
    const uint64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL((to_bricks_kernel<T>), dim3((uint32_t)blocks), dim3(256), 0, s, (const T*)src, (T*)dst, N,
                       nb, total);
    return hipGetLastError();
}

hipError_t launch_to_bricks(const void* src, void* dst, int dtype, int N, hipStream_t s)
{
    switch (dtype) {
    case VI_U8: return launch_t<uint8_t>(src, dst, N, s);
    case VI_U16:
    case VI_F16: return launch_t<uint16_t>(src, dst, N, s);
    default: return launch_t<uint32_t>(src, dst, N, s);
    }
}

// Quad layout: one thread per slot (brick order as above); the slot holds
// its voxel's 2x2 neighbourhood in x and y, indices clamped to N-1, stored
// with one 4-element store.  Padding slots hold zeros (never read).
template <typename T, typename T4>
__global__ __launch_bounds__(256) void to_quads_kernel(const T* __restrict__ src, T4* __restrict__ dst, int N,
                                                       uint32_t nb, uint64_t total)
{
    const uint64_t idx = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    if (idx >= total) return;
    const uint32_t b = (uint32_t)(idx >> 6), w = (uint32_t)(idx & 63u);
    const uint32_t bx = b % nb, by = (b / nb) % nb, bz = b / (nb * nb);
    const int x = (int)(bx * 4u + (w & 3u)), y = (int)(by * 4u + ((w >> 2) & 3u)), z = (int)(bz * 4u + (w >> 4));
    T4 q;
    q.x = q.y = q.z = q.w = T(0);
    if (x < N && y < N && z < N) {
        const int x1 = min(x + 1, N - 1), y1 = min(y + 1, N - 1);
        const size_t r0 = ((size_t)z * N + y) * N, r1 = ((size_t)z * N + y1) * N;
        q.x = src[r0 + x];
        q.y = src[r0 + x1];
        q.z = src[r1 + x];
        q.w = src[r1 + x1];
    }
    dst[idx] = q;
}

template <typename T, typename T4>
static hipError_t launch_q(const void* src, void* dst, int N, hipStream_t s)
{
    const uint32_t NP = round_up((uint32_t)N, 4u), nb = NP / 4u;
    const uint64_t total = (uint64_t)NP * NP * NP;
    const uint64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL((to_quads_kernel<T, T4>), dim3((uint32_t)blocks), dim3(256), 0, s, (const T*)src, (T4*)dst,
                       N, nb, total);
    return hipGetLastError();
}

hipError_t launch_to_quads(const void* src, void* dst, int dtype, int N, hipStream_t s)
{
    switch (dtype) {
    case VI_U8: return launch_q<uint8_t, uchar4>(src, dst, N, s);
    case VI_U16:
    case VI_F16: return launch_q<uint16_t, ushort4>(src, dst, N, s);
    default: return launch_q<uint32_t, uint4>(src, dst, N, s);
    }
}

// Empty-space map: one thread per cell, min/max of the normalised voxel
// values over the cell's voxels plus one more along each axis (clamped).
template <typename VT, int LAYOUT>
__global__ __launch_bounds__(256) void minmax_kernel(const VT* __restrict__ vol, VolIndex I, int N, float scale,
                                                     int shift, uint32_t nc, float2* __restrict__ out)
{
    const uint32_t c = blockIdx.x * 256u + threadIdx.x;
    if (c >= nc * nc * nc) return;
    const int cx = (int)(c % nc), cy = (int)((c / nc) % nc), cz = (int)(c / (nc * nc));
    const int B = 1 << shift;
    const int x0 = cx * B, y0 = cy * B, z0 = cz * B;
    const int x1 = min(x0 + B, N - 1), y1 = min(y0 + B, N - 1), z1 = min(z0 + B, N - 1);
    float lo = 1.0f, hi = 0.0f;
    for (int z = z0; z <= z1; ++z) {
        const uint32_t oz = vol_oz<LAYOUT>(I, z);
        for (int y = y0; y <= y1; ++y) {
            const uint32_t oy = oz + vol_oy<LAYOUT>(I, y);
            for (int x = x0; x <= x1; ++x) {
                // a quad slot's first element is its own voxel
                const uint32_t o = oy + vol_ox<LAYOUT>(I, x);
                const float v = LAYOUT == VI_LAYOUT_QUAD4 ? voxel_norm(vol + 4 * (size_t)o, 0u, scale)
                                                          : voxel_norm(vol, o, scale);
                lo = fminf(lo, v);
                hi = fmaxf(hi, v);
            }
        }
    }
    out[c] = make_float2(lo, hi);
}

template <typename VT>
static hipError_t launch_mm(const void* vol, int layout, VolIndex I, int N, float scale, int shift, float* out,
                            hipStream_t s)
{
    const uint32_t nc = ((uint32_t)N + (1u << shift) - 1) >> shift;
    const uint32_t cells = nc * nc * nc;
    dim3 grid((cells + 255) / 256), block(256);
    if (layout == VI_LAYOUT_QUAD4)
        hipLaunchKernelGGL((minmax_kernel<VT, VI_LAYOUT_QUAD4>), grid, block, 0, s, (const VT*)vol, I, N, scale,
                           shift, nc, (float2*)out);
    else if (layout == VI_LAYOUT_BRICK4)
        hipLaunchKernelGGL((minmax_kernel<VT, VI_LAYOUT_BRICK4>), grid, block, 0, s, (const VT*)vol, I, N, scale,
                           shift, nc, (float2*)out);
    else
        hipLaunchKernelGGL((minmax_kernel<VT, VI_LAYOUT_LINEAR>), grid, block, 0, s, (const VT*)vol, I, N, scale,
                           shift, nc, (float2*)out);
    return hipGetLastError();
}

hipError_t launch_minmax(const void* vol, int dtype, int layout, uint32_t vsy, uint32_t vsz, int N, float scale,
                         int shift, float* out, hipStream_t s)
{
    const VolIndex I = {1u, vsy, vsz};
    switch (dtype) {
    case VI_U8: return launch_mm<uint8_t>(vol, layout, I, N, scale, shift, out, s);
    case VI_U16: return launch_mm<uint16_t>(vol, layout, I, N, scale, shift, out, s);
    case VI_F16: return launch_mm<__half>(vol, layout, I, N, scale, shift, out, s);
    default: return launch_mm<float>(vol, layout, I, N, scale, shift, out, s);
    }
}

// Occupancy bits for one transfer function: one thread per 32-cell word,
// bit i = cell 32w+i may hold opacity (the negation of the map's emptiness
// test against the table's next-opaque indices, built in LDS per block).
__global__ __launch_bounds__(256) void occupancy_kernel(const float2* __restrict__ mm, uint32_t cells,
                                                        const float* __restrict__ tf, int K, uint32_t* __restrict__ bits)
{
    extern __shared__ int s_next[];
    build_next_opaque(s_next, tf, K);
    __syncthreads();
    const uint32_t w = blockIdx.x * 256u + threadIdx.x;
    const uint32_t words = (cells + 31u) / 32u;
    if (w >= words) return;
    const float Km1 = (float)(K - 1);
    uint32_t b = 0;
    for (uint32_t i = 0; i < 32u; ++i) {
        const uint32_t c = w * 32u + i;
        if (c < cells && !cell_empty(mm[c], s_next, Km1, K)) b |= 1u << i;
    }
    bits[w] = b;
}

// Super-cell bits: super-cell (X, Y, Z) covers cells 4X .. 4X+3 (and so on,
// clipped at nc) and is set when any of them is.  One lane per super-cell;
// each half-wave's ballot is one word.
__global__ __launch_bounds__(256) void super_kernel(const uint32_t* __restrict__ bits, uint32_t nc,
                                                    uint32_t* __restrict__ sbits)
{
    const uint32_t snc = (nc + 3u) / 4u, scells = snc * snc * snc;
    const uint32_t sc = blockIdx.x * 256u + threadIdx.x;
    bool any = false;
    if (sc < scells) {
        const uint32_t X = sc % snc, Y = (sc / snc) % snc, Z = sc / (snc * snc);
        for (uint32_t z = 4u * Z; z < min(4u * Z + 4u, nc); ++z)
            for (uint32_t y = 4u * Y; y < min(4u * Y + 4u, nc); ++y)
                for (uint32_t x = 4u * X; x < min(4u * X + 4u, nc); ++x) {
                    const uint32_t c = (z * nc + y) * nc + x;
                    any = any || ((bits[c >> 5] >> (c & 31u)) & 1u);
                }
    }
    const uint64_t m = __ballot(any);
    const uint32_t lane = threadIdx.x & 63u;
    if ((lane & 31u) == 0u && sc < scells) sbits[sc >> 5] = (uint32_t)(lane ? (m >> 32) : m);
}

hipError_t launch_occupancy(const float* minmax, uint32_t nc, const float* tf, int K, uint32_t* bits,
                            hipStream_t s)
{
    const uint32_t cells = nc * nc * nc, words = (cells + 31u) / 32u;
    hipLaunchKernelGGL(occupancy_kernel, dim3((words + 255u) / 256u), dim3(256), sizeof(int) * (size_t)K, s,
                       (const float2*)minmax, cells, tf, K, bits);
    const uint32_t snc = (nc + 3u) / 4u;
    hipLaunchKernelGGL(super_kernel, dim3((snc * snc * snc + 255u) / 256u), dim3(256), 0, s, (const uint32_t*)bits,
                       nc, bits + words);
    return hipGetLastError();
}

}  // namespace vi
