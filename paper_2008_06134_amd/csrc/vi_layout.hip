// vi_layout.hip -- volume layout conversion: linear raw[z][y][x] -> 4x4x4
// bricks (one 64-element brick = one 128-byte line at 16 bits).  One thread
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

}  // namespace vi
