// vi_probe.hip -- measurement probes for the benchmark, not part of the method.
//
// Reads an L2-resident buffer many times over so that the on-chip gather
// traffic of the render frames can be quoted against a rate measured on the
// same GPU.  Each workgroup of 256 lanes reads one 4 KiB chunk (a float4 per
// lane) per iteration and walks the buffer's chunks in a stride coprime to
// their count, so a CU's recent chunks exceed its L1 and nearly every read
// is served by L2.  Built into its own library (libvi_probe.so), which only
// the benchmark loads.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__global__ __launch_bounds__(256) void l2_read_kernel(const float4* __restrict__ buf, uint32_t chunks, uint32_t step,
                                                      uint32_t iters, float* __restrict__ out)
{
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    uint32_t c = blockIdx.x % chunks;
    for (uint32_t k = 0; k < iters; ++k) {
        const float4 v = buf[(size_t)c * 256u + threadIdx.x];
        acc.x += v.x;
        acc.y += v.y;
        acc.z += v.z;
        acc.w += v.w;
        c += step;
        if (c >= chunks) c -= chunks;
    }
    out[(size_t)blockIdx.x * 256u + threadIdx.x] = acc.x + acc.y + acc.z + acc.w;
}

}  // namespace

// Read `chunks` 4 KiB chunks of `buf` (device, chunks * 4096 bytes, 16-byte
// aligned) `iters` times per workgroup over `blocks` workgroups, stepping
// `step` chunks (step < chunks, coprime to chunks); writes one float per
// lane to `out` (device, blocks * 256 floats).  Returns 0 or the HIP error.
extern "C" int vi_probe_l2_read(const void* buf, uint32_t chunks, uint32_t step, uint32_t iters, uint32_t blocks,
                                float* out, hipStream_t stream)
{
    if (!buf || !out || chunks == 0 || step == 0 || step >= chunks || blocks == 0) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(l2_read_kernel, dim3(blocks), dim3(256), 0, stream, (const float4*)buf, chunks, step, iters,
                       out);
    return (int)hipGetLastError();
}

// Store-only probe of the attenuation build's write pattern: `rows`
// workgroups of 1024 lanes, workgroup j writing elements
// org + j * pitch + i (i < width) of every one of `layers` layers, `lstride`
// elements apart, one float per lane per layer, as the build stores a run of
// a layer.  With org, pitch and lstride multiples of 32 floats every wave's
// store covers whole 128-byte lines; otherwise its stores straddle lines.
namespace {

__global__ __launch_bounds__(1024) void store_rows_kernel(float* __restrict__ out, uint32_t width, uint32_t layers,
                                                          uint32_t org, uint32_t pitch, uint32_t lstride)
{
    const uint32_t i = threadIdx.x;
    if (i >= width) return;
    uint32_t at = org + blockIdx.x * pitch + i;
    float v = 1.0f;
    for (uint32_t k = 0; k < layers; ++k) {
        out[at] = v;
        v *= 0.999f;
        at += lstride;
    }
}

}  // namespace

// `out` (device) holds at least org + (layers - 1) * lstride + (rows - 1) * pitch
// + width floats (the caller checks); width <= 1024.  Returns 0 or the HIP error.
extern "C" int vi_probe_store_rows(float* out, uint32_t rows, uint32_t width, uint32_t layers, uint32_t org,
                                   uint32_t pitch, uint32_t lstride, hipStream_t stream)
{
    if (!out || rows == 0 || width == 0 || width > 1024 || layers == 0) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(store_rows_kernel, dim3(rows), dim3(1024), 0, stream, out, width, layers, org, pitch, lstride);
    return (int)hipGetLastError();
}
