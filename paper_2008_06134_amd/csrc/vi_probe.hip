// vi_probe.hip -- measurement probe for the benchmark, not part of the method.
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
