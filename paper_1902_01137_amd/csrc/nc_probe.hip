// Random-read rate of the device: the ceiling of a tracer whose every
// tentative collision reads one 4-byte value at an unpredictable address.
// Not part of the transport method; it gives the roofline its measured peak.
#include <hip/hip_runtime.h>
#include <cstdint>
#include "nc_internal.hpp"

namespace nc {

__device__ inline uint32_t mix32(uint32_t x)
{
    // integer finaliser (a bijection on 32 bits): spreads consecutive
    // counters over the whole buffer
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

// Each thread issues `loads` independent 4-byte reads (8 in flight per
// batch) at hashed addresses below mask + 1 and writes their sum.
__global__ __launch_bounds__(256) void gather_rate_kernel(const float *__restrict__ buf, uint32_t mask, int loads,
                                                          uint32_t seed, float *__restrict__ out)
{
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    float acc = 0.0f;
    for (int i = 0; i < loads; i += 8) {
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = buf[mix32(tid * 0x9E3779B9U + (uint32_t)(i + j) * 0x85EBCA6BU + seed) & mask];
#pragma unroll
        for (int j = 0; j < 8; ++j) acc += v[j];
    }
    out[tid] = acc;
}

hipError_t launch_gather_rate(const nc_ctx *ctx, const float *buf, uint32_t mask, int threads, int loads,
                              uint32_t seed, float *out)
{
    hipLaunchKernelGGL(gather_rate_kernel, dim3(threads / 256), dim3(256), 0, ctx->stream, buf, mask, loads, seed,
                       out);
    return hipGetLastError();
}

}  // namespace nc
