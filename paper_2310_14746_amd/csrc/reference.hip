// The sweep's access pattern without its collision: a bandwidth reference
// (see include/hlbm_reference.h).  It uses the sweep's gather and stores, so
// the loads and stores are the sweep's own instructions.
#include "hlbm.h"
#include "hlbm_reference.h"
#include "cell.hpp"

namespace hlbm {

__global__ __launch_bounds__(1024) void stream_pattern_kernel(const float* __restrict__ src,
                                                              float* __restrict__ dst,
                                                              const float* __restrict__ dfield, uint32_t P,
                                                              uint32_t nx, uint32_t ny, uint32_t nz)
{
    using L = D3Q19;
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nx) return;
    const uint32_t y = blockIdx.y, z = blockIdx.z;
    float g[L::Q];
    gather_periodic<L, StoreF32>(src, P, 0u, nx, ny, nz, x, y, z, 1.0f, g);
    const uint32_t cell = x + nx * (y + ny * z);
    g[0] += 0.0f * ld(dfield, cell);  // the porosity read the sweep makes
#pragma unroll
    for (int i = 0; i < L::Q; ++i) st_stream(dst + (size_t)i * P, cell, g[i]);
}

}  // namespace hlbm

extern "C" int hlbm_ref_stream_pattern(const void* src, void* dst, const void* d, int nx, int ny, int nz,
                                       int row_pad_bytes, int block_x, void* stream)
{
    if (!src || !dst || !d) return HLBM_EINVAL;
    if (nx < 1 || ny < 1 || nz < 1 || nx > 1024 || ny > 1024 || nz > 1024) return HLBM_EINVAL;
    if (row_pad_bytes < 0 || row_pad_bytes % 4) return HLBM_EINVAL;
    if (block_x < 64 || block_x > 1024 || block_x % 64) return HLBM_EINVAL;
    const uint32_t N = (uint32_t)nx * (uint32_t)ny * (uint32_t)nz;
    const uint32_t P = N + (uint32_t)(row_pad_bytes / 4);
    const dim3 grid((unsigned)((nx + block_x - 1) / block_x), (unsigned)ny, (unsigned)nz);
    hipLaunchKernelGGL(hlbm::stream_pattern_kernel, grid, dim3((unsigned)block_x), 0,
                       static_cast<hipStream_t>(stream), static_cast<const float*>(src), static_cast<float*>(dst),
                       static_cast<const float*>(d), P, (uint32_t)nx, (uint32_t)ny, (uint32_t)nz);
    return hipGetLastError() == hipSuccess ? HLBM_OK : HLBM_EDEVICE;
}
