// Memory-hierarchy probe: the bandwidth and latency of the read patterns the
// BVH traversal issues, over a working set of a chosen size.  The traversal's
// bytes are 128-byte node lines (and 48-byte triangle records) read at
// scattered addresses, one line per lane, from a tree that usually fits the
// L2 caches or the Infinity Cache rather than HBM; its roof is the rate at
// which the chip serves such lines at the tree's size, which this kernel
// measures.
//
//   pattern 0  streaming read: 16-byte vectors, grid-stride, coalesced.
//   pattern 1  gather: each lane reads whole 128-byte lines (8 x 16 bytes, as
//              a 4-wide node is read) at pseudo-random line indices; the
//              indices do not depend on loaded data, so many lines are in
//              flight per lane (throughput).
//   pattern 2  chase: as 1, but each line index depends on the data of the
//              previous line (one line in flight per lane: latency).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "rpr_device.hpp"
#include "rpr_internal.hpp"

namespace rpr {
namespace {

// A 32-bit integer mixer (xorshift-multiply rounds): a well spread line index
// from a lane's running state.
__device__ __forceinline__ uint32_t mix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x7FEB352Du;
    h ^= h >> 15;
    h *= 0x846CA68Bu;
    h ^= h >> 16;
    return h;
}

template <int PATTERN>
__global__ void k_probe(const float4* __restrict__ buf, int64_t n_vec, int iters, float* __restrict__ sink)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    float acc = 0.0f;
    if constexpr (PATTERN == 0) {
        for (int it = 0; it < iters; ++it)
            for (int64_t i = tid; i < n_vec; i += nth) {
                const float4 v = gld(buf + i);
                acc += (v.x + v.y) + (v.z + v.w);
            }
    } else {
        const uint64_t n_lines = (uint64_t)(n_vec / 8);
        uint32_t h = mix32((uint32_t)tid * 0x9E3779B9u + 0x632BE5ABu);
        for (int it = 0; it < iters; ++it) {
            h = mix32(h + (uint32_t)it);
            const uint64_t line = ((uint64_t)h * n_lines) >> 32;  // uniform in [0, n_lines)
            const float4* p = buf + 8 * line;
            float4 v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = gld(p + j);
#pragma unroll
            for (int j = 0; j < 8; ++j) acc += (v[j].x + v[j].y) + (v[j].z + v[j].w);
            if constexpr (PATTERN == 2) h ^= __float_as_uint(acc) & 1u;  // next index waits for this line
        }
    }
    sink[tid] = acc;
}

}  // namespace
}  // namespace rpr

using namespace rpr;

extern "C" int memory_probe(const void* buf, int64_t bytes, int32_t pattern, int32_t iters, int32_t grid,
                            int32_t block, float* sink, void* hip_stream)
{
    if (!buf || !sink) return set_error(RPR_EINVAL, "memory_probe: null buffer");
    if (bytes < 128 || bytes % 128 != 0) return set_error(RPR_EINVAL, "memory_probe: bytes must be a multiple of 128");
    if (bytes / 128 > ((int64_t)1 << 32)) return set_error(RPR_EINVAL, "memory_probe: more than 2^32 lines");
    if (pattern < 0 || pattern > 2) return set_error(RPR_EINVAL, "memory_probe: pattern must be 0, 1 or 2");
    if (iters < 1) return set_error(RPR_EINVAL, "memory_probe: iters must be >= 1");
    if (grid < 1 || block < kWave || block > 1024 || block % kWave != 0)
        return set_error(RPR_EINVAL, "memory_probe: bad launch shape");
    if (((uintptr_t)buf) % 16 != 0) return set_error(RPR_EINVAL, "memory_probe: buffer not 16-byte aligned");
    const float4* b = (const float4*)buf;
    const int64_t n_vec = bytes / 16;
    hipStream_t st = (hipStream_t)hip_stream;
    if (pattern == 0) hipLaunchKernelGGL(k_probe<0>, dim3(grid), dim3(block), 0, st, b, n_vec, iters, sink);
    else if (pattern == 1) hipLaunchKernelGGL(k_probe<1>, dim3(grid), dim3(block), 0, st, b, n_vec, iters, sink);
    else hipLaunchKernelGGL(k_probe<2>, dim3(grid), dim3(block), 0, st, b, n_vec, iters, sink);
    RPR_HIP_TRY(hipGetLastError());
    return RPR_OK;
}
