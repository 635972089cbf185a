// mgp_probe.hip -- memory-system probes of the C ABI (include/mgp.h): the
// streaming-read rate of this device at a given buffer size, and the rate of
// the Megopolis accept loop's own read pattern without its arithmetic, which
// the benchmark reports as ceilings beside the loop's achieved rate.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "mgp.h"
#include "mgp_internal.h"

namespace mgp {

constexpr uint32_t kProbeThreads = 256;
constexpr int kProbeUnroll = 4;  // float4 loads in flight per thread

// Reads every float4 of a[0, n4) `passes` times (grid-stride, kProbeUnroll
// loads in flight per thread). Pass p reads element (t + p rot) mod n4 where
// the single pass would read t, so a block's next pass lands about 38% of the
// buffer away and is not served by the L2 that its previous pass filled.
// Block b's sum goes to sink[b] so that no load is dropped. n4 < 2^30.
__global__ __launch_bounds__(kProbeThreads) void k_probe_read(const float4* __restrict__ a, uint32_t n4,
                                                              uint32_t passes, uint32_t rot, float* __restrict__ sink)
{
    const uint32_t stride = gridDim.x * kProbeThreads;
    const uint32_t t0 = blockIdx.x * kProbeThreads + threadIdx.x;
    float acc = 0.0f;
    uint32_t shift = 0;
    for (uint32_t p = 0; p < passes; ++p) {
        uint32_t t = t0;
        for (; t + (kProbeUnroll - 1) * stride < n4; t += kProbeUnroll * stride) {
            float4 v[kProbeUnroll];
#pragma unroll
            for (int u = 0; u < kProbeUnroll; ++u) {
                uint32_t j = t + u * stride + shift;
                j = j >= n4 ? j - n4 : j;
                v[u] = a[j];
            }
#pragma unroll
            for (int u = 0; u < kProbeUnroll; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
        }
        for (; t < n4; t += stride) {
            uint32_t j = t + shift;
            j = j >= n4 ? j - n4 : j;
            const float4 v = a[j];
            acc += (v.x + v.y) + (v.z + v.w);
        }
        shift += rot;
        shift = shift >= n4 ? shift - n4 : shift;
    }
    __shared__ float part[kProbeThreads / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63u) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.0f;
        for (uint32_t k = 0; k < kProbeThreads / 64; ++k) s += part[k];
        sink[blockIdx.x] = s;
    }
}

// The candidate reads of the four-particle Megopolis loop over a mirrored
// weight array, and nothing else: thread t of block b holds the particles
// i0 + P_STRIDE p (i0 = b BT P + t, P_STRIDE = BT), every step shares one
// offset o, and particle i reads M[(i & ~31) + (o & ~31) + ((i + o) & 31)],
// five steps' loads issued together per round as the loop does. No random
// draws, no accept step: the kernel's time is what the access pattern alone
// costs. The values are summed per block; the sum is written only if it is
// negative, which non-negative contents never are, so no load is elided.
template <int P, int BT>
__global__ __launch_bounds__(BT) void k_probe_pattern(const char* __restrict__ M, const uint32_t* __restrict__ offs,
                                                      uint32_t n, uint32_t rounds, float* __restrict__ sink)
{
    constexpr uint32_t kStrideBytes = 4u * BT;
    const uint32_t i0 = blockIdx.x * (BT * P) + threadIdx.x;
    const uint32_t ia4 = (i0 & ~31u) * 4u;
    const uint32_t il4 = (i0 & 31u) * 4u;
    float acc[P];
#pragma unroll
    for (int p = 0; p < P; ++p) acc[p] = 0.0f;
    for (uint32_t q = 0; q < rounds; ++q) {
        float wj[5][P];
#pragma unroll
        for (uint32_t s = 0; s < 5; ++s) {
            uint32_t o = offs[q * 5u + s];
            o = o < n ? o : n - 1u;
            const uint32_t voff = ia4 | ((il4 + (o & 31u) * 4u) & 124u);
            const char* base = M + (o & ~31u) * 4u;
#pragma unroll
            for (int p = 0; p < P; ++p) wj[s][p] = *reinterpret_cast<const float*>(base + voff + kStrideBytes * p);
        }
#pragma unroll
        for (uint32_t s = 0; s < 5; ++s)
#pragma unroll
            for (int p = 0; p < P; ++p) acc[p] += wj[s][p];
    }
    float tot = 0.0f;
#pragma unroll
    for (int p = 0; p < P; ++p) tot += acc[p];
    if (tot < 0.0f) sink[blockIdx.x] = tot;
}

}  // namespace mgp

using namespace mgp;

extern "C" int mgp_probe_stream_read(const void* buf_dev, size_t bytes, int32_t passes, int32_t blocks,
                                     float* sink_dev, void* stream)
{
    clear_error();
    if (!buf_dev || !sink_dev) return fail(MGP_EINVAL, "buf_dev and sink_dev must not be NULL");
    if (bytes == 0 || bytes % 16u != 0) return fail(MGP_EINVAL, "bytes must be a positive multiple of 16");
    if (((uintptr_t)buf_dev & 15u) != 0) return fail(MGP_EINVAL, "buf_dev must be 16-byte aligned");
    if (passes < 1 || blocks < 1) return fail(MGP_EINVAL, "passes and blocks must be >= 1");
    if (bytes / 16u >= (1u << 30)) return fail(MGP_ERANGE, "bytes must be below 16 GiB");
    const uint32_t n4 = (uint32_t)(bytes / 16u);
    // about 0.382 n4 (the golden section), a multiple of 256 vectors so that
    // every wave's loads stay on whole 4 KB stretches
    const uint32_t rot = (uint32_t)(((uint64_t)n4 * 1640531527ull >> 32) & ~255ull) % n4;
    hipLaunchKernelGGL(k_probe_read, dim3((uint32_t)blocks), dim3(kProbeThreads), 0, static_cast<hipStream_t>(stream),
                       static_cast<const float4*>(buf_dev), n4, (uint32_t)passes, rot, sink_dev);
    return check_launch("probe kernel");
}

extern "C" int mgp_probe_pattern_read(const float* mirror_dev, size_t mirror_bytes, uint32_t n,
                                      const uint32_t* offsets_dev, int32_t steps, float* sink_dev, void* stream)
{
    constexpr int kP = 4;
    constexpr int kBT = 256;
    clear_error();
    if (!mirror_dev || !offsets_dev || !sink_dev) return fail(MGP_EINVAL, "pointers must not be NULL");
    if (n < (uint32_t)(kP * kBT) || n % (uint32_t)(kP * kBT) != 0)
        return fail(MGP_EINVAL, "n must be a positive multiple of %d", kP * kBT);
    if (n > (1u << 29)) return fail(MGP_ERANGE, "n above 2^29");
    if (steps < 5 || steps % 5 != 0) return fail(MGP_EINVAL, "steps must be a positive multiple of 5");
    if (mirror_bytes < 4ull * (2ull * n + (uint64_t)(kP * kBT)))
        return fail(MGP_EINVAL, "mirror_bytes must cover 2n + %d floats", kP * kBT);
    if (((uintptr_t)mirror_dev & 3u) != 0) return fail(MGP_EINVAL, "mirror_dev must be 4-byte aligned");
    hipLaunchKernelGGL((k_probe_pattern<kP, kBT>), dim3(n / (uint32_t)(kP * kBT)), dim3(kBT), 0,
                       static_cast<hipStream_t>(stream), reinterpret_cast<const char*>(mirror_dev), offsets_dev, n,
                       (uint32_t)steps / 5u, sink_dev);
    return check_launch("pattern probe kernel");
}
