// Streaming-read reference kernel: reads a device buffer once with 16-byte
// loads spread over the whole device and folds every word into one xor, so
// that nothing can be skipped. It measures the read bandwidth a plain stream
// reaches on this device, the ceiling the scan kernels are compared with
// besides the HBM specification.
#include <hip/hip_runtime.h>

#include "mag_internal.hpp"

namespace mag {
namespace {

constexpr int kStreamThreads = 256;
constexpr int kStreamUnroll = 4;      // 16-byte loads in flight per thread

// Thread t of the grid reads the 16-byte vectors t, t + T, t + 2T, ...
// (T = threads in the grid), kStreamUnroll at a time; the tail past the last
// whole vector is read bytewise by thread 0. sink[blockIdx] gets the block's
// xor.
__global__ __launch_bounds__(kStreamThreads) void k_stream_read(const uint4 *src, uint64_t nvec,
                                                                const uint8_t *tail, uint32_t ntail,
                                                                uint32_t *sink) {
    __shared__ uint32_t s_x[kStreamThreads / 64];
    const uint64_t T = (uint64_t)gridDim.x * kStreamThreads;
    uint64_t i = (uint64_t)blockIdx.x * kStreamThreads + threadIdx.x;
    uint32_t x = 0;
    for (; i + (kStreamUnroll - 1) * T < nvec; i += kStreamUnroll * T) {
        uint4 v[kStreamUnroll];
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u) v[u] = src[i + u * T];
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u) x ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    for (; i < nvec; i += T) {
        const uint4 v = src[i];
        x ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (uint32_t b = 0; b < ntail; ++b) x ^= (uint32_t)tail[b] << (8 * (b & 3));
    for (int off = 32; off > 0; off >>= 1) x ^= __shfl_xor(x, off);
    if ((threadIdx.x & 63) == 0) s_x[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t y = 0;
        for (int w = 0; w < kStreamThreads / 64; ++w) y ^= s_x[w];
        sink[blockIdx.x] = y;
    }
}

}  // namespace

uint32_t stream_read_grid() {
    static uint32_t grid = 0;
    if (!grid) {
        int dev = 0, ncu = 0, occ = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_stream_read, kStreamThreads, 0) !=
                hipSuccess) {
            (void)hipGetLastError();
            return 0;
        }
        grid = (uint32_t)(ncu * occ);
    }
    return grid;
}

mag_status launch_stream_read(const uint8_t *d, uint64_t n, uint32_t *sink, hipStream_t stream) {
    const uint32_t grid = stream_read_grid();
    if (!grid) return fail(MAG_E_DEVICE, "cannot size the streaming-read grid");
    const uint64_t nvec = n / 16;
    hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(kStreamThreads), 0, stream,
                       reinterpret_cast<const uint4 *>(d), nvec, d + nvec * 16, (uint32_t)(n % 16), sink);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? MAG_OK : hip_fail(e, "streaming-read launch");
}

}  // namespace mag
