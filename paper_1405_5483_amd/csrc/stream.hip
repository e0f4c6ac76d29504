// Streaming-read reference kernel: reads a device buffer once with 16-byte
// loads spread over the whole device and folds every word into one xor, so
// that nothing can be skipped. It measures the read bandwidth a plain stream
// reaches on this device, the ceiling the scan kernels are compared with
// besides the HBM specification.
#include <hip/hip_runtime.h>

#include "mag_internal.hpp"

namespace mag {
namespace {

constexpr int kStreamThreads = 1024;
constexpr uint64_t kStreamTileVec = 2048;   // 32 KiB tiles: two 16-byte loads per thread

// One workgroup per compute unit (the fastest layout measured: faster than a
// grid-stride sweep of small workgroups). Workgroup g reads tiles g, g + G, ...
// of kStreamTileVec 16-byte vectors, each thread issuing both of its loads of
// a tile before using either; the tail past the last whole vector is read
// bytewise by thread 0. sink[blockIdx] gets the workgroup's xor.
__global__ __launch_bounds__(kStreamThreads) void k_stream_read(const uint4 *src, uint64_t nvec,
                                                                const uint8_t *tail, uint32_t ntail,
                                                                uint32_t *sink) {
    __shared__ uint32_t s_x[kStreamThreads / 64];
    const uint64_t ntiles = (nvec + kStreamTileVec - 1) / kStreamTileVec;
    uint32_t x = 0;
    for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const uint64_t i0 = t * kStreamTileVec + threadIdx.x, i1 = i0 + kStreamThreads;
        const uint4 a = i0 < nvec ? src[i0] : make_uint4(0u, 0u, 0u, 0u);
        const uint4 b = i1 < nvec ? src[i1] : make_uint4(0u, 0u, 0u, 0u);
        x ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w;
    }
    static_assert(kStreamTileVec == 2 * kStreamThreads, "two vectors per thread per tile");
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
        const int ncu = device_compute_units();
        if (ncu < 1) return 0;
        grid = (uint32_t)ncu;
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
