// Single-job dense scan: a persistent grid walks tiles of
// kDenseScanTile start positions with the Bloom bitmap staged in LDS
// (see dense.hpp).
#include <hip/hip_runtime.h>

#include <cstddef>

#include "dense.hpp"

namespace mag {
namespace {

using namespace dev;

constexpr int kNT = kDenseScanThreads;
constexpr int kQueue = 128;
static_assert(kQueue >= (int)kDenseQueue, "dense_test fills up to kDenseQueue starts");

constexpr uint32_t kBloomWordsMax = 1u << (kBloomMaxLog2 - 5);

// At least 4 waves per SIMD: at most 128 VGPRs, so one workgroup of 16
// waves fills a compute unit. The bitmap and the queues are static LDS
// (144 KiB, the bitmap at address 0): a Bloom word's address is then its
// index times 4, with no base to add per probe.
__global__ __launch_bounds__(kNT, 4) void k_dense(DenseArgs a) {
    __shared__ __align__(16) uint32_t s_bloom[kBloomWordsMax];
    __shared__ uint64_t s_queue[(kNT / 64) * kQueue];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // the kernel's only argument is `a`, at the start of the argument segment
    const VerifyArgs *vargs = (const VerifyArgs *)((const __attribute__((address_space(4))) char *)
                                                       __builtin_amdgcn_kernarg_segment_ptr() +
                                                   offsetof(DenseArgs, v));
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(a.bloom);
        uint4 *dst = reinterpret_cast<uint4 *>(s_bloom);
        for (uint32_t v = tid; v < a.bloom_vec; v += kNT) dst[v] = src[v];
    }
    __syncthreads();
    uint64_t *queue = s_queue + wave * kQueue;
    uint32_t qn = 0;
    uint64_t nhit = 0;
    const uint32_t hw = a.v.hw, mw = a.v.mw, lastmask = a.v.lastmask;
    // a tile's resource, size and the offset of its first position
    auto tile_at = [&](uint64_t tile, __amdgpu_buffer_rsrc_t &rs, uint32_t &nrec, uint32_t &p0) {
        const int64_t x0 = (int64_t)tile * kDenseScanTile;
        int64_t b1 = x0 + kDenseScanTile + 40;            // bytes the tile's windows touch
        if (b1 > (int64_t)a.n) b1 = (int64_t)a.n;
        const uint64_t pa0 = (a.delta + (uint64_t)x0) & ~15ull;
        const uint64_t pa1 = (a.delta + (uint64_t)b1 + 15) & ~15ull;
        rs = tile_rsrc(a.tbase + pa0, (uint32_t)(pa1 - pa0));
        nrec = (uint32_t)(pa1 - pa0);
        p0 = (uint32_t)(a.delta + (uint64_t)x0 - pa0);
    };
    // the next tile's bytes are loaded before the current tile's windows are tested
    uint64_t tile = blockIdx.x;
    uint32_t W[10], Wn[10];
    uint32_t p0 = 0;
    if (tile < a.ntiles) {
        __amdgpu_buffer_rsrc_t rs;
        uint32_t nrec;
        tile_at(tile, rs, nrec, p0);
        dense_load<kNT>(rs, nrec, p0, tid, W);
    }
    for (; tile < a.ntiles; tile += gridDim.x) {
        const uint64_t nt = tile + gridDim.x;
        uint32_t p0n = 0;
        if (nt < a.ntiles) {
            __amdgpu_buffer_rsrc_t rs;
            uint32_t nrec;
            tile_at(nt, rs, nrec, p0n);
            dense_load<kNT>(rs, nrec, p0n, tid, Wn);
        }
        const int64_t x0 = (int64_t)tile * kDenseScanTile;
        dense_test_any(W, p0 & 3u, x0 + 16 * (int64_t)tid, a.last, s_bloom, a.bshift, hw, mw, lastmask,
                       queue, qn, vargs, lane, nhit);
#pragma unroll
        for (int t = 0; t < 10; ++t) W[t] = Wn[t];
        p0 = p0n;
    }
    if (qn) drain_partial(vargs, queue, qn, lane);
    unsigned long long nh = nhit;
    for (int off = 32; off > 0; off >>= 1) nh += __shfl_xor(nh, off);
    if (lane == 0 && nh) {
        atomicAdd((unsigned long long *)&a.counters[1], nh);
        atomicAdd((unsigned long long *)&a.counters[2], nh);
    }
}

}  // namespace

mag_status launch_dense(const DenseArgs &a, size_t bloom_bytes, hipStream_t stream) {
    if (!a.ntiles) return MAG_OK;
    if (bloom_bytes > (size_t)kBloomWordsMax * 4 || a.bloom_vec * 16ull != bloom_bytes)
        return fail(MAG_E_INVALID, "Bloom bitmap does not fit the dense kernel's LDS array");
    const size_t shmem = 0;
    static int ncu = 0;
    if (!ncu) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) {
            ncu = 0;
            return hip_fail(e, "dense scan sizing");
        }
    }
    const int occ = cached_occupancy((const void *)k_dense, kNT, shmem);
    if (occ < 1) return fail(MAG_E_UNSUPPORTED, "dense scan does not fit on a compute unit");
    uint64_t grid = (uint64_t)ncu * occ;
    if (grid > a.ntiles) grid = a.ntiles;
    hipLaunchKernelGGL(k_dense, dim3((uint32_t)grid), dim3(kNT), shmem, stream, a);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? MAG_OK : hip_fail(e, "dense scan launch");
}

}  // namespace mag
