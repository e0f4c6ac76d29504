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
// (148 KiB with the found-key buffers, the bitmap at address 0): a Bloom
// word's address is then its index times 4, with no base to add per probe.
__global__ __launch_bounds__(kNT, 4) void k_dense(DenseArgs a) {
    __shared__ __align__(16) uint32_t s_bloom[kBloomWordsMax];
    __shared__ uint64_t s_queue[(kNT / 64) * kQueue];
    __shared__ uint64_t s_found[(kNT / 64) * kFoundBuf];
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
    uint64_t *fbuf = s_found + wave * kFoundBuf;
    uint32_t qn = 0, fbn = 0;
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
                       queue, qn, vargs, lane, nhit, FoundBuf{fbuf, &fbn, kFoundBuf});
#pragma unroll
        for (int t = 0; t < 10; ++t) W[t] = Wn[t];
        p0 = p0n;
    }
    if (qn) fbn = drain_partial_found(vargs, queue, qn, lane, fbuf, fbn);
    unsigned long long nh = nhit;
    for (int off = 32; off > 0; off >>= 1) nh += __shfl_xor(nh, off);
    __shared__ uint64_t s_wg[3 * (kNT / 64)];
    workgroup_out<kNT / 64>(vargs, fbuf, fbn, nh, nh, a.counters, s_wg);
}

// The one-probe dense scan (slice_test): the same grid and bitmap staging as
// k_dense; tiles of slice_scan_tile(P) positions, wave w covering positions
// 63 P w .. 63 P (w + 1) - 1 of its tile, each lane loading the words its
// probes read, from the word that holds its first position. Each wave keeps the loads of
// its next two tiles in flight while it tests the current one (three
// register sets, used in turn). AL: the text starts on a 4-byte boundary, so
// no byte realignment is needed (tiles are a multiple of 4 positions long).
template <int K, int P, bool AL>
__global__ __launch_bounds__(kNT, 4) void k_dense_slices(DenseArgs a) {
    constexpr int kTile = slice_scan_tile(P);
    constexpr int kLW = SliceLane<P>::load_words(AL);
    __shared__ __align__(16) uint32_t s_bits[kBloomWordsMax];
    __shared__ uint64_t s_queue[(kNT / 64) * kQueue];
    __shared__ uint64_t s_found[(kNT / 64) * kFoundBuf];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const VerifyArgs *vargs = (const VerifyArgs *)((const __attribute__((address_space(4))) char *)
                                                       __builtin_amdgcn_kernarg_segment_ptr() +
                                                   offsetof(DenseArgs, v));
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(a.bloom);
        uint4 *dst = reinterpret_cast<uint4 *>(s_bits);
        for (uint32_t v = tid; v < a.bloom_vec; v += kNT) dst[v] = src[v];
    }
    __syncthreads();
    uint64_t *queue = s_queue + wave * kQueue;
    uint64_t *fbuf = s_found + wave * kFoundBuf;
    uint32_t qn = 0, nhit = 0, fbn = 0;
    // byte offset of this lane's first position in its tile
    const uint32_t lane_off = (uint32_t)(P * (kSliceOwners * wave + lane));
    // Tiles whose lanes' 2P bytes all lie inside the text take whole 16-byte
    // loads (the pipelined loop below), the last ones (at most two) single
    // range-checked dwords. Resource offsets are taken from the 16-byte-aligned
    // text base, which the text's first tile byte follows by d = delta & 3
    // within its word.
    const uint64_t pa_end = (a.delta + a.n) & ~3ull;  // whole words of text from tbase
    uint64_t nfull = 0;
    {
        const uint64_t need = kTile + 4u * kLW + 16;   // a tile's bytes from its word
        nfull = pa_end >= need ? (pa_end - need) / kTile + 1 : 0;
        if (nfull > a.ntiles) nfull = a.ntiles;
    }
    const uint32_t d = (uint32_t)(a.delta & 3u);
    auto load = [&](uint64_t tile, uint32_t (&W)[kLW]) {
        // the word holding the tile's first position, and a resource from the
        // 16-byte boundary below it over the tile's lanes' bytes
        const uint64_t w0 = (a.delta & ~3ull) + tile * (uint64_t)kTile;
        const uint64_t pa0 = w0 & ~15ull;
        const __amdgpu_buffer_rsrc_t rs = tile_rsrc(a.tbase + pa0, kTile + 4u * kLW + 32u);
        const int at = (int)(w0 - pa0 + lane_off);
#pragma unroll
        for (int v = 0; v < kLW / 4; ++v) {
            const uint4 x = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, at + 16 * v, 0, 0));
            W[4 * v] = x.x; W[4 * v + 1] = x.y; W[4 * v + 2] = x.z; W[4 * v + 3] = x.w;
        }
        constexpr int r0 = kLW & ~3;
        if constexpr (kLW % 4 == 1) {
            W[r0] = __builtin_amdgcn_raw_buffer_load_b32(rs, at + 4 * r0, 0, 0);
        } else if constexpr (kLW % 4 == 2) {
            const auto x = __builtin_amdgcn_raw_buffer_load_b64(rs, at + 4 * r0, 0, 0);
            W[r0] = x[0]; W[r0 + 1] = x[1];
        } else if constexpr (kLW % 4 == 3) {
            const auto x = __builtin_amdgcn_raw_buffer_load_b96(rs, at + 4 * r0, 0, 0);
            W[r0] = x[0]; W[r0 + 1] = x[1]; W[r0 + 2] = x[2];
        }
    };
    auto run = [&](uint64_t tile, const uint32_t (&W)[kLW]) {
        const int64_t xb = (int64_t)tile * kTile + lane_off;
        slice_test<K, P, AL, true>(W, d, xb, a.last - xb + 1, s_bits, a.bshift, queue, qn, vargs, lane, nhit,
                                   fbuf, fbn);
    };
    const uint64_t G = gridDim.x;
    uint64_t tile = blockIdx.x;
    uint32_t Wa[kLW], Wb[kLW], Wc[kLW];
    // every step issues the same loads (past the last full tile they reload
    // it), so the wait before a tile's use counts the same loads after it on
    // every path and the two tiles ahead stay in flight
    const uint64_t lastfull = nfull ? nfull - 1 : 0;
    auto ahead = [&](uint64_t t) { return t < lastfull ? t : lastfull; };
    if (tile < nfull) {
        load(tile, Wa);
        load(ahead(tile + G), Wb);
    }
    while (tile < nfull) {
        load(ahead(tile + 2 * G), Wc);
        run(tile, Wa);
        if ((tile += G) >= nfull) break;
        load(ahead(tile + 2 * G), Wa);
        run(tile, Wb);
        if ((tile += G) >= nfull) break;
        load(ahead(tile + 2 * G), Wb);
        run(tile, Wc);
        tile += G;
    }
    // the tail tiles, dword by dword within the text's resource
    for (tile = nfull + ((blockIdx.x + G - nfull % G) % G); tile < a.ntiles; tile += G) {
        const int64_t x0 = (int64_t)tile * kTile;
        int64_t b1 = x0 + kTile + 4 * kLW + 16;
        if (b1 > (int64_t)a.n) b1 = (int64_t)a.n;
        const uint64_t pa0 = (a.delta + (uint64_t)x0) & ~15ull;
        const uint64_t pa1 = (a.delta + (uint64_t)b1 + 15) & ~15ull;
        const __amdgpu_buffer_rsrc_t rs = tile_rsrc(a.tbase + pa0, (uint32_t)(pa1 - pa0));
        const uint32_t p0 = (uint32_t)(a.delta + (uint64_t)x0 - pa0);
        const uint32_t at = (p0 & ~3u) + lane_off;
        uint32_t W[kLW];
#pragma unroll
        for (int t = 0; t < kLW; ++t) W[t] = ld32(rs, at + 4u * t);
        run(tile, W);
    }
    if (qn) fbn = drain_partial_found(vargs, queue, qn, lane, fbuf, fbn);
    unsigned long long nh = nhit;
    for (int off = 32; off > 0; off >>= 1) nh += __shfl_xor(nh, off);
    __shared__ uint64_t s_wg[3 * (kNT / 64)];
    workgroup_out<kNT / 64>(vargs, fbuf, fbn, nh, nh, a.counters, s_wg);
}

int compute_units(int &ncu) {
    if (ncu) return 0;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) {
        ncu = 0;
        hip_fail(e, "dense scan sizing");
        return -1;
    }
    return 0;
}

template <int K, int P>
mag_status launch_slices_kp(const DenseArgs &a, hipStream_t stream) {
    static int ncu = 0;
    if (compute_units(ncu)) return MAG_E_DEVICE;
    const bool al = (a.delta & 3) == 0;
    const void *fn = al ? (const void *)k_dense_slices<K, P, true> : (const void *)k_dense_slices<K, P, false>;
    const int occ = cached_occupancy(fn, kNT, 0);
    if (occ < 1) return fail(MAG_E_UNSUPPORTED, "dense scan does not fit on a compute unit");
    uint64_t grid = (uint64_t)ncu * occ;
    if (grid > a.ntiles) grid = a.ntiles;
    if (al)
        hipLaunchKernelGGL((k_dense_slices<K, P, true>), dim3((uint32_t)grid), dim3(kNT), 0, stream, a);
    else
        hipLaunchKernelGGL((k_dense_slices<K, P, false>), dim3((uint32_t)grid), dim3(kNT), 0, stream, a);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? MAG_OK : hip_fail(e, "dense scan launch");
}

template <int K>
mag_status launch_slices_k(const DenseArgs &a, int P, hipStream_t stream) {
    return P == 32 ? launch_slices_kp<K, 32>(a, stream) : launch_slices_kp<K, 16>(a, stream);
}

}  // namespace

mag_status launch_dense_slices(const DenseArgs &a, size_t bitmap_bytes, int k, int P, hipStream_t stream) {
    if (!a.ntiles) return MAG_OK;
    if (bitmap_bytes > (size_t)kBloomWordsMax * 4 || a.bloom_vec * 16ull != bitmap_bytes)
        return fail(MAG_E_INVALID, "slice bitmap does not fit the dense kernel's LDS array");
    if (P != 16 && P != 32) return fail(MAG_E_INVALID, "positions per lane must be 16 or 32");
    switch (k) {
        case 1: return launch_slices_k<1>(a, P, stream);
        case 2: return launch_slices_k<2>(a, P, stream);
        case 3: return launch_slices_k<3>(a, P, stream);
        case 4: return launch_slices_k<4>(a, P, stream);
        case 5: return launch_slices_k<5>(a, P, stream);
        case 6: return launch_slices_k<6>(a, P, stream);
        case 7: return launch_slices_k<7>(a, P, stream);
        case 8: return launch_slices_k<8>(a, P, stream);
    }
    return fail(MAG_E_INVALID, "slices per pattern outside [1, 8]");
}

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
