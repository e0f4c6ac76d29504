// Canonical output order: occurrences sorted ascending by (pos, id).
//
// The scan emits 64-bit keys (pos << idbits | id) in arbitrary order; keys are
// unique, since every (pos, id) is reported once. The finishing kernel (one
// workgroup, launched right after the scan) publishes the occurrence count and
// the work counters, and sorts up to kSmallMax keys in LDS with a bitonic
// network. Larger outputs are sorted by a stable LSD radix sort with 8-bit
// digits: either inside the finishing kernel by its one workgroup (when the
// host does not know the count), or by per-digit histogram / offset / scatter
// kernels across the whole device that the host enqueues once it has read the
// count. No kernel waits on another workgroup.
#include <hip/hip_runtime.h>

#include "mag_internal.hpp"

namespace mag {
namespace {

constexpr int kFinishThreads = 1024;
constexpr uint32_t kSmallMax = 8192;
constexpr uint32_t kRankMax = 2048;           // rank counting below this, bitonic above
constexpr int kRadixThreads = 256;
constexpr uint32_t kRadixChunk = 4096;      // keys per block and pass in the device-wide sort
constexpr uint32_t kMaxRadixBlocks = 2048;

__global__ void k_fill_u64(uint64_t *p, uint64_t count, uint64_t value) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        p[i] = value;
}

__device__ __forceinline__ uint32_t lanes_below_mask(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ mag_match to_record(uint64_t key, int idbits) {
    mag_match r;
    r.pos = key >> idbits;
    r.pattern_id = (uint32_t)(key & ((1ull << idbits) - 1ull));
    r.reserved = 0;
    return r;
}

// Lanes of this wave whose (valid) digit equals the lane's own, as a mask.
__device__ __forceinline__ uint64_t same_digit_lanes(bool valid, uint32_t d) {
    uint64_t eq = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const uint64_t bb = __ballot(valid && ((d >> b) & 1u));
        eq &= ((d >> b) & 1u) ? bb : ~bb;
    }
    return eq;
}

// Stable scatter of src[beg, end) by digit (key >> shift) & 255 into dst, the
// digit d's run for this block starting at s_off[d]. Rounds of blockDim.x
// consecutive keys; within a round, waves in order and lanes in order, so
// equal digits keep their input order. s_wcnt is [waves][256] of zeros on
// entry and on exit.
__device__ void stable_scatter(const uint64_t *src, uint64_t *dst, uint64_t beg, uint64_t end,
                               int shift, uint64_t *s_off, uint32_t (*s_wcnt)[256]) {
    const uint32_t tid = threadIdx.x, wave = tid >> 6, nwaves = blockDim.x >> 6;
    for (uint64_t base = beg; base < end; base += blockDim.x) {
        const uint64_t i = base + tid;
        const bool valid = i < end;
        const uint64_t key = valid ? src[i] : 0ull;
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        const uint64_t eq = same_digit_lanes(valid, d);
        const uint32_t rank = lanes_below_mask(eq);
        if (valid && rank == 0) s_wcnt[wave][d] = (uint32_t)__popcll(eq);
        __syncthreads();
        if (valid) {
            uint64_t off = s_off[d];
            for (uint32_t v = 0; v < wave; ++v) off += s_wcnt[v][d];
            dst[off + rank] = key;
        }
        __syncthreads();
        for (uint32_t dd = tid; dd < 256; dd += blockDim.x) {
            uint32_t add = 0;
            for (uint32_t v = 0; v < nwaves; ++v) {
                add += s_wcnt[v][dd];
                s_wcnt[v][dd] = 0;
            }
            s_off[dd] += add;
        }
        __syncthreads();
    }
}

struct FinishArgs {
    uint64_t *keys;        // two buffers of cap keys: [0, cap) holds the scan output
    uint64_t cap;
    uint64_t *counters;    // read, published, then returned to zero
    uint64_t *d_count;
    mag_stats *d_stats;
    uint64_t samples;
    mag_match *out;
    int idbits, nbits;
    int host_sorts;        // large outputs are left to the device-wide sort
};

__global__ __launch_bounds__(kFinishThreads) void k_finish(FinishArgs a) {
    __shared__ uint64_t s_keys[kSmallMax];
    __shared__ uint32_t s_hist[256];
    __shared__ uint32_t s_wcnt[kFinishThreads / 64][256];
    __shared__ uint64_t s_off[256];
    const uint32_t tid = threadIdx.x;
    const uint64_t z = a.counters[0];
    const uint64_t cw = a.counters[1], nv = a.counters[2];
    __syncthreads();      // every thread has read the counters
    if (tid == 0) {
        *a.d_count = z;
        if (a.d_stats) {
            a.d_stats->samples = a.samples;
            a.d_stats->cand_windows = cw;
            a.d_stats->verifications = nv;
            a.d_stats->matches = z;
        }
        // leave the counters at zero for the next scan of this plan
        a.counters[0] = 0;
        a.counters[1] = 0;
        a.counters[2] = 0;
        a.counters[3] = 0;
    }
    if (z > a.cap || z == 0) return;      // overflow leaves the records unspecified

    if (z <= kRankMax) {
        // keys are unique: a key's output slot is the number of smaller keys.
        // Each key's count is split over `parts` threads (8 independent sums
        // each, so LDS reads overlap) and combined with LDS atomics.
        uint32_t *s_rank = reinterpret_cast<uint32_t *>(&s_wcnt[0][0]);   // kRankMax entries
        for (uint32_t i = tid; i < z; i += kFinishThreads) {
            s_keys[i] = a.keys[i];
            s_rank[i] = 0;
        }
        __syncthreads();
        const uint32_t parts = z <= kFinishThreads ? kFinishThreads / (uint32_t)z : 1u;
        const uint32_t span = ((uint32_t)z + parts - 1) / parts;
        for (uint32_t w = tid; w < (uint32_t)z * parts; w += kFinishThreads) {
            const uint32_t i = w / parts, part = w % parts;
            const uint64_t key = s_keys[i];
            const uint32_t j0 = part * span, j1 = j0 + span < z ? j0 + span : (uint32_t)z;
            uint32_t acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            uint32_t j = j0;
            for (; j + 8 <= j1; j += 8) {
#pragma unroll
                for (int u = 0; u < 8; ++u) acc[u] += s_keys[j + u] < key ? 1u : 0u;
            }
            for (; j < j1; ++j) acc[0] += s_keys[j] < key ? 1u : 0u;
            atomicAdd(&s_rank[i], acc[0] + acc[1] + acc[2] + acc[3] + acc[4] + acc[5] + acc[6] + acc[7]);
        }
        __syncthreads();
        for (uint32_t i = tid; i < z; i += kFinishThreads)
            a.out[s_rank[i]] = to_record(s_keys[i], a.idbits);
        return;
    }
    if (z <= kSmallMax) {
        uint32_t N = 1;
        while (N < z) N <<= 1;
        for (uint32_t i = tid; i < N; i += kFinishThreads) s_keys[i] = i < z ? a.keys[i] : ~0ull;
        __syncthreads();
        for (uint32_t k = 2; k <= N; k <<= 1) {
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                for (uint32_t i = tid; i < N; i += kFinishThreads) {
                    const uint32_t p = i ^ j;
                    if (p > i) {
                        const uint64_t x = s_keys[i], y = s_keys[p];
                        const bool up = (i & k) == 0;
                        if ((x > y) == up) { s_keys[i] = y; s_keys[p] = x; }
                    }
                }
                __syncthreads();
            }
        }
        for (uint32_t i = tid; i < z; i += kFinishThreads) a.out[i] = to_record(s_keys[i], a.idbits);
        return;
    }
    if (a.host_sorts) return;

    // one-workgroup LSD radix sort over global memory
    for (uint32_t v = tid; v < (kFinishThreads / 64) * 256; v += kFinishThreads)
        (&s_wcnt[0][0])[v] = 0;
    uint64_t *src = a.keys, *dst = a.keys + a.cap;
    const int passes = (a.nbits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        if (tid < 256) s_hist[tid] = 0;
        __syncthreads();
        for (uint64_t i = tid; i < z; i += kFinishThreads)
            atomicAdd(&s_hist[(src[i] >> shift) & 255u], 1u);
        __syncthreads();
        if (tid == 0) {
            uint64_t run = 0;
            for (int d = 0; d < 256; ++d) {
                s_off[d] = run;
                run += s_hist[d];
            }
        }
        __syncthreads();
        stable_scatter(src, dst, 0, z, shift, s_off, s_wcnt);
        uint64_t *t = src;
        src = dst;
        dst = t;
        __syncthreads();
    }
    for (uint64_t i = tid; i < z; i += kFinishThreads) a.out[i] = to_record(src[i], a.idbits);
}

// ---- device-wide LSD radix sort, one launch per phase and digit

__global__ __launch_bounds__(kRadixThreads) void k_radix_hist(const uint64_t *src, uint64_t z,
                                                              int shift, uint32_t *cnt) {
    __shared__ uint32_t s_hist[256];
    const uint32_t g = blockIdx.x, G = gridDim.x, tid = threadIdx.x;
    s_hist[tid] = 0;
    __syncthreads();
    const uint64_t beg = (uint64_t)g * kRadixChunk;
    const uint64_t end = beg + kRadixChunk < z ? beg + kRadixChunk : z;
    for (uint64_t i = beg + tid; i < end; i += kRadixThreads)
        atomicAdd(&s_hist[(src[i] >> shift) & 255u], 1u);
    __syncthreads();
    cnt[(size_t)tid * G + g] = s_hist[tid];
}

// cnt (digit-major, [256][G]) -> exclusive start offsets, in place (64-bit out)
__global__ __launch_bounds__(256) void k_radix_offsets(const uint32_t *cnt, uint64_t *off, uint32_t G) {
    __shared__ uint64_t s_tot[256];
    const uint32_t d = threadIdx.x;
    uint64_t run = 0;
    for (uint32_t g = 0; g < G; ++g) run += cnt[(size_t)d * G + g];
    s_tot[d] = run;
    __syncthreads();
    if (d == 0) {
        uint64_t acc = 0;
        for (int i = 0; i < 256; ++i) {
            const uint64_t t = s_tot[i];
            s_tot[i] = acc;
            acc += t;
        }
    }
    __syncthreads();
    uint64_t acc = s_tot[d];
    for (uint32_t g = 0; g < G; ++g) {
        off[(size_t)d * G + g] = acc;
        acc += cnt[(size_t)d * G + g];
    }
}

__global__ __launch_bounds__(kRadixThreads) void k_radix_scatter(const uint64_t *src, uint64_t *dst,
                                                                 uint64_t z, int shift,
                                                                 const uint64_t *off) {
    __shared__ uint64_t s_off[256];
    __shared__ uint32_t s_wcnt[kRadixThreads / 64][256];
    const uint32_t g = blockIdx.x, G = gridDim.x, tid = threadIdx.x;
    s_off[tid] = off[(size_t)tid * G + g];
    for (int v = 0; v < kRadixThreads / 64; ++v) s_wcnt[v][tid] = 0;
    __syncthreads();
    const uint64_t beg = (uint64_t)g * kRadixChunk;
    const uint64_t end = beg + kRadixChunk < z ? beg + kRadixChunk : z;
    stable_scatter(src, dst, beg, end, shift, s_off, s_wcnt);
}

__global__ void k_expand(const uint64_t *keys, uint64_t z, mag_match *out, int idbits) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < z; i += stride)
        out[i] = to_record(keys[i], idbits);
}

}  // namespace

mag_status launch_fill_u64(uint64_t *ptr, uint64_t count, uint64_t value, hipStream_t stream) {
    if (!count) return MAG_OK;
    uint64_t blocks = (count + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_fill_u64, dim3((uint32_t)blocks), dim3(256), 0, stream, ptr, count, value);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MAG_OK : hip_fail(e, "fill launch");
}

uint32_t small_sort_max() { return kSmallMax; }

mag_status launch_finish(Scratch &sc, uint64_t cap, uint64_t samples, uint64_t *d_count,
                         mag_stats *d_stats, mag_match *out, int idbits, int nbits, bool host_sorts,
                         hipStream_t stream) {
    FinishArgs a;
    a.keys = sc.keys;
    a.cap = cap;
    a.counters = sc.counters;
    a.d_count = d_count;
    a.d_stats = d_stats;
    a.samples = samples;
    a.out = out;
    a.idbits = idbits;
    a.nbits = nbits;
    a.host_sorts = host_sorts ? 1 : 0;
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kFinishThreads), 0, stream, a);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MAG_OK : hip_fail(e, "finish launch");
}

mag_status ensure_radix_scratch(Scratch &sc, uint64_t z) {
    const uint64_t G = (z + kRadixChunk - 1) / kRadixChunk;
    if (G > kMaxRadixBlocks * 64ull) return fail(MAG_E_UNSUPPORTED, "too many occurrences to sort");
    if (sc.radix_blocks >= G && sc.hist) return MAG_OK;
    (void)hipFree(sc.hist);
    (void)hipFree(sc.radix_off);
    sc.hist = nullptr;
    sc.radix_off = nullptr;
    sc.radix_blocks = 0;
    hipError_t e = hipMalloc(&sc.hist, (size_t)256 * G * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&sc.radix_off, (size_t)256 * G * sizeof(uint64_t));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(MAG_E_NOMEM, "device allocation of radix counts failed");
    }
    sc.radix_blocks = G;
    return MAG_OK;
}

mag_status launch_radix_sort(Scratch &sc, uint64_t z, uint64_t cap, mag_match *out, int idbits,
                             int nbits, hipStream_t stream) {
    if (z <= kSmallMax || z > cap) return MAG_OK;    // done by the finishing kernel / overflow
    mag_status s = ensure_radix_scratch(sc, z);
    if (s != MAG_OK) return s;
    const uint32_t G = (uint32_t)((z + kRadixChunk - 1) / kRadixChunk);
    uint64_t *src = sc.keys, *dst = sc.keys + cap;
    const int passes = (nbits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        hipLaunchKernelGGL(k_radix_hist, dim3(G), dim3(kRadixThreads), 0, stream,
                           (const uint64_t *)src, z, shift, sc.hist);
        hipLaunchKernelGGL(k_radix_offsets, dim3(1), dim3(256), 0, stream,
                           (const uint32_t *)sc.hist, sc.radix_off, G);
        hipLaunchKernelGGL(k_radix_scatter, dim3(G), dim3(kRadixThreads), 0, stream,
                           (const uint64_t *)src, dst, z, shift, (const uint64_t *)sc.radix_off);
        uint64_t *t = src;
        src = dst;
        dst = t;
    }
    uint64_t blocks = (z + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_expand, dim3((uint32_t)blocks), dim3(256), 0, stream,
                       (const uint64_t *)src, z, out, idbits);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MAG_OK : hip_fail(e, "radix sort launch");
}

}  // namespace mag
