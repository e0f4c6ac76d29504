// Canonical output order: occurrences sorted ascending by (pos, id).
//
// The scan emits 64-bit keys (pos << idbits | id) in arbitrary order. One
// cooperative launch finishes a scan without any host round trip: it publishes
// the occurrence count and the work counters, then sorts the keys and expands
// them into 16-byte records. Up to kSmallMax keys are sorted by workgroup 0
// alone with a bitonic network in LDS; more go through a stable LSD radix sort
// (8-bit digits) across the whole grid, with grid-wide barriers between the
// count, offset and scatter phases of each digit.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include "mag_internal.hpp"

namespace cg = cooperative_groups;

namespace mag {
namespace {

constexpr int kSortThreads = 256;
constexpr uint32_t kSmallMax = 8192;
constexpr int kMaxGroups = 256;

__global__ void k_fill_u64(uint64_t *p, uint64_t count, uint64_t value) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        p[i] = value;
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
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

struct FinishArgs {
    uint64_t *keys;        // two buffers of cap keys: [0, cap) holds the scan output
    uint64_t cap;
    const uint64_t *counters;
    uint64_t *d_count;
    mag_stats *d_stats;
    uint64_t samples;
    uint32_t *cnt;         // 256 * gridDim.x digit counts
    mag_match *out;
    int idbits, nbits;
};

__global__ __launch_bounds__(kSortThreads) void k_finish(FinishArgs a) {
    __shared__ uint64_t s_keys[kSmallMax];
    __shared__ uint32_t s_hist[256];
    __shared__ uint32_t s_wcnt[kSortThreads / 64][256];
    __shared__ uint64_t s_off[256];

    const uint32_t tid = threadIdx.x, w = blockIdx.x, G = gridDim.x;
    const uint64_t z = a.counters[0];
    if (w == 0 && tid == 0) {
        *a.d_count = z;
        if (a.d_stats) {
            a.d_stats->samples = a.samples;
            a.d_stats->cand_windows = a.counters[1];
            a.d_stats->verifications = a.counters[2];
            a.d_stats->matches = z;
        }
    }
    if (z > a.cap || z == 0) return;      // overflow leaves the records unspecified

    if (z <= kSmallMax) {
        if (w != 0) return;
        uint32_t N = 1;
        while (N < z) N <<= 1;
        for (uint32_t i = tid; i < N; i += kSortThreads) s_keys[i] = i < z ? a.keys[i] : ~0ull;
        __syncthreads();
        for (uint32_t k = 2; k <= N; k <<= 1) {
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                for (uint32_t i = tid; i < N; i += kSortThreads) {
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
        for (uint32_t i = tid; i < z; i += kSortThreads) a.out[i] = to_record(s_keys[i], a.idbits);
        return;
    }

    // ---- stable LSD radix sort over the grid (z > kSmallMax for every group)
    cg::grid_group grid = cg::this_grid();
    const uint64_t chunk = (z + G - 1) / G;
    const uint64_t beg = (uint64_t)w * chunk < z ? (uint64_t)w * chunk : z;
    const uint64_t end = beg + chunk < z ? beg + chunk : z;
    const uint32_t wave = tid >> 6;
    uint64_t *src = a.keys, *dst = a.keys + a.cap;
    const int passes = (a.nbits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        s_hist[tid] = 0;
        for (int v = 0; v < kSortThreads / 64; ++v) s_wcnt[v][tid] = 0;
        __syncthreads();
        for (uint64_t i = beg + tid; i < end; i += kSortThreads)
            atomicAdd(&s_hist[(src[i] >> shift) & 255u], 1u);
        __syncthreads();
        a.cnt[(size_t)tid * G + w] = s_hist[tid];
        grid.sync();

        // digit d = tid: keys of digit d in groups before w, and in all groups
        uint64_t pre = 0, tot = 0;
        for (uint32_t v = 0; v < G; ++v) {
            const uint32_t c = a.cnt[(size_t)tid * G + v];
            tot += c;
            if (v < w) pre += c;
        }
        s_off[tid] = tot;
        __syncthreads();
        if (tid == 0) {
            uint64_t run = 0;
            for (int d = 0; d < 256; ++d) {
                const uint64_t t = s_off[d];
                s_off[d] = run;
                run += t;
            }
        }
        __syncthreads();
        s_off[tid] += pre;
        __syncthreads();

        for (uint64_t base = beg; base < end; base += kSortThreads) {
            const uint64_t i = base + tid;
            const bool valid = i < end;
            const uint64_t key = valid ? src[i] : 0ull;
            const uint32_t d = (uint32_t)(key >> shift) & 255u;
            uint64_t eq = __ballot(valid);
            for (int b = 0; b < 8; ++b) {
                const uint64_t bb = __ballot(valid && ((d >> b) & 1u));
                eq &= ((d >> b) & 1u) ? bb : ~bb;
            }
            const uint32_t rank = lanes_below(eq);
            if (valid && rank == 0) s_wcnt[wave][d] = (uint32_t)__popcll(eq);
            __syncthreads();
            if (valid) {
                uint64_t off = s_off[d];
                for (uint32_t v = 0; v < wave; ++v) off += s_wcnt[v][d];
                dst[off + rank] = key;
            }
            __syncthreads();
            uint32_t add = 0;
            for (int v = 0; v < kSortThreads / 64; ++v) {
                add += s_wcnt[v][tid];
                s_wcnt[v][tid] = 0;
            }
            s_off[tid] += add;
            __syncthreads();
        }
        grid.sync();
        uint64_t *t = src;
        src = dst;
        dst = t;
    }
    const uint64_t stride = (uint64_t)G * kSortThreads;
    for (uint64_t i = (uint64_t)w * kSortThreads + tid; i < z; i += stride)
        a.out[i] = to_record(src[i], a.idbits);
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

int finish_groups() {
    static int groups = 0;
    if (groups) return groups;
    int dev = 0, ncu = 0, occ = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_finish, kSortThreads, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    int g = ncu * occ;
    groups = g > kMaxGroups ? kMaxGroups : g;
    return groups;
}

mag_status launch_finish(Scratch &sc, uint64_t cap, uint64_t samples, uint64_t *d_count,
                         mag_stats *d_stats, mag_match *out, int idbits, int nbits,
                         hipStream_t stream) {
    const int G = sc.sort_groups;
    FinishArgs a;
    a.keys = sc.keys;
    a.cap = cap;
    a.counters = sc.counters;
    a.d_count = d_count;
    a.d_stats = d_stats;
    a.samples = samples;
    a.cnt = sc.hist;
    a.out = out;
    a.idbits = idbits;
    a.nbits = nbits;
    void *args[] = {&a};
    hipError_t e = hipLaunchCooperativeKernel((const void *)k_finish, dim3(G), dim3(kSortThreads),
                                              args, 0, stream);
    if (e != hipSuccess) return hip_fail(e, "finish launch");
    return MAG_OK;
}

}  // namespace mag
