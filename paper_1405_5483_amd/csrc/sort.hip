// Canonical output order: occurrences sorted ascending by (pos, id).
//
// The scan emits 64-bit keys (pos << idbits | id, batched scans add the job
// number above the position) in arbitrary order; keys are unique, since every
// (pos, id) is reported once. The finishing kernel (launched right after the
// scan) publishes the occurrence count and the work counters and ranks up to
// kSmallMax keys: each of its workgroups stages the keys in LDS and places
// kFinishKeys of them, so a small output is sorted by several compute units
// at once. Larger outputs are sorted by a stable LSD radix sort with 8-bit
// digits across the whole device: per pass a histogram, a scan of the counts
// and a scatter kernel. Those kernels read the count from device memory (the
// finishing kernel leaves it in counters[kSortCountSlot]), so they can be
// enqueued before the host knows it: the grid is sized for an upper bound and
// workgroups past the real count return at once. No kernel waits on another
// workgroup.
#include <hip/hip_runtime.h>

#include "mag_internal.hpp"

namespace mag {
namespace {

constexpr uint32_t kFinishWaves = 8;               // ranking waves per finishing workgroup
constexpr uint32_t kRankThreads = kFinishWaves * 64;
constexpr int kFinishThreads = kRankThreads + 64;  // plus the counter wave
constexpr uint32_t kSmallMax = 8192;
constexpr uint32_t kFinishKeys = 64;              // keys ranked per finishing workgroup
constexpr uint32_t kFinishGrid = kSmallMax / kFinishKeys;
constexpr uint32_t kFinishEager = 1024;           // keys loaded before the count is known
static_assert(kFinishEager % kRankThreads == 0, "whole eager rounds");
constexpr int kRadixThreads = 256;
constexpr uint32_t kRadixChunk = 4096;        // keys per chunk of the device-wide sort
constexpr uint32_t kRadixGrid = 1024;         // workgroups per radix kernel (they loop over chunks)
constexpr uint32_t kRadixChunkSmall = 1024;   // keys per chunk while that gives at most kRadixGrid chunks

// Keys per chunk for z keys: short sorts take small chunks, so that more
// workgroups share them and each scatters fewer rounds one after another.
__host__ __device__ inline uint64_t radix_chunk_keys(uint64_t z) {
    return z <= (uint64_t)kRadixGrid * kRadixChunkSmall ? kRadixChunkSmall : kRadixChunk;
}
__host__ __device__ inline uint64_t radix_chunk_count(uint64_t z) {
    const uint64_t k = radix_chunk_keys(z);
    return (z + k - 1) / k;
}

__global__ void k_fill_u64(uint64_t *p, uint64_t count, uint64_t value) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        p[i] = value;
}

__device__ __forceinline__ uint32_t lanes_below_mask(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Workgroup barrier that orders LDS accesses only: outstanding global loads
// and atomics of the waves stay in flight across it.
__device__ __forceinline__ void lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ mag_match to_record(uint64_t key, int idbits, uint64_t posmask) {
    mag_match r;
    r.pos = (key >> idbits) & posmask;
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

// Stable scatter of one chunk src[beg, end) (K keys, the last chunk fewer)
// by digit d = (key >> shift) & 255 into dst, digit d's run for this chunk
// starting at s_off[d]. The chunk is ordered by digit in LDS first: wave w
// takes keys [w K/4, (w+1) K/4) of the chunk, in input order, and ranks each
// among equal digits with ballots. The ordered chunk is then written out by
// consecutive threads to consecutive addresses of each digit's run, so the
// global writes come in runs of whole cache lines rather than one key per
// digit and round. s_run[wave][256] is zero on entry and on exit.
__device__ uint64_t block_exclusive_scan256(uint64_t v, uint64_t *s_tmp, uint64_t *total);
constexpr int kScatterWaves = kRadixThreads / 64;
static_assert(kRadixChunk % kRadixThreads == 0 && kRadixChunkSmall % kRadixThreads == 0,
              "chunks are whole rounds of every wave");
constexpr int kScatterMaxRounds = kRadixChunk / kRadixThreads;   // keys per lane
__device__ void chunk_scatter(const uint64_t *src, uint64_t *dst, uint64_t beg, uint64_t end, uint64_t K,
                              int shift, const uint64_t *s_off, uint64_t *s_keys,
                              uint32_t (*s_run)[256], uint32_t *s_start, uint64_t *s_tmp, mag_match *out,
                              int idbits, uint64_t posmask) {
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t n = (uint32_t)(end - beg);
    const uint32_t per = (uint32_t)(K / kScatterWaves);          // keys per wave, a multiple of 64
    const uint32_t rounds = per / 64;
    const uint32_t w0 = wave * per;
    uint64_t key[kScatterMaxRounds];
    uint32_t at[kScatterMaxRounds];                            // place among the wave's equal digits
#pragma unroll
    for (int r = 0; r < kScatterMaxRounds; ++r) {
        const uint32_t i = w0 + 64u * r + lane;
        key[r] = (r < (int)rounds && i < n) ? src[beg + i] : 0ull;
    }
#pragma unroll
    for (int r = 0; r < kScatterMaxRounds; ++r) {
        if (r >= (int)rounds) continue;      // wave-uniform
        const bool valid = w0 + 64u * r + lane < n;
        const uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
        const uint64_t eq = same_digit_lanes(valid, d);
        const uint32_t rank = lanes_below_mask(eq);
        const uint32_t before = valid ? s_run[wave][d] : 0u;
        at[r] = before + rank;
        // the lanes of one digit read the count before its first lane adds to it
        if (valid && rank == 0) s_run[wave][d] = before + (uint32_t)__popcll(eq);
    }
    __syncthreads();
    {
        // digit tid: its start in the ordered chunk, and each wave's start within it
        uint32_t c[kScatterWaves], tot = 0;
#pragma unroll
        for (int v = 0; v < kScatterWaves; ++v) {
            c[v] = s_run[v][tid];
            tot += c[v];
        }
        uint64_t all;
        const uint32_t st = (uint32_t)block_exclusive_scan256(tot, s_tmp, &all);
        s_start[tid] = st;
        uint32_t acc = st;
#pragma unroll
        for (int v = 0; v < kScatterWaves; ++v) {
            s_run[v][tid] = acc;
            acc += c[v];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kScatterMaxRounds; ++r) {
        if (r < (int)rounds && w0 + 64u * r + lane < n) {
            const uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
            s_keys[s_run[wave][d] + at[r]] = key[r];
        }
    }
    __syncthreads();
    for (uint32_t i = tid; i < n; i += kRadixThreads) {
        const uint64_t k = s_keys[i];
        const uint32_t d = (uint32_t)(k >> shift) & 255u;
        const uint64_t at = s_off[d] + (i - s_start[d]);
        if (out) out[at] = to_record(k, idbits, posmask);
        else dst[at] = k;
    }
#pragma unroll
    for (int v = 0; v < kScatterWaves; ++v) s_run[v][tid] = 0;
    __syncthreads();
}

// Exclusive prefix sum over a 256-thread block (one value per thread); the
// block total goes to *total. s_tmp holds 4 words.
__device__ uint64_t block_exclusive_scan256(uint64_t v, uint64_t *s_tmp, uint64_t *total) {
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint64_t inc = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t o = __shfl_up(inc, off);
        if (lane >= (uint32_t)off) inc += o;
    }
    if (lane == 63) s_tmp[wave] = inc;
    __syncthreads();
    uint64_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const uint64_t t = s_tmp[w];
        if (w < (int)wave) before += t;
        all += t;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

struct FinishArgs {
    const uint64_t *keys;  // the scan's keys, [0, cap)
    uint64_t cap;
    uint64_t *counters;    // read, published, then returned to zero
    uint64_t *d_count;
    mag_stats *d_stats;
    StatsInfo info;
    uint64_t samples;
    mag_match *out;
    uint64_t *sorted;      // optional: the sorted keys of small outputs too
    uint64_t posmask;
    uint64_t *seg_count;   // optional: deferred-start segment counters, returned to zero
    int idbits;
};

__global__ __launch_bounds__(kFinishThreads) void k_finish(FinishArgs a) {
    __shared__ uint64_t s_keys[kSmallMax];
    __shared__ uint64_t s_z;
    __shared__ uint32_t s_rank[kFinishKeys];
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63, wave = tid >> 6;
    // waves 0 .. kFinishWaves-1 rank; the last wave reads the counters and
    // reports the workgroup's arrival. The first kFinishEager keys are read
    // alongside the counters (slots past the count hold stale keys and are
    // never used).
    const uint32_t eager = a.cap < kFinishEager ? (uint32_t)a.cap : kFinishEager;
    uint64_t ek[kFinishEager / kRankThreads];
    if (wave < kFinishWaves) {
#pragma unroll
        for (uint32_t u = 0; u < kFinishEager / kRankThreads; ++u) {
            const uint32_t i = u * kRankThreads + tid;
            ek[u] = i < eager ? a.keys[i] : 0ull;
        }
    } else if (lane == 0) {
        const uint64_t z = a.counters[0];
        s_z = z;
        if (blockIdx.x == 0) {
            *a.d_count = z;
            if (a.d_stats) {
                a.d_stats->samples = a.samples;
                a.d_stats->cand_windows = a.counters[1];
                a.d_stats->verifications = a.counters[2];
                a.d_stats->matches = z;
                a.d_stats->q = a.info.q;
                a.d_stats->k = a.info.k;
                a.d_stats->sigma_prime = a.info.sigma_prime;
                a.d_stats->m_prime = a.info.m_prime;
                a.d_stats->plan_ms = a.info.plan_ms;
                a.d_stats->scan_ms = 0.0f;
            }
            // the count stays for the device-wide sort
            a.counters[kSortCountSlot] = z;
        }
    }
    // the verification kernel has read the segment counts (it ran before)
    if (blockIdx.x == 0 && a.seg_count)
        for (uint32_t i = tid; i < kPendingSegments; i += kFinishThreads) a.seg_count[i] = 0;
    __syncthreads();
    const uint64_t z = s_z;
    const uint32_t base = blockIdx.x * kFinishKeys;
    const bool ranks = z <= a.cap && z != 0 && z <= kSmallMax && base < z;

    if (wave == kFinishWaves) {
        // every workgroup has read the counters once it arrives here; the
        // last to arrive returns them (and the arrival count) to zero for the
        // next scan. This wave loads nothing else, so the ranking waves never
        // wait for the arrival; it joins their two barriers meanwhile.
        unsigned long long arrival = 0;
        if (lane == 0) {
            // an opaque (per-lane) slot index keeps the compiler from
            // combining the wave's atomics, which would wait for the result
            // right away
            uint32_t slot = kFinishDoneSlot;
            asm volatile("" : "+v"(slot));
            arrival = atomicAdd((unsigned long long *)&a.counters[slot], 1ull);
        }
        if (ranks) {
            lds_sync();
            lds_sync();
        }
        if (lane == 0 && arrival == gridDim.x - 1) {
            for (int c = 0; c < 4; ++c)
                __hip_atomic_store(&a.counters[c], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.counters[kFinishDoneSlot], 0ull, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        return;
    }
    if (!ranks) return;

    // keys are unique: a key's output slot is the number of smaller keys.
    // Every workgroup stages all z keys in LDS (eight loads in flight per
    // thread) and ranks kFinishKeys of them, one per lane; each wave counts
    // over its share of the keys (8 independent sums, so LDS reads overlap)
    // and the shares are combined with LDS atomics.
    const uint32_t zz = (uint32_t)z;
#pragma unroll
    for (uint32_t u = 0; u < kFinishEager / kRankThreads; ++u) {
        const uint32_t i = u * kRankThreads + tid;
        if (i < zz) s_keys[i] = ek[u];
    }
    for (uint32_t b = kFinishEager; b < zz; b += 8 * kRankThreads) {
        uint64_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t i = b + u * kRankThreads + tid;
            v[u] = i < zz ? a.keys[i] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t i = b + u * kRankThreads + tid;
            if (i < zz) s_keys[i] = v[u];
        }
    }
    if (tid < kFinishKeys) s_rank[tid] = 0;
    lds_sync();
    const uint32_t i = base + lane;
    const uint64_t key = i < zz ? s_keys[i] : 0ull;
    const uint32_t share = (zz + kFinishWaves - 1) / kFinishWaves;
    const uint32_t j0 = wave * share < zz ? wave * share : zz;
    const uint32_t j1 = j0 + share < zz ? j0 + share : zz;
    uint32_t acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    uint32_t j = j0;
    for (; j + 8 <= j1; j += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] += s_keys[j + u] < key ? 1u : 0u;
    }
    for (; j < j1; ++j) acc[0] += s_keys[j] < key ? 1u : 0u;
    const uint32_t below = acc[0] + acc[1] + acc[2] + acc[3] + acc[4] + acc[5] + acc[6] + acc[7];
    if (below) atomicAdd(&s_rank[lane], below);
    lds_sync();
    if (i < zz) {
        const uint32_t r = s_rank[lane];
        a.out[r] = to_record(key, a.idbits, a.posmask);
        if (a.sorted) a.sorted[r] = key;
    }
}

// ---- device-wide LSD radix sort. The count z is read from *zp; every kernel
// returns at once unless kSmallMax < z <= cap. Keys are cut into chunks of
// radix_chunk_keys(z); cnt and off are digit-major [256][C], C = ceil(z / chunk).

__device__ __forceinline__ bool radix_active(const uint64_t *zp, uint64_t cap, uint64_t *z) {
    *z = *zp;
    return *z > kSmallMax && *z <= cap;
}

__global__ __launch_bounds__(kRadixThreads) void k_radix_hist(const uint64_t *src, const uint64_t *zp,
                                                              uint64_t cap, int shift, uint32_t *cnt) {
    __shared__ uint32_t s_hist[256];
    uint64_t z;
    if (!radix_active(zp, cap, &z)) return;
    const uint64_t K = radix_chunk_keys(z), C = (z + K - 1) / K;
    const uint32_t tid = threadIdx.x;
    for (uint64_t c = blockIdx.x; c < C; c += gridDim.x) {
        s_hist[tid] = 0;
        __syncthreads();
        const uint64_t beg = c * K;
        const uint64_t end = beg + K < z ? beg + K : z;
        // four loads in flight before their digits are counted
        for (uint64_t i = beg + tid; i < end; i += 4 * kRadixThreads) {
            uint64_t k4[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint64_t j = i + (uint64_t)r * kRadixThreads;
                k4[r] = j < end ? src[j] : 0ull;
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (i + (uint64_t)r * kRadixThreads < end) atomicAdd(&s_hist[(k4[r] >> shift) & 255u], 1u);
        }
        __syncthreads();
        cnt[(size_t)tid * C + c] = s_hist[tid];
        __syncthreads();
    }
}

// One workgroup per digit d: off[d][c] = sum of cnt[d][c' < c], tot[d] = row sum.
__global__ __launch_bounds__(256) void k_radix_scan(const uint32_t *cnt, uint64_t *off, uint64_t *tot,
                                                    const uint64_t *zp, uint64_t cap) {
    __shared__ uint64_t s_tmp[4];
    uint64_t z;
    if (!radix_active(zp, cap, &z)) return;
    const uint64_t K = radix_chunk_keys(z), C = (z + K - 1) / K;
    const uint32_t d = blockIdx.x, tid = threadIdx.x;
    uint64_t carry = 0;
    for (uint64_t base = 0; base < C; base += 256) {
        const uint64_t c = base + tid;
        const uint64_t v = c < C ? cnt[(size_t)d * C + c] : 0;
        uint64_t part;
        const uint64_t ex = block_exclusive_scan256(v, s_tmp, &part);
        if (c < C) off[(size_t)d * C + c] = carry + ex;
        carry += part;
    }
    if (tid == 0) tot[d] = carry;
}

// out (the last pass of a sort whose records need no job offsets; else
// null): the records are written in place of the sorted keys.
__global__ __launch_bounds__(kRadixThreads) void k_radix_scatter(const uint64_t *src, uint64_t *dst,
                                                                 const uint64_t *zp, uint64_t cap,
                                                                 int shift, const uint64_t *off,
                                                                 const uint64_t *tot, mag_match *out,
                                                                 int idbits, uint64_t posmask) {
    __shared__ uint64_t s_base[256];
    __shared__ uint64_t s_off[256];
    __shared__ uint64_t s_tmp[4];
    __shared__ uint32_t s_start[256];
    __shared__ uint32_t s_run[kScatterWaves][256];
    __shared__ uint64_t s_keys[kRadixChunk];
    uint64_t z;
    if (!radix_active(zp, cap, &z)) return;
    const uint64_t K = radix_chunk_keys(z), C = (z + K - 1) / K;
    const uint32_t tid = threadIdx.x;
    uint64_t all;
    s_base[tid] = block_exclusive_scan256(tot[tid], s_tmp, &all);
    for (int v = 0; v < kScatterWaves; ++v) s_run[v][tid] = 0;
    for (uint64_t c = blockIdx.x; c < C; c += gridDim.x) {
        s_off[tid] = s_base[tid] + off[(size_t)tid * C + c];
        __syncthreads();
        const uint64_t beg = c * K;
        const uint64_t end = beg + K < z ? beg + K : z;
        chunk_scatter(src, dst, beg, end, K, shift, s_off, s_keys, s_run, s_start, s_tmp, out, idbits, posmask);
    }
}

// Records of the sorted keys. Batches (jbase not null) key positions in their
// texts laid end to end: a record's position is made relative to its job's
// text, jbase[j] (njobs + 1 ascending offsets) being job j's first byte, the
// job the last j with jbase[j] <= the position (empty jobs share their offset
// with the next). The offsets are staged in LDS when they fit.
constexpr uint32_t kExpandJobsLds = 2048;
__global__ __launch_bounds__(256) void k_expand(const uint64_t *keys, const uint64_t *zp, uint64_t cap,
                                                mag_match *out, int idbits, uint64_t posmask,
                                                const uint64_t *jbase, uint32_t njobs) {
    __shared__ uint64_t s_jb[kExpandJobsLds];
    uint64_t z;
    if (!radix_active(zp, cap, &z)) return;
    const bool staged = jbase && njobs <= kExpandJobsLds;
    if (staged)
        for (uint32_t t = threadIdx.x; t < njobs; t += blockDim.x) s_jb[t] = jbase[t];
    __syncthreads();
    const uint64_t *jb = staged ? s_jb : jbase;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < z; i += stride) {
        mag_match r = to_record(keys[i], idbits, posmask);
        if (jb) r.pos -= jb[job_of_position(jb, njobs, r.pos)];
        out[i] = r;
    }
}

// Chunks of the largest count a sort of at most `bound` keys can take.
uint64_t radix_chunks(uint64_t bound) {
    const uint64_t small = (uint64_t)kRadixGrid * kRadixChunkSmall;
    const uint64_t a = radix_chunk_count(bound < small ? bound : small), b = radix_chunk_count(bound);
    return a > b ? a : b;
}

uint32_t radix_grid(uint64_t bound) {
    const uint64_t C = radix_chunks(bound);
    return (uint32_t)(C < kRadixGrid ? (C ? C : 1) : kRadixGrid);
}

}  // namespace

uint64_t radix_scratch_chunks(uint64_t bound) { return radix_chunks(bound); }

mag_status launch_fill_u64(uint64_t *ptr, uint64_t count, uint64_t value, hipStream_t stream) {
    if (!count) return MAG_OK;
    uint64_t blocks = (count + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_fill_u64, dim3((uint32_t)blocks), dim3(256), 0, stream, ptr, count, value);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MAG_OK : hip_fail(e, "fill launch");
}

uint32_t small_sort_max() { return kSmallMax; }

int radix_passes(int nbits, int lo) { return nbits > lo ? (nbits - lo + 7) / 8 : 0; }

mag_status launch_finish(Scratch &sc, uint64_t cap, uint64_t samples, uint64_t *d_count,
                         mag_stats *d_stats, const StatsInfo &info, mag_match *out, int idbits,
                         uint64_t posmask, uint64_t *sorted, hipStream_t stream) {
    FinishArgs a;
    a.keys = sc.keys;
    a.cap = cap;
    a.counters = sc.counters;
    a.d_count = d_count;
    a.d_stats = d_stats;
    a.info = info;
    a.samples = samples;
    a.out = out;
    a.sorted = sorted;
    a.posmask = posmask;
    a.seg_count = sc.seg_count;
    a.idbits = idbits;
    hipLaunchKernelGGL(k_finish, dim3(kFinishGrid), dim3(kFinishThreads), 0, stream, a);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MAG_OK : hip_fail(e, "finish launch");
}

mag_status ensure_radix_scratch(Scratch &sc, uint64_t bound, hipStream_t stream) {
    const uint64_t C = radix_chunks(bound);
    if (sc.radix_chunks >= C && sc.hist) return MAG_OK;
    hipError_t e = hipStreamSynchronize(stream);     // earlier sorts may still use the old buffers
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    (void)hipFree(sc.hist);
    (void)hipFree(sc.radix_off);
    sc.hist = nullptr;
    sc.radix_off = nullptr;
    sc.radix_chunks = 0;
    e = hipMalloc(&sc.hist, (size_t)256 * C * sizeof(uint32_t));
    // offsets [256][C], then the 256 digit totals
    if (e == hipSuccess) e = hipMalloc(&sc.radix_off, ((size_t)256 * C + 256) * sizeof(uint64_t));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(MAG_E_NOMEM, "device allocation of radix counts failed");
    }
    sc.radix_chunks = C;
    return MAG_OK;
}

mag_status launch_radix_sort(Scratch &sc, uint64_t bound, uint64_t cap, int nbits, int lo, hipStream_t stream,
                             mag_match *out, int idbits, uint64_t posmask) {
    if (bound <= kSmallMax) return MAG_OK;
    if (sc.radix_chunks < radix_chunks(bound) || !sc.hist)
        return fail(MAG_E_INVALID, "radix scratch smaller than the bound");
    if (bound > cap) bound = cap;
    const uint32_t G = radix_grid(bound);
    const uint64_t *zp = sc.counters + kSortCountSlot;
    uint64_t *src = sc.keys, *dst = sc.keys + cap;
    uint64_t *tot = sc.radix_off + (size_t)256 * sc.radix_chunks;
    const int passes = radix_passes(nbits, lo);
    for (int p = 0; p < passes; ++p) {
        const int shift = lo + 8 * p;
        hipLaunchKernelGGL(k_radix_hist, dim3(G), dim3(kRadixThreads), 0, stream,
                           (const uint64_t *)src, zp, cap, shift, sc.hist);
        hipLaunchKernelGGL(k_radix_scan, dim3(256), dim3(256), 0, stream, (const uint32_t *)sc.hist,
                           sc.radix_off, tot, zp, cap);
        hipLaunchKernelGGL(k_radix_scatter, dim3(G), dim3(kRadixThreads), 0, stream,
                           (const uint64_t *)src, dst, zp, cap, shift, (const uint64_t *)sc.radix_off,
                           (const uint64_t *)tot, p + 1 == passes ? out : nullptr, idbits, posmask);
        uint64_t *t = src;
        src = dst;
        dst = t;
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MAG_OK : hip_fail(e, "radix sort launch");
}

uint64_t *sorted_keys(Scratch &sc, uint64_t cap, int nbits, int lo) {
    return (radix_passes(nbits, lo) & 1) ? sc.keys + cap : sc.keys;
}

mag_status launch_expand(Scratch &sc, uint64_t bound, uint64_t cap, int nbits, int lo, mag_match *out,
                         int idbits, uint64_t posmask, hipStream_t stream, const uint64_t *jbase,
                         uint32_t njobs) {
    if (bound <= kSmallMax) return MAG_OK;
    if (bound > cap) bound = cap;
    uint64_t blocks = (bound + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_expand, dim3((uint32_t)blocks), dim3(256), 0, stream,
                       (const uint64_t *)sorted_keys(sc, cap, nbits, lo),
                       (const uint64_t *)(sc.counters + kSortCountSlot), cap, out, idbits, posmask, jbase,
                       njobs);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MAG_OK : hip_fail(e, "expand launch");
}

}  // namespace mag
