// Batched MAG scans: many independent (text, pattern set) jobs in one
// persistent launch.
//
// Every job is cut into tiles (512 * words-per-lane samples; dense jobs
// kDenseTilePositions start positions); the tiles of all
// jobs form one global sequence (job after job) that the host splits into
// contiguous ranges of about equal text bytes, one per workgroup, so a
// workgroup restages a job's alphabet map and mask table in LDS only when its
// range crosses into the next job. Per tile the kernel runs the two phases of
// the single-job scan with all of its threads: the mask entries of the
// tile's samples (with the job's q, k, sigma' and table; q selects one of
// eight compile-time variants per tile), then the Shift-Or recurrence over
// each lane's run of entries, with ballot-compacted candidate windows and
// exact verification of their start positions. Keys carry the job number
// above the position, so one device-wide sort orders the whole output job by
// job, and a last kernel finds each job's first record. Nothing waits on the
// host, so the launch sequence can be captured in a hipGraph.
//
// Batched jobs keep their state in 32 bits: W = k*m' <= 32 and k < 32.
#include <hip/hip_runtime.h>

#include "batch.hpp"
#include "scan_common.hpp"

namespace mag {
static_assert(kBatchQueue >= (int)kDenseQueue, "dense tiles fill up to kDenseQueue starts");
namespace {

using namespace dev;

constexpr int kBT = kBatchThreads;
constexpr int kWaves = kBT / 64;
static_assert(kBatchMaxWarm % 4 == 0, "lane runs are whole vectors");

__device__ __forceinline__ uint32_t uni32(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
// readfirstlane returns int: each half goes through uint32_t so that the low
// word is not sign-extended into the high one
__device__ __forceinline__ uint64_t uni64(uint64_t x) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}
template <typename T>
__device__ __forceinline__ T *uniptr(T *p) {
    return reinterpret_cast<T *>(uni64(reinterpret_cast<uint64_t>(p)));
}

// Entries are read and written as 16-byte vectors of four u32 entries;
// vector V lives at V ^ ((V >> 3) & 7). A Shift-Or read step has the lanes
// kLaneVecs vectors apart; with the swizzle any eight consecutive lanes read
// eight different 16-byte bank groups. Phase A's stores of consecutive
// vectors stay conflict-free.
__device__ __forceinline__ uint32_t swz(uint32_t V) { return V ^ ((V >> 3) & 7u); }

template <int ESZ>
__device__ __forceinline__ uint32_t lds_entry(const uint8_t *s_tab, uint32_t g) {
    if constexpr (ESZ == 1) return s_tab[g];
    else if constexpr (ESZ == 2) return reinterpret_cast<const uint16_t *>(s_tab)[g];
    else return reinterpret_cast<const uint32_t *>(s_tab)[g];
}

template <int ESZ>
__device__ __forceinline__ uint32_t l2_entry(__amdgpu_buffer_rsrc_t trs, uint32_t g) {
    if constexpr (ESZ == 1) return __builtin_amdgcn_raw_buffer_load_b8(trs, (int)g, 0, 0);
    else if constexpr (ESZ == 2) return __builtin_amdgcn_raw_buffer_load_b16(trs, (int)(2 * g), 0, 0);
    else return __builtin_amdgcn_raw_buffer_load_b32(trs, (int)(4 * g), 0, 0);
}

// Mask entries (as u32) of samples X0-w0 .. X0+TS-1 of one job: entry of
// sample X0+s goes to E index s + w0. Thread tid computes vectors tid,
// tid + kBT, ... two at a time (both loads issued before the lookups).
template <int TS, int Q, int ESZ>
__device__ void phase_a(uint4 *s_E, __amdgpu_buffer_rsrc_t rs, int32_t p0, uint32_t kq, uint32_t sp,
                        const uint8_t *s_mu, const uint8_t *s_tab, __amdgpu_buffer_rsrc_t trs,
                        bool tlds, int w0, int64_t X0, int64_t X, int tid) {
    const uint32_t none = ESZ == 1 ? 0xFFu : ESZ == 2 ? 0xFFFFu : 0xFFFFFFFFu;
    const int nvec = (TS + w0) / 4;
    for (int V = tid; V < nvec; V += 2 * kBT) {
        GramWords w[2][4];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int s = 4 * (V + h * kBT) - w0;
#pragma unroll
            for (int u = 0; u < 4; ++u)
                w[h][u] = gram_words<Q>(rs, (uint32_t)(p0 + (s + u) * (int32_t)kq));
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int Vh = V + h * kBT;
            if (Vh >= nvec) break;
            const int s = 4 * Vh - w0;
            uint32_t e[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t g = gram_code<Q, true>(w[h][u], s_mu, sp);
                e[u] = tlds ? lds_entry<ESZ>(s_tab, g) : l2_entry<ESZ>(trs, g);
                const int64_t x = X0 + s + u;
                if (x < 0 || x >= X) e[u] = none;
            }
            s_E[swz((uint32_t)Vh)] = make_uint4(e[0], e[1], e[2], e[3]);
        }
    }
}

template <int TS, int Q>
__device__ __forceinline__ void phase_a_q(uint32_t esz, uint4 *s_E, __amdgpu_buffer_rsrc_t rs,
                                          int32_t p0, uint32_t kq, uint32_t sp, const uint8_t *s_mu,
                                          const uint8_t *s_tab, __amdgpu_buffer_rsrc_t trs, bool tlds,
                                          int w0, int64_t X0, int64_t X, int tid) {
    if (esz == 1) phase_a<TS, Q, 1>(s_E, rs, p0, kq, sp, s_mu, s_tab, trs, tlds, w0, X0, X, tid);
    else if (esz == 2) phase_a<TS, Q, 2>(s_E, rs, p0, kq, sp, s_mu, s_tab, trs, tlds, w0, X0, X, tid);
    else phase_a<TS, Q, 4>(s_E, rs, p0, kq, sp, s_mu, s_tab, trs, tlds, w0, X0, X, tid);
}

constexpr uint64_t kNoTile = ~0ull;

// Wave 0 of a workgroup picks the workgroup with the most unclaimed tiles
// (other than `me`) and claims one of them; kNoTile when none is left. The
// claim counters only grow, so a tile is never handed out twice, and once
// every range is exhausted it stays so.
__device__ uint64_t steal_tile(uint64_t *next, const uint64_t *ranges, uint32_t G, uint32_t me,
                               int lane) {
    for (;;) {
        uint64_t best = 0;                       // (remaining << 16) | workgroup
        for (uint32_t base = 0; base < G; base += 64) {
            const uint32_t v = base + (uint32_t)lane;
            if (v < G && v != me) {
                const uint64_t nx = __hip_atomic_load(&next[v], __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
                const uint64_t end = ranges[3 * v + 1];
                const uint64_t rem = nx < end ? end - nx : 0;
                const uint64_t key = (rem << 16) | v;
                if (rem && key > best) best = key;
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const uint64_t o = __shfl_xor(best, off);
            best = o > best ? o : best;
        }
        if (best == 0) return kNoTile;
        const uint32_t v = (uint32_t)(best & 0xFFFF);
        unsigned long long c = 0;
        if (lane == 0) c = atomicAdd((unsigned long long *)&next[v], 1ull);
        c = __shfl(c, 0);
        if (c < ranges[3 * v + 1]) return c;
    }
}

// TS: samples per filter tile (512 * words per lane).
template <int TS>
__global__ __launch_bounds__(kBT, 4) void k_batch(const JobDesc *__restrict__ jobs, uint32_t njobs,
                                               const uint64_t *__restrict__ ranges,
                                               uint64_t *next, uint64_t *counters) {
    constexpr int kS = TS / kBT;                 // samples per lane in the Shift-Or phase
    constexpr int kLaneVecs = kS / 4;            // 16-byte vectors of u32 entries per lane
    static_assert(kS % 4 == 0, "lane runs are whole vectors");
    // static LDS of a fixed size: every carved-out array sits at a known
    // address, so LDS accesses need no base added at run time
    __shared__ __align__(16) uint8_t smem[batch_lds_bytes(TS)];
    uint8_t *s_mu = smem;
    uint64_t *s_ctl = reinterpret_cast<uint64_t *>(smem + 256);          // claimed tiles, 2 slots
    uint64_t *s_queue = reinterpret_cast<uint64_t *>(smem + 256 + 16);
    uint4 *s_E = reinterpret_cast<uint4 *>(smem + 256 + 16 + kWaves * kBatchQueue * 8);
    uint8_t *s_tab = smem + 256 + 16 + kWaves * kBatchQueue * 8 + batch_entry_bytes(TS);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint64_t *queue = s_queue + wave * kBatchQueue;
    uint32_t qn = 0;
    // While the workgroup runs dense tiles, the entry buffer (used only by
    // filter tiles) holds each wave's found keys, written to the output with
    // one atomic add per buffer instead of one per verification round; the
    // buffers are flushed before a filter tile's mask entries overwrite them.
    constexpr uint32_t kFoundCap = batch_entry_bytes(TS) / 8 / kWaves;
    uint64_t *fbuf = reinterpret_cast<uint64_t *>(s_E) + wave * kFoundCap;
    uint32_t fbn = 0;
    uint64_t ncand = 0, nver = 0;
    const uint32_t me = blockIdx.x, G = gridDim.x;
    const uint64_t own_end = uni64(ranges[3 * me + 1]);
    bool own_done = false;

    // first tile
    if (wave == 0) {
        unsigned long long c = 0;
        if (lane == 0) c = atomicAdd((unsigned long long *)&next[me], 1ull);
        c = __shfl(c, 0);
        uint64_t t = c;
        if (c >= own_end) {
            own_done = true;
            t = steal_tile(next, ranges, G, me, lane);
        }
        if (lane == 0) s_ctl[0] = t;
    }
    __syncthreads();

    // the current job, in scalar registers
    int cur = -1;
    const VerifyArgs *vp = nullptr;
    const uint8_t *tbase = nullptr;
    __amdgpu_buffer_rsrc_t trs = tile_rsrc(nullptr, 0);
    uint64_t delta = 0, n = 0, X = 0, tfirst = 0, tend = 0;
    uint32_t q = 1, k = 1, kq = 1, mprime = 1, W = 1, sp = 1, esz = 1, w0 = 0, tlds = 0, m = 1;
    uint32_t dense = 0, bshift = 32, hw = 1, mw = 1, lastmask = 0;

    for (uint32_t slot = 0;; slot ^= 1) {
        const uint64_t g = uni64(s_ctl[slot]);
        if (g == kNoTile) break;
        // wave 0 asks for the next tile now and settles the claim after phase A
        unsigned long long pending = 0;
        if (wave == 0 && !own_done && lane == 0)
            pending = atomicAdd((unsigned long long *)&next[me], 1ull);
        if (cur < 0 || g < tfirst || g >= tend) {
            if (cur >= 0 && qn) {
                drain_partial(vp, queue, qn, lane);   // starts of the previous job
                qn = 0;
            }
            // the job holding tile g: the last one whose first tile is <= g
            // (jobs without tiles share their first tile with the next job)
            uint32_t lo = 0, hi = njobs - 1;
            while (lo < hi) {
                const uint32_t mid = (lo + hi + 1) / 2;
                if (jobs[mid].tile_first <= g) lo = mid;
                else hi = mid - 1;
            }
            const uint32_t j = uni32(lo);
            const JobDesc &J = jobs[j];
            cur = (int)j;
            vp = &J.v;
            tbase = uniptr(J.tbase);
            delta = uni64(J.delta);
            n = uni64(J.n);
            X = uni64(J.X);
            tfirst = uni64(J.tile_first);
            tend = tfirst + uni64(J.ntiles);
            q = uni32(J.q);
            k = uni32(J.k);
            kq = uni32(J.kq);
            mprime = uni32(J.mprime);
            W = uni32(J.W);
            sp = uni32(J.sp) & 0x1FFu;      // sigma' <= 256: keeps 24-bit Horner steps
            esz = uni32(J.esz);
            w0 = uni32(J.w0);
            tlds = uni32(J.tlds);
            m = uni32(J.v.m);
            dense = uni32(J.dense);
            bshift = uni32(J.bshift);
            hw = uni32(J.v.hw);
            mw = uni32(J.v.mw);
            lastmask = uni32(J.v.lastmask);
            const uint32_t tvec = uni32(J.table_vec);
            const uint8_t *mu = uniptr(J.mu);
            const uint8_t *table = uniptr(reinterpret_cast<const uint8_t *>(J.table));
            trs = tile_rsrc(table, tvec * 16u);
            __syncthreads();                // the previous tile is done with the LDS tables
            for (int i = tid; i < 256; i += kBT) s_mu[i] = mu[i];
            if (tlds) {
                const uint4 *src = reinterpret_cast<const uint4 *>(table);
                uint4 *dst = reinterpret_cast<uint4 *>(s_tab);
                for (uint32_t v = tid; v < tvec; v += kBT) dst[v] = src[v];
            }
        }
        const int64_t X0 = (int64_t)(g - tfirst) * (dense ? kDenseTilePositions : TS);
        if (dense) {
            // start positions X0 .. X0 + kDenseTilePositions - 1 against the Bloom bitmap in s_tab
            int64_t e1 = X0 + kDenseTilePositions + 40;
            if (e1 > (int64_t)n) e1 = (int64_t)n;
            const uint64_t da0 = (delta + (uint64_t)X0) & ~15ull;
            const uint64_t da1 = (delta + (uint64_t)e1 + 15) & ~15ull;
            const __amdgpu_buffer_rsrc_t drs = tile_rsrc(tbase + da0, (uint32_t)(da1 - da0));
            __syncthreads();                // the bitmap is staged
            if (wave == 0) {
                uint64_t t = kNoTile;
                if (!own_done) {
                    const uint64_t c = __shfl(pending, 0);
                    if (c < own_end) t = c;
                    else own_done = true;
                }
                if (t == kNoTile) t = steal_tile(next, ranges, G, me, lane);
                if (lane == 0) s_ctl[slot ^ 1] = t;
            }
            dense_tile<kBT>(drs, (uint32_t)(da1 - da0), (uint32_t)(delta + (uint64_t)X0 - da0), X0,
                            (int64_t)n - (int64_t)m,
                            reinterpret_cast<const uint32_t *>(s_tab), bshift, hw, mw, lastmask, queue,
                            qn, vp, tid, lane, nver, FoundBuf{fbuf, &fbn, kFoundCap});
            __syncthreads();                // s_ctl for the next tile
            continue;
        }
        // text bytes the tile's samples touch, warm-up included
        int64_t b0 = (X0 - (int64_t)w0) * kq;
        if (b0 < 0) b0 = 0;
        int64_t b1 = (X0 + TS) * (int64_t)kq + kMaxQ;
        if (b1 > (int64_t)n) b1 = (int64_t)n;
        if (b1 < b0) b1 = b0;
        const uint64_t pa0 = (delta + (uint64_t)b0) & ~15ull;
        const uint64_t pa1 = (delta + (uint64_t)b1 + 15) & ~15ull;
        const __amdgpu_buffer_rsrc_t rs = tile_rsrc(tbase + pa0, (uint32_t)(pa1 - pa0));
        const int32_t p0 = (int32_t)((int64_t)delta - (int64_t)pa0 + X0 * (int64_t)kq);
        if (fbn) {                          // found keys of earlier dense tiles
            flush_found_args(vp, fbuf, fbn);
            fbn = 0;
        }
        __syncthreads();                    // tables staged; the previous tile's entries consumed
        switch (q) {
            case 1: phase_a_q<TS, 1>(esz, s_E, rs, p0, kq, sp, s_mu, s_tab, trs, tlds, (int)w0, X0, (int64_t)X, tid); break;
            case 2: phase_a_q<TS, 2>(esz, s_E, rs, p0, kq, sp, s_mu, s_tab, trs, tlds, (int)w0, X0, (int64_t)X, tid); break;
            case 3: phase_a_q<TS, 3>(esz, s_E, rs, p0, kq, sp, s_mu, s_tab, trs, tlds, (int)w0, X0, (int64_t)X, tid); break;
            case 4: phase_a_q<TS, 4>(esz, s_E, rs, p0, kq, sp, s_mu, s_tab, trs, tlds, (int)w0, X0, (int64_t)X, tid); break;
            case 5: phase_a_q<TS, 5>(esz, s_E, rs, p0, kq, sp, s_mu, s_tab, trs, tlds, (int)w0, X0, (int64_t)X, tid); break;
            case 6: phase_a_q<TS, 6>(esz, s_E, rs, p0, kq, sp, s_mu, s_tab, trs, tlds, (int)w0, X0, (int64_t)X, tid); break;
            case 7: phase_a_q<TS, 7>(esz, s_E, rs, p0, kq, sp, s_mu, s_tab, trs, tlds, (int)w0, X0, (int64_t)X, tid); break;
            default: phase_a_q<TS, 8>(esz, s_E, rs, p0, kq, sp, s_mu, s_tab, trs, tlds, (int)w0, X0, (int64_t)X, tid); break;
        }
        if (wave == 0) {
            uint64_t t = kNoTile;
            if (!own_done) {
                const uint64_t c = __shfl(pending, 0);
                if (c < own_end) t = c;
                else own_done = true;
            }
            if (t == kNoTile) t = steal_tile(next, ranges, G, me, lane);
            if (lane == 0) s_ctl[slot ^ 1] = t;
        }
        __syncthreads();

        // Shift-Or over the lane's kS samples, after w0 warm-up entries (only
        // the last m' entries reach the candidate bits, so older ones are harmless)
        const uint32_t kmask = (1u << k) - 1u;           // k < 32
        const uint32_t topshift = W - k;
        const int64_t last = (int64_t)n - (int64_t)m;    // last valid start position
        const uint32_t vb = (uint32_t)tid * kLaneVecs;
        uint32_t D = 0xFFFFFFFFu;
        for (uint32_t v = 0; v < w0 / 4; ++v) {
            const uint4 raw = s_E[swz(vb + v)];
            D = (D << k) | raw.x;
            D = (D << k) | raw.y;
            D = (D << k) | raw.z;
            D = (D << k) | raw.w;
        }
#pragma unroll
        for (int v = 0; v < kLaneVecs; ++v) {
            const uint4 raw = s_E[swz(vb + w0 / 4 + v)];
            const uint32_t ent[4] = {raw.x, raw.y, raw.z, raw.w};
            const uint32_t Dstart = D;
            uint32_t all = 0xFFFFFFFFu;      // a 0 in a candidate bit: some entry fired
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                D = (D << k) | ent[u];
                all &= D;
            }
            if (!__ballot((((~all) >> topshift) & kmask) != 0u)) continue;
            // slow path: step through the vector again, queueing the start
            // positions of every candidate window
            const int64_t xv = X0 + (int64_t)tid * kS + 4 * v;
            uint32_t R = Dstart;
            for (int u = 0; u < 4; ++u) {
                R = (R << k) | ent[u];
                uint32_t c = ((~R) >> topshift) & kmask;
                if (!__ballot(c != 0u)) continue;
                const int64_t topx = (xv + u - (int64_t)mprime + 1) * (int64_t)kq;
                for (;;) {
                    const bool has = c != 0u;
                    const uint64_t hb = __ballot(has);
                    if (!hb) break;
                    ncand += (uint64_t)__popcll(hb);
                    const uint32_t bit = has ? (uint32_t)__builtin_ctz(c) : 0u;
                    if (has) c &= c - 1u;
                    const int64_t top = topx - (int64_t)bit * q;
                    for (uint32_t sft = 0; sft < q; ++sft) {
                        const int64_t i0 = top - sft;
                        const bool ok = has && i0 >= 0 && i0 <= last;
                        const uint64_t bal = __ballot(ok);
                        if (ok) {
                            queue[qn + lanes_below(bal)] = (uint64_t)i0;
                            ++nver;
                        }
                        qn += (uint32_t)__popcll(bal);
                        if (qn >= 64) {
                            qn -= 64;
                            drain64(vp, queue, qn, lane);
                        }
                    }
                }
            }
        }
    }
    if (cur >= 0 && qn) drain_partial(vp, queue, qn, lane);
    if (fbn) flush_found_args(vp, fbuf, fbn);
    if (lane == 0 && ncand) atomicAdd((unsigned long long *)&counters[1], (unsigned long long)ncand);
    unsigned long long nv = nver;
    for (int off = 32; off > 0; off >>= 1) nv += __shfl_xor(nv, off);
    if (lane == 0 && nv) atomicAdd((unsigned long long *)&counters[2], nv);
}

// Claim counters back to the first tile of each workgroup's range.
__global__ void k_batch_init(const uint64_t *ranges, uint64_t *next, uint32_t G) {
    const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w < G) next[w] = ranges[3 * w];
}

// offsets[j] = first record of job j (binary search of the sorted keys on the
// job field), offsets[njobs] = the count. One thread per entry.
__global__ void k_batch_offsets(const uint64_t *sorted, const uint64_t *zp, uint64_t cap,
                                uint64_t *offsets, uint32_t njobs, int job_shift) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > njobs) return;
    const uint64_t z = *zp;
    uint64_t at = 0;
    if (j == njobs) {
        at = z;
    } else if (z <= cap) {
        uint64_t lo = 0, hi = z;
        while (lo < hi) {
            const uint64_t mid = lo + (hi - lo) / 2;
            if ((sorted[mid] >> job_shift) < j) lo = mid + 1;
            else hi = mid;
        }
        at = lo;
    }
    offsets[j] = at;
}

}  // namespace

mag_status batch_configure() { return MAG_OK; }   // the kernel's LDS is static

namespace {
const void *batch_kernel(int words_per_lane) {
    switch (words_per_lane) {
        case 8: return (const void *)k_batch<8 * kBT>;
        case 32: return (const void *)k_batch<32 * kBT>;
        default: return (const void *)k_batch<16 * kBT>;
    }
}
}  // namespace

int batch_occupancy(int words_per_lane) {
    batch_configure();
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, batch_kernel(words_per_lane), kBT, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return occ;
}

mag_status launch_batch(const BatchLaunch &b, hipStream_t stream) {
    if (!b.total_tiles || !b.grid) return MAG_OK;
    hipLaunchKernelGGL(k_batch_init, dim3((b.grid + 255) / 256), dim3(256), 0, stream, b.ranges,
                       b.next, b.grid);
    switch (b.words_per_lane) {
        case 8:
            hipLaunchKernelGGL(k_batch<8 * kBT>, dim3(b.grid), dim3(kBT), 0, stream, b.jobs, b.njobs,
                               b.ranges, b.next, b.counters);
            break;
        case 32:
            hipLaunchKernelGGL(k_batch<32 * kBT>, dim3(b.grid), dim3(kBT), 0, stream, b.jobs, b.njobs,
                               b.ranges, b.next, b.counters);
            break;
        default:
            hipLaunchKernelGGL(k_batch<16 * kBT>, dim3(b.grid), dim3(kBT), 0, stream, b.jobs, b.njobs,
                               b.ranges, b.next, b.counters);
            break;
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MAG_OK : hip_fail(e, "batch scan launch");
}

mag_status launch_batch_offsets(const uint64_t *sorted, const uint64_t *zp, uint64_t cap,
                                uint64_t *d_offsets, uint32_t njobs, int job_shift,
                                hipStream_t stream) {
    const uint32_t threads = 256;
    const uint32_t blocks = (njobs + 1 + threads - 1) / threads;
    hipLaunchKernelGGL(k_batch_offsets, dim3(blocks), dim3(threads), 0, stream, sorted, zp, cap,
                       d_offsets, njobs, job_shift);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MAG_OK : hip_fail(e, "batch offsets launch");
}

namespace {

constexpr int kBatchVerifyThreads = 256;

// The deferred starts of batched jobs (entry = job << kBatchJobShift |
// start), spread over the buffer's segments like the single-job
// verification kernel. Each lane reads its own job's verification
// arguments; all jobs share the batch's counters, key buffer and capacity,
// so the wave's collective output reservation still applies.
__global__ __launch_bounds__(kBatchVerifyThreads) void k_batch_verify(const JobDesc *jobs,
                                                                      const uint64_t *pending,
                                                                      const uint64_t *seg_count,
                                                                      uint64_t seg_cap) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t wave = ((uint64_t)blockIdx.x * kBatchVerifyThreads + threadIdx.x) >> 6;
    const uint64_t waves = ((uint64_t)gridDim.x * kBatchVerifyThreads) >> 6;
    const uint64_t per = waves >= kPendingSegments ? waves / kPendingSegments : 1;
    const uint64_t posmask = (1ull << kBatchJobShift) - 1ull;
    for (uint64_t w = wave; w < per * kPendingSegments; w += waves) {
        const uint32_t seg = (uint32_t)(w % kPendingSegments);
        const uint64_t sub = w / kPendingSegments;
        const uint64_t count = seg_count[seg];
        const uint64_t total = count < seg_cap ? count : seg_cap;
        const uint64_t *src = pending + (uint64_t)seg * seg_cap;
        for (uint64_t c = sub * 64; c < total; c += per * 64) {
            const uint64_t i = c + lane;
            const bool active = i < total;
            const uint64_t e = active ? src[i] : 0ull;
            VerifyArgs v;
            __builtin_memcpy(&v, &jobs[(uint32_t)(e >> kBatchJobShift)].v, sizeof(v));
            verify_wave(v, e & posmask, active);
        }
    }
}

}  // namespace

mag_status launch_batch_verify(const JobDesc *jobs, const uint64_t *pending, const uint64_t *seg_count,
                               uint64_t seg_cap, hipStream_t stream) {
    static uint32_t grid = 0;
    if (!grid) {
        const int ncu = device_compute_units();
        const int occ = cached_occupancy((const void *)k_batch_verify, kBatchVerifyThreads, 0);
        if (ncu < 1 || occ < 1) return fail(MAG_E_DEVICE, "cannot size the batch verification");
        grid = (uint32_t)(ncu * occ);
    }
    hipLaunchKernelGGL(k_batch_verify, dim3(grid), dim3(kBatchVerifyThreads), 0, stream, jobs, pending,
                       seg_count, seg_cap);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? MAG_OK : hip_fail(e, "batch verification launch");
}

}  // namespace mag
