// Batched MAG scans: many independent (text, pattern set) jobs in one
// persistent launch.
//
// Every filter job is cut into tiles of 1024 * words-per-lane samples; the
// tiles of all filter jobs form one global sequence (job after job) that the
// host splits into contiguous ranges of about equal text bytes, one per
// workgroup, so a workgroup restages a job's alphabet map and mask table in
// LDS only when its range crosses into the next job. Dense jobs run in their
// own persistent launch (k_batch_dense, below) with the single-job dense
// kernels' tiles and bitmaps. Per tile the kernel runs the two phases of
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

// TS: samples per filter tile (1024 * words per lane).
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

    __shared__ uint64_t s_found[kWaves * kFoundBuf];      // the waves' found-key buffers

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint64_t *queue = s_queue + wave * kBatchQueue;
    uint64_t *fbuf = s_found + wave * kFoundBuf;
    uint32_t qn = 0, fbn = 0;
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

    for (uint32_t slot = 0;; slot ^= 1) {
        const uint64_t g = uni64(s_ctl[slot]);
        if (g == kNoTile) break;
        // wave 0 asks for the next tile now and settles the claim after phase A
        unsigned long long pending = 0;
        if (wave == 0 && !own_done && lane == 0)
            pending = atomicAdd((unsigned long long *)&next[me], 1ull);
        if (cur < 0 || g < tfirst || g >= tend) {
            if (cur >= 0 && qn) {
                fbn = drain_partial_found(vp, queue, qn, lane, fbuf, fbn);   // starts of the previous job
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
        const int64_t X0 = (int64_t)(g - tfirst) * TS;
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
                            fbn = drain64_found(vp, queue, qn, lane, fbuf, fbn);
                        }
                    }
                }
            }
        }
    }
    if (cur >= 0 && qn) fbn = drain_partial_found(vp, queue, qn, lane, fbuf, fbn);
    unsigned long long nv = nver;
    for (int off = 32; off > 0; off >>= 1) nv += __shfl_xor(nv, off);
    __shared__ uint64_t s_wg[3 * (kBT / 64)];
    workgroup_out<kBT / 64>(vp, fbuf, fbn, ncand, nv, counters, s_wg);
}

// ---- dense jobs ----
//
// One 1024-thread workgroup per compute unit, as in the single-job dense
// kernels: the job's bitmap (the slice bitmap of the one-probe mode, or the
// Bloom bitmap, up to 128 KiB) in a static LDS array at address 0, per-wave
// queues and found-key buffers after it. Tiles are those of the single-job
// kernels (kBatchSliceTile or kDenseScanTile start positions); workgroups
// claim them from contiguous ranges of the dense tile sequence and steal as
// the filter launch does, and restage the bitmap when the job changes. When
// a job's bitmap leaves at least half of its array free, the free part holds
// the waves' found-key buffers (up to 1,024 keys each instead of
// kFoundBuf): jobs with short DNA patterns find a match at several percent
// of their start positions, and one output reservation per kFoundBuf keys
// would serialize them on the output counter.
constexpr int kDT = kDenseScanThreads;
constexpr int kDQueue = 128;
static_assert(kDQueue >= (int)kDenseQueue, "dense_test fills up to kDenseQueue starts");
constexpr uint32_t kDBitsWords = 1u << (kBloomMaxLog2 - 5);

// A claimed dense tile is the job's `chunk` consecutive sub-tiles of the
// single-job kernels' size; a wave tests one sub-tile while the loads of the
// next are in flight (the loads are unconditional, clamped to the last
// sub-tile, so that the wait before a sub-tile counts the same loads on every
// path), and the workgroup meets at a barrier once per claimed tile.

// The slice sub-tiles x0 + s kBatchSliceTile, s < nsub, of one claimed tile:
// lane L < 63 of wave w owns the 16 start positions from 16 (63 w + L) of
// each. rs covers the tile's bytes from a 16-byte boundary and p0 is the
// resource offset of x0; loads past the resource read zeros, which only
// positions past `last` see.
template <int K>
__device__ __forceinline__ void slice_chunk(__amdgpu_buffer_rsrc_t rs, uint32_t p0, int64_t x0, int nsub,
                                            int64_t last, const uint32_t *s_bits, uint32_t bshift,
                                            uint64_t *queue, uint32_t &qn, const VerifyArgs *vp, int lane,
                                            int wave, uint32_t &nhit, uint64_t *fbuf, uint32_t &fbn,
                                            uint32_t fbcap) {
    constexpr int P = kBatchSliceLane;
    constexpr int kLW = SliceLane<P>::load_words(false);
    static_assert(kLW == 7, "one 16-byte and one 12-byte load per lane");
    const uint32_t lane_off = (uint32_t)(P * (kSliceOwners * wave + lane));
    auto load = [&](int sub, uint32_t (&W)[kLW]) {
        const int at = (int)((p0 & ~3u) + (uint32_t)sub * kBatchSliceTile + lane_off);
        const uint4 x = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, at, 0, 0));
        const auto y = __builtin_amdgcn_raw_buffer_load_b96(rs, at + 16, 0, 0);
        W[0] = x.x; W[1] = x.y; W[2] = x.z; W[3] = x.w;
        W[4] = y[0]; W[5] = y[1]; W[6] = y[2];
    };
    auto test = [&](int sub, const uint32_t (&W)[kLW]) {
        const int64_t xb = x0 + (int64_t)sub * kBatchSliceTile + lane_off;
        slice_test<K, P, false>(W, p0 & 3u, xb, last - xb + 1, s_bits, bshift, queue, qn, vp, lane, nhit, fbuf,
                                fbn, fbcap);
    };
    uint32_t Wa[kLW], Wb[kLW];
    load(0, Wa);
    for (int sub = 0; sub < nsub; sub += 2) {
        load(sub + 1 < nsub ? sub + 1 : nsub - 1, Wb);
        test(sub, Wa);
        if (sub + 1 >= nsub) break;
        load(sub + 2 < nsub ? sub + 2 : nsub - 1, Wa);
        test(sub + 1, Wb);
    }
}

// Emits the occurrences of the queued starts of a job with exact codes:
// entry = start | code << 48. code_ids[code] is the pattern id | kCodeDirect
// when the code's distinct pattern has one id (one load per start), else the
// distinct pattern's index + 1, whose ids the id runs give. All 64 lanes call
// it; lanes at or past `count` hold no entry.
constexpr int kCodeShift = 48;
__device__ static __attribute__((noinline)) uint32_t drain_codes(const VerifyArgs *v, const uint64_t *queue,
                                                                uint32_t from, uint32_t count,
                                                                const uint32_t *code_ids, uint64_t *fbuf,
                                                                uint32_t fbn, uint32_t fcap) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const uint32_t lane = __lane_id();
    const bool active = lane < count;
    const uint64_t e = active ? queue[from + lane] : 0ull;
    __builtin_amdgcn_wave_barrier();
    const uint32_t ent = active ? code_ids[e >> kCodeShift] : 0u;
    VerifyArgs args;
    __builtin_memcpy(&args, v, sizeof(args));
    const bool direct = (ent & kCodeDirect) != 0;
    uint32_t b = ent & ~kCodeDirect, c = direct ? 1u : 0u;
    if (!direct && ent) {
        b = args.idstart[ent - 1];
        c = args.idstart[ent] - b;
    }
    return emit_runs_buffered(args, e & ((1ull << kCodeShift) - 1), c,
                              [&](uint32_t t) { return direct ? b : args.ids[b + t]; }, fbuf, fbn, fcap);
}

// The 16 start positions xb .. xb + 15 of one lane in a job with exact codes
// (W: the 40 bytes from the word holding xb, d = xb's byte offset in it).
// Each byte's code is (b >> shift) & 3; four bytes' codes are packed into one
// byte and the lane's 24 bytes into 48 bits, so a window's code is one funnel
// shift and a mask, and one LDS bit test decides it. A byte is a pattern byte
// iff the code's byte (a byte permute of rep) equals it; a window holding
// another byte is dropped (the lanes of a wave check this only when one of
// them holds such a byte). Passing starts are queued with their codes and
// emitted 64 at a time.
__device__ __forceinline__ void code_test(const uint32_t (&W)[10], uint32_t d, int64_t xb, int64_t last,
                                          const uint32_t *s_bits, uint32_t shift, uint32_t rep,
                                          uint32_t cmask, uint32_t m, uint64_t *queue, uint32_t &qn,
                                          const VerifyArgs *vp, const uint32_t *code_ids, int lane,
                                          uint64_t &nhit, uint64_t *fbuf, uint32_t &fbn, uint32_t fcap) {
    uint32_t V[6], x[6], q[6];
    uint32_t bad = 0;
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        V[t] = __builtin_amdgcn_alignbyte(W[t + 1], W[t], d);
        const uint32_t T = (V[t] >> shift) & 0x03030303u;
        x[t] = __builtin_amdgcn_perm(rep, rep, T) ^ V[t];    // nonzero bytes: not pattern bytes
        bad |= x[t];
        const uint32_t pp = T | (T >> 6);
        q[t] = pp | (pp >> 12);                             // the 4 codes in bits 0..7
    }
    const uint32_t lo16 = __builtin_amdgcn_perm(q[1], q[0], 0x0C0C0400u);
    const uint32_t hi16 = __builtin_amdgcn_perm(q[3], q[2], 0x0C0C0400u);
    const uint32_t Slo = __builtin_amdgcn_perm(hi16, lo16, 0x05040100u);   // codes of bytes 0..15
    const uint32_t Shi = __builtin_amdgcn_perm(q[5], q[4], 0x0C0C0400u);   // bytes 16..23
    // the 16 bitmap words are read before any is used, so that the reads
    // overlap (one at a time, each waits out the LDS latency)
    uint32_t code[16], word[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) code[u] = (u ? __builtin_amdgcn_alignbit(Shi, Slo, 2u * u) : Slo) & cmask;
#pragma unroll
    for (int u = 0; u < 16; ++u) word[u] = s_bits[code[u] >> 5];
    __builtin_amdgcn_sched_barrier(0);
    uint32_t hm = 0;
#pragma unroll
    for (int u = 0; u < 16; ++u) hm |= __builtin_amdgcn_ubfe(word[u], code[u], 1u) << u;
    if (__ballot(bad != 0) && bad) {
        // byte k of the lane is not a pattern byte: drop the windows holding it
        uint32_t badk = 0;
#pragma unroll
        for (int k = 0; k < 23; ++k)
            badk |= (((x[k >> 2] >> (8 * (k & 3))) & 0xFFu) != 0u ? 1u : 0u) << k;
        const uint32_t wmask = (1u << m) - 1u;
#pragma unroll
        for (int u = 0; u < 16; ++u)
            if ((badk >> u) & wmask) hm &= ~(1u << u);
    }
    const int64_t room = last - xb + 1;
    if (room < 16) hm &= room <= 0 ? 0u : ((1u << (uint32_t)room) - 1u);
    nhit += (uint32_t)__popc(hm);
    while (__ballot(hm != 0)) {
        const bool act = hm != 0;
        const uint32_t u = act ? (uint32_t)__builtin_ctz(hm) : 0u;
        hm &= hm - 1u;
        const uint64_t bal = __ballot(act);
        if (act) {
            const uint32_t code = __builtin_amdgcn_alignbit(Shi, Slo, 2u * u) & cmask;
            queue[qn + lanes_below(bal)] = (uint64_t)(xb + u) | ((uint64_t)code << kCodeShift);
        }
        qn += (uint32_t)__popcll(bal);
        if (qn >= 64) {
            qn -= 64;
            fbn = drain_codes(vp, queue, qn, 64, code_ids, fbuf, fbn, fcap);
        }
    }
}

__global__ __launch_bounds__(kDT, 4) void k_batch_dense(const JobDesc *__restrict__ jobs, uint32_t njobs,
                                                     const uint64_t *__restrict__ ranges, uint64_t *next,
                                                     uint64_t *counters) {
    __shared__ __align__(16) uint32_t s_bits[kDBitsWords];
    __shared__ uint64_t s_queue[(kDT / 64) * kDQueue];
    __shared__ uint64_t s_found[(kDT / 64) * kFoundBuf];
    __shared__ uint64_t s_ctl[2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint64_t *queue = s_queue + wave * kDQueue;
    uint64_t *fbuf = s_found + wave * kFoundBuf;
    uint32_t fcap = kFoundBuf;
    uint32_t qn = 0, fbn = 0, nslice = 0;
    uint64_t nbloom = 0;
    const uint32_t me = blockIdx.x, G = gridDim.x;
    const uint64_t own_end = uni64(ranges[3 * me + 1]);
    bool own_done = false;
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

    int cur = -1;
    const VerifyArgs *vp = nullptr;
    const uint8_t *tbase = nullptr;
    uint64_t delta = 0, n = 0, tfirst = 0, tend = 0;
    uint32_t m = 1, slice_k = 0, bshift = 32, hw = 1, mw = 1, lastmask = 0, tile = kDenseScanTile, chunk = 1;
    uint32_t code_shift = 0, code_rep = 0, code_mask = 0;
    const uint32_t *code_ids = nullptr;
    for (uint32_t slot = 0;; slot ^= 1) {
        const uint64_t g = uni64(s_ctl[slot]);
        if (g == kNoTile) break;
        unsigned long long pending = 0;
        if (wave == 0 && !own_done && lane == 0)
            pending = atomicAdd((unsigned long long *)&next[me], 1ull);
        if (cur < 0 || g < tfirst || g >= tend) {
            if (cur >= 0 && qn) {                // the previous job's starts
                if (code_mask) fbn = drain_codes(vp, queue, 0, qn, code_ids, fbuf, fbn, fcap);
                else fbn = drain_partial_found(vp, queue, qn, lane, fbuf, fbn, fcap);
                qn = 0;
            }
            if (fbn) {                      // the buffer may lie where the next bitmap goes
                flush_found_args(vp, fbuf, fbn);
                fbn = 0;
            }
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
            tfirst = uni64(J.tile_first);
            tend = tfirst + uni64(J.ntiles);
            m = uni32(J.v.m);
            slice_k = uni32(J.slice_k);
            bshift = uni32(J.bshift);
            hw = uni32(J.v.hw);
            mw = uni32(J.v.mw);
            lastmask = uni32(J.v.lastmask);
            code_shift = uni32(J.code_shift);
            code_rep = uni32(J.code_rep);
            code_mask = uni32(J.code_mask);
            code_ids = uniptr(J.code_ids);
            tile = slice_k ? (uint32_t)kBatchSliceTile : (uint32_t)kDenseScanTile;   // one sub-tile
            chunk = uni32(J.chunk);
            const uint32_t tvec = uni32(J.table_vec);
            const uint4 *src = reinterpret_cast<const uint4 *>(uniptr(J.table));
            const uint32_t spare = (kDBitsWords * 4u - tvec * 16u) / (8u * (kDT / 64));   // keys per wave
            if (spare >= kDBitsWords * 4u / 2u / (8u * (kDT / 64))) {
                fcap = spare < 1024u ? spare : 1024u;
                fbuf = reinterpret_cast<uint64_t *>(reinterpret_cast<uint8_t *>(s_bits) + tvec * 16u) +
                       (uint32_t)wave * fcap;
            } else {
                fcap = kFoundBuf;
                fbuf = s_found + wave * kFoundBuf;
            }
            __syncthreads();                // the previous tile is done with the bitmap
            uint4 *dst = reinterpret_cast<uint4 *>(s_bits);
            for (uint32_t v = tid; v < tvec; v += kDT) dst[v] = src[v];
        }
        const int64_t X0 = (int64_t)(g - tfirst) * tile * chunk;
        const int64_t last = (int64_t)n - (int64_t)m;
        // sub-tiles holding start positions up to `last`
        const int64_t left = last - X0 + 1;
        const int nsub = left >= (int64_t)tile * chunk ? (int)chunk : (int)((left + tile - 1) / tile);
        int64_t e1 = X0 + (int64_t)tile * chunk + 48;    // bytes the tile's windows and probes touch
        if (e1 > (int64_t)n) e1 = (int64_t)n;
        const uint64_t da0 = (delta + (uint64_t)X0) & ~15ull;
        const uint64_t da1 = (delta + (uint64_t)e1 + 15) & ~15ull;
        const __amdgpu_buffer_rsrc_t drs = tile_rsrc(tbase + da0, (uint32_t)(da1 - da0));
        const uint32_t p0 = (uint32_t)(delta + (uint64_t)X0 - da0);
        const uint32_t nrec = (uint32_t)(da1 - da0);
        __syncthreads();                    // the bitmap is staged
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
        // every tile holds a start position (tiles = ceil(positions / tile size))
        if (slice_k) {
            switch (slice_k) {
                case 1: slice_chunk<1>(drs, p0, X0, nsub, last, s_bits, bshift, queue, qn, vp, lane, wave, nslice, fbuf, fbn, fcap); break;
                case 2: slice_chunk<2>(drs, p0, X0, nsub, last, s_bits, bshift, queue, qn, vp, lane, wave, nslice, fbuf, fbn, fcap); break;
                case 3: slice_chunk<3>(drs, p0, X0, nsub, last, s_bits, bshift, queue, qn, vp, lane, wave, nslice, fbuf, fbn, fcap); break;
                case 4: slice_chunk<4>(drs, p0, X0, nsub, last, s_bits, bshift, queue, qn, vp, lane, wave, nslice, fbuf, fbn, fcap); break;
                case 5: slice_chunk<5>(drs, p0, X0, nsub, last, s_bits, bshift, queue, qn, vp, lane, wave, nslice, fbuf, fbn, fcap); break;
                case 6: slice_chunk<6>(drs, p0, X0, nsub, last, s_bits, bshift, queue, qn, vp, lane, wave, nslice, fbuf, fbn, fcap); break;
                case 7: slice_chunk<7>(drs, p0, X0, nsub, last, s_bits, bshift, queue, qn, vp, lane, wave, nslice, fbuf, fbn, fcap); break;
                default: slice_chunk<8>(drs, p0, X0, nsub, last, s_bits, bshift, queue, qn, vp, lane, wave, nslice, fbuf, fbn, fcap); break;
            }
        } else {
            // Bloom or exact-code sub-tiles: 16 positions per thread
            const bool codes = code_mask != 0;
            auto test = [&](int sub, const uint32_t (&W)[10]) {
                const int64_t xb = X0 + (int64_t)sub * tile + 16 * (int64_t)tid;
                if (codes)
                    code_test(W, p0 & 3u, xb, last, s_bits, code_shift, code_rep, code_mask, m, queue, qn, vp,
                              code_ids, lane, nbloom, fbuf, fbn, fcap);
                else
                    dense_test_any(W, p0 & 3u, xb, last, s_bits, bshift, hw, mw, lastmask, queue, qn, vp, lane,
                                   nbloom, FoundBuf{fbuf, &fbn, fcap});
            };
            uint32_t Wa[10], Wb[10];
            dense_load<kDT>(drs, nrec, p0, tid, Wa);
            for (int sub = 0; sub < nsub; sub += 2) {
                dense_load<kDT>(drs, nrec, p0 + (uint32_t)(sub + 1 < nsub ? sub + 1 : nsub - 1) * tile, tid, Wb);
                test(sub, Wa);
                if (sub + 1 >= nsub) break;
                dense_load<kDT>(drs, nrec, p0 + (uint32_t)(sub + 2 < nsub ? sub + 2 : nsub - 1) * tile, tid, Wa);
                test(sub + 1, Wb);
            }
        }
        __syncthreads();                    // s_ctl for the next tile
    }
    if (cur >= 0 && qn) {
        if (code_mask) fbn = drain_codes(vp, queue, 0, qn, code_ids, fbuf, fbn, fcap);
        else fbn = drain_partial_found(vp, queue, qn, lane, fbuf, fbn, fcap);
    }
    unsigned long long nh = nbloom + nslice;
    for (int off = 32; off > 0; off >>= 1) nh += __shfl_xor(nh, off);
    __shared__ uint64_t s_wg[3 * (kDT / 64)];
    workgroup_out<kDT / 64>(vp, fbuf, fbn, nh, nh, counters, s_wg);
}

// Claim counters back to the first tile of each workgroup's range.
__global__ void k_batch_init(const uint64_t *ranges, uint64_t *next, uint32_t G) {
    const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w < G) next[w] = ranges[3 * w];
}

// offsets[j] = first record of job j (binary search of the sorted keys on the
// job field), offsets[njobs] = the count. One thread per entry.
__global__ void k_batch_offsets(const uint64_t *sorted, const uint64_t *zp, uint64_t cap,
                                uint64_t *offsets, uint32_t njobs, const uint64_t *jbase, int idbits) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > njobs) return;
    const uint64_t z = *zp;
    uint64_t at = 0;
    if (j == njobs) {
        at = z;
    } else if (z <= cap) {
        const uint64_t first = jbase[j] << idbits;    // the job's smallest key
        uint64_t lo = 0, hi = z;
        while (lo < hi) {
            const uint64_t mid = lo + (hi - lo) / 2;
            if (sorted[mid] < first) lo = mid + 1;
            else hi = mid;
        }
        at = lo;
    }
    offsets[j] = at;
}

// The records the finishing kernel wrote (outputs of at most small_max keys;
// larger ones are made relative in k_expand): each position less its job's
// first byte in the batch's texts (see k_expand).
__global__ __launch_bounds__(256) void k_batch_rebase(mag_match *out, const uint64_t *zp, uint64_t cap,
                                                      uint64_t small_max, const uint64_t *jbase,
                                                      uint32_t njobs) {
    const uint64_t z = *zp;
    if (z > cap || z > small_max) return;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < z; i += stride)
        out[i].pos -= jbase[job_of_position(jbase, njobs, out[i].pos)];
}

}  // namespace

mag_status batch_configure() { return MAG_OK; }   // the kernel's LDS is static

namespace {
const void *batch_kernel(int words_per_lane) {
    switch (words_per_lane) {
        case 8: return (const void *)k_batch<8 * kBT>;
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
        default:
            hipLaunchKernelGGL(k_batch<16 * kBT>, dim3(b.grid), dim3(kBT), 0, stream, b.jobs, b.njobs,
                               b.ranges, b.next, b.counters);
            break;
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MAG_OK : hip_fail(e, "batch scan launch");
}

int batch_dense_occupancy() {
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)k_batch_dense, kDT, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return occ;
}

mag_status launch_batch_dense(const BatchLaunch &b, hipStream_t stream) {
    if (!b.total_tiles || !b.grid) return MAG_OK;
    hipLaunchKernelGGL(k_batch_init, dim3((b.grid + 255) / 256), dim3(256), 0, stream, b.ranges,
                       b.next, b.grid);
    hipLaunchKernelGGL(k_batch_dense, dim3(b.grid), dim3(kDT), 0, stream, b.jobs, b.njobs, b.ranges, b.next,
                       b.counters);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MAG_OK : hip_fail(e, "batch dense scan launch");
}

mag_status launch_batch_offsets(const uint64_t *sorted, const uint64_t *zp, uint64_t cap,
                                uint64_t *d_offsets, uint32_t njobs, const uint64_t *jbase, int idbits,
                                mag_match *out, hipStream_t stream) {
    const uint32_t threads = 256;
    const uint32_t blocks = (njobs + 1 + threads - 1) / threads;
    hipLaunchKernelGGL(k_batch_offsets, dim3(blocks), dim3(threads), 0, stream, sorted, zp, cap,
                       d_offsets, njobs, jbase, idbits);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "batch offsets launch");
    if (!out || !cap || !njobs) return MAG_OK;
    const uint64_t small = small_sort_max();
    const uint64_t most = std::min<uint64_t>(cap, small);
    const uint32_t rblocks = (uint32_t)std::min<uint64_t>((most + threads - 1) / threads, 1024);
    hipLaunchKernelGGL(k_batch_rebase, dim3(rblocks), dim3(threads), 0, stream, out, zp, cap, small, jbase,
                       njobs);
    e = hipGetLastError();
    return e == hipSuccess ? MAG_OK : hip_fail(e, "batch rebase launch");
}

namespace {

constexpr int kBatchVerifyThreads = 256;
constexpr uint32_t kVerifyFound = 256;   // found keys buffered per wave

// The deferred starts of batched jobs (entry = job << kBatchJobShift |
// start), spread over the buffer's segments like the single-job
// verification kernel. Each lane reads its own job's verification
// arguments; all jobs share the batch's counters, key buffer and capacity,
// so the wave's collective output reservation still applies. Found keys
// collect in a per-wave LDS buffer (rounds with a lane of an unequal-length
// job emit directly).
__global__ __launch_bounds__(kBatchVerifyThreads) void k_batch_verify(const JobDesc *jobs,
                                                                      const uint64_t *pending,
                                                                      const uint64_t *seg_count,
                                                                      uint64_t seg_cap) {
    __shared__ uint64_t s_found[(kBatchVerifyThreads / 64) * kVerifyFound];
    __shared__ uint64_t s_wg[3 * (kBatchVerifyThreads / 64)];
    uint64_t *fbuf = s_found + (threadIdx.x >> 6) * kVerifyFound;
    uint32_t fbn = 0;
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
            const uint64_t i0 = e & posmask;
            if (__ballot(active && v.var) == 0)
                fbn = emit_found_buffered(v, i0, active ? find_pattern(v, i0) : 0u, fbuf, fbn, kVerifyFound);
            else
                verify_wave(v, i0, active);
        }
    }
    workgroup_out<kBatchVerifyThreads / 64>(&jobs[0].v, fbuf, fbn, 0, 0, nullptr, s_wg);
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
