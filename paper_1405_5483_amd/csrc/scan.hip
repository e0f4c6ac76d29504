// MAG scan kernel for gfx950: the sampled Shift-Or filter over superimposed
// q-gram classes (Sections 3.1-3.2) with fused exact verification.
//
// Sample x is the text q-gram at byte x*k*q; its code is the Horner value of
// the mapped bytes (Section 3.2, "Implementation") and B[code] is its Shift-Or
// mask. Window (x, j) is a candidate when bit (m'-1)k + j of
// D_x = (D_{x-1} << k) | B[g_x] is 0; it stands for the q start positions
// i0 = (x-m'+1)kq - jq - s (s < q). Each start position maps to exactly one
// (x, j, s), so every position is verified at most once.
//
// A workgroup owns tiles of TS consecutive samples. Its waves have two roles,
// working one tile apart on two LDS buffers of mask entries E:
//  - producer waves take consecutive samples (coalesced 32-bit buffer loads of
//    the q bytes, range-checked so any text alignment works; the next rounds'
//    words are prefetched), map the bytes through mu, look the code up in the
//    mask table (LDS when it fits, else global/L2) and store the entry in E;
//    no sample depends on another, so every lookup can be in flight;
//  - consumer lanes run the Shift-Or recurrence over a contiguous run of S
//    entries of the previous tile's E, after the W0 entries before it (warm-up:
//    only the last m' entries reach the candidate bits, so each window is
//    evaluated by exactly one lane). E is read 16 bytes at a time and a wave
//    leaves the register-only fast path only when one of its lanes has a
//    candidate (ballot); it then queues the start positions of the candidate
//    windows in LDS with a ballot + mbcnt prefix.
// One barrier per tile separates the rounds. Full queues (64 starts) are
// verified one start per lane by an out-of-line function: the window's bytes
// are read from the text (L2), the hash of its first 16 bytes probes an
// open-addressing table of the distinct patterns, a fingerprint hit is
// confirmed by a full word compare, and every id of the matching pattern is
// emitted as a 64-bit key (pos << idbits | id).
//
// The gram length Q is a compile-time parameter: this file is compiled once per
// Q (MAG_SCAN_Q) and scan_dispatch.cpp picks the object.
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "mag_internal.hpp"
#include "scan_args.hpp"
#include "scan_common.hpp"

#ifndef MAG_SCAN_Q
#error "compile with -DMAG_SCAN_Q=<1..8>"
#endif

namespace mag {
namespace {

constexpr int Q = MAG_SCAN_Q;
constexpr int kNT = kScanThreads;
constexpr int kProducerWaves = kScanProducerWaves;
constexpr int kConsumerWaves = kNT / 64 - kScanProducerWaves;
constexpr int kProducerThreads = kProducerWaves * 64;
constexpr int kQueue = 128;          // per-wave queue of start positions (64-bit)
using namespace dev;

#ifndef MAG_SCAN_GROUP
#define MAG_SCAN_GROUP 4
#endif
constexpr int kGroup = MAG_SCAN_GROUP;
#ifndef MAG_SCAN_PREFETCH
#define MAG_SCAN_PREFETCH 2
#endif
constexpr int kPrefetch = MAG_SCAN_PREFETCH;   // rounds of loads in flight in phase A

template <int G>
__device__ __forceinline__ void load_group(GramWords (&w)[G], __amdgpu_buffer_rsrc_t rs, int32_t p0,
                                           int s, uint32_t kq) {
#pragma unroll
    for (int u = 0; u < G; ++u) w[u] = gram_words<Q>(rs, (uint32_t)(p0 + (s + u) * (int32_t)kq));
}

template <bool INTERIOR, bool MUL24, bool TLDS, int G, typename ET>
__device__ __forceinline__ void process_group(const GramWords (&w)[G], ET *s_E, int s, int W0,
                                              uint32_t sp, const uint8_t *s_mu, const ET *s_tab,
                                              const ET *g_tab, int64_t X0, uint64_t X) {
    const ET none = (ET)~(ET)0;
    uint32_t g[G];
#pragma unroll
    for (int u = 0; u < G; ++u) g[u] = gram_code<Q, MUL24>(w[u], s_mu, sp);
    ET e[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
        e[u] = TLDS ? s_tab[g[u]] : g_tab[g[u]];
        if (!INTERIOR) {
            const int64_t x = X0 + s + u;
            if (x < 0 || x >= (int64_t)X) e[u] = none;
        }
    }
#pragma unroll
    for (int u = 0; u < G; u += 4) store4(s_E + (s + W0 + u), e + u);
}

template <bool INTERIOR, bool MUL24, bool TLDS, typename ET>
__device__ __forceinline__ void phase_a(ET *s_E, __amdgpu_buffer_rsrc_t rs, int32_t p0, uint32_t kq,
                                        uint32_t sp, const uint8_t *s_mu, const ET *s_tab,
                                        const ET *g_tab, int W0, uint32_t TS, int64_t X0, uint64_t X,
                                        int tid) {
    constexpr int G = kGroup;
    const int step = G * kProducerThreads;
    int s = G * tid - W0;
    if (kPrefetch >= 2) {
        // two rounds in flight while a third is processed
        GramWords b0[G], b1[G];
        load_group<G>(b0, rs, p0, s, kq);
        load_group<G>(b1, rs, p0, s + step, kq);
        for (;;) {
            if (s >= (int)TS) break;
            process_group<INTERIOR, MUL24, TLDS, G>(b0, s_E, s, W0, sp, s_mu, s_tab, g_tab, X0, X);
            load_group<G>(b0, rs, p0, s + 2 * step, kq);
            s += step;
            if (s >= (int)TS) break;
            process_group<INTERIOR, MUL24, TLDS, G>(b1, s_E, s, W0, sp, s_mu, s_tab, g_tab, X0, X);
            load_group<G>(b1, rs, p0, s + 2 * step, kq);
            s += step;
        }
    } else {
        GramWords cur[G];
        load_group<G>(cur, rs, p0, s, kq);
        for (; s < (int)TS; s += step) {
            GramWords nxt[G];
            load_group<G>(nxt, rs, p0, s + step, kq);
            process_group<INTERIOR, MUL24, TLDS, G>(cur, s_E, s, W0, sp, s_mu, s_tab, g_tab, X0, X);
#pragma unroll
            for (int u = 0; u < G; ++u) cur[u] = nxt[u];
        }
    }
}

template <typename ET, typename DT, bool TLDS, bool MUL24>
__global__ __launch_bounds__(kNT) void k_scan(ScanArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    constexpr int EPV = 16 / (int)sizeof(ET);            // entries per 16-byte LDS read
    uint8_t *s_mu = smem;
    uint64_t *s_queue = reinterpret_cast<uint64_t *>(smem + 256);
    ET *s_E0 = reinterpret_cast<ET *>(smem + 256 + kConsumerWaves * kQueue * 8);
    ET *s_E1 = reinterpret_cast<ET *>(smem + 256 + kConsumerWaves * kQueue * 8 + a.e_lds);
    ET *s_tab = reinterpret_cast<ET *>(smem + 256 + kConsumerWaves * kQueue * 8 + 2 * a.e_lds);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const bool producer = wave < kProducerWaves;
    // the kernel's only argument is `a`, at the start of the argument segment
    const VerifyArgs *vargs = (const VerifyArgs *)((const __attribute__((address_space(4))) char *)
                                                       __builtin_amdgcn_kernarg_segment_ptr() +
                                                   offsetof(ScanArgs, v));
    for (int i = tid; i < 256; i += kNT) s_mu[i] = a.mu[i];
    if (TLDS) {
        const uint4 *src = reinterpret_cast<const uint4 *>(a.table);
        uint4 *dst = reinterpret_cast<uint4 *>(s_tab);
        for (uint32_t v = tid; v < a.table_vec; v += kNT) dst[v] = src[v];
    }
    const ET *g_tab = reinterpret_cast<const ET *>(a.table);
    // every wave stages part of the map and the table; producers read all of it
    __syncthreads();

    // consumer state
    const int ct = tid - kProducerThreads;                // consumer lane index
    uint64_t *queue = s_queue + (producer ? 0 : (wave - kProducerWaves)) * kQueue;
    uint32_t qn = 0;
    uint64_t ncand = 0, nver = 0;
    const uint32_t kmask = a.k >= 32 ? 0xFFFFFFFFu : ((1u << a.k) - 1u);
    const uint32_t topshift = a.W - a.k;
    // sigma' <= 256: the mask tells the compiler so, and Horner keeps 24-bit multiply-adds
    const uint32_t sp = a.sp & 0x1FFu, k = a.k, kq = a.kq, S = a.S, TS = a.tile_samples;
    const int W0 = (int)a.w0;                             // warm-up entries kept before a tile
    const int64_t last = (int64_t)a.n - (int64_t)a.m;   // last valid start position

    // Producer waves fill E for this workgroup's it-th tile while consumer
    // waves run the Shift-Or over the (it-1)-th, in alternating buffers; one
    // barrier per round.
    const uint64_t nlocal = a.ntiles > blockIdx.x ? (a.ntiles - 1 - blockIdx.x) / gridDim.x + 1 : 0;
    for (uint64_t it = 0; it <= nlocal; ++it) {
        if (producer) {
            if (it < nlocal) {
                const int64_t X0 = (int64_t)(blockIdx.x + it * gridDim.x) * TS;
                // text bytes the tile's samples touch, warm-up included
                int64_t b0 = (X0 - (int64_t)W0) * kq;
                if (b0 < 0) b0 = 0;
                int64_t b1 = (X0 + (int64_t)TS) * kq + kMaxQ;
                if (b1 > (int64_t)a.n) b1 = (int64_t)a.n;
                if (b1 < b0) b1 = b0;
                const uint64_t pa0 = (a.delta + (uint64_t)b0) & ~15ull;
                const uint64_t pa1 = (a.delta + (uint64_t)b1 + 15) & ~15ull;
                const __amdgpu_buffer_rsrc_t rs = tile_rsrc(a.tbase + pa0, (uint32_t)(pa1 - pa0));
                const int64_t pbase = (int64_t)a.delta - (int64_t)pa0;
                const bool interior = X0 - W0 >= 0 && X0 + (int64_t)TS <= (int64_t)a.X;
                const int32_t p0 = (int32_t)(pbase + X0 * (int64_t)kq);   // resource offset of sample X0
                ET *E = (it & 1) ? s_E1 : s_E0;
                if (interior)
                    phase_a<true, MUL24, TLDS>(E, rs, p0, kq, sp, s_mu, s_tab, g_tab, W0, TS, X0, a.X, tid);
                else
                    phase_a<false, MUL24, TLDS>(E, rs, p0, kq, sp, s_mu, s_tab, g_tab, W0, TS, X0, a.X, tid);
            }
        } else if (it >= 1) {
            // Shift-Or over the lane's S samples. The W0 entries before them
            // warm the state up (only the last m' entries reach the candidate
            // bits, so the extra older ones are harmless).
            const int64_t X0 = (int64_t)(blockIdx.x + (it - 1) * gridDim.x) * TS;
            const ET *E = ((it - 1) & 1) ? s_E1 : s_E0;
            const uint4 *vE = reinterpret_cast<const uint4 *>(E) + (uint32_t)ct * (S / EPV);
            DT D = ~(DT)0;
            for (int v = 0; v < W0 / EPV; ++v) {
                const uint4 raw = vE[v];
                ET ent[EPV];
                __builtin_memcpy(ent, &raw, 16);
#pragma unroll
                for (int u = 0; u < EPV; ++u) D = (D << k) | (DT)ent[u];
            }
            vE += W0 / EPV;
            for (uint32_t v = 0; v < S / EPV; ++v) {
                const uint4 raw = vE[v];
                ET ent[EPV];
                __builtin_memcpy(ent, &raw, 16);
                const DT Dstart = D;
                DT all = ~(DT)0;     // a 0 in a candidate bit of the AND: some entry fired
#pragma unroll
                for (int u = 0; u < EPV; ++u) {
                    D = (D << k) | (DT)ent[u];
                    all &= D;
                }
                const uint32_t anyc = (uint32_t)((~all) >> topshift) & kmask;
                if (!__ballot(anyc != 0)) continue;
                // slow path: replay the vector once to mark which entries
                // fired, then visit only those: recompute the state there and
                // queue the start positions of each candidate window
                uint32_t fired = 0;
                {
                    DT R = Dstart;
#pragma unroll
                    for (int u = 0; u < EPV; ++u) {
                        R = (R << k) | (DT)ent[u];
                        fired |= ((((uint32_t)((~R) >> topshift)) & kmask) != 0u ? 1u : 0u) << u;
                    }
                }
                const int64_t xv = X0 + (int64_t)((uint32_t)ct * S + v * EPV);
                for (;;) {
                    const bool hasu = fired != 0;
                    if (!__ballot(hasu)) break;
                    const int u = hasu ? __builtin_ctz(fired) : 0;
                    if (hasu) fired &= fired - 1u;
                    DT R = Dstart;
                    for (int t = 0; t <= u; ++t) R = (R << k) | (DT)entry_at<ET>(raw, t);
                    uint32_t c = hasu ? ((uint32_t)((~R) >> topshift) & kmask) : 0u;
                    const int64_t topx = (xv + u - (int64_t)a.mprime + 1) * (int64_t)kq;
                    for (;;) {
                        const bool has = c != 0;
                        const uint64_t hb = __ballot(has);
                        if (!hb) break;
                        ncand += (uint64_t)__popcll(hb);
                        const uint32_t bit = has ? __builtin_ctz(c) : 0u;
                        if (has) c &= c - 1u;
                        const int64_t top = topx - (int64_t)bit * Q;
#pragma unroll
                        for (int sft = 0; sft < Q; ++sft) {
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
                                drain64(vargs, queue, qn, lane);
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    if (!producer) {
        // starts still queued
        if (qn) drain_partial(vargs, queue, qn, lane);
        if (lane == 0 && ncand)
            atomicAdd((unsigned long long *)&a.counters[1], (unsigned long long)ncand);
        unsigned long long nv = nver;
        for (int off = 32; off > 0; off >>= 1) nv += __shfl_xor(nv, off);
        if (lane == 0 && nv) atomicAdd((unsigned long long *)&a.counters[2], nv);
    }
}

template <typename ET, typename DT, bool TLDS, bool MUL24>
mag_status launch_one(const ScanArgs &a, size_t shmem, int ncu, hipStream_t stream) {
    auto fn = k_scan<ET, DT, TLDS, MUL24>;
    static int configured_bytes = 0;    // per instantiation
    if ((int)shmem > configured_bytes) {
        // not every runtime needs the opt-in; a real LDS overflow fails the launch below
        (void)hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)shmem);
        (void)hipGetLastError();
        configured_bytes = (int)shmem;
    }
    int occ = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, kNT, shmem);
    if (e != hipSuccess) return hip_fail(e, "occupancy query (scan)");
    if (occ < 1) return fail(MAG_E_UNSUPPORTED, "scan kernel does not fit on a compute unit");
    uint64_t grid = (uint64_t)ncu * (uint64_t)occ;
    if (grid > a.ntiles) grid = a.ntiles;
    if (grid == 0) return MAG_OK;
    hipLaunchKernelGGL(fn, dim3((uint32_t)grid), dim3(kNT), shmem, stream, a);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "scan launch");
    return MAG_OK;
}

template <typename ET, typename DT>
mag_status launch_et(const ScanArgs &a, bool tlds, bool mul24, size_t shmem, int ncu,
                     hipStream_t stream) {
    if (tlds) return launch_one<ET, DT, true, true>(a, shmem, ncu, stream);   // LDS tables are small
    return mul24 ? launch_one<ET, DT, false, true>(a, shmem, ncu, stream)
                 : launch_one<ET, DT, false, false>(a, shmem, ncu, stream);
}

}  // namespace

#define MAG_CAT2(a, b) a##b
#define MAG_CAT(a, b) MAG_CAT2(a, b)

mag_status MAG_CAT(launch_scan_q, MAG_SCAN_Q)(const ScanArgs &a, int esz, bool wide, bool tlds,
                                             bool mul24, size_t shmem, int ncu, hipStream_t stream) {
    switch (esz) {
        case 1: return launch_et<uint8_t, uint32_t>(a, tlds, mul24, shmem, ncu, stream);
        case 2: return launch_et<uint16_t, uint32_t>(a, tlds, mul24, shmem, ncu, stream);
        case 4:
            if (wide) return launch_et<uint32_t, uint64_t>(a, tlds, mul24, shmem, ncu, stream);
            return launch_et<uint32_t, uint32_t>(a, tlds, mul24, shmem, ncu, stream);
        default: return launch_et<uint64_t, uint64_t>(a, tlds, mul24, shmem, ncu, stream);
    }
}

}  // namespace mag
