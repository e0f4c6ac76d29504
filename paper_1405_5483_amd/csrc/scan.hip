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
//    words are prefetched), turn the bytes into the gram's code (Horner over
//    mu, the bit fields of the bit-field map, or the hash of the alphabet
//    mapping on q-grams), look the code up in the mask table (LDS when it
//    fits, else global/L2; whole or packed 1/2/4-bit entries) and store the
//    entry in E;
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
static_assert(MAG_SCAN_PREFETCH >= 1, "at least one round of loads in flight");
constexpr int kPrefetch = MAG_SCAN_PREFETCH;   // rounds of loads in flight in phase A
#ifndef MAG_SCAN_VEC
#define MAG_SCAN_VEC 1
#endif
// Words per sample when consecutive samples sit in consecutive words (stride
// = 4 * kWordsPerSample bytes, word-aligned): a thread's group of samples is
// then read with 16-byte loads.
constexpr int kWordsPerSample = (Q + 3) / 4;

// How phase A turns a gram into its code: Horner with 24-bit multiply-adds,
// Horner with 32-bit ones, the bit-field map's field extraction, the hash of
// the alphabet mapping on q-grams (blen = log2 sigma'), or (SMAG) a code the
// encoding kernel already wrote, 16 or 32 bits wide.
constexpr int kCodeMul24 = 0, kCodeMul32 = 1, kCodeBits = 2, kCodeHash = 3;
constexpr int kCodePre16 = 4, kCodePre32 = 5;
constexpr int kCodeNibbles = 6;   // bit-field map with 4-bit fields, Q <= 4
constexpr bool is_pre(int code) { return code == kCodePre16 || code == kCodePre32; }

// ALIGNED: the words come from the 16-byte-load path, gram at w0's first byte.
template <int CODE, bool ALIGNED = false>
__device__ __forceinline__ uint32_t code_of(const GramWords &w, const uint8_t *s_mu, uint32_t sp,
                                            uint32_t bshift, uint32_t blen) {
    if constexpr (CODE == kCodeBits) return gram_code_bits<Q, ALIGNED>(w, bshift, blen);
    else if constexpr (CODE == kCodeNibbles) return gram_code_nibbles<(Q <= 4 ? Q : 4), ALIGNED>(w, bshift);
    else if constexpr (CODE == kCodeHash) return gram_code_hash<Q, ALIGNED>(w, blen);
    // encoded codes arrive through a resource that may extend into the
    // buffer's unwritten tail (samples past the last one read it before their
    // entry is discarded): clamp to the largest valid code, carried in sp
    else if constexpr (CODE == kCodePre16) return min((w.w0 >> (8u * w.sh)) & 0xFFFFu, sp);
    else if constexpr (CODE == kCodePre32) return min(w.w0, sp);
    else return gram_code<Q, CODE == kCodeMul24, ALIGNED>(w, s_mu, sp);
}

// Source words of G consecutive samples, the first at resource offset o and
// the others `stride` bytes apart: the text words of each q-gram, or the
// word holding each encoded code.
template <int CODE, int G, bool VEC>
__device__ __forceinline__ void load_group(GramWords (&w)[G], __amdgpu_buffer_rsrc_t rs, uint32_t o,
                                           uint32_t stride) {
    if constexpr (VEC) {
        // G samples in G * kWordsPerSample consecutive words starting at the
        // word-aligned offset o: one 16-byte load per 4 words
        static_assert(G % 4 == 0, "whole 16-byte loads");
        uint32_t words[G * kWordsPerSample];
#pragma unroll
        for (int v = 0; v < G * kWordsPerSample / 4; ++v) {
            const auto x = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(o + 16u * v), 0, 0);
            words[4 * v] = x[0];
            words[4 * v + 1] = x[1];
            words[4 * v + 2] = x[2];
            words[4 * v + 3] = x[3];
        }
#pragma unroll
        for (int u = 0; u < G; ++u) {
            w[u].w0 = words[u * kWordsPerSample];
            w[u].w1 = kWordsPerSample > 1 ? words[u * kWordsPerSample + 1] : 0u;
            w[u].w2 = 0u;
            w[u].sh = 0u;
        }
        return;
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
        const uint32_t at = o + (uint32_t)u * stride;
        if constexpr (is_pre(CODE)) {
            w[u].w0 = ld32(rs, at & ~3u);
            w[u].sh = at & 3u;
            w[u].w1 = w[u].w2 = 0u;
        } else {
            w[u] = gram_words<Q>(rs, at);
        }
    }
}

template <bool INTERIOR, int CODE, bool TLDS, int PB, bool VEC, int G, typename ET>
__device__ __forceinline__ void process_group(const GramWords (&w)[G], ET *s_E, int s, int W0,
                                              uint32_t sp, uint32_t bshift, uint32_t blen,
                                              const uint8_t *s_mu, const ET *s_tab, const ET *g_tab,
                                              int64_t X0, uint64_t X) {
    const ET none = (ET)~(ET)0;
    uint32_t g[G];
#pragma unroll
    for (int u = 0; u < G; ++u) g[u] = code_of<CODE, VEC>(w[u], s_mu, sp, bshift, blen);
    ET e[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
        e[u] = table_entry<PB>(TLDS ? s_tab : g_tab, g[u]);
        if (!INTERIOR) {
            const int64_t x = X0 + s + u;
            if (x < 0 || x >= (int64_t)X) e[u] = none;
        }
    }
#pragma unroll
    for (int u = 0; u < G; u += 4) store4(s_E + (s + W0 + u), e + u);
}

template <bool INTERIOR, int CODE, bool TLDS, int PB, bool VEC, typename ET>
__device__ __forceinline__ void phase_a(ET *s_E, __amdgpu_buffer_rsrc_t rs, int32_t p0, uint32_t kq /* source stride */,
                                        uint32_t sp, uint32_t bshift, uint32_t blen,
                                        const uint8_t *s_mu, const ET *s_tab,
                                        const ET *g_tab, int W0, uint32_t TS, int64_t X0, uint64_t X,
                                        int tid) {
    constexpr int G = kGroup;
    constexpr int P = kPrefetch;
    const int step = G * kProducerThreads;
    int s = G * tid - W0;
    // P rounds of words in flight: round r is processed while rounds r+1 ..
    // r+P-1 load, and its buffer is refilled with round r+P at once. The
    // thread's round count is known up front, so the steady-state loop has
    // no exit between rounds (an exit there lets the compiler sink a refill
    // past the next round's wait). Refills past the last round read outside
    // the tile's resource (zeros) and are never processed. Offsets advance by
    // adds (one multiply per tile).
    const int nr = s < (int)TS ? ((int)TS - s + step - 1) / step : 0;
    const uint32_t ostep = (uint32_t)step * kq;
    uint32_t o = (uint32_t)(p0 + s * (int32_t)kq);
    GramWords buf[P][G];
#pragma unroll
    for (int r = 0; r < P; ++r) load_group<CODE, G, VEC>(buf[r], rs, o + (uint32_t)r * ostep, kq);
    o += (uint32_t)P * ostep;
    int r0 = 0;
    for (; r0 + P <= nr; r0 += P) {
#pragma unroll
        for (int r = 0; r < P; ++r) {
            process_group<INTERIOR, CODE, TLDS, PB, VEC, G>(buf[r], s_E, s, W0, sp, bshift, blen, s_mu, s_tab,
                                                  g_tab, X0, X);
            load_group<CODE, G, VEC>(buf[r], rs, o, kq);
            o += ostep;
            s += step;
            // keep the refill here: hoisting the next round's work above it
            // would wait for every outstanding load before reissuing any
            __builtin_amdgcn_sched_barrier(0);
        }
    }
#pragma unroll
    for (int r = 0; r < P - 1; ++r) {
        if (r0 + r >= nr) return;
        process_group<INTERIOR, CODE, TLDS, PB, VEC, G>(buf[r], s_E, s, W0, sp, bshift, blen, s_mu, s_tab,
                                              g_tab, X0, X);
        s += step;
    }
}

template <typename ET, typename DT, bool TLDS, int CODE, int PB>
__global__ __launch_bounds__(kNT) void k_scan(ScanArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    constexpr int EPV = 16 / (int)sizeof(ET);            // entries per 16-byte LDS read
    uint8_t *s_mu = smem;
    uint64_t *s_queue = reinterpret_cast<uint64_t *>(smem + 256);
    ET *s_E0 = reinterpret_cast<ET *>(smem + 256 + kConsumerWaves * kQueue * 8);
    ET *s_E1 = reinterpret_cast<ET *>(smem + 256 + kConsumerWaves * kQueue * 8 + a.e_lds);
    ET *s_tab = reinterpret_cast<ET *>(smem + 256 + kConsumerWaves * kQueue * 8 + 2 * a.e_lds);

    // the consumer waves' found-key buffers
    __shared__ uint64_t s_found[kConsumerWaves * kFoundBuf];
    static_assert(sizeof(s_found) <= kScanStaticLds, "static LDS beside the dynamic part");

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
    uint64_t *fbuf = s_found + (producer ? 0 : (wave - kProducerWaves)) * kFoundBuf;
    uint32_t qn = 0, fbn = 0;
    uint64_t ncand = 0, nver = 0;
    const uint32_t kmask = a.k >= 32 ? 0xFFFFFFFFu : ((1u << a.k) - 1u);
    const uint32_t topshift = a.W - a.k;
    // sigma' <= 256: the mask tells the compiler so, and Horner keeps 24-bit multiply-adds
    // sigma' (Horner codes, <= 256), or the largest valid code (encoded codes)
    const uint32_t sp = is_pre(CODE) ? a.maxcode : (a.sp & 0x1FFu);
    const uint32_t k = a.k, kq = a.kq, S = a.S, TS = a.tile_samples;
    const uint32_t stride = a.stride;                     // source bytes from one sample to the next
    const uint32_t bshift = a.bshift & 7u;                // bit-field map (CODE == kCodeBits)
    const uint32_t blen = a.blen & 31u;                   // field width, or log2 sigma' (kCodeHash)
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
                int64_t b0 = (X0 - (int64_t)W0) * stride;
                if (b0 < 0) b0 = 0;
                int64_t b1 = (X0 + (int64_t)TS) * stride + kMaxQ;
                if (b1 > (int64_t)a.src_bytes) b1 = (int64_t)a.src_bytes;
                if (b1 < b0) b1 = b0;
                const uint64_t pa0 = (a.delta + (uint64_t)b0) & ~15ull;
                const uint64_t pa1 = (a.delta + (uint64_t)b1 + 15) & ~15ull;
                const __amdgpu_buffer_rsrc_t rs = tile_rsrc(a.tbase + pa0, (uint32_t)(pa1 - pa0));
                const int64_t pbase = (int64_t)a.delta - (int64_t)pa0;
                const bool interior = X0 - W0 >= 0 && X0 + (int64_t)TS <= (int64_t)a.X;
                const int32_t p0 = (int32_t)(pbase + X0 * (int64_t)stride);   // resource offset of sample X0
                ET *E = (it & 1) ? s_E1 : s_E0;
                // consecutive samples in consecutive words: 16-byte loads
                const bool vec = MAG_SCAN_VEC && !is_pre(CODE) &&
                                 stride == 4u * kWordsPerSample && (p0 & 3) == 0;
                if (interior) {
                    if (vec)
                        phase_a<true, CODE, TLDS, PB, true>(E, rs, p0, stride, sp, bshift, blen, s_mu, s_tab, g_tab, W0, TS, X0, a.X, tid);
                    else
                        phase_a<true, CODE, TLDS, PB, false>(E, rs, p0, stride, sp, bshift, blen, s_mu, s_tab, g_tab, W0, TS, X0, a.X, tid);
                } else {
                    phase_a<false, CODE, TLDS, PB, false>(E, rs, p0, stride, sp, bshift, blen, s_mu, s_tab, g_tab, W0, TS, X0, a.X, tid);
                }
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
                                fbn = drain64_found(vargs, queue, qn, lane, fbuf, fbn);
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    unsigned long long nv = 0;
    if (!producer) {
        // starts still queued
        if (qn) fbn = drain_partial_found(vargs, queue, qn, lane, fbuf, fbn);
        nv = nver;
        for (int off = 32; off > 0; off >>= 1) nv += __shfl_xor(nv, off);
    }
    // the entry buffers (at least 4 KiB) are free after the last round's barrier
    workgroup_out<kNT / 64>(vargs, fbuf, producer ? 0u : fbn, producer ? 0ull : ncand, nv, a.counters,
                            reinterpret_cast<uint64_t *>(s_E0));
}

template <typename ET, typename DT, bool TLDS, int CODE, int PB = 0>
mag_status launch_one(const ScanArgs &a, size_t shmem, int ncu, hipStream_t stream) {
    auto fn = k_scan<ET, DT, TLDS, CODE, PB>;
    static int configured_bytes = 0;    // per instantiation
    if ((int)shmem > configured_bytes) {
        // not every runtime needs the opt-in; a real LDS overflow fails the launch below
        (void)hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)shmem);
        (void)hipGetLastError();
        configured_bytes = (int)shmem;
    }
    const int occ = cached_occupancy((const void *)fn, kNT, shmem);
    if (occ < 1) return fail(MAG_E_UNSUPPORTED, "scan kernel does not fit on a compute unit");
    uint64_t grid = (uint64_t)ncu * (uint64_t)occ;
    if (grid > a.ntiles) grid = a.ntiles;
    if (grid == 0) return MAG_OK;
    hipLaunchKernelGGL(fn, dim3((uint32_t)grid), dim3(kNT), shmem, stream, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "scan launch");
    return MAG_OK;
}

// Chooses the table form: packed 1/2/4-bit entries (1-byte entry types
// only) or whole entries, staged in LDS or read from global memory.
template <typename ET, typename DT, int CODE>
mag_status launch_tables(const ScanArgs &a, bool tlds, size_t shmem, int ncu, hipStream_t stream) {
    if constexpr (sizeof(ET) == 1) {
        if (a.pbits == 1)
            return tlds ? launch_one<ET, DT, true, CODE, 1>(a, shmem, ncu, stream)
                        : launch_one<ET, DT, false, CODE, 1>(a, shmem, ncu, stream);
        if (a.pbits == 2)
            return tlds ? launch_one<ET, DT, true, CODE, 2>(a, shmem, ncu, stream)
                        : launch_one<ET, DT, false, CODE, 2>(a, shmem, ncu, stream);
        if (a.pbits == 4)
            return tlds ? launch_one<ET, DT, true, CODE, 4>(a, shmem, ncu, stream)
                        : launch_one<ET, DT, false, CODE, 4>(a, shmem, ncu, stream);
    }
    if (a.pbits) return fail(MAG_E_UNSUPPORTED, "packed mask entries need W <= 4");
    return tlds ? launch_one<ET, DT, true, CODE, 0>(a, shmem, ncu, stream)
                : launch_one<ET, DT, false, CODE, 0>(a, shmem, ncu, stream);
}

template <typename ET, typename DT>
mag_status launch_et(const ScanArgs &a, bool tlds, bool mul24, size_t shmem, int ncu,
                     hipStream_t stream) {
    if (a.pre == 2) return launch_tables<ET, DT, kCodePre16>(a, tlds, shmem, ncu, stream);
    if (a.pre == 4) return launch_tables<ET, DT, kCodePre32>(a, tlds, shmem, ncu, stream);
    if (a.qgram) return launch_tables<ET, DT, kCodeHash>(a, tlds, shmem, ncu, stream);
    if (tlds) {   // LDS tables are small: 24-bit Horner steps always suffice
        if (Q <= 4 && a.blen == 4) return launch_one<ET, DT, true, kCodeNibbles>(a, shmem, ncu, stream);
        return a.blen ? launch_one<ET, DT, true, kCodeBits>(a, shmem, ncu, stream)
                      : launch_one<ET, DT, true, kCodeMul24>(a, shmem, ncu, stream);
    }
    return mul24 ? launch_one<ET, DT, false, kCodeMul24>(a, shmem, ncu, stream)
                 : launch_one<ET, DT, false, kCodeMul32>(a, shmem, ncu, stream);
}

// SMAG's encoding pass (Section 3.2, "Implementation"): the code of every
// complete non-overlapping q-gram T[yQ .. yQ+Q), written as CT. A block takes
// kEncodeThreads * kEncodePerThread consecutive grams per step; thread t
// writes grams t, t + kEncodeThreads, ... of the step, so stores coalesce.
constexpr int kEncodeThreads = 256, kEncodePerThread = 4;

template <int CODE, typename CT>
__global__ __launch_bounds__(kEncodeThreads) void k_encode(EncodeArgs e) {
    __shared__ uint8_t s_mu[256];
    for (int i = threadIdx.x; i < 256; i += kEncodeThreads) s_mu[i] = e.mu[i];
    __syncthreads();
    constexpr uint64_t kBlockGrams = (uint64_t)kEncodeThreads * kEncodePerThread;
    const uint32_t sp = e.sp & 0x1FFu, bshift = e.bshift & 7u, blen = e.blen & 31u;
    CT *out = reinterpret_cast<CT *>(e.codes);
    for (uint64_t y0 = (uint64_t)blockIdx.x * kBlockGrams; y0 < e.G; y0 += (uint64_t)gridDim.x * kBlockGrams) {
        // the step's text bytes (and the word after the last gram); loads
        // past the resource read zeros and belong to no complete gram
        const uint64_t b0 = y0 * Q;
        uint64_t b1 = (y0 + kBlockGrams) * Q + 8;
        if (b1 > e.n) b1 = e.n;
        const uint64_t pa0 = (e.delta + b0) & ~15ull;
        const uint64_t pa1 = (e.delta + b1 + 15) & ~15ull;
        const __amdgpu_buffer_rsrc_t rs = tile_rsrc(e.tbase + pa0, (uint32_t)(pa1 - pa0));
        const uint32_t pbase = (uint32_t)(e.delta + b0 - pa0);
#pragma unroll
        for (int u = 0; u < kEncodePerThread; ++u) {
            const uint64_t y = y0 + (uint64_t)u * kEncodeThreads + threadIdx.x;
            if (y < e.G) {
                const GramWords w = gram_words<Q>(rs, pbase + (uint32_t)((y - y0) * Q));
                out[y] = (CT)code_of<CODE>(w, s_mu, sp, bshift, blen);
            }
        }
    }
}

template <int CODE>
mag_status launch_encode_code(const EncodeArgs &e, int csz, hipStream_t stream) {
    const uint64_t steps = (e.G + kEncodeThreads * kEncodePerThread - 1) / (kEncodeThreads * kEncodePerThread);
    const uint32_t grid = (uint32_t)(steps < (1u << 20) ? steps : (1u << 20));
    if (csz == 2) hipLaunchKernelGGL((k_encode<CODE, uint16_t>), dim3(grid), dim3(kEncodeThreads), 0, stream, e);
    else hipLaunchKernelGGL((k_encode<CODE, uint32_t>), dim3(grid), dim3(kEncodeThreads), 0, stream, e);
    const hipError_t err = hipGetLastError();
    return err == hipSuccess ? MAG_OK : hip_fail(err, "encode launch");
}

}  // namespace

#define MAG_CAT2(a, b) a##b
#define MAG_CAT(a, b) MAG_CAT2(a, b)

mag_status MAG_CAT(launch_encode_q, MAG_SCAN_Q)(const EncodeArgs &e, int csz, bool mul24,
                                               hipStream_t stream) {
    if (e.G == 0) return MAG_OK;
    if (e.qgram) return launch_encode_code<kCodeHash>(e, csz, stream);
    if (e.blen) return launch_encode_code<kCodeBits>(e, csz, stream);
    return mul24 ? launch_encode_code<kCodeMul24>(e, csz, stream)
                 : launch_encode_code<kCodeMul32>(e, csz, stream);
}

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
