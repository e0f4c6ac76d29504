// Device helpers shared by the single-job scan kernel and the batched kernel:
// range-checked text loads, q-gram codes, mask-entry packing and the
// out-of-line exact verification of start positions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mag_internal.hpp"
#include "verify.hpp"

namespace mag {
namespace dev {

constexpr uint32_t kBufferWord3 = 0x00020000u;   // raw 32-bit buffer resource (gfx9)

__device__ __forceinline__ uint32_t ld32(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, 0);
}

// The 32-bit words holding the q bytes of the gram that starts at resource
// offset p (the third word only for q > 4).
struct GramWords {
    uint32_t w0, w1, w2, sh;
};

template <int Q>
__device__ __forceinline__ GramWords gram_words(__amdgpu_buffer_rsrc_t rs, uint32_t p) {
    GramWords g;
    const uint32_t a = p & ~3u;
    g.sh = p & 3;
    g.w0 = ld32(rs, a);
    g.w1 = ld32(rs, a + 4);
    g.w2 = Q > 4 ? ld32(rs, a + 8) : 0u;
    return g;
}

// Code of a q-gram: Horner over the mapped bytes, last byte first. With MUL24
// every partial value is below 2^24 (the host checks sigma'^(q-1) < 2^24), so
// the full-rate 24-bit multiply-add is exact.
template <int Q, bool MUL24, bool ALIGNED = false>
__device__ __forceinline__ uint32_t gram_code(const GramWords &gw, const uint8_t *s_mu, uint32_t sp) {
    // ALIGNED: the gram starts at w0's first byte (w1 holds bytes 4..7)
    const uint32_t lo = ALIGNED ? gw.w0 : __builtin_amdgcn_alignbyte(gw.w1, gw.w0, gw.sh);
    const uint32_t hi = Q <= 4 ? 0u : ALIGNED ? gw.w1 : __builtin_amdgcn_alignbyte(gw.w2, gw.w1, gw.sh);
    uint32_t g = 0;
#pragma unroll
    for (int t = Q - 1; t >= 0; --t) {
        const uint32_t byte = t < 4 ? __builtin_amdgcn_ubfe(lo, 8 * t, 8)
                                    : __builtin_amdgcn_ubfe(hi, 8 * (t - 4), 8);
        const uint32_t c = s_mu[byte];
        if (t == Q - 1) g = c;
        else if (MUL24) g = __umul24(g, sp) + c;
        else g = g * sp + c;
    }
    return g;
}

// Code of a q-gram under the bit-field map of Section 3.3: the l bits from
// bit `shift` of every byte, S[0]'s field lowest. Equal to gram_code with
// mu(c) = (c >> shift) & (2^l - 1), without the map table.
template <int Q, bool ALIGNED = false>
__device__ __forceinline__ uint32_t gram_code_bits(const GramWords &gw, uint32_t shift, uint32_t l) {
    const uint32_t lo = ALIGNED ? gw.w0 : __builtin_amdgcn_alignbyte(gw.w1, gw.w0, gw.sh);
    const uint32_t hi = Q <= 4 ? 0u : ALIGNED ? gw.w1 : __builtin_amdgcn_alignbyte(gw.w2, gw.w1, gw.sh);
    uint32_t g = 0;
#pragma unroll
    for (int t = 0; t < Q; ++t) {
        const uint32_t field = t < 4 ? __builtin_amdgcn_ubfe(lo, 8 * t + shift, l)
                                     : __builtin_amdgcn_ubfe(hi, 8 * (t - 4) + shift, l);
        g |= field << (l * t);
    }
    return g;
}

// gram_code_bits for 4-bit fields (sigma' = 16) and Q <= 4: mask the gram's
// nibbles in place, fold each pair of bytes into one (f0 | f1 << 4 and
// f2 | f3 << 4; the rotate's wrapped bits land in byte 3, which is not
// gathered), and gather bytes 0 and 2.
template <int Q, bool ALIGNED = false>
__device__ __forceinline__ uint32_t gram_code_nibbles(const GramWords &gw, uint32_t shift) {
    static_assert(Q >= 1 && Q <= 4, "one word per gram");
    const uint32_t lo = ALIGNED ? gw.w0 : __builtin_amdgcn_alignbyte(gw.w1, gw.w0, gw.sh);
    constexpr uint32_t m = Q == 4 ? 0x0F0F0F0Fu : Q == 3 ? 0x000F0F0Fu : Q == 2 ? 0x00000F0Fu : 0x0Fu;
    const uint32_t x = (lo >> shift) & m;
    const uint32_t y = x | __builtin_amdgcn_alignbit(x, x, 4);
    return __builtin_amdgcn_perm(0u, y, 0x0C0C0200u);
}

// Code of a q-gram under the alphabet mapping on q-grams (Section 3.3): the
// top hbits (<= 28) bits of MurmurHash3's 64-bit finalizer of the gram's raw
// bytes (S[0] in the low byte). The finalizer's last xor-shift leaves the high
// word alone, so only the high word of the second product is formed.
template <int Q, bool ALIGNED = false>
__device__ __forceinline__ uint32_t gram_code_hash(const GramWords &gw, uint32_t hbits) {
    uint32_t lo = ALIGNED ? gw.w0 : __builtin_amdgcn_alignbyte(gw.w1, gw.w0, gw.sh);
    uint32_t hi = Q <= 4 ? 0u : ALIGNED ? gw.w1 : __builtin_amdgcn_alignbyte(gw.w2, gw.w1, gw.sh);
    if (Q < 4) lo &= (1u << (8 * Q)) - 1u;
    if (Q > 4 && Q < 8) hi &= (1u << (8 * (Q - 4))) - 1u;
    lo ^= hi >> 1;                                                     // x ^= x >> 33
    const uint64_t x = (((uint64_t)hi << 32) | lo) * 0xFF51AFD7ED558CCDull;
    const uint32_t xh = (uint32_t)(x >> 32);
    const uint32_t xl = (uint32_t)x ^ (xh >> 1);                       // x ^= x >> 33
    constexpr uint32_t c2lo = 0x1A85EC53u, c2hi = 0xC4CEB9FEu;
    const uint32_t top = __umulhi(xl, c2lo) + xl * c2hi + xh * c2lo;   // high word of x * C2
    return hbits ? top >> (32u - hbits) : 0u;
}

// Entry g of a mask table: whole entries of type ET, or (PB = 1, 2, 4) PB-bit
// entries packed little-endian into 32-bit words, returned with the bits
// above PB set (they are past W).
template <int PB, typename ET>
__device__ __forceinline__ ET table_entry(const ET *tab, uint32_t g) {
    if constexpr (PB == 0) {
        return tab[g];
    } else {
        constexpr uint32_t kPer = 32 / PB;
        const uint32_t word = reinterpret_cast<const uint32_t *>(tab)[g / kPer];
        return (ET)(((word >> ((g % kPer) * PB)) & ((1u << PB) - 1u)) | (0xFFu << PB));
    }
}

// Raw buffer resource over [base, base + bytes). The operands are wave-uniform;
// readfirstlane says so to the compiler, which otherwise may keep them in
// vector registers and wrap every load in a loop over distinct values.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(const uint8_t *base, uint32_t bytes) {
    const uint64_t b = reinterpret_cast<uint64_t>(base);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    const uint32_t n = __builtin_amdgcn_readfirstlane(bytes);
    void *p = reinterpret_cast<void *>(((uint64_t)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, (int)n, (int)kBufferWord3);
}

// Out-of-line verification of the start positions of a wave, one per lane
// (lanes with active false only take part in the wave's output reservation;
// every lane must call it). `v` points at the verification arguments in
// memory (the scan kernel passes their place in its kernel-argument segment,
// the batched kernel its job table), so they are read on this cold path and
// occupy no registers in the scan loops. With a pending buffer the starts are
// appended to it (one atomic per wave) for the verification kernel; lanes
// whose slot falls past its capacity verify here instead.
__device__ static __attribute__((noinline)) void verify_one(const VerifyArgs *v, uint64_t i0,
                                                            bool active) {
    VerifyArgs args;
    __builtin_memcpy(&args, v, sizeof(args));
    if (args.pending) {
        const uint64_t mask = __ballot(active);
        if (!mask) return;
        const uint32_t cnt = (uint32_t)__popcll(mask);
        const uint32_t lane = __lane_id();
        const uint32_t first = (uint32_t)__builtin_ctzll(__ballot(true));
        // one counter per segment keeps the atomics apart and spreads a small
        // grid's starts over many verifying waves; a multiplicative hash of
        // the wave's number (golden-ratio constant, top bits) uses every
        // segment whichever waves of a workgroup verify
        static_assert(kPendingSegments == 256, "segment = top 8 bits of the hash");
        const uint32_t seg = ((blockIdx.x * 16u + (threadIdx.x >> 6)) * 0x9E3779B1u) >> 24;
        unsigned long long got = 0;
        if (lane == first) got = atomicAdd((unsigned long long *)&args.seg_count[seg], (unsigned long long)cnt);
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)got);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(got >> 32));
        const uint64_t base = ((uint64_t)hi << 32) | lo;
        const uint64_t slot = base + lanes_below(mask);
        const bool stored = active && slot < args.seg_cap;
        if (stored) args.pending[(uint64_t)seg * args.seg_cap + slot] = i0 | args.pending_tag;
        if (base + cnt <= args.seg_cap) return;
        active = active && !stored;
    }
    verify_wave(args, i0, active);
}

// verify_one with the keys of inline verification collected in the wave's
// LDS buffer fbuf (holding fbn keys; see emit_found_buffered); returns the
// new count. Deferred and unequal-length scans take verify_one's path.
// verify_found_inline is the body, for kernels with registers to spare: a
// call makes the callee wait for every load the caller has in flight (its
// prefetched text among them), the inlined body only for its own.
__device__ __forceinline__ uint32_t verify_found_inline(const VerifyArgs *v, uint64_t i0, bool active,
                                                        uint64_t *fbuf, uint32_t fbn, uint32_t cap) {
    VerifyArgs args;
    __builtin_memcpy(&args, v, sizeof(args));
    if (args.pending || args.var) {
        verify_one(v, i0, active);
        return fbn;
    }
    return emit_found_buffered(args, i0, active ? find_pattern(args, i0) : 0u, fbuf, fbn, cap);
}
__device__ static __attribute__((noinline)) uint32_t verify_one_buffered(const VerifyArgs *v, uint64_t i0,
                                                                         bool active, uint64_t *fbuf,
                                                                         uint32_t fbn, uint32_t cap) {
    return verify_found_inline(v, i0, active, fbuf, fbn, cap);
}

__device__ static __attribute__((noinline)) void flush_found_args(const VerifyArgs *v, const uint64_t *fbuf,
                                                                  uint32_t fbn) {
    VerifyArgs args;
    __builtin_memcpy(&args, v, sizeof(args));
    flush_found(args, fbuf, fbn);
}

// The end of a persistent kernel: the found keys left in the waves' LDS
// buffers (fbn in each wave's fbuf; none without buffers) go to the output,
// and the waves' statistics c1, c2 (wave totals) to counters[1] and
// counters[2], with one atomic add per counter for the whole workgroup.
// Atomic adds to one address are serialized across the device, and
// thousands of waves adding at their ends kept the kernels running for tens
// of microseconds after their last tile. v may be null where no wave of the
// workgroup holds a key. Every thread of the workgroup calls it; s_wg holds
// 3 * WAVES words of LDS. Out of line, so that the scan loops' registers do
// not pay for it.
template <int WAVES>
__device__ __attribute__((noinline)) void workgroup_out(const VerifyArgs *v, const uint64_t *fbuf,
                                                        uint32_t fbn, uint64_t c1, uint64_t c2,
                                                        uint64_t *counters, uint64_t *s_wg) {
    static_assert(WAVES <= 64, "one lane per wave");
    const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6;
    if (lane == 0) {
        s_wg[wave] = fbn;
        s_wg[WAVES + wave] = c1;
        s_wg[2 * WAVES + wave] = c2;
    }
    __syncthreads();
    if (wave == 0) {
        const bool in = lane < (uint32_t)WAVES;
        const uint64_t n = in ? s_wg[lane] : 0ull;
        uint64_t t1 = in ? s_wg[WAVES + lane] : 0ull, t2 = in ? s_wg[2 * WAVES + lane] : 0ull;
        uint64_t inc = n;                     // inclusive prefix of the waves' key counts
#pragma unroll
        for (int off = 1; off < WAVES; off <<= 1) {
            const uint64_t o = __shfl_up(inc, off);
            if (lane >= (uint32_t)off) inc += o;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            t1 += __shfl_xor(t1, off);
            t2 += __shfl_xor(t2, off);
        }
        const uint64_t total = __shfl(inc, WAVES - 1);
        unsigned long long base = 0;
        if (lane == 0) {
            if (total) base = atomicAdd((unsigned long long *)&v->counters[0], (unsigned long long)total);
            if (t1) atomicAdd((unsigned long long *)&counters[1], (unsigned long long)t1);
            if (t2) atomicAdd((unsigned long long *)&counters[2], (unsigned long long)t2);
        }
        base = __shfl(base, 0);
        if (in) s_wg[lane] = base + inc - n;  // the wave's first output slot
    }
    __syncthreads();
    if (fbn) {
        const uint64_t at = s_wg[wave];
        uint64_t *keys = v->keys;
        const uint64_t cap = v->cap;
        for (uint32_t i = lane; i < fbn; i += 64)
            if (at + i < cap) keys[at + i] = fbuf[i];
    }
}

// Verifies the 64 start positions queue[from .. from+64) of this wave, one per
// lane. The queue is written by other lanes of the same wave.
__device__ __forceinline__ void drain64(const VerifyArgs *v, const uint64_t *queue, uint32_t from,
                                        int lane) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const uint64_t e = queue[from + lane];
    __builtin_amdgcn_wave_barrier();
    verify_one(v, e, true);
}

// drain64 / drain_partial with the wave's found-key buffer (INL: the
// verification inlined, see verify_found_inline).
template <bool INL = false>
__device__ __forceinline__ uint32_t drain64_found(const VerifyArgs *v, const uint64_t *queue, uint32_t from,
                                                  int lane, uint64_t *fbuf, uint32_t fbn,
                                                  uint32_t cap = kFoundBuf) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const uint64_t e = queue[from + lane];
    __builtin_amdgcn_wave_barrier();
    if constexpr (INL) return verify_found_inline(v, e, true, fbuf, fbn, cap);
    else return verify_one_buffered(v, e, true, fbuf, fbn, cap);
}

__device__ __forceinline__ uint32_t drain_partial_found(const VerifyArgs *v, const uint64_t *queue,
                                                        uint32_t qn, int lane, uint64_t *fbuf, uint32_t fbn,
                                                        uint32_t cap = kFoundBuf) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const bool active = (uint32_t)lane < qn;
    const uint64_t e = active ? queue[lane] : 0ull;
    __builtin_amdgcn_wave_barrier();
    return verify_one_buffered(v, e, active, fbuf, fbn, cap);
}

// Verifies the first qn queued starts of this wave (qn < 64).
__device__ __forceinline__ void drain_partial(const VerifyArgs *v, const uint64_t *queue, uint32_t qn,
                                              int lane) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const bool active = (uint32_t)lane < qn;
    const uint64_t e = active ? queue[lane] : 0ull;
    __builtin_amdgcn_wave_barrier();
    verify_one(v, e, active);
}

// Entry t (runtime index) of a 16-byte vector of mask entries.
template <typename ET>
__device__ __forceinline__ ET entry_at(const uint4 &raw, int t) {
    constexpr int per_word = 4 / (int)(sizeof(ET) < 4 ? sizeof(ET) : 4);
    if constexpr (sizeof(ET) == 8) {
        const uint32_t lo = t == 0 ? raw.x : raw.z, hi = t == 0 ? raw.y : raw.w;
        return (ET)(((uint64_t)hi << 32) | lo);
    } else {
        const int w = t / per_word;
        const uint32_t word = w == 0 ? raw.x : w == 1 ? raw.y : w == 2 ? raw.z : raw.w;
        return (ET)(word >> (8 * sizeof(ET) * (t % per_word)));
    }
}

template <typename ET>
__device__ __forceinline__ void store4(ET *dst, const ET e[4]) {
    if constexpr (sizeof(ET) == 1) {
        *reinterpret_cast<uint32_t *>(dst) = (uint32_t)e[0] | ((uint32_t)e[1] << 8) |
                                             ((uint32_t)e[2] << 16) | ((uint32_t)e[3] << 24);
    } else if constexpr (sizeof(ET) == 2) {
        *reinterpret_cast<uint2 *>(dst) = make_uint2((uint32_t)e[0] | ((uint32_t)e[1] << 16),
                                                     (uint32_t)e[2] | ((uint32_t)e[3] << 16));
    } else if constexpr (sizeof(ET) == 4) {
        *reinterpret_cast<uint4 *>(dst) = make_uint4(e[0], e[1], e[2], e[3]);
    } else {
        uint4 *d = reinterpret_cast<uint4 *>(dst);
        d[0] = make_uint4((uint32_t)e[0], (uint32_t)(e[0] >> 32), (uint32_t)e[1], (uint32_t)(e[1] >> 32));
        d[1] = make_uint4((uint32_t)e[2], (uint32_t)(e[2] >> 32), (uint32_t)e[3], (uint32_t)(e[3] >> 32));
    }
}

// Phase A for one tile: mask entries of samples X0-W0 .. X0+TS-1 into
// E[s + W0]. Each thread takes G consecutive samples per round; the words of
// the next round are loaded before the current round's lookups, so global
// latency overlaps LDS work, and each round's entries leave in G/4 LDS
// stores. Outside interior tiles, samples before the text or past the last
// sample get the all-ones (no match) entry. Loads past the tile are
// range-checked by the buffer resource and their entries are never read.

}  // namespace dev
}  // namespace mag
