// Exact verification of one start position (Section 3.2: the filter only
// prunes; every surviving position is checked against the patterns). Used
// inline by the filter kernels and by the verification kernel that drains the
// start positions they defer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mag_internal.hpp"

namespace mag {

struct VerifyArgs {
    const uint8_t *tbase;      // text pointer rounded down to 16 bytes
    uint64_t delta;            // text - tbase
    uint64_t last_word;        // offset from tbase of the last 32-bit word holding text bytes
    uint32_t m, mw, hw, lastmask;
    uint32_t slot_shift, slot_mask, idbits, pad_;
    const uint64_t *slots;     // (hash << 32) | (u + 1), 0 = empty
    const uint32_t *pwords, *idstart, *ids;
    uint64_t *keys;            // output keys key_or + (pos << idbits) | id
    uint64_t cap;
    uint64_t key_or;           // batched scans: the job's first byte in the batch's texts << idbits
    uint64_t *counters;        // [0] = occurrences found
    uint64_t *pending;         // deferred start positions (NULL: verify inline), kPendingSegments
                               // segments of seg_cap entries; wave w of workgroup g appends to
                               // (16 g + w) % segments
    uint64_t *seg_count;       // starts appended to each segment (may exceed seg_cap)
    uint64_t seg_cap;
    uint64_t pending_tag;      // OR'ed into each deferred start (batches: job << 40)
    // patterns of unequal lengths (var = 1): slots lead to groups of distinct
    // patterns that share their first m bytes (m = the shortest length);
    // group g is distinct patterns gstart[g] .. gstart[g+1]-1, pattern u has
    // plen[u] bytes in words pwords[pwoff[u] ..]
    uint64_t n;                // text bytes
    const uint32_t *pwoff, *plen, *gstart;
    uint32_t var, pad2_;
    // word filter in front of the probe slots (NULL: none): words wfilter[h >> wf_shift]
    const uint64_t *wfilter;
    uint32_t wf_shift, pad3_;
};

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// 32-bit text word at physical byte offset `a` (a multiple of 4) from the
// 16-byte-aligned text base; offsets past the last word that holds text bytes
// are clamped to it, so no load leaves the caller's buffer (the clamped
// bytes are never used).
__device__ __forceinline__ uint32_t gword(const VerifyArgs &a, uint64_t off) {
    off = off < a.last_word ? off : a.last_word;
    return *reinterpret_cast<const uint32_t *>(a.tbase + off);
}

#ifndef MAG_CMP_WORDS
#define MAG_CMP_WORDS 4
#endif
constexpr uint32_t kCmpWords = MAG_CMP_WORDS;   // pattern words compared per round trip

// Whether the words words0 .. words0+nw-1 of the window starting at byte
// offset `base` + sh equal pw[0 .. nw) (nw <= kCmpWords; the last word masked by
// lastmask when it is the pattern's last). The chunk's text and pattern words
// are all loaded before any compare, so they arrive in one round trip.
__device__ inline bool words_equal(const VerifyArgs &a, uint64_t base, uint32_t sh, uint32_t words0,
                                   uint32_t nw, const uint32_t *pw, uint32_t lastmask, bool last) {
    uint32_t tw[kCmpWords + 1], pv[kCmpWords];
#pragma unroll
    for (int t = 0; t <= kCmpWords; ++t) tw[t] = (uint32_t)t <= nw ? gword(a, base + 4 * (words0 + t)) : 0u;
#pragma unroll
    for (int t = 0; t < kCmpWords; ++t) pv[t] = (uint32_t)t < nw ? pw[t] : 0u;
    uint32_t diff = 0;
#pragma unroll
    for (int t = 0; t < kCmpWords; ++t) {
        if ((uint32_t)t < nw) {
            uint32_t x = __builtin_amdgcn_alignbyte(tw[t + 1], tw[t], sh);
            if (last && (uint32_t)t == nw - 1) x &= lastmask;
            diff |= x ^ pv[t];
        }
    }
    return diff == 0;
}

// Whether the window at byte offset base + sh equals the nw-word pattern at
// pw (last word masked by lastmask), compared kCmpWords words at a time.
__device__ inline bool window_equal(const VerifyArgs &a, uint64_t base, uint32_t sh, uint32_t nw,
                                    const uint32_t *pw, uint32_t lastmask) {
    for (uint32_t c = 0; c < nw; c += kCmpWords) {
        const uint32_t k = nw - c < kCmpWords ? nw - c : kCmpWords;
        if (!words_equal(a, base, sh, c, k, pw + c, lastmask, c + k == nw)) return false;
    }
    return true;
}

// Index + 1 of the distinct pattern that equals the window at start position
// i0, or 0 if none does. On a fingerprint hit the window's and the pattern's
// words are loaded together before they are compared (kCmpWords words per
// round trip), so a verification waits for a few memory round trips.
__device__ inline uint32_t find_pattern(const VerifyArgs &a, uint64_t i0) {
    const uint64_t p = a.delta + i0;
    const uint64_t base = p & ~3ull;
    const uint32_t sh = (uint32_t)(p & 3);
    uint32_t w[kHashWords + 1];
#pragma unroll
    for (int t = 0; t <= kHashWords; ++t) w[t] = t <= (int)a.hw ? gword(a, base + 4 * t) : 0u;
    uint32_t hv[kHashWords];
#pragma unroll
    for (int t = 0; t < kHashWords; ++t) {
        uint32_t x = 0;
        if (t < (int)a.hw) {
            x = __builtin_amdgcn_alignbyte(w[t + 1], w[t], sh);
            if (t == (int)a.mw - 1) x &= a.lastmask;
        }
        hv[t] = x;
    }
    const uint32_t h = window_hash(hv, (int)a.hw);
    if (a.wfilter) {
        // a hash that fails the word filter is no pattern's: one load decides
        const uint64_t mask = word_filter_mask(h);
        if ((a.wfilter[h >> a.wf_shift] & mask) != mask) return 0;
    }
    uint32_t slot = h >> a.slot_shift;
    for (;;) {
        const uint64_t e = a.slots[slot];
        if (e == 0) return 0;
        if ((uint32_t)(e >> 32) == h) {
            const uint32_t u = (uint32_t)e - 1u;
            if (window_equal(a, base, sh, a.mw, a.pwords + (size_t)u * a.mw, a.lastmask))
                return u + 1;     // distinct patterns: at most one can be equal
        }
        slot = (slot + 1) & a.slot_mask;
    }
}

// Unequal lengths: index + 1 of the group whose shared first m bytes equal
// the window's, or 0.
__device__ inline uint32_t find_group(const VerifyArgs &a, uint64_t i0) {
    const uint64_t p = a.delta + i0;
    const uint64_t base = p & ~3ull;
    const uint32_t sh = (uint32_t)(p & 3);
    uint32_t hv[kHashWords];
    uint32_t lo = gword(a, base);
#pragma unroll
    for (int t = 0; t < kHashWords; ++t) {
        uint32_t x = 0;
        if (t < (int)a.hw) {
            const uint32_t hi = gword(a, base + 4 * t + 4);
            x = __builtin_amdgcn_alignbyte(hi, lo, sh);
            lo = hi;
            if (t == (int)a.mw - 1) x &= a.lastmask;
        }
        hv[t] = x;
    }
    const uint32_t h = window_hash(hv, (int)a.hw);
    uint32_t slot = h >> a.slot_shift;
    for (;;) {
        const uint64_t e = a.slots[slot];
        if (e == 0) return 0;
        if ((uint32_t)(e >> 32) == h) {
            const uint32_t g = (uint32_t)e - 1u;
            const uint32_t *pw = a.pwords + a.pwoff[a.gstart[g]];
            bool eq = true;
            uint32_t w0 = gword(a, base);
            for (uint32_t t = 0; t < a.mw; ++t) {
                const uint32_t w1 = gword(a, base + 4 * t + 4);
                uint32_t x = __builtin_amdgcn_alignbyte(w1, w0, sh);
                w0 = w1;
                uint32_t y = pw[t];
                if (t == a.mw - 1) {
                    x &= a.lastmask;
                    y &= a.lastmask;
                }
                if (x != y) { eq = false; break; }
            }
            if (eq) return g + 1;     // groups have distinct prefixes
        }
        slot = (slot + 1) & a.slot_mask;
    }
}

// Unequal lengths: does distinct pattern u occur at start position i0?
__device__ inline bool member_matches(const VerifyArgs &a, uint64_t i0, uint32_t u) {
    const uint32_t len = a.plen[u];
    if (i0 + len > a.n) return false;
    const uint32_t *pw = a.pwords + a.pwoff[u];
    const uint64_t p = a.delta + i0;
    const uint64_t base = p & ~3ull;
    const uint32_t sh = (uint32_t)(p & 3);
    const uint32_t words = (len + 3) / 4;
    const uint32_t lastmask = (len & 3) ? ((1u << (8 * (len & 3))) - 1u) : 0xFFFFFFFFu;
    return window_equal(a, base, sh, words, pw, lastmask);
}

// Unequal lengths: every member of the window's group that fits before the
// text's end and equals the text there emits all its ids. Lanes walk their
// own groups in step; each step's ids leave in ballot rounds (one atomic add
// per round).
__device__ inline void verify_wave_var(const VerifyArgs &a, uint64_t i0, bool active) {
    const uint32_t g1 = active ? find_group(a, i0) : 0u;
    uint32_t it = 0, end = 0;
    if (g1) {
        it = a.gstart[g1 - 1];
        end = a.gstart[g1];
    }
    const uint32_t lane = __lane_id();
    const uint32_t first = (uint32_t)__builtin_ctzll(__ballot(true));
    const uint64_t emit = a.key_or + (i0 << a.idbits);
    while (__ballot(it < end)) {
        uint32_t b = 0, c = 0;
        if (it < end) {
            const uint32_t u = it++;
            if (member_matches(a, i0, u)) {
                b = a.idstart[u];
                c = a.idstart[u + 1] - b;
            }
        }
        for (uint32_t t = 0;; ++t) {
            const bool has = t < c;
            const uint64_t mask = __ballot(has);
            if (!mask) break;
            unsigned long long got = 0;
            if (lane == first)
                got = atomicAdd((unsigned long long *)&a.counters[0], (unsigned long long)__popcll(mask));
            const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)got);
            const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(got >> 32));
            if (has) {
                const uint64_t at = (((uint64_t)hi << 32) | lo) + lanes_below(mask);
                if (at < a.cap) a.keys[at] = emit | (uint64_t)a.ids[b + t];
            }
        }
    }
}

// Verifies the start positions of the wave's lanes that have `active` set
// and emits every (i0, id) occurrence, reserving output room with one atomic
// add per wave so that outputs with many occurrences do not serialize on the
// counter. With all 64 lanes executing (the scan kernels call it so) a wave
// prefix sum gives each lane its slots at once; otherwise round t writes the
// t-th id of each lane's run of equal patterns, from ballots only.
__device__ inline void emit_found(const VerifyArgs &a, uint64_t i0, uint32_t u1);

__device__ inline void verify_wave(const VerifyArgs &a, uint64_t i0, bool active) {
    if (a.var) {
        verify_wave_var(a, i0, active);
        return;
    }
    emit_found(a, i0, active ? find_pattern(a, i0) : 0u);
}

// Emits every id of distinct pattern u1 - 1 (none for u1 = 0) at start i0,
// reserving output room with one atomic add per wave.
__device__ inline void emit_found(const VerifyArgs &a, uint64_t i0, uint32_t u1) {
    uint32_t b = 0, c = 0;
    if (u1) {
        b = a.idstart[u1 - 1];
        c = a.idstart[u1] - b;
    }
    const uint64_t exec = __ballot(true);
    const uint32_t lane = __lane_id();
    const uint64_t emit = a.key_or + (i0 << a.idbits);
    if (exec == ~0ull) {
        uint32_t inc = c;                     // inclusive prefix of c over the wave
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(inc, off);
            if (lane >= (uint32_t)off) inc += o;
        }
        const uint32_t total = __shfl(inc, 63);
        if (total == 0) return;
        unsigned long long base = 0;
        if (lane == 63) base = atomicAdd((unsigned long long *)&a.counters[0], (unsigned long long)total);
        base = __shfl(base, 63);
        const uint64_t at = base + inc - c;
        for (uint32_t t = 0; t < c; ++t)
            if (at + t < a.cap) a.keys[at + t] = emit | (uint64_t)a.ids[b + t];
        return;
    }
    const uint32_t first = (uint32_t)__builtin_ctzll(exec);
    for (uint32_t t = 0;; ++t) {
        const bool has = t < c;
        const uint64_t mask = __ballot(has);
        if (!mask) break;
        unsigned long long base = 0;
        if (lane == first)
            base = atomicAdd((unsigned long long *)&a.counters[0], (unsigned long long)__popcll(mask));
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)base);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
        if (has) {
            const uint64_t at = (((uint64_t)hi << 32) | lo) + lanes_below(mask);
            if (at < a.cap) a.keys[at] = emit | (uint64_t)a.ids[b + t];
        }
    }
}

// Per-wave buffering of output keys (every scan kernel): a wave collects its
// keys in an LDS buffer of kFoundBuf keys and writes them to the output with
// one atomic add per buffer, instead of one atomic add on the output counter
// per round that finds a match (atomic adds to one address are serialized
// across the device). All 64 lanes call these.
constexpr uint32_t kFoundBuf = 64;

// Writes buf[0 .. n) (n wave-uniform) to the output.
__device__ inline void flush_found(const VerifyArgs &a, const uint64_t *buf, uint32_t n) {
    if (!n) return;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const uint32_t lane = __lane_id();
    unsigned long long got = 0;
    if (lane == 0) got = atomicAdd((unsigned long long *)&a.counters[0], (unsigned long long)n);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)got);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(got >> 32));
    const uint64_t base = ((uint64_t)hi << 32) | lo;
    for (uint32_t i = lane; i < n; i += 64)
        if (base + i < a.cap) a.keys[base + i] = buf[i];
    __builtin_amdgcn_wave_barrier();
}

// Buffered emission of id runs: each lane emits c keys, emit | id_at(t) for
// t < c, into buf (holding fbn of at most cap keys); returns the new count.
// Keys that do not fit flush the buffer first; a round with more keys than
// the buffer holds goes to the output directly, with one atomic add.
template <typename IdAt>
__device__ inline uint32_t emit_runs_buffered(const VerifyArgs &a, uint64_t i0, uint32_t c, IdAt id_at,
                                              uint64_t *buf, uint32_t fbn, uint32_t cap) {
    const uint32_t lane = __lane_id();
    uint32_t inc, total;                      // inclusive prefix of c over the wave, its sum
    const uint64_t one = __ballot(c != 0);
    if (__ballot(c > 1) == 0) {               // at most one key per lane: ballots only
        inc = lanes_below(one) + c;
        total = (uint32_t)__popcll(one);
    } else {
        inc = c;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(inc, off);
            if (lane >= (uint32_t)off) inc += o;
        }
        total = __builtin_amdgcn_readlane(inc, 63);
    }
    if (total == 0) return fbn;
    if (fbn + total > cap) {
        flush_found(a, buf, fbn);
        fbn = 0;
    }
    const uint64_t emit = a.key_or + (i0 << a.idbits);
    if (total > cap) {
        unsigned long long base = 0;
        if (lane == 63) base = atomicAdd((unsigned long long *)&a.counters[0], (unsigned long long)total);
        base = __shfl(base, 63);
        const uint64_t at = base + inc - c;
        for (uint32_t t = 0; t < c; ++t)
            if (at + t < a.cap) a.keys[at + t] = emit | (uint64_t)id_at(t);
        return 0;
    }
    const uint32_t at = fbn + inc - c;
    for (uint32_t t = 0; t < c; ++t) buf[at + t] = emit | (uint64_t)id_at(t);
    return fbn + total;
}

// emit_found into buf: every id of distinct pattern u1 - 1 (none for u1 = 0)
// at start i0 (see emit_runs_buffered).
__device__ inline uint32_t emit_found_buffered(const VerifyArgs &a, uint64_t i0, uint32_t u1, uint64_t *buf,
                                               uint32_t fbn, uint32_t cap = kFoundBuf) {
    uint32_t b = 0, c = 0;
    if (u1) {
        b = a.idstart[u1 - 1];
        c = a.idstart[u1] - b;
    }
    return emit_runs_buffered(a, i0, c, [&](uint32_t t) { return a.ids[b + t]; }, buf, fbn, cap);
}

}  // namespace mag
