// Dense mode: every start position is tested against a Bloom bitmap of the
// patterns' first min(m, 16) bytes; those that pass go to the exact
// verification of Section 3.2. This is the filter that passes every window
// (sigma' = 1), done without per-window overhead: one hash and kBloomBits LDS
// bit tests per position. Shared by the single-job dense kernel and the batched
// kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mag_internal.hpp"
#include "scan_common.hpp"

namespace mag {

// The single-job dense kernel: one 1024-thread workgroup holds a compute
// unit's 16 wave slots (4 per SIMD at up to 128 VGPRs) beside a Bloom bitmap
// of up to 128 KiB, where two 512-thread ones would not fit.
#ifndef MAG_DENSE_SCAN_THREADS
#define MAG_DENSE_SCAN_THREADS 1024
#endif
constexpr int kDenseScanThreads = MAG_DENSE_SCAN_THREADS;
constexpr int kDenseScanTile = 16 * kDenseScanThreads;
constexpr uint32_t kDenseQueue = 128;   // per-wave queue the callers provide (starts)
// one-probe dense kernel: 63 owning lanes of P (16 or 32, the words per
// lane) positions per wave; a tile is the workgroup's 16 waves
constexpr int slice_scan_tile(int P) { return P * 63 * (kDenseScanThreads / 64); }

struct DenseArgs {
    const uint8_t *tbase;      // text pointer rounded down to 16 bytes
    uint64_t delta;            // text - tbase
    uint64_t n;
    int64_t last;              // last start position, n - m
    uint64_t ntiles;
    uint32_t bshift;           // 32 - log2(Bloom bits)
    uint32_t bloom_vec;        // 16-byte vectors of the bitmap
    const uint32_t *bloom;
    uint64_t *counters;        // [1] positions past the bitmap [2] verifications
    VerifyArgs v;
};

mag_status launch_dense(const DenseArgs &a, size_t bloom_bytes, hipStream_t stream);
// The one-probe dense kernel: a.bloom is the slice bitmap, k its slices per
// pattern, P the positions per lane (16 or 32), a.ntiles counts tiles of
// slice_scan_tile(P) positions.
mag_status launch_dense_slices(const DenseArgs &a, size_t bitmap_bytes, int k, int P, hipStream_t stream);

namespace dev {

// One tile of the dense mode: start positions x0 .. x0 + 16*NT - 1 (those up
// to `last`). Thread tid takes the 16 consecutive positions from
// x0 + 16*tid: two 16-byte loads and one 8-byte load (consecutive lanes read
// consecutive 16-byte blocks) give the bytes of all 16 windows. rs covers the
// tile's bytes, nrec is its size and p0 the resource offset of position x0.
// A thread whose 40 bytes reach past the resource (only at the end of a
// text) loads single dwords, each range-checked on its own, so no text byte
// comes back as an out-of-range zero. Positions that pass the bitmap go to
// this wave's queue; full queues are verified at once.
// The 40 bytes thread tid needs, [a, a + 40) with a = (p0 & ~3) + 16*tid.
template <int NT>
__device__ __forceinline__ void dense_load(__amdgpu_buffer_rsrc_t rs, uint32_t nrec, uint32_t p0, int tid,
                                           uint32_t (&W)[10]) {
    const uint32_t a = (p0 & ~3u) + 16u * (uint32_t)tid;
    if (a + 40u <= nrec) {
        const uint4 v0 = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)a, 0, 0));
        const uint4 v1 = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(a + 16), 0, 0));
        const uint2 v2 = __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)(a + 32), 0, 0));
        W[0] = v0.x; W[1] = v0.y; W[2] = v0.z; W[3] = v0.w;
        W[4] = v1.x; W[5] = v1.y; W[6] = v1.z; W[7] = v1.w;
        W[8] = v2.x; W[9] = v2.y;
    } else {
#pragma unroll
        for (int t = 0; t < 10; ++t) W[t] = ld32(rs, a + 4u * t);
    }
}

// Found-key buffer of a wave (see emit_found_buffered): buf holds *n of at
// most cap keys; buf == nullptr emits every verification round directly.
struct FoundBuf {
    uint64_t *buf = nullptr;
    uint32_t *n = nullptr;
    uint32_t cap = 0;
};

__device__ __forceinline__ void queue_hits(uint32_t hm, int64_t xb, int64_t last, uint64_t *queue,
                                           uint32_t &qn, const VerifyArgs *vp, int lane, uint64_t &nhit,
                                           FoundBuf fb);

// Tests the 16 windows of thread tid (positions xb .. xb + 15, xb = x0 +
// 16*tid; d = p0 & 3) whose bytes are in W, and queues those that pass.
// FAST: the hash takes 4 whole words (m >= 16, or m a multiple of 4 from 13
// up), so no word count or last-word mask is read at run time. The hits of
// the 16 positions are collected in a mask first; a wave prefix sum then
// places all of the wave's hits in its queue at once when they fit (the queue
// holds fewer than 64 starts between calls), and otherwise they are queued
// position by position with ballots, draining full queues as before.
template <bool FAST>
__device__ __forceinline__ void dense_test(const uint32_t (&W)[10], uint32_t d, int64_t xb, int64_t last,
                                           const uint32_t *s_bloom, uint32_t bshift, uint32_t hw,
                                           uint32_t mw, uint32_t lastmask, uint64_t *queue, uint32_t &qn,
                                           const VerifyArgs *vp, int lane, uint64_t &nhit, FoundBuf fb) {
    uint32_t V[9];                              // bytes from position xb on
#pragma unroll
    for (int t = 0; t < 9; ++t) V[t] = __builtin_amdgcn_alignbyte(W[t + 1], W[t], d);
    uint32_t hm = 0;                            // bit 4i+s: position xb+4i+s passed the bitmap
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        // the probes of 4 positions: all bitmap words are read before any is
        // used, so that the LDS reads overlap
        uint32_t p[4][kBloomBits], word[4][kBloomBits];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            uint32_t w[4];
#pragma unroll
            for (int t = 0; t < 4; ++t)
                w[t] = s ? __builtin_amdgcn_alignbyte(V[i + t + 1], V[i + t], s) : V[i + t];
            uint32_t h;
            if constexpr (FAST) {
                h = prefilter_hash4(w);
            } else {
                if (mw <= 4) {
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        if ((uint32_t)t == mw - 1) w[t] &= lastmask;
                }
                h = prefilter_hash(w, (int)hw);
            }
#pragma unroll
            for (int j = 0; j < kBloomBits; ++j) p[s][j] = bloom_probe(h, j);
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int j = 0; j < kBloomBits; ++j) word[s][j] = s_bloom[p[s][j] >> (bshift + 5)];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            uint32_t b = 1u;
#pragma unroll
            for (int j = 0; j < kBloomBits; ++j) b &= word[s][j] >> (p[s][j] & 31u);
            hm |= (b & 1u) << (4 * i + s);
        }
    }
    queue_hits(hm, xb, last, queue, qn, vp, lane, nhit, fb);
}

// Queues the positions xb + u of this lane whose bit u (u < 16) is set in hm
// and that do not pass `last`; verifies full queues, their keys going to the
// found-key buffer fb when it has one. Every lane of the wave calls it.
__device__ __forceinline__ void queue_hits(uint32_t hm, int64_t xb, int64_t last, uint64_t *queue,
                                           uint32_t &qn, const VerifyArgs *vp, int lane, uint64_t &nhit,
                                           FoundBuf fb) {
    auto drain = [&](uint32_t from) {
        if (fb.buf) *fb.n = drain64_found(vp, queue, from, lane, fb.buf, *fb.n, fb.cap);
        else drain64(vp, queue, from, lane);
    };
    // positions past the last start
    const int64_t room = last - xb + 1;
    if (room < 16) hm &= room <= 0 ? 0u : ((1u << (uint32_t)room) - 1u);
    if (!__ballot(hm != 0)) return;
    const uint32_t c = (uint32_t)__popc(hm);
    uint32_t inc = c;                           // inclusive prefix of c over the wave
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(inc, off);
        if (lane >= off) inc += o;
    }
    const uint32_t total = __shfl(inc, 63);
    nhit += c;
    if (qn + total <= kDenseQueue) {
        uint32_t at = qn + inc - c;
        for (uint32_t m = hm; m; m &= m - 1u) queue[at++] = (uint64_t)(xb + __builtin_ctz(m));
        qn += total;
        while (qn >= 64) {
            qn -= 64;
            drain(qn);
        }
        return;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const bool hit = (hm >> u) & 1u;
        const uint64_t bal = __ballot(hit);
        if (!bal) continue;
        if (hit) queue[qn + lanes_below(bal)] = (uint64_t)(xb + u);
        qn += (uint32_t)__popcll(bal);
        if (qn >= 64) {
            qn -= 64;
            drain(qn);
        }
    }
}

// One-probe dense mode (slice_hash). A wave covers 63 * P consecutive start
// positions (P = 16 or 32): lane L < 63 owns the P from xb = its wave's first
// + P L, and lane 63 probes the P that follow the wave's last (the next
// wave's first), so that every owner finds the probes of the positions up to
// P - 1 past its own in the next lane. W holds load_words(AL) words from the
// word that contains xb (d = xb's byte offset in it; AL: d = 0): exactly the
// words the probes read, so that no loaded register is left dead (a dead
// load's register, reused, makes the wave wait for that load before the
// prefetched tiles behind it arrive). Bit u of a lane's
// probe mask is the bitmap bit of the slice at xb + u; position xb + u passes
// when bits u, u + 2, .., u + 2(K-1) of the mask extended by the next lane's
// are all set.
constexpr int kSliceOwners = 63;
template <int P> struct SliceLane {
    static constexpr int kWords = P / 4 + 2;         // realigned words: bytes xb .. xb + P + 7
    // words loaded per lane: one more when xb is not word-aligned
    static constexpr int load_words(bool al) { return kWords + (al ? 0 : 1); }
};

template <int P, bool AL>
__device__ __forceinline__ void slice_words(const uint32_t (&W)[SliceLane<P>::load_words(AL)], uint32_t d,
                                            uint32_t (&V)[SliceLane<P>::kWords]) {
#pragma unroll
    for (int t = 0; t < SliceLane<P>::kWords; ++t)
        V[t] = AL ? W[t] : __builtin_amdgcn_alignbyte(W[t + 1], W[t], d);
}

template <int P>
__device__ __forceinline__ uint32_t slice_probes(const uint32_t (&V)[SliceLane<P>::kWords],
                                                 const uint32_t *s_bits, uint32_t bshift) {
    uint32_t A[P + 3];                          // A[i]: the word of bytes xb+i .. xb+i+3
#pragma unroll
    for (int i = 0; i < P + 3; ++i)
        A[i] = (i & 3) ? __builtin_amdgcn_alignbyte(V[i / 4 + 1], V[i / 4], i & 3) : V[i / 4];
    uint32_t hm = 0;
    const uint32_t ashift = bshift + 3;
#pragma unroll
    for (int u = 0; u < P; ++u) {
        const uint32_t h = __umul24(A[u + 3], kSliceK2) + __umul24(A[u], kSliceK1);
        const uint32_t w = *reinterpret_cast<const uint32_t *>(
            reinterpret_cast<const char *>(s_bits) + ((h >> ashift) & ~3u));
        hm |= __builtin_amdgcn_ubfe(w, h >> bshift, 1u) << u;
    }
    return hm;
}

// One lane-run of the one-probe dense mode: probes, the K-slice test, and the
// queueing of the passing positions (room: starts left from xb, <= 0 when
// none), one per lane and round with a ballot; found keys collect in the
// wave's buffer fbuf (fbn keys). Every lane of the wave calls it. INL:
// verification inlined (drain64_found).
template <int K, int P, bool AL, bool INL = false>
__device__ __forceinline__ void slice_test(const uint32_t (&W)[SliceLane<P>::load_words(AL)], uint32_t d,
                                           int64_t xb, int64_t room, const uint32_t *s_bits,
                                           uint32_t bshift, uint64_t *queue, uint32_t &qn,
                                           const VerifyArgs *vp, int lane, uint32_t &nhit, uint64_t *fbuf,
                                           uint32_t &fbn, uint32_t fbcap = kFoundBuf) {
    uint32_t V[SliceLane<P>::kWords];
    slice_words<P, AL>(W, d, V);
    const uint32_t hm = slice_probes<P>(V, s_bits, bshift);
    uint32_t pass = hm;
    if constexpr (K > 1) {
        // the next lane's probes of the positions after this lane's
        const uint32_t nx = __shfl_down(hm, 1);
        if constexpr (P == 32) {
            const uint64_t ext = (uint64_t)hm | ((uint64_t)nx << 32);
            uint64_t pw = ext;
#pragma unroll
            for (int j = 1; j < K; ++j) pw &= ext >> (kSliceStride * j);
            pass = (uint32_t)pw;
        } else {
            const uint32_t ext = hm | (nx << 16);
#pragma unroll
            for (int j = 1; j < K; ++j) pass &= ext >> (kSliceStride * j);
            pass &= 0xFFFFu;
        }
    }
    if (lane >= kSliceOwners) pass = 0u;
    if (room < P) pass &= room <= 0 ? 0u : (uint32_t)((1ull << (uint32_t)room) - 1u);
    nhit += (uint32_t)__popc(pass);
    while (__ballot(pass != 0)) {
        const bool act = pass != 0;
        const uint32_t u = act ? (uint32_t)__builtin_ctz(pass) : 0u;
        pass &= pass - 1u;
        const uint64_t bal = __ballot(act);
        if (act) queue[qn + lanes_below(bal)] = (uint64_t)(xb + u);
        qn += (uint32_t)__popcll(bal);
        if (qn >= 64) {
            qn -= 64;
            fbn = drain64_found<INL>(vp, queue, qn, lane, fbuf, fbn, fbcap);
        }
    }
}

// dense_test with the hash form chosen from the pattern length.
__device__ __forceinline__ void dense_test_any(const uint32_t (&W)[10], uint32_t d, int64_t xb,
                                               int64_t last, const uint32_t *s_bloom, uint32_t bshift,
                                               uint32_t hw, uint32_t mw, uint32_t lastmask,
                                               uint64_t *queue, uint32_t &qn, const VerifyArgs *vp,
                                               int lane, uint64_t &nhit, FoundBuf fb = {}) {
    if (hw == 4 && (mw > 4 || lastmask == 0xFFFFFFFFu))
        dense_test<true>(W, d, xb, last, s_bloom, bshift, hw, mw, lastmask, queue, qn, vp, lane, nhit, fb);
    else
        dense_test<false>(W, d, xb, last, s_bloom, bshift, hw, mw, lastmask, queue, qn, vp, lane, nhit, fb);
}

}  // namespace dev
}  // namespace mag
