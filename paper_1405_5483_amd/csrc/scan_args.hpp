// Arguments of the scan kernel, shared by its per-q objects and the dispatcher.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mag.h"
#include "verify.hpp"

namespace mag {

#ifndef MAG_SCAN_THREADS
#define MAG_SCAN_THREADS 1024
#endif
#ifndef MAG_SCAN_PRODUCERS
#define MAG_SCAN_PRODUCERS 12
#endif
constexpr int kScanThreads = MAG_SCAN_THREADS;        // threads per scan workgroup
constexpr int kScanProducerWaves = MAG_SCAN_PRODUCERS; // waves that compute mask entries
constexpr int kScanConsumerLanes = kScanThreads - 64 * kScanProducerWaves;  // Shift-Or lanes
constexpr uint64_t kScanLdsMax = 160 * 1024;   // LDS of one workgroup on gfx950
constexpr uint64_t kScanStaticLds = 4096;       // the scan kernel's static LDS, at most

struct ScanArgs {
    const uint8_t *tbase;      // text pointer rounded down to 16 bytes
    uint64_t delta;            // text - tbase
    uint64_t n, X, ntiles;     // text bytes, samples, tiles
    uint64_t src_bytes;        // bytes phase A reads from: the text, or (SMAG) the encoded text
    uint32_t stride;           // source bytes between samples: kq, or k * code bytes
    uint32_t k, kq, mprime, W, sp, m;
    uint32_t S;                // samples per consumer lane
    uint32_t tile_samples;     // kScanConsumerLanes * S
    uint32_t e_lds;            // bytes of LDS for one buffer of a tile's mask entries
    uint32_t table_vec;        // 16-byte vectors of the mask table (LDS copy)
    uint32_t w0;               // entries kept before a tile's first sample (>= m'-1)
    uint32_t bshift, blen;     // bit-field map: field shift and width l (blen 0: map table);
                               // q-gram map: blen = log2 sigma'
    uint32_t qgram;            // 1: codes are hashed q-grams (no mu)
    uint32_t pbits;            // bits per packed table entry (1, 2, 4), 0: whole entries
    uint32_t pre;              // SMAG: bytes per encoded code (2 or 4), 0: codes on the fly
    uint32_t maxcode;          // SMAG: largest valid code (n_codes - 1)
    const uint8_t *mu;
    const void *table;
    uint64_t *counters;        // [1] candidate windows [2] verifications
    VerifyArgs v;              // verification of the queued start positions
};

VerifyArgs make_verify_args(const mag_plan *p, const ScanLaunch &s);

// Encoding of the whole text for SMAG: the code of every complete
// non-overlapping q-gram, csz (2 or 4) bytes each.
struct EncodeArgs {
    const uint8_t *tbase;      // text pointer rounded down to 16 bytes
    uint64_t delta, n, G;      // text - tbase, text bytes, grams
    void *codes;
    const uint8_t *mu;
    uint32_t sp, bshift, blen, qgram;
};

#define MAG_DECLARE_SCAN_Q(q)                                                            \
    mag_status launch_scan_q##q(const ScanArgs &a, int esz, bool wide, bool tlds,        \
                                bool mul24, size_t shmem, int ncu, hipStream_t stream);  \
    mag_status launch_encode_q##q(const EncodeArgs &e, int csz, bool mul24, hipStream_t stream);
MAG_DECLARE_SCAN_Q(1)
MAG_DECLARE_SCAN_Q(2)
MAG_DECLARE_SCAN_Q(3)
MAG_DECLARE_SCAN_Q(4)
MAG_DECLARE_SCAN_Q(5)
MAG_DECLARE_SCAN_Q(6)
MAG_DECLARE_SCAN_Q(7)
MAG_DECLARE_SCAN_Q(8)
#undef MAG_DECLARE_SCAN_Q

}  // namespace mag
