// Batched scans: the per-job descriptors that the persistent kernel reads and
// its launch entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dense.hpp"
#include "mag_internal.hpp"
#include "verify.hpp"

namespace mag {

constexpr int kBatchThreads = 1024;               // threads per workgroup
// Filter tiles hold 1024 * words-per-lane samples, words per lane (the
// Shift-Or run of one lane) 8 or 16 (default), chosen per batch: 1024-thread
// workgroups with 64 KiB tables in LDS leave room for the entries of 16
// words per lane, and ran the batch's filter jobs in 0.50 ms against 0.66
// with 512 threads (one workgroup per compute unit either way). Dense jobs run in
// a launch of their own (k_batch_dense): tiles of kBatchSliceTile start
// positions with the slice bitmap, else kDenseScanTile with the Bloom bitmap.
constexpr int kBatchWordsDefault = 16;
constexpr int kBatchMaxWarm = 32;                // warm-up entries before a tile (>= m' - 1)
constexpr int kBatchQueue = 128;                 // per-wave queue of start positions
// mask entries of one tile of TS samples as u32, in whole groups of eight
// 16-byte vectors
constexpr uint32_t batch_entry_bytes(int TS) { return ((TS + kBatchMaxWarm) * 4 + 127) / 128 * 128; }
constexpr uint32_t kBatchTableLds = 64 * 1024;   // larger mask tables are read from L2
constexpr int kBatchSliceLane = 16;              // start positions per lane of a slice tile
constexpr int kBatchSliceTile = slice_scan_tile(kBatchSliceLane);
// a dense job's claimed tile: up to this many sub-tiles of kBatchSliceTile
// or kDenseScanTile start positions (JobDesc::chunk: fewer for jobs whose
// positions pass often, whose sub-tiles take longer)
constexpr int kBatchDenseChunk = 8;
// alphabet map, two claimed-tile slots, queues, entries, table
constexpr uint32_t batch_lds_bytes(int TS) {
    return 256 + 16 + (kBatchThreads / 64) * kBatchQueue * 8 + batch_entry_bytes(TS) + kBatchTableLds;
}

// One job as the kernel sees it. Written by the host at bind time.
struct JobDesc {
    const uint8_t *tbase;      // text pointer rounded down to 16 bytes
    uint64_t delta;            // text - tbase
    uint64_t n, X;             // text bytes, samples
    uint64_t tile_first;       // global index of the job's first tile
    uint64_t ntiles;
    const uint8_t *mu;         // the plan's alphabet map (256 B)
    const void *table;         // its mask table
    uint32_t q, k, kq, mprime, W, sp, esz, w0;
    uint32_t tlds;             // table staged in LDS
    uint32_t table_vec;        // 16-byte vectors of the table
    uint32_t dense;            // test every start position; `table` is then the job's bitmap
    uint32_t bshift;           // 32 - log2(bitmap bits) of a dense job
    uint32_t slice_k;          // dense job: slices per pattern of its slice bitmap (0: Bloom bitmap)
    uint32_t chunk;            // dense job: sub-tiles per claimed tile (1 .. kBatchDenseChunk)
    // dense job with exact window codes (code_mask != 0; `table` is then the
    // code bitmap): the field shift, the bytes of the four codes and the
    // code of each distinct pattern's index + 1
    uint32_t code_shift, code_rep, code_mask;
    const uint32_t *code_ids;
    VerifyArgs v;              // verification, with the job number in key_or
};

struct BatchLaunch {
    const JobDesc *jobs;
    uint32_t njobs;
    const uint64_t *ranges;    // per workgroup: first tile, end tile, job of the first tile
    uint64_t *next;            // per workgroup: next unclaimed tile of its range
    uint32_t grid;
    uint64_t total_tiles;
    uint64_t *counters;
    uint32_t words_per_lane;   // 8 or 16: filter tiles of 1024 * words samples
};

// Workgroups of the batch kernel with `words_per_lane` that fit on one
// compute unit (0 on error).
int batch_occupancy(int words_per_lane);
mag_status batch_configure();
mag_status launch_batch(const BatchLaunch &b, hipStream_t stream);
// The dense jobs' launch: b.jobs holds only dense jobs, with their own tile
// sequence, ranges and claims; one 1024-thread workgroup per compute unit.
int batch_dense_occupancy();
mag_status launch_batch_dense(const BatchLaunch &b, hipStream_t stream);
// Verifies the starts that batched jobs deferred: entry = job << kBatchJobShift
// | start (batch.hip).
constexpr int kBatchJobShift = 40;
mag_status launch_batch_verify(const JobDesc *jobs, const uint64_t *pending, const uint64_t *seg_count,
                               uint64_t seg_cap, hipStream_t stream);
// offsets[j] = first record of job j in the sorted keys (the first key at
// or above jbase[j] << idbits), offsets[njobs] = count; for outputs the
// finishing kernel sorted (at most small_sort_max keys), each record's
// position less its job's jbase (out: their records).
mag_status launch_batch_offsets(const uint64_t *sorted, const uint64_t *zp, uint64_t cap,
                                uint64_t *d_offsets, uint32_t njobs, const uint64_t *jbase, int idbits,
                                mag_match *out, hipStream_t stream);

}  // namespace mag
