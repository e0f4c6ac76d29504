// C ABI of batched scans (include/mag.h): a batch binds many (text, plan)
// jobs, lays their tiles out for one persistent launch and enqueues scan,
// sort and per-job offsets without host synchronization.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "batch.hpp"
#include "scan_args.hpp"

namespace mag {
namespace {

int ceil_log2(uint64_t v) {
    int b = 0;
    while (b < 64 && (1ull << b) < v) ++b;
    return b;
}

// Fixed cost of a tile (barriers, setup) in text-byte equivalents, for the
// split of the tile sequence among workgroups.
constexpr uint64_t kTileOverheadBytes = 2048;
// A dense start position that passes (its key emitted or its window
// verified) costs about this many positions that fail (measured on jobs of
// exact codes with DNA patterns, whose emission took longer than their test).
constexpr double kDensePassCost = 32.0;
// Jobs with texts up to this size may defer their verification; the batch's
// deferred-start buffer holds this many entries (starts past a segment's
// share are verified inline, so the result never depends on it).
constexpr uint64_t kBatchDeferMaxText = 1 << 20;
constexpr uint64_t kBatchPendingEntries = 1 << 23;

// Contiguous tile ranges of about equal weight, one per workgroup, over a
// tile sequence laid out job after job (tiles_of[j] tiles of job j, weight(j,
// t) of its tile t): ranges[3w] = first tile, [3w+1] = end, [3w+2] = the job
// of the first tile.
template <typename Weight>
std::vector<uint64_t> split_ranges(uint64_t grid, const std::vector<uint64_t> &tiles_of, uint64_t total_tiles,
                                   Weight weight) {
    std::vector<uint64_t> ranges(3 * std::max<uint64_t>(grid, 1), 0);
    if (!grid) return ranges;
    const uint32_t njobs = (uint32_t)tiles_of.size();
    long double total = 0;
    for (uint32_t j = 0; j < njobs; ++j)
        for (uint64_t t = 0; t < tiles_of[j]; ++t) total += (long double)weight(j, t);
    std::vector<uint64_t> begin(grid + 1, total_tiles);
    std::vector<uint32_t> job_of(grid, 0);
    uint64_t next_wg = 0, g = 0;
    long double run = 0;
    for (uint32_t j = 0; j < njobs; ++j) {
        for (uint64_t t = 0; t < tiles_of[j]; ++t, ++g) {
            uint64_t w = (uint64_t)(run * (long double)grid / total);
            if (w >= grid) w = grid - 1;
            while (next_wg <= w) {
                begin[next_wg] = g;
                job_of[next_wg] = j;
                ++next_wg;
            }
            run += (long double)weight(j, t);
        }
    }
    for (uint64_t wg = 0; wg < grid; ++wg) {
        ranges[3 * wg] = begin[wg];
        ranges[3 * wg + 1] = begin[wg + 1] > begin[wg] ? begin[wg + 1] : begin[wg];
        ranges[3 * wg + 2] = begin[wg] < total_tiles ? job_of[wg] : 0;
    }
    return ranges;
}

template <typename T>
mag_status grow(T **p, size_t *have, size_t want_bytes, const char *what) {
    if (*p && *have >= want_bytes) return MAG_OK;
    (void)hipFree(*p);
    *p = nullptr;
    *have = 0;
    if (hipMalloc(p, want_bytes ? want_bytes : 16) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(MAG_E_NOMEM, std::string("device allocation failed: ") + what);
    }
    *have = want_bytes;
    return MAG_OK;
}

}  // namespace
}  // namespace mag

struct mag_batch {
    std::vector<mag_plan *> plans;
    std::mutex mtx;
    int device = -1;
    bool bound = false;
    uint64_t cap = 0;
    int idbits = 1, posbits = 1, nbits = 3;   // posbits: the batch's text bytes
    uint64_t total_tiles = 0;
    uint64_t *d_jbase = nullptr;     // njobs + 1: each job's first byte in the batch's texts
    size_t jbase_bytes = 0;
    uint32_t grid = 0;
    mag::JobDesc *d_jobs = nullptr;
    size_t jobs_bytes = 0;
    uint64_t *d_ranges = nullptr;
    size_t ranges_bytes = 0;
    uint64_t *d_next = nullptr;      // tile claim counters, one per workgroup
    size_t next_bytes = 0;
    // the dense jobs' launch: its job table, tile ranges and claims
    uint32_t ndense = 0;
    uint64_t dense_tiles = 0;
    uint32_t dense_grid = 0;
    mag::JobDesc *d_djobs = nullptr;
    size_t djobs_bytes = 0;
    uint64_t *d_dranges = nullptr;
    size_t dranges_bytes = 0;
    uint64_t *d_dnext = nullptr;
    size_t dnext_bytes = 0;
    bool defer = false;              // some job defers its verification
    int words_per_lane = mag::kBatchWordsDefault;   // filter tiles of 1024 * words samples
    int bound_words = mag::kBatchWordsDefault;      // the value the bound tile layout uses
    mag::Scratch sc;
};

using namespace mag;

extern "C" {

mag_status mag_batch_create(mag_plan *const *plans, uint32_t njobs, mag_batch **out) {
    if (!out) return fail(MAG_E_INVALID, "out is NULL");
    *out = nullptr;
    if (njobs && !plans) return fail(MAG_E_INVALID, "plans is NULL");
    if (njobs > (1u << 24)) return fail(MAG_E_UNSUPPORTED, "more than 2^24 jobs in one batch");
    for (uint32_t j = 0; j < njobs; ++j) {
        const mag_plan *p = plans[j];
        if (!p) return fail(MAG_E_INVALID, "plans[" + std::to_string(j) + "] is NULL");
        if (p->var)
            return fail(MAG_E_UNSUPPORTED, "batched jobs need patterns of one length (job " +
                                               std::to_string(j) + ")");
        if (p->r == 0 || p->dense) continue;   // no filter state in these jobs
        if (p->map_kind == MAG_MAP_QGRAM)
            return fail(MAG_E_UNSUPPORTED, "batched filter jobs need a per-byte alphabet map (job " +
                                               std::to_string(j) + " maps q-grams)");
        if (p->W > 32 || p->k >= 32)
            return fail(MAG_E_UNSUPPORTED, "batched jobs need W = k*m' <= 32 and k < 32 (job " +
                                               std::to_string(j) + ")");
        uint64_t partial = 1;
        for (int t = 0; t + 1 < p->q; ++t) partial *= (uint64_t)p->sigma_prime;
        if (partial >= (1ull << 24))
            return fail(MAG_E_UNSUPPORTED, "batched jobs need sigma'^(q-1) < 2^24 (job " +
                                               std::to_string(j) + ")");
    }
    mag_batch *b = new (std::nothrow) mag_batch();
    if (!b) return fail(MAG_E_NOMEM, "host allocation failed");
    b->plans.assign(plans, plans + njobs);
    *out = b;
    return MAG_OK;
}

void mag_batch_destroy(mag_batch *b) {
    if (!b) return;
    if (b->device >= 0) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(b->device);
        (void)hipFree(b->d_jobs);
        (void)hipFree(b->d_ranges);
        (void)hipFree(b->d_next);
        (void)hipFree(b->d_djobs);
        (void)hipFree(b->d_dranges);
        (void)hipFree(b->d_dnext);
        (void)hipFree(b->d_jbase);
        (void)hipFree(b->sc.counters);
        (void)hipFree(b->sc.keys);
        (void)hipFree(b->sc.hist);
        (void)hipFree(b->sc.radix_off);
        (void)hipFree(b->sc.pending);
        (void)hipFree(b->sc.seg_count);
        (void)hipSetDevice(cur);
    }
    delete b;
}

mag_status mag_batch_bind(mag_batch *b, const uint8_t *const *d_texts, const uint64_t *n,
                          uint64_t out_cap, void *stream_) {
    if (!b) return fail(MAG_E_INVALID, "batch is NULL");
    const uint32_t njobs = (uint32_t)b->plans.size();
    if (njobs && (!d_texts || !n)) return fail(MAG_E_INVALID, "d_texts or n is NULL");
    for (uint32_t j = 0; j < njobs; ++j)
        if (n[j] && !d_texts[j]) return fail(MAG_E_INVALID, "d_texts[" + std::to_string(j) + "] is NULL");
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    std::lock_guard<std::mutex> lock(b->mtx);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (b->device >= 0 && b->device != dev) return fail(MAG_E_INVALID, "batch was bound on another device");
    b->bound = false;
    for (mag_plan *p : b->plans) {
        std::lock_guard<std::mutex> pl(p->mtx);
        mag_status s = ensure_device(p);
        if (s != MAG_OK) return s;
    }
    // earlier runs may still read the job table or the scratch
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    b->device = dev;

    // key layout: (the job's first byte in the texts laid end to end +
    // position) << idbits | pattern id, so that keys sort by job, then
    // position, and the sort passes over the bits of the total text length
    // only (1.1 GB: 31 bits, 4 passes; job and longest-job bits took 33)
    int idbits = 1, posbits = 1, jposbits = 1;
    std::vector<uint64_t> jbase(njobs + 1, 0);
    for (uint32_t j = 0; j < njobs; ++j) {
        idbits = std::max(idbits, ceil_log2(std::max<uint64_t>(b->plans[j]->r, 2)));
        jposbits = std::max(jposbits, ceil_log2(std::max<uint64_t>(n[j] + 1, 2)));
        if (n[j] > ~0ull - jbase[j]) return fail(MAG_E_UNSUPPORTED, "texts longer than 2^64 bytes in all");
        jbase[j + 1] = jbase[j] + n[j];
    }
    posbits = std::max(posbits, ceil_log2(std::max<uint64_t>(jbase[njobs] + 1, 2)));
    if (idbits + posbits > 64)
        return fail(MAG_E_UNSUPPORTED, "text positions and ids need more than 64 key bits");

    // scratch
    Scratch &sc = b->sc;
    if (!sc.counters) {
        size_t have = 0;
        mag_status s = grow(&sc.counters, &have, kCounterWords * sizeof(uint64_t), "batch counters");
        if (s != MAG_OK) return s;
        // the finishing kernel of every run returns the counters to zero
        e = hipMemset(sc.counters, 0, kCounterWords * sizeof(uint64_t));
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "clearing batch counters");
    }
    const uint64_t kcap = std::max<uint64_t>(out_cap, 1024);
    if (!sc.keys || sc.keys_cap < kcap) {
        size_t have = 0;
        (void)hipFree(sc.keys);
        sc.keys = nullptr;
        sc.keys_cap = 0;
        mag_status s = grow(&sc.keys, &have, (size_t)kcap * 2 * sizeof(uint64_t), "batch sort keys");
        if (s != MAG_OK) return s;
        sc.keys_cap = kcap;
    }
    if (out_cap > small_sort_max()) {
        mag_status s = ensure_radix_scratch(sc, out_cap, stream);
        if (s != MAG_OK) return s;
    }

    // jobs and their tiles
    std::vector<JobDesc> jobs(njobs);
    std::vector<uint8_t> defer(njobs, 0);
    std::vector<uint64_t> tiles_of(njobs), tile_bytes_full(njobs), tail_samples(njobs), tile_samples(njobs);
    const int wpl = b->words_per_lane;
    uint64_t total_tiles = 0;
    // dense jobs: their own tile sequence (tiles of the single-job dense kernels)
    std::vector<JobDesc> djobs;
    std::vector<uint32_t> djob_of;   // the batch's job number of each dense job
    std::vector<uint64_t> dtiles_of, dtile_pos, dtail_pos, dstage_bytes;
    std::vector<double> dcost;
    uint64_t dense_tiles = 0;
    for (uint32_t j = 0; j < njobs; ++j) {
        const mag_plan *p = b->plans[j];
        JobDesc &J = jobs[j];
        std::memset(&J, 0, sizeof(J));
        const uint64_t kq = (uint64_t)p->k * p->q;
        const bool scans = p->r > 0 && n[j] >= p->m && n[j] >= (uint64_t)p->q;
        // filter: samples; dense: start positions
        const uint64_t X = !scans ? 0 : p->dense ? n[j] - p->m + 1 : (n[j] - p->q) / kq + 1;
        const uintptr_t t = reinterpret_cast<uintptr_t>(d_texts[j]);
        J.tbase = reinterpret_cast<const uint8_t *>(t & ~(uintptr_t)15);
        J.delta = t & 15;
        J.n = n[j];
        J.X = X;
        J.tile_first = total_tiles;
        const bool slices = p->dense && p->slice_k > 0;
        const bool codes = p->dense && p->code_shift >= 0;
        // dense jobs: the expected share of start positions that pass (the
        // codes of the distinct patterns among the 4^m, else the bitmap's
        // estimate), and the cost of a position relative to one that fails;
        // claimed tiles of costly positions are shorter, so that the last
        // tiles of the launch end close together
        const double pass = codes ? (double)p->n_unique / (double)(1ull << (2 * p->m))
                            : slices ? p->slice_fp : p->dense ? p->bloom_fp : 0.0;
        const double cost = 1.0 + kDensePassCost * pass;
        const uint32_t chunk = (uint32_t)std::max(1.0, std::min((double)kBatchDenseChunk,
                                                                std::floor(kBatchDenseChunk / cost)));
        const uint64_t TS = slices ? (uint64_t)kBatchSliceTile * chunk
                            : p->dense ? (uint64_t)kDenseScanTile * chunk
                                       : (uint64_t)kBatchThreads * wpl;
        J.ntiles = (X + TS - 1) / TS;
        J.mu = p->dev.mu;
        J.table = p->dev.table;
        J.q = p->q;
        J.k = p->k;
        J.kq = (uint32_t)kq;
        J.mprime = p->mprime;
        J.W = p->W;
        J.sp = p->sigma_prime;
        J.esz = p->esz;
        J.w0 = ((uint32_t)p->mprime - 1 + 3) / 4 * 4;
        J.tlds = p->table.size() <= kBatchTableLds ? 1 : 0;
        J.table_vec = (uint32_t)((p->table.size() + 15) / 16);
        J.dense = p->dense ? 1u : 0u;
        J.chunk = chunk;
        if (codes) {
            // exact window codes: the code bitmap (at most 8 KiB) in LDS
            J.table = p->dev.code_bits;
            J.tlds = 1;
            J.table_vec = (uint32_t)(p->code_bits.size() * 4 / 16);
            J.code_shift = (uint32_t)p->code_shift;
            J.code_rep = p->code_rep;
            J.code_mask = (uint32_t)((1ull << (2 * p->m)) - 1);
            J.code_ids = p->dev.code_ids;
        } else if (p->dense) {
            // the slice bitmap of the one-probe mode at full size, else the
            // Bloom bitmap's batched copy (at most 32 KiB, which leaves the
            // rest of the LDS array to the found-key buffers)
            J.table = slices ? p->dev.slices : p->dev.bloom_batch;
            J.tlds = 1;
            J.table_vec = (uint32_t)((slices ? p->slices.size() : p->bloom_batch.size()) * 4 / 16);
            J.bshift = 32u - (uint32_t)(slices ? p->bloom_log2 : std::min(p->bloom_log2, kBloomBatchLog2));
            J.slice_k = slices ? (uint32_t)p->slice_k : 0u;
        }
        ScanLaunch sl;
        sl.text = d_texts[j];
        sl.n = n[j];
        sl.keys = sc.keys;
        sl.cap = out_cap;
        sl.counters = sc.counters;
        sl.idbits = idbits;
        J.v = make_verify_args(p, sl);
        J.v.key_or = jbase[j] << idbits;
        // a short text with many patterns keeps one workgroup verifying for
        // long; its starts go to the batch verification kernel instead
        const double expect = slices ? p->slice_fp * (double)X
                              : p->dense ? p->bloom_fp * (double)X : p->est_verif * (double)n[j];
        const double vwaves = (double)std::max<uint64_t>(J.ntiles, 1) *
                              ((p->dense ? kDenseScanThreads : kBatchThreads) / 64);
        if (X && n[j] <= kBatchDeferMaxText && jposbits <= kBatchJobShift &&
            ((double)p->r * p->m * 4 >= (double)n[j] || expect >= kDeferPerWave * vwaves))
            defer[j] = 1;
        if (p->dense) {
            // the job leaves the filter launch's sequence (no tiles there)
            JobDesc D = J;
            D.tile_first = dense_tiles;
            djobs.push_back(D);
            djob_of.push_back(j);
            dtiles_of.push_back(J.ntiles);
            dtile_pos.push_back(TS);
            dtail_pos.push_back(X - (J.ntiles ? (J.ntiles - 1) * TS : 0));
            dstage_bytes.push_back((uint64_t)J.table_vec * 16);
            dcost.push_back(cost);
            dense_tiles += J.ntiles;
            J.ntiles = 0;
        }
        tiles_of[j] = J.ntiles;
        tile_bytes_full[j] = TS * kq;
        tile_samples[j] = TS;
        tail_samples[j] = X - (J.ntiles ? (J.ntiles - 1) * TS : 0);
        total_tiles += J.ntiles;
    }

    // contiguous tile ranges of about equal weight, one per workgroup, for
    // each of the two launches
    const int ncu = device_compute_units();
    const int occ = batch_occupancy(wpl);
    const int docc = batch_dense_occupancy();
    if (ncu < 1 || occ < 1 || docc < 1) return fail(MAG_E_DEVICE, "cannot size the batch launch");
    uint64_t grid = (uint64_t)ncu * occ;
    if (grid > total_tiles) grid = total_tiles;
    const std::vector<uint64_t> ranges = split_ranges(grid, tiles_of, total_tiles, [&](uint32_t j, uint64_t t) {
        const uint64_t samples = t + 1 < tiles_of[j] ? tile_samples[j] : tail_samples[j];
        return samples * jobs[j].kq + kTileOverheadBytes;
    });
    uint64_t dgrid = (uint64_t)ncu * docc;
    if (dgrid > dense_tiles) dgrid = dense_tiles;
    const std::vector<uint64_t> dranges = split_ranges(dgrid, dtiles_of, dense_tiles, [&](uint32_t d, uint64_t t) {
        // a dense tile reads one byte per position but hashes every one of
        // them (more for positions that pass); a job's first tile also
        // stages its bitmap
        const uint64_t pos = t + 1 < dtiles_of[d] ? dtile_pos[d] : dtail_pos[d];
        return (uint64_t)((double)pos * 4 * dcost[d]) + kTileOverheadBytes + (t == 0 ? dstage_bytes[d] : 0);
    });
    // deferred starts: one buffer for the batch, its segment counters zeroed
    // here once and by the finishing kernel of every run
    b->defer = false;
    for (uint32_t j = 0; j < njobs; ++j) b->defer = b->defer || defer[j];
    if (b->defer) {
        if (!sc.pending) {
            e = hipMalloc(&sc.pending, kBatchPendingEntries * sizeof(uint64_t));
            if (e == hipSuccess) e = hipMalloc(&sc.seg_count, kPendingSegments * sizeof(uint64_t));
            if (e == hipSuccess) e = hipMemset(sc.seg_count, 0, kPendingSegments * sizeof(uint64_t));
            if (e == hipSuccess) e = hipDeviceSynchronize();
            if (e != hipSuccess) return hip_fail(e, "deferred-start buffer of the batch");
            sc.pending_cap = kBatchPendingEntries;
        }
        for (uint32_t j = 0; j < njobs; ++j) {
            if (!defer[j]) continue;
            jobs[j].v.pending = sc.pending;
            jobs[j].v.seg_count = sc.seg_count;
            jobs[j].v.seg_cap = sc.pending_cap / kPendingSegments;
            jobs[j].v.pending_tag = (uint64_t)j << kBatchJobShift;
        }
    }
    mag_status s = grow(&b->d_jobs, &b->jobs_bytes, std::max<size_t>(njobs, 1) * sizeof(JobDesc), "job table");
    if (s != MAG_OK) return s;
    s = grow(&b->d_ranges, &b->ranges_bytes, ranges.size() * sizeof(uint64_t), "tile ranges");
    if (s != MAG_OK) return s;
    s = grow(&b->d_next, &b->next_bytes, std::max<size_t>(grid, 1) * sizeof(uint64_t), "tile claims");
    if (s != MAG_OK) return s;
    // the dense jobs carry the deferred-start fields set above
    for (size_t d = 0; d < djobs.size(); ++d) djobs[d].v = jobs[djob_of[d]].v;
    s = grow(&b->d_djobs, &b->djobs_bytes, std::max<size_t>(djobs.size(), 1) * sizeof(JobDesc), "dense job table");
    if (s != MAG_OK) return s;
    s = grow(&b->d_dranges, &b->dranges_bytes, dranges.size() * sizeof(uint64_t), "dense tile ranges");
    if (s != MAG_OK) return s;
    s = grow(&b->d_dnext, &b->dnext_bytes, std::max<size_t>(dgrid, 1) * sizeof(uint64_t), "dense tile claims");
    if (s != MAG_OK) return s;
    s = grow(&b->d_jbase, &b->jbase_bytes, jbase.size() * sizeof(uint64_t), "job text offsets");
    if (s != MAG_OK) return s;
    if (njobs) e = hipMemcpy(b->d_jobs, jobs.data(), njobs * sizeof(JobDesc), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_jbase, jbase.data(), jbase.size() * sizeof(uint64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_ranges, ranges.data(), ranges.size() * sizeof(uint64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess && !djobs.empty())
        e = hipMemcpy(b->d_djobs, djobs.data(), djobs.size() * sizeof(JobDesc), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_dranges, dranges.data(), dranges.size() * sizeof(uint64_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "upload of the job table");
    b->ndense = (uint32_t)djobs.size();
    b->dense_tiles = dense_tiles;
    b->dense_grid = (uint32_t)dgrid;
    b->cap = out_cap;
    b->idbits = idbits;
    b->posbits = posbits;
    b->nbits = idbits + posbits;
    b->total_tiles = total_tiles;
    b->grid = (uint32_t)grid;
    b->bound_words = wpl;
    b->bound = true;
    return MAG_OK;
}

mag_status mag_batch_set_words_per_lane(mag_batch *b, int32_t words_per_lane) {
    if (!b) return fail(MAG_E_INVALID, "batch is NULL");
    if (words_per_lane != 8 && words_per_lane != 16)
        return fail(MAG_E_INVALID, "words_per_lane must be 8 or 16");
    std::lock_guard<std::mutex> lock(b->mtx);
    b->words_per_lane = words_per_lane;
    return MAG_OK;
}

mag_status mag_batch_run_async(mag_batch *b, mag_match *d_out, uint64_t *d_offsets,
                               uint64_t *d_count, void *stream_) {
    if (!b) return fail(MAG_E_INVALID, "batch is NULL");
    if (!d_offsets || !d_count) return fail(MAG_E_INVALID, "d_offsets or d_count is NULL");
    std::lock_guard<std::mutex> lock(b->mtx);
    if (!b->bound) return fail(MAG_E_INVALID, "batch has no bound texts");
    if (b->cap && !d_out) return fail(MAG_E_INVALID, "d_out is NULL");
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    const uint32_t njobs = (uint32_t)b->plans.size();
    Scratch &sc = b->sc;
    const uint64_t posmask = (1ull << b->posbits) - 1ull;
    // batched plans have equal-length patterns: no pass over the id bits
    const int lo = sort_low_bit(false, b->idbits);
    uint64_t *sorted = sorted_keys(sc, b->cap, b->nbits, lo);

    BatchLaunch bl;
    bl.jobs = b->d_jobs;
    bl.njobs = njobs;
    bl.ranges = b->d_ranges;
    bl.next = b->d_next;
    bl.grid = b->grid;
    bl.total_tiles = b->total_tiles;
    bl.counters = sc.counters;
    bl.words_per_lane = (uint32_t)b->bound_words;
    BatchLaunch dl = bl;
    dl.jobs = b->d_djobs;
    dl.njobs = b->ndense;
    dl.ranges = b->d_dranges;
    dl.next = b->d_dnext;
    dl.grid = b->dense_grid;
    dl.total_tiles = b->dense_tiles;
    ProfileMarks prof;
    mag_status s = profile_start(prof, stream);
    if (s == MAG_OK) s = launch_batch(bl, stream);
    if (s == MAG_OK) s = launch_batch_dense(dl, stream);
    profile_mark(prof, stream);
    if (s == MAG_OK && b->defer)
        s = launch_batch_verify(b->d_jobs, sc.pending, sc.seg_count, sc.pending_cap / kPendingSegments,
                                stream);
    if (s == MAG_OK)
        s = launch_finish(sc, b->cap, 0, d_count, nullptr, StatsInfo{}, d_out, b->idbits, posmask, sorted,
                          stream);
    if (s == MAG_OK && b->cap > small_sort_max()) {
        s = launch_radix_sort(sc, b->cap, b->cap, b->nbits, lo, stream);
        if (s == MAG_OK)
            s = launch_expand(sc, b->cap, b->cap, b->nbits, lo, d_out, b->idbits, posmask, stream, b->d_jbase,
                              njobs);
    }
    // per-job offsets of the sorted keys (and the positions of records the
    // finishing kernel wrote made relative to their jobs' texts)
    if (s == MAG_OK)
        s = launch_batch_offsets(sorted, sc.counters + kSortCountSlot, b->cap, d_offsets, njobs, b->d_jbase,
                                 b->idbits, d_out, stream);
    profile_commit(prof, stream);
    return s;
}

mag_status mag_scan_batch(const mag_job *jobs, uint32_t njobs, mag_match *d_out, uint64_t out_cap,
                          uint64_t *offsets, void *stream_) {
    if (!jobs || !offsets) return fail(MAG_E_INVALID, "jobs or offsets is NULL");
    if (out_cap && !d_out) return fail(MAG_E_INVALID, "d_out is NULL");
    if (njobs == 0) {
        offsets[0] = 0;
        return MAG_OK;
    }
    std::vector<mag_plan *> plans(njobs);
    std::vector<const uint8_t *> texts(njobs);
    std::vector<uint64_t> n(njobs);
    for (uint32_t j = 0; j < njobs; ++j) {
        if (!jobs[j].plan) return fail(MAG_E_INVALID, "a job's plan is NULL");
        if (jobs[j].n && !jobs[j].d_text) return fail(MAG_E_INVALID, "a job's text is NULL");
        plans[j] = jobs[j].plan;
        texts[j] = jobs[j].d_text;
        n[j] = jobs[j].n;
    }
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    mag_batch *b = nullptr;
    mag_status s = mag_batch_create(plans.data(), njobs, &b);
    if (s != MAG_OK) return s;
    uint64_t *d_tmp = nullptr;     // the job offsets and the total, then the count
    s = mag_batch_bind(b, texts.data(), n.data(), out_cap, stream_);
    if (s == MAG_OK) {
        const hipError_t e = hipMalloc(&d_tmp, ((size_t)njobs + 2) * sizeof(uint64_t));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            d_tmp = nullptr;
            s = fail(MAG_E_NOMEM, "device allocation of the batch offsets failed");
        }
    }
    if (s == MAG_OK) s = mag_batch_run_async(b, d_out, d_tmp, d_tmp + njobs + 1, stream_);
    if (s == MAG_OK) {
        hipError_t e = hipMemcpyAsync(offsets, d_tmp, ((size_t)njobs + 1) * sizeof(uint64_t),
                                      hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) s = hip_fail(e, "reading the batch offsets");
    } else if (d_tmp) {
        (void)hipStreamSynchronize(stream);    // nothing of ours may still use the buffers
    }
    if (d_tmp) (void)hipFree(d_tmp);
    mag_batch_destroy(b);
    if (s == MAG_OK && offsets[njobs] > out_cap)
        s = fail(MAG_E_OVERFLOW, "the jobs have more occurrences than out_cap");
    return s;
}

}  // extern "C"
