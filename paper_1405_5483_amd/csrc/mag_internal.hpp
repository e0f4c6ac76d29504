// Internal declarations of the MAG library: the plan, the verification hash
// (shared by the host builder and the device kernels) and the kernel launch
// entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/mag.h"

namespace mag {

constexpr int kMaxM = 64;           // longest pattern the library verifies
constexpr int kMaxQ = 8;            // longest q-gram
constexpr int kMaxW = 64;           // automaton bits
constexpr int kMaxK = 32;           // candidate mask of one window fits 32 bits
constexpr uint32_t kCodeDirect = 1u << 31;   // code_ids entry holding a pattern id (ids < 2^31)
constexpr uint64_t kMaxTableBytes = 1ull << 30;
constexpr int kDefaultTableBudget = 96 * 1024;
// alphabet mapping on q-grams: sigma' = 2^b codes with b <= 28; the heuristic
// aims at kQgramLoad codes per distinct gram of the fullest class within
// kQgramTableBudget bytes of table
constexpr int kMaxQgramLog2 = 28;
constexpr int kQgramTableBudget = 8 << 20;
constexpr int kQgramLoad = 32;
// filter scans expected to verify at least this many start positions defer
// them to the verification kernel (measured: below it, and for the dense
// mode, whose verification overlaps its ALU-bound position tests, inline
// verification is as fast or faster)
constexpr double kDeferMinVerifications = 1 << 24;
constexpr uint64_t kPendingMax = 1ull << 26;
constexpr uint32_t kPendingSegments = 256;   // deferred-start buffer segments, one counter each
// A scan whose grid covers less than half the compute units also defers when
// each of its verifying waves would face at least this many starts: inline,
// those few waves would verify them one queue after another.
constexpr double kDeferPerWave = 64;
constexpr uint64_t kSmallGridTileSamples = 4096;   // filter tile size of short texts
constexpr int kHashWords = 4;       // the verification hash reads the first 16 bytes
// Scratch counters: [0] occurrences [1] candidate windows [2] verifications,
// [4] and [8..11] the count and stats that mag_scan reads back, and
// [kSortCountSlot] the count that the device-wide sort reads, and
// [kFinishDoneSlot] the finishing workgroups that have read the counters.
constexpr int kSortCountSlot = 12;
constexpr int kFinishDoneSlot = 13;
constexpr int kStatsSlot = 16;          // mag_scan's mag_stats (7 words)
constexpr int kCounterWords = 32;       // counter words of a scan's scratch

// The plan fields a scan's finishing kernel writes into mag_stats.
struct StatsInfo {
    int32_t q = 0, k = 0, sigma_prime = 0, m_prime = 0;
    float plan_ms = 0.0f;
};

// Fingerprint of the first min(m, 16) bytes of a pattern or text window, given
// as little-endian 32-bit words with bytes past m zeroed. It only has to spread
// keys over the probe table; equality is decided by a full compare. It is a
// multiply / xor-shift mix in the style of MurmurHash3's 32-bit finalizer
// (fmix32) and uses that finalizer's two multipliers, 0x85EBCA6B and
// 0xC2B2AE35: one multiply and xor-shift per word, then fmix32's last three
// steps.
__host__ __device__ inline uint32_t window_hash(const uint32_t *w, int nwords) {
    uint32_t h = 0x9E3779B9u;
    for (int t = 0; t < nwords; ++t) {
        h ^= w[t];
        h *= 0x85EBCA6Bu;
        h ^= h >> 15;
    }
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

// Dense mode (every start position tested): a Bloom bitmap of 2^B bits over
// the same first min(m, 16) bytes, kBloomBits bits per distinct pattern
// (bloom_bit of bloom_probe of the hash). B grows with the number of
// distinct patterns; batched scans use a copy with at most kBloomBatchLog2
// bits, built from the same hashes.
#ifndef MAG_BLOOM_BITS
#define MAG_BLOOM_BITS 3
#endif
constexpr int kBloomBits = MAG_BLOOM_BITS;
constexpr int kBloomMinLog2 = 12;
constexpr int kBloomMaxLog2 = 20;
constexpr int kBloomBatchLog2 = 18;
// MAG_MODE_AUTO scans densely when the filter is expected to verify at least
// this many start positions per text byte.
constexpr double kDenseVerifPerByte = 0.1;
// A learned pick with sigma' = 2^l switches to the bit-field map when that
// map's expected verifications per byte are at most 1.25x the greedy map's
// plus this.
constexpr double kLearnedBitsSlack = 1e-5;

__host__ __device__ inline uint32_t prefilter_hash(const uint32_t *w, int nwords) {
    uint32_t x = w[0];
    if (nwords > 1) x ^= (w[1] << 7) | (w[1] >> 25);
    if (nwords > 2) x ^= (w[2] << 14) | (w[2] >> 18);
    if (nwords > 3) x ^= (w[3] << 21) | (w[3] >> 11);
    return x * 0x9E3779B1u;
}

// prefilter_hash(w, 4) on the device: the same value, with its first three
// terms in one 3-input XOR (v_bitop3, truth table 0x96).
__device__ inline uint32_t prefilter_hash4(const uint32_t *w) {
    const uint32_t x = __builtin_amdgcn_bitop3_b32(w[0], (w[1] << 7) | (w[1] >> 25),
                                                   (w[2] << 14) | (w[2] >> 18), 0x96);
    return (x ^ ((w[3] << 21) | (w[3] >> 11))) * 0x9E3779B1u;
}

// Bloom probe j of a hash: g = h ^ (h >> 16) rotated left by 11j. g folds
// the well-mixed high half of the product into its low half, so the
// rotations stay independent on low-entropy texts (DNA); a few ALU ops
// replace a multiplicative remix per probe. A probe p of a 2^B-bit bitmap
// names bit p & 31 of 32-bit word p >> (37 - B) (bloom_bit): the low five
// bits serve as the shift count as they are.
__host__ __device__ inline uint32_t bloom_probe(uint32_t h, int j) {
    const uint32_t g = h ^ (h >> 16);
    const uint32_t r = (uint32_t)(11 * j) & 31u;
    return r ? (g << r) | (g >> (32u - r)) : g;
}
__host__ __device__ inline uint32_t bloom_bit(uint32_t p, int B) {
    return ((p >> (37 - B)) << 5) | (p & 31u);
}

// Dense mode with one bitmap probe per start position (the "sliced" bitmap):
// each distinct pattern sets one bit for each of its first k 6-byte slices at
// offsets 0, 2, .., 2(k-1), and a start position passes when the bits of its
// own slices at those offsets are all set. Consecutive positions share their
// probes (position x's slice at offset 2j is position x+2j's slice at offset
// 0), so a scan reads one bitmap word per position whatever k is. The slice
// hash sums two 24-bit products, one per half of the slice (bytes o..o+2 and
// o+3..o+5, little-endian), so it maps to full-rate 24-bit multiplies on the
// device; the multipliers are the top 24 bits of the 32-bit golden-ratio
// constant 0x9E3779B9 (Knuth's multiplicative hashing) and of MurmurHash3's
// finalizer multiplier 0x85EBCA6B, made odd. A slice hash h names bit
// (h >> (32 - B)) & 31 of 32-bit word h >> (37 - B) of a 2^B-bit bitmap.
constexpr uint32_t kSliceK1 = 0x9E3779u;
constexpr uint32_t kSliceK2 = 0x85EBCBu;
constexpr int kSliceBytes = 6;
constexpr int kSliceStride = 2;
constexpr int kSliceMaxK = 8;
__host__ __device__ inline uint32_t slice_hash(uint32_t lo, uint32_t hi) {
    return (hi & 0xFFFFFFu) * kSliceK2 + (lo & 0xFFFFFFu) * kSliceK1;
}

// Word filter in front of the probe slots of the one-probe dense mode: a
// blocked Bloom filter of 2^F 64-bit words over the distinct patterns' window
// hashes h (window_hash). Pattern h sets, in word h >> (32 - F), the bits
// word_filter_mask(h): kWordFilterBits 6-bit fields of h times the 32-bit
// golden-ratio constant. A start whose hash fails it matches no pattern, so
// its verification costs one 8-byte load instead of a walk over the slots.
constexpr int kWordFilterBits = 5;
__host__ __device__ inline uint64_t word_filter_mask(uint32_t h) {
    const uint32_t x = h * 0x9E3779B1u;
    uint64_t m = 0;
    for (int j = 0; j < kWordFilterBits; ++j) m |= 1ull << ((x >> (6 * j)) & 63u);
    return m;
}

// Everything a scan needs on the device. Plain pointers into one allocation.
struct DeviceTables {
    uint8_t *base = nullptr;        // the single allocation
    const uint8_t *mu = nullptr;    // 256 B
    const void *table = nullptr;    // n_codes * entry_bytes
    const uint64_t *slots = nullptr;   // 2^slot_bits probe slots: (hash << 32) | (u + 1)
    const uint32_t *pwords = nullptr;  // n_unique * mw words
    const uint32_t *idstart = nullptr; // n_unique + 1
    const uint32_t *ids = nullptr;     // r
    const uint32_t *bloom = nullptr;   // 2^bloom_log2 bits
    const uint32_t *bloom_batch = nullptr;  // 2^min(bloom_log2, kBloomBatchLog2) bits
    const uint32_t *slices = nullptr;  // 2^bloom_log2 bits of the one-probe dense mode
    const uint32_t *code_bits = nullptr;  // exact codes (build_codes)
    const uint32_t *code_ids = nullptr;
    const uint64_t *wfilter = nullptr; // 2^wf_bits words: the word filter (one-probe dense mode)
    const uint32_t *pwoff = nullptr;   // unequal lengths: word offset of each distinct pattern
    const uint32_t *plen = nullptr;    //   its length
    const uint32_t *gstart = nullptr;  //   first distinct pattern of each prefix group (+ end)
};

struct Scratch {
    int device = -1;
    uint64_t *counters = nullptr;   // 16 words, see kSortCountSlot
    uint64_t *keys = nullptr;       // two key buffers of keys_cap entries each
    uint64_t keys_cap = 0;
    uint32_t *hist = nullptr;       // device-wide radix sort: digit counts [256][chunks]
    uint64_t *radix_off = nullptr;  // their start offsets [256][chunks], then 256 digit totals
    uint64_t radix_chunks = 0;
    uint64_t *pending = nullptr;    // start positions deferred to the verification kernel
    uint64_t pending_cap = 0;
    uint64_t *seg_count = nullptr;  // kPendingSegments counters (cleared by the finishing kernel)
    void *codes = nullptr;          // SMAG: the encoded text
    uint64_t codes_bytes = 0;
};

}  // namespace mag

struct mag_plan {
    // pattern set
    uint32_t r = 0, m = 0, mw = 0;
    std::vector<uint8_t> patterns;

    // filter parameters
    int q = 1, k = 1, sigma_prime = 1, L = 0, mprime = 0, W = 0, esz = 1;
    int q_formula = 0;               // Section 3.2's q for this pattern set, before kMaxQ
    int map_kind = MAG_MAP_GREEDY, select = MAG_SELECT_HEURISTIC;
    int bits_shift = 0;              // s of the bit-field map
    int qbits = 0;                   // log2 sigma' of the q-gram map
    int entry_bits = 8;              // stored bits per table entry (1, 2, 4: packed)
    uint8_t mu[256] = {0};
    uint64_t n_codes = 0;
    std::vector<uint8_t> table;      // n_codes * esz bytes, or packed entries

    // verification set: distinct patterns, their ids, and a probe table
    uint32_t n_unique = 0, slot_bits = 1;
    std::vector<uint32_t> pwords, idstart, ids;
    std::vector<uint64_t> slots;

    // dense mode: test every start position against the Bloom bitmaps
    int mode = MAG_MODE_AUTO, dense = 0, bloom_log2 = mag::kBloomMinLog2;
    double est_verif = 0.0;          // estimated verifications per text byte of the filter
    double bloom_fp = 0.0;           // estimated share of start positions the Bloom bitmap passes
    int verify = MAG_VERIFY_AUTO;    // inline or deferred verification
    int encode = 0;                  // 1: SMAG, the text is encoded before the search
    // unequal lengths: m is the shortest length and the filter sees every
    // pattern's first m bytes; verification uses the full patterns
    int var = 0;
    uint32_t m_max = 0;
    std::vector<uint8_t> fbytes;     // the full patterns, concatenated
    std::vector<uint64_t> foff;      // r + 1 offsets into fbytes
    std::vector<uint32_t> pwoff, plen, gstart;
    uint64_t verify_buffer = 0;      // deferred-start buffer entries (0: sized per scan)
    std::vector<uint32_t> bloom, bloom_batch;
    // exact codes of the batched dense scans (build_codes): when the pattern
    // bytes are at most four and a 2-bit field (b >> code_shift) & 3 tells
    // them apart, and 2m <= 16, a window's code (field t at bits 2t) is exact
    // for windows of pattern bytes; code_bits has bit c set when code c is a
    // distinct pattern's, code_ids[c] is that pattern's id | kCodeDirect when
    // it has one id, else its index + 1, and code_rep holds the byte of each
    // code (another code's byte for unused ones), so that a window byte b is
    // a pattern byte iff rep[(b >> code_shift) & 3] == b.
    int code_shift = -1;             // -1: no exact codes
    uint32_t code_rep = 0;
    std::vector<uint32_t> code_bits, code_ids;
    // one-probe dense mode: slice_k slices per distinct pattern in a bitmap of
    // 2^bloom_log2 bits (slice_k = 0: the dense mode uses the Bloom bitmap)
    int dense_probe = MAG_DENSE_PROBE_AUTO;
    float plan_ms = 0.0f;            // host time of mag_plan_create
    // tile shape asked for at creation (0 = auto): text bytes per tile, or
    // entries (samples, start positions) per lane (filter_lane_entries and
    // dense_lane_positions resolve them)
    int chunk_bytes = 0, words_per_lane = 0;
    int slice_k = 0;
    double slice_fp = 0.0;           // estimated share of start positions it passes
    std::vector<uint32_t> slices;
    int wf_bits = 0;                 // log2 words of the word filter (0: none)
    std::vector<uint64_t> wfilter;

    // device side
    std::mutex mtx;
    int device = -1;
    mag::DeviceTables dev;
    mag::Scratch scratch;
};

namespace mag {

// Benchmark timing (capi.cpp): while mag_profile_enable is on and `stream` is
// not being captured, profile_start records an event before a scan's first
// kernel, profile_mark(1) one after its scan kernel and profile_commit one
// after its last kernel and keeps the record for mag_profile_read.
struct ProfileMarks {
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    bool on = false;
};
mag_status profile_start(ProfileMarks &pm, hipStream_t stream);
void profile_mark(ProfileMarks &pm, hipStream_t stream);
void profile_commit(ProfileMarks &pm, hipStream_t stream);

// Positions per lane of the one-probe dense kernel (16 or 32) for a plan's
// chunk_bytes / words_per_lane, or by default for a scan of `positions`
// start positions on `ncu` compute units (scan_dispatch.cpp).
int dense_lane_positions(const mag_plan *p, uint64_t positions, int ncu);

// Thread-local error text (capi.cpp).
mag_status fail(mag_status s, const std::string &msg);
mag_status hip_fail(hipError_t e, const char *what);

// Uploads the plan's tables and scratch counters to the current device on
// first use; fails if the plan lives on another device (capi.cpp).
mag_status ensure_device(mag_plan *p);

// q by Section 3.2's formula: log base max(sigma, 2) of r*m, rounded half
// up, clamped to [1, (m+1)/2] (at least one gram position).
int heuristic_q_formula(int sigma, uint32_t r, uint32_t m);
// q of the fixed heuristic as the library runs it: the formula's q, at most
// kMaxQ (the longest gram the scan kernels are built for).
int heuristic_q(int sigma, uint32_t r, uint32_t m);

// Verifications per text byte the filter of a built plan is expected to make,
// from the class densities its mask table gives under the pattern-set byte
// frequencies (plan.cpp); -1 when the table is too large to evaluate.
double estimate_verifications(const mag_plan *p);

// Host plan builder (plan.cpp).
mag_status build_plan(mag_plan *p, const uint8_t *patterns, uint32_t r, uint32_t m,
                      const mag_params *params);
// Patterns of unequal lengths: bytes[offsets[i] .. offsets[i+1]) is pattern i.
mag_status build_plan_var(mag_plan *p, const uint8_t *bytes, const uint64_t *offsets, uint32_t r,
                          const mag_params *params);

// Kernel launches (scan.hip, sort.hip).
struct VerifyArgs;
struct ScanLaunch {
    const uint8_t *text = nullptr;
    uint64_t n = 0;
    uint64_t *keys = nullptr;      // key output, capacity cap
    uint64_t cap = 0;
    uint64_t *counters = nullptr;  // [0] occurrences [1] candidate windows [2] verifications
                                   // [3] deferred starts
    int idbits = 0;
    uint64_t *pending = nullptr;   // deferred start positions (NULL: verify inline)
    uint64_t pending_cap = 0;      // entries, split into kPendingSegments segments
    uint64_t *seg_count = nullptr;
    const void *codes = nullptr;   // SMAG: the encoded text (NULL: codes on the fly)
    int csz = 0;                   // bytes per encoded code (2 or 4)
};
mag_status launch_scan(const mag_plan *p, const ScanLaunch &s, hipStream_t stream);
// SMAG: writes the code of every complete non-overlapping q-gram of
// text[0..n) to codes, csz (2 or 4) bytes each (scan_dispatch.cpp).
mag_status launch_encode(const mag_plan *p, const uint8_t *text, uint64_t n, void *codes, int csz,
                         hipStream_t stream);
// Bytes per encoded code of a plan: 2 when every code fits 16 bits, else 4.
int encoded_code_bytes(const mag_plan *p);
// Resident workgroups per compute unit of kernel `fn` at `threads` threads
// and `shmem` bytes of dynamic LDS, queried once per (kernel, threads, size)
// and then served from a cache (capi.cpp); 0 after an error (detail in the
// thread's last error).
int cached_occupancy(const void *fn, int threads, size_t shmem);
// Compute units of the current device, queried once (scan_dispatch.cpp); 0
// after an error.
int device_compute_units();
// Streaming-read reference (stream.hip): reads d[0..n) once; sink needs
// stream_read_grid() words.
mag_status launch_stream_read(const uint8_t *d, uint64_t n, uint32_t *sink, hipStream_t stream);
uint32_t stream_read_grid();
// Verifies the start positions a filter kernel deferred to v.pending
// (segment counts in v.seg_count) with a full-occupancy grid (verify.hip).
mag_status launch_verify(const VerifyArgs &v, hipStream_t stream);
mag_status launch_fill_u64(uint64_t *ptr, uint64_t count, uint64_t value, hipStream_t stream);
// Occurrence counts up to this many are sorted inside the finishing kernel.
uint32_t small_sort_max();
// Publishes the count (and the stats if d_stats), leaves the count in
// counters[kSortCountSlot], returns the other counters to zero, and sorts
// outputs of up to small_sort_max() occurrences into `out` (and their keys
// into `sorted` if not null). Records hold ((key >> idbits) & posmask, key's
// low idbits).
mag_status launch_finish(Scratch &sc, uint64_t cap, uint64_t samples, uint64_t *d_count,
                         mag_stats *d_stats, const StatsInfo &info, mag_match *out, int idbits,
                         uint64_t posmask, uint64_t *sorted, hipStream_t stream);
// Device-wide radix sort of the keys for counts in (small_sort_max(), cap],
// with grids sized for counts up to `bound`: the scratch for `bound`, the
// passes over key bits lo .. nbits - 1, and the records. The passes are
// stable, so bits below lo keep the order in which the keys were written.
mag_status ensure_radix_scratch(Scratch &sc, uint64_t bound, hipStream_t stream);
// Chunks of the device-wide radix sort's counts for outputs of up to `bound`
// keys (its scratch: 256 * chunks u32 counts, 256 * chunks + 256 u64 offsets).
uint64_t radix_scratch_chunks(uint64_t bound);
// out (not null): the last pass writes the records ((key >> idbits) &
// posmask, the id bits) instead of the sorted keys, which then need no
// launch_expand (when radix_passes(nbits, lo) > 0).
mag_status launch_radix_sort(Scratch &sc, uint64_t bound, uint64_t cap, int nbits, int lo, hipStream_t stream,
                             mag_match *out = nullptr, int idbits = 0, uint64_t posmask = 0);
int radix_passes(int nbits, int lo);
// jbase (batches; njobs + 1 offsets): positions made relative to their jobs'
// texts (see k_expand).
mag_status launch_expand(Scratch &sc, uint64_t bound, uint64_t cap, int nbits, int lo, mag_match *out,
                         int idbits, uint64_t posmask, hipStream_t stream, const uint64_t *jbase = nullptr,
                         uint32_t njobs = 0);
// The job of position p of a batch's texts laid end to end: the last j <
// njobs with jb[j] <= p (jb: njobs + 1 ascending first bytes; njobs >= 1).
__host__ __device__ inline uint32_t job_of_position(const uint64_t *jb, uint32_t njobs, uint64_t p) {
    uint32_t lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) / 2;
        if (jb[mid] <= p) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}
// The key buffer that holds the sorted keys after the radix passes.
uint64_t *sorted_keys(Scratch &sc, uint64_t cap, int nbits, int lo);
// Lowest key bit the radix passes sort on. With equal-length patterns every
// start matches one distinct pattern, whose ids are written one after another
// in ascending order (id runs, emit_found), so the id bits need no pass; with
// unequal lengths several members of a prefix group can match one start, in
// member order, and the ids are sorted too.
inline int sort_low_bit(bool var, int idbits) { return var ? 0 : idbits; }

}  // namespace mag
