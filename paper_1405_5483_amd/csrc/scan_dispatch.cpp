// Host side of the scan launch: tile sizing and the choice among the per-q
// kernel objects (scan.hip compiled once per q).
#include "dense.hpp"
#include "mag_internal.hpp"
#include "scan_args.hpp"

namespace mag {

namespace {

constexpr uint64_t kTableLdsMax = 64 * 1024;   // mask tables up to this size are staged in LDS
#ifndef MAG_SCAN_TILE_BYTES
#define MAG_SCAN_TILE_BYTES (32 * 1024)
#endif
constexpr uint32_t kEntryBytesPerTile = MAG_SCAN_TILE_BYTES;   // one of the two mask-entry buffers

int compute_units() { return device_compute_units(); }

}  // namespace

int device_compute_units() {
    static int ncu = 0;
    if (ncu) return ncu;
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    ncu = v;
    return ncu;
}

VerifyArgs make_verify_args(const mag_plan *p, const ScanLaunch &s) {
    VerifyArgs v{};
    const uintptr_t t = reinterpret_cast<uintptr_t>(s.text);
    v.tbase = reinterpret_cast<const uint8_t *>(t & ~(uintptr_t)15);
    v.delta = t & 15;
    v.last_word = s.n ? ((v.delta + s.n - 1) & ~3ull) : 0;
    v.m = p->m;
    v.mw = p->mw;
    v.hw = p->mw < (uint32_t)kHashWords ? p->mw : (uint32_t)kHashWords;
    v.lastmask = (p->m & 3) ? ((1u << (8 * (p->m & 3))) - 1u) : 0xFFFFFFFFu;
    v.slot_shift = 32 - p->slot_bits;
    v.slot_mask = (uint32_t)((1ull << p->slot_bits) - 1);
    v.idbits = (uint32_t)s.idbits;
    v.slots = p->dev.slots;
    v.pwords = p->dev.pwords;
    v.idstart = p->dev.idstart;
    v.ids = p->dev.ids;
    v.keys = s.keys;
    v.cap = s.cap;
    v.counters = s.counters;
    v.pending = s.pending;
    v.seg_count = s.seg_count;
    v.seg_cap = s.pending_cap / kPendingSegments;
    v.n = s.n;
    v.var = (uint32_t)p->var;
    v.pwoff = p->dev.pwoff;
    v.plen = p->dev.plen;
    v.gstart = p->dev.gstart;
    v.wfilter = p->dev.wfilter;
    v.wf_shift = p->wf_bits ? 32u - (uint32_t)p->wf_bits : 0u;
    return v;
}

int encoded_code_bytes(const mag_plan *p) { return p->n_codes <= 65536 ? 2 : 4; }

namespace {
// 24-bit Horner steps are exact when every partial code stays below 2^24
bool horner_mul24(const mag_plan *p) {
    uint64_t partial = 1;
    for (int t = 0; t + 1 < p->q; ++t) partial *= (uint64_t)p->sigma_prime;
    return partial < (1ull << 24);
}
}  // namespace

mag_status launch_encode(const mag_plan *p, const uint8_t *text, uint64_t n, void *codes, int csz,
                         hipStream_t stream) {
    if (n < (uint64_t)p->q) return MAG_OK;
    EncodeArgs e{};
    const uintptr_t t = reinterpret_cast<uintptr_t>(text);
    e.tbase = reinterpret_cast<const uint8_t *>(t & ~(uintptr_t)15);
    e.delta = t & 15;
    e.n = n;
    e.G = (n - p->q) / p->q + 1;
    e.codes = codes;
    e.mu = p->dev.mu;
    e.sp = (uint32_t)p->sigma_prime;
    if (p->map_kind == MAG_MAP_QGRAM) {
        e.qgram = 1;
        e.blen = (uint32_t)p->qbits;
    } else if (p->map_kind == MAG_MAP_BITS && p->sigma_prime > 1) {
        e.bshift = (uint32_t)p->bits_shift;
        uint32_t l = 0;
        while ((1 << l) < p->sigma_prime) ++l;
        e.blen = l;
    }
    const bool mul24 = horner_mul24(p);
    switch (p->q) {
        case 1: return launch_encode_q1(e, csz, mul24, stream);
        case 2: return launch_encode_q2(e, csz, mul24, stream);
        case 3: return launch_encode_q3(e, csz, mul24, stream);
        case 4: return launch_encode_q4(e, csz, mul24, stream);
        case 5: return launch_encode_q5(e, csz, mul24, stream);
        case 6: return launch_encode_q6(e, csz, mul24, stream);
        case 7: return launch_encode_q7(e, csz, mul24, stream);
        case 8: return launch_encode_q8(e, csz, mul24, stream);
        default: return fail(MAG_E_UNSUPPORTED, "q outside [1, 8]");
    }
}

int dense_lane_positions(const mag_plan *p, uint64_t positions, int ncu) {
    if (p->words_per_lane > 0) return p->words_per_lane >= 24 ? 32 : 16;
    if (p->chunk_bytes > 0) return p->chunk_bytes >= slice_scan_tile(24) ? 32 : 16;
    // 32 halves the per-tile work per position (measured on the 1 GiB protein
    // scan: 0.522 against 0.574 ms) wherever the larger tiles still give
    // every compute unit at least two
    return positions >= 2ull * (uint64_t)(ncu > 0 ? ncu : 256) * (uint64_t)slice_scan_tile(32) ? 32 : 16;
}

mag_status launch_scan(const mag_plan *p, const ScanLaunch &s, hipStream_t stream) {
    if (s.n < (uint64_t)p->q || p->r == 0) return MAG_OK;
    const int ncu = compute_units();
    if (ncu < 1) return fail(MAG_E_DEVICE, "cannot query the compute unit count");
    ScanArgs a{};
    const uintptr_t t = reinterpret_cast<uintptr_t>(s.text);
    a.tbase = reinterpret_cast<const uint8_t *>(t & ~(uintptr_t)15);
    a.delta = t & 15;
    a.n = s.n;
    a.k = p->k;
    a.kq = p->k * p->q;
    a.mprime = p->mprime;
    a.W = p->W;
    a.sp = p->sigma_prime;
    a.m = p->m;
    a.X = (s.n - p->q) / a.kq + 1;
    a.src_bytes = s.n;
    a.stride = a.kq;
    if (s.codes) {
        // SMAG: phase A reads sample x's code at entry x*k of the encoded text
        a.tbase = static_cast<const uint8_t *>(s.codes);
        a.delta = 0;
        a.src_bytes = ((s.n - p->q) / p->q + 1) * (uint64_t)s.csz;
        a.stride = p->k * (uint32_t)s.csz;
        a.pre = (uint32_t)s.csz;
        a.maxcode = (uint32_t)(p->n_codes - 1);
    }

    const uint32_t esz = (uint32_t)p->esz;
    const uint32_t epv = 16 / esz;                      // entries per 16-byte LDS read
    // lane runs start on 16-byte vector boundaries: S is a multiple of epv
    uint32_t S = kEntryBytesPerTile / (kScanConsumerLanes * esz) / epv * epv;
    if (p->words_per_lane > 0 || p->chunk_bytes > 0) {
        // the plan's tile shape: entries per lane, or text bytes per tile
        // (256 lanes of kq bytes per entry), within the LDS left beside the
        // mask table (two entry buffers)
        S = p->words_per_lane > 0 ? (uint32_t)p->words_per_lane
                                  : (uint32_t)((uint64_t)p->chunk_bytes / ((uint64_t)kScanConsumerLanes * a.kq));
        const uint64_t tab = p->table.size() <= kTableLdsMax ? p->table.size() : 0;
        const uint64_t room = (kScanLdsMax - kScanStaticLds - 256 - (kScanConsumerLanes / 64) * 128 * 8 - tab) / 2;
        const uint64_t cap = (room - 128 * esz) / esz / kScanConsumerLanes;   // w0 + 16 <= 80 entries
        if (S > cap) S = (uint32_t)cap;
        S = S / epv * epv;
        if (S < epv) S = epv;
    } else {
        if (S < epv) S = epv;
        // small texts: shorter lane runs so that every compute unit gets tiles
        while (S > epv && (a.X + (uint64_t)kScanConsumerLanes * S - 1) /
                                  ((uint64_t)kScanConsumerLanes * S) < 2ull * (uint64_t)ncu)
            S -= epv;
    }
    a.S = S;
    a.tile_samples = kScanConsumerLanes * S;
    a.ntiles = (a.X + a.tile_samples - 1) / a.tile_samples;
    const uint32_t warm = p->mprime - 1;
    const uint32_t align = epv > 8 ? epv : 8;          // phase A writes groups of up to 8 entries
    a.w0 = (warm + align - 1) / align * align;
    // entries 0 .. TS+w0-1 are read; phase A's last group ends at most 7
    // entries past them
    a.e_lds = (uint32_t)((((uint64_t)a.tile_samples + a.w0 + 16) * esz + 15) & ~15ull);

    if (p->map_kind == MAG_MAP_BITS && p->sigma_prime > 1) {
        a.bshift = (uint32_t)p->bits_shift;
        uint32_t l = 0;
        while ((1 << l) < p->sigma_prime) ++l;
        a.blen = l;
    }
    if (p->map_kind == MAG_MAP_QGRAM) {
        a.qgram = 1;
        a.blen = (uint32_t)p->qbits;
        a.pbits = p->entry_bits < 8 ? (uint32_t)p->entry_bits : 0u;
    }
    a.mu = p->dev.mu;
    a.table = p->dev.table;
    a.counters = s.counters;
    a.v = make_verify_args(p, s);

    const uint64_t tbytes = p->table.size();
    const bool tlds = tbytes <= kTableLdsMax;
    a.table_vec = (uint32_t)((tbytes + 15) / 16);
    const size_t shmem = 256 + (size_t)(kScanConsumerLanes / 64) * 128 * 8 + 2 * (size_t)a.e_lds +
                         (tlds ? (size_t)a.table_vec * 16 : 0);
    const bool wide = p->W > 32 || p->k >= 32;
    const bool mul24 = horner_mul24(p);
    switch (p->q) {
        case 1: return launch_scan_q1(a, p->esz, wide, tlds, mul24, shmem, ncu, stream);
        case 2: return launch_scan_q2(a, p->esz, wide, tlds, mul24, shmem, ncu, stream);
        case 3: return launch_scan_q3(a, p->esz, wide, tlds, mul24, shmem, ncu, stream);
        case 4: return launch_scan_q4(a, p->esz, wide, tlds, mul24, shmem, ncu, stream);
        case 5: return launch_scan_q5(a, p->esz, wide, tlds, mul24, shmem, ncu, stream);
        case 6: return launch_scan_q6(a, p->esz, wide, tlds, mul24, shmem, ncu, stream);
        case 7: return launch_scan_q7(a, p->esz, wide, tlds, mul24, shmem, ncu, stream);
        case 8: return launch_scan_q8(a, p->esz, wide, tlds, mul24, shmem, ncu, stream);
        default: return fail(MAG_E_UNSUPPORTED, "q outside [1, 8]");
    }
}

}  // namespace mag
