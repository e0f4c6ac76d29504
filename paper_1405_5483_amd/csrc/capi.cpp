// C ABI of the MAG library (declared in include/mag.h): plan life cycle,
// device upload, scratch management and the scan entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <string>
#include <vector>

#include "dense.hpp"
#include "mag_internal.hpp"
#include "scan_args.hpp"

namespace mag {

namespace {
thread_local std::string g_last_error;

// benchmark timing: events recorded around each scan's two kernels
struct ProfileRecord {
    hipEvent_t ev[3];   // before the scan, after the scan, after the finishing kernel
};
std::mutex g_prof_mtx;
bool g_prof_on = false;
std::vector<ProfileRecord> g_prof;

hipEvent_t make_event() {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

uint64_t round16(uint64_t v) { return (v + 15) & ~15ull; }

}  // namespace

mag_status profile_start(ProfileMarks &pm, hipStream_t stream) {
    pm = ProfileMarks{};
    {
        std::lock_guard<std::mutex> pl(g_prof_mtx);
        if (!g_prof_on) return MAG_OK;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return MAG_OK;
    }
    if (cs != hipStreamCaptureStatusNone) return MAG_OK;
    for (auto &ev : pm.ev) {
        ev = make_event();
        if (!ev) return fail(MAG_E_DEVICE, "hipEventCreate");
    }
    pm.on = true;
    (void)hipEventRecord(pm.ev[0], stream);
    return MAG_OK;
}

void profile_mark(ProfileMarks &pm, hipStream_t stream) {
    if (pm.on) (void)hipEventRecord(pm.ev[1], stream);
}

void profile_commit(ProfileMarks &pm, hipStream_t stream) {
    if (!pm.on) return;
    (void)hipEventRecord(pm.ev[2], stream);
    std::lock_guard<std::mutex> pl(g_prof_mtx);
    g_prof.push_back(ProfileRecord{{pm.ev[0], pm.ev[1], pm.ev[2]}});
    pm.on = false;
}

namespace {

int ceil_log2(uint64_t v) {
    int b = 0;
    while (b < 64 && (1ull << b) < v) ++b;
    return b;
}

// Grows the key buffers to hold 2 * cap keys. Waits for `stream` first so no
// earlier scan still uses the old buffer.
mag_status ensure_keys(mag_plan *p, uint64_t cap, hipStream_t stream) {
    Scratch &sc = p->scratch;
    if (sc.keys_cap >= cap && sc.keys) return MAG_OK;
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (sc.keys) {
        (void)hipFree(sc.keys);
        sc.keys = nullptr;
        sc.keys_cap = 0;
    }
    uint64_t want = cap < 1024 ? 1024 : cap;
    e = hipMalloc(&sc.keys, want * 2 * sizeof(uint64_t));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(MAG_E_NOMEM, "device allocation of sort keys failed");
    }
    sc.keys_cap = want;
    return MAG_OK;
}

// Pending-start buffer of at least `cap` entries (grown like the key buffers).
mag_status ensure_pending(mag_plan *p, uint64_t cap, hipStream_t stream) {
    Scratch &sc = p->scratch;
    if (sc.pending_cap >= cap && sc.pending) return MAG_OK;
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (sc.pending) {
        (void)hipFree(sc.pending);
        sc.pending = nullptr;
        sc.pending_cap = 0;
    }
    e = hipMalloc(&sc.pending, cap * sizeof(uint64_t));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(MAG_E_NOMEM, "device allocation of the deferred-start buffer failed");
    }
    sc.pending_cap = cap;
    if (!sc.seg_count) {
        // zero once here; afterwards the finishing kernel of every scan clears them
        e = hipMalloc(&sc.seg_count, kPendingSegments * sizeof(uint64_t));
        if (e == hipSuccess) e = hipMemsetAsync(sc.seg_count, 0, kPendingSegments * sizeof(uint64_t), stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "deferred-start counters");
    }
    return MAG_OK;
}

// Encoded-text buffer of at least `bytes` bytes (SMAG).
mag_status ensure_codes(mag_plan *p, uint64_t bytes, hipStream_t stream) {
    Scratch &sc = p->scratch;
    if (sc.codes_bytes >= bytes && sc.codes) return MAG_OK;
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (sc.codes) {
        (void)hipFree(sc.codes);
        sc.codes = nullptr;
        sc.codes_bytes = 0;
    }
    e = hipMalloc(&sc.codes, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(MAG_E_NOMEM, "device allocation of the encoded text failed");
    }
    sc.codes_bytes = bytes;
    return MAG_OK;
}

// Capacity of the deferred-start buffer for a scan expected to verify
// `expect` start positions, or 0 to verify inline.
uint64_t pending_capacity(double expect) {
    if (expect >= 0.0 && expect < (double)(1 << 20)) return 0;
    const double want = expect < 0.0 ? (double)(1ull << 24) : 2.0 * expect;
    uint64_t cap = 1ull << 20;
    while ((double)cap < want && cap < kPendingMax) cap <<= 1;
    return cap;
}

}  // namespace

int cached_occupancy(const void *fn, int threads, size_t shmem) {
    static std::mutex mtx;
    static std::map<std::tuple<const void *, int, size_t>, int> cache;
    const auto key = std::make_tuple(fn, threads, shmem);
    {
        std::lock_guard<std::mutex> lock(mtx);
        const auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    int occ = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, threads, shmem);
    if (e != hipSuccess) {
        hip_fail(e, "occupancy query");
        return 0;
    }
    std::lock_guard<std::mutex> lock(mtx);
    cache[key] = occ;
    return occ;
}

mag_status fail(mag_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

mag_status hip_fail(hipError_t e, const char *what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return MAG_E_DEVICE;
}

// Uploads the plan's tables to the current device on first use.
mag_status ensure_device(mag_plan *p) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (p->device >= 0) {
        if (p->device != dev)
            return fail(MAG_E_INVALID, "plan was uploaded to another device");
        return MAG_OK;
    }
    const uint64_t o_mu = 0;
    const uint64_t o_tab = 256;
    const uint64_t o_slots = round16(o_tab + round16(p->table.size()) + 16);
    const uint64_t o_pw = round16(o_slots + p->slots.size() * 8);
    const uint64_t o_ids0 = round16(o_pw + p->pwords.size() * 4 + 16);
    const uint64_t o_ids = round16(o_ids0 + p->idstart.size() * 4);
    const uint64_t o_bloom = round16(o_ids + p->ids.size() * 4 + 16);
    const uint64_t o_bloomb = round16(o_bloom + p->bloom.size() * 4);
    const uint64_t o_sl = round16(o_bloomb + p->bloom_batch.size() * 4 + 16);
    const uint64_t o_cb = round16(o_sl + p->slices.size() * 4 + 16);
    const uint64_t o_ci = round16(o_cb + p->code_bits.size() * 4);
    const uint64_t o_wf = round16(o_ci + p->code_ids.size() * 4 + 16);
    const uint64_t o_pwoff = round16(o_wf + p->wfilter.size() * 8 + 16);
    const uint64_t o_plen = round16(o_pwoff + p->pwoff.size() * 4);
    const uint64_t o_gstart = round16(o_plen + p->plen.size() * 4);
    const uint64_t total = round16(o_gstart + p->gstart.size() * 4 + 16);
    uint8_t *base = nullptr;
    e = hipMalloc(&base, total);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(MAG_E_NOMEM, "device allocation of plan tables failed");
    }
    std::string host(total, '\0');
    std::memcpy(&host[o_mu], p->mu, 256);
    if (!p->table.empty()) std::memcpy(&host[o_tab], p->table.data(), p->table.size());
    if (!p->slots.empty()) std::memcpy(&host[o_slots], p->slots.data(), p->slots.size() * 8);
    if (!p->pwords.empty()) std::memcpy(&host[o_pw], p->pwords.data(), p->pwords.size() * 4);
    if (!p->idstart.empty()) std::memcpy(&host[o_ids0], p->idstart.data(), p->idstart.size() * 4);
    if (!p->ids.empty()) std::memcpy(&host[o_ids], p->ids.data(), p->ids.size() * 4);
    if (!p->bloom.empty()) std::memcpy(&host[o_bloom], p->bloom.data(), p->bloom.size() * 4);
    if (!p->bloom_batch.empty())
        std::memcpy(&host[o_bloomb], p->bloom_batch.data(), p->bloom_batch.size() * 4);
    if (!p->slices.empty()) std::memcpy(&host[o_sl], p->slices.data(), p->slices.size() * 4);
    if (!p->code_bits.empty()) std::memcpy(&host[o_cb], p->code_bits.data(), p->code_bits.size() * 4);
    if (!p->code_ids.empty()) std::memcpy(&host[o_ci], p->code_ids.data(), p->code_ids.size() * 4);
    if (!p->wfilter.empty()) std::memcpy(&host[o_wf], p->wfilter.data(), p->wfilter.size() * 8);
    if (!p->pwoff.empty()) std::memcpy(&host[o_pwoff], p->pwoff.data(), p->pwoff.size() * 4);
    if (!p->plen.empty()) std::memcpy(&host[o_plen], p->plen.data(), p->plen.size() * 4);
    if (!p->gstart.empty()) std::memcpy(&host[o_gstart], p->gstart.data(), p->gstart.size() * 4);
    e = hipMemcpy(base, host.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(base);
        return hip_fail(e, "upload of plan tables");
    }
    p->dev.base = base;
    p->dev.mu = base + o_mu;
    p->dev.table = base + o_tab;
    p->dev.slots = reinterpret_cast<const uint64_t *>(base + o_slots);
    p->dev.pwords = reinterpret_cast<const uint32_t *>(base + o_pw);
    p->dev.idstart = reinterpret_cast<const uint32_t *>(base + o_ids0);
    p->dev.ids = reinterpret_cast<const uint32_t *>(base + o_ids);
    p->dev.bloom = reinterpret_cast<const uint32_t *>(base + o_bloom);
    p->dev.bloom_batch = reinterpret_cast<const uint32_t *>(base + o_bloomb);
    p->dev.slices = reinterpret_cast<const uint32_t *>(base + o_sl);
    p->dev.code_bits = reinterpret_cast<const uint32_t *>(base + o_cb);
    p->dev.code_ids = reinterpret_cast<const uint32_t *>(base + o_ci);
    p->dev.wfilter = p->wfilter.empty() ? nullptr : reinterpret_cast<const uint64_t *>(base + o_wf);
    p->dev.pwoff = reinterpret_cast<const uint32_t *>(base + o_pwoff);
    p->dev.plen = reinterpret_cast<const uint32_t *>(base + o_plen);
    p->dev.gstart = reinterpret_cast<const uint32_t *>(base + o_gstart);

    // fixed scratch: counters[4], the count and the stats of mag_scan
    Scratch &sc = p->scratch;
    sc.device = dev;
    e = hipMalloc(&sc.counters, kCounterWords * sizeof(uint64_t));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(MAG_E_NOMEM, "device allocation of scan scratch failed");
    }
    // the finishing kernel of every scan returns the counters to zero
    e = hipMemset(sc.counters, 0, kCounterWords * sizeof(uint64_t));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "clearing scan counters");
    p->device = dev;
    return MAG_OK;
}

}  // namespace mag

using namespace mag;

extern "C" {

int32_t mag_version(void) { return 100; }

mag_status mag_stream_read(const uint8_t *d, uint64_t n, uint32_t *d_sink, void *stream) {
    if (!d_sink || (n && !d)) return fail(MAG_E_INVALID, "NULL argument");
    if (reinterpret_cast<uintptr_t>(d) & 15) return fail(MAG_E_INVALID, "d must be 16-byte aligned");
    return launch_stream_read(d, n, d_sink, reinterpret_cast<hipStream_t>(stream));
}

uint32_t mag_stream_read_sink_words(void) { return stream_read_grid(); }

const char *mag_status_string(mag_status s) {
    switch (s) {
        case MAG_OK: return "ok";
        case MAG_E_INVALID: return "invalid argument";
        case MAG_E_UNSUPPORTED: return "unsupported";
        case MAG_E_NOMEM: return "out of memory";
        case MAG_E_DEVICE: return "device error";
        case MAG_E_OVERFLOW: return "output overflow";
    }
    return "unknown status";
}

const char *mag_last_error(void) { return g_last_error.c_str(); }

mag_status mag_profile_enable(int enable) {
    std::lock_guard<std::mutex> pl(g_prof_mtx);
    g_prof_on = enable != 0;
    return MAG_OK;
}

mag_status mag_profile_read(double *scan_ms, double *finish_ms, uint64_t *launches) {
    if (!scan_ms || !finish_ms || !launches) return fail(MAG_E_INVALID, "NULL argument");
    std::vector<ProfileRecord> recs;
    {
        std::lock_guard<std::mutex> pl(g_prof_mtx);
        recs.swap(g_prof);
    }
    double acc[2] = {0, 0};
    mag_status st = MAG_OK;
    for (auto &r : recs) {
        hipError_t e = hipEventSynchronize(r.ev[2]);
        for (int i = 0; i < 2 && e == hipSuccess; ++i) {
            float t = 0;
            e = hipEventElapsedTime(&t, r.ev[i], r.ev[i + 1]);
            acc[i] += t;
        }
        if (e != hipSuccess && st == MAG_OK) st = hip_fail(e, "reading profile events");
        for (auto ev : r.ev) (void)hipEventDestroy(ev);
    }
    *scan_ms = acc[0];
    *finish_ms = acc[1];
    *launches = recs.size();
    return st;
}

mag_status mag_plan_create(const uint8_t *patterns, uint32_t r, uint32_t m,
                           const mag_params *params, mag_plan **out) {
    if (!out) return fail(MAG_E_INVALID, "out is NULL");
    *out = nullptr;
    if (params) {
        for (int v : params->reserved)
            if (v) return fail(MAG_E_INVALID, "mag_params.reserved must be zero");
    }
    mag_plan *p = new (std::nothrow) mag_plan();
    if (!p) return fail(MAG_E_NOMEM, "host allocation failed");
    mag_status s;
    try {
        const auto t0 = std::chrono::steady_clock::now();
        s = build_plan(p, patterns, r, m, params);
        p->plan_ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    } catch (const std::bad_alloc &) {
        s = fail(MAG_E_NOMEM, "host allocation failed while building the plan");
    }
    if (s != MAG_OK) {
        delete p;
        return s;
    }
    *out = p;
    return MAG_OK;
}

mag_status mag_plan_create_var(const uint8_t *bytes, const uint64_t *offsets, uint32_t r,
                               const mag_params *params, mag_plan **out) {
    if (!out) return fail(MAG_E_INVALID, "out is NULL");
    *out = nullptr;
    if (params) {
        for (int v : params->reserved)
            if (v) return fail(MAG_E_INVALID, "mag_params.reserved must be zero");
    }
    mag_plan *p = new (std::nothrow) mag_plan();
    if (!p) return fail(MAG_E_NOMEM, "host allocation failed");
    mag_status s;
    try {
        const auto t0 = std::chrono::steady_clock::now();
        s = build_plan_var(p, bytes, offsets, r, params);
        p->plan_ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    } catch (const std::bad_alloc &) {
        s = fail(MAG_E_NOMEM, "host allocation failed while building the plan");
    }
    if (s != MAG_OK) {
        delete p;
        return s;
    }
    *out = p;
    return MAG_OK;
}

void mag_plan_destroy(mag_plan *p) {
    if (!p) return;
    if (p->device >= 0) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(p->device);
        (void)hipFree(p->dev.base);
        (void)hipFree(p->scratch.counters);
        (void)hipFree(p->scratch.hist);
        (void)hipFree(p->scratch.radix_off);
        (void)hipFree(p->scratch.keys);
        (void)hipFree(p->scratch.pending);
        (void)hipFree(p->scratch.seg_count);
        (void)hipFree(p->scratch.codes);
        (void)hipSetDevice(cur);
    }
    delete p;
}

mag_status mag_plan_info(const mag_plan *p, mag_plan_desc *d) {
    if (!p || !d) return fail(MAG_E_INVALID, "NULL argument");
    std::memset(d, 0, sizeof(*d));
    d->q = p->q;
    d->k = p->k;
    d->sigma_prime = p->sigma_prime;
    d->L = p->L;
    d->m_prime = p->mprime;
    d->W = p->W;
    d->entry_bytes = p->esz;
    d->map_kind = p->map_kind;
    d->select = p->select;
    d->r = p->r;
    d->m = p->m;
    d->n_unique = p->n_unique;
    d->dense = p->dense;
    d->bloom_log2 = p->bloom_log2;
    d->bits_shift = p->bits_shift;
    d->entry_bits = p->entry_bits;
    d->n_codes = p->n_codes;
    d->table_bytes = p->table.size();
    d->est_verif = p->est_verif;
    d->m_max = p->m_max;
    d->var = (uint32_t)p->var;
    d->q_formula = p->q_formula;
    d->dense_slices = p->slice_k;
    d->dense_pass = p->slice_k ? p->slice_fp : p->bloom_fp;
    return MAG_OK;
}

mag_status mag_plan_get_params(const mag_plan *p, mag_params *o) {
    if (!p || !o) return fail(MAG_E_INVALID, "NULL argument");
    std::memset(o, 0, sizeof(*o));
    o->select = MAG_SELECT_EXPLICIT;
    o->map_kind = p->map_kind;
    o->q = p->q;
    o->k = p->k;
    o->sigma_prime = p->sigma_prime;
    o->table_budget = 0;
    o->mode = p->dense ? MAG_MODE_DENSE : MAG_MODE_FILTER;
    o->verify = p->verify;
    o->verify_buffer = (int32_t)p->verify_buffer;
    o->encode = p->encode;
    o->dense_probe = p->dense_probe;
    o->chunk_bytes = p->chunk_bytes;
    o->words_per_lane = p->words_per_lane;
    return MAG_OK;
}

mag_status mag_plan_export(const mag_plan *p, uint8_t *mu_out, void *table_out, uint64_t table_cap) {
    if (!p) return fail(MAG_E_INVALID, "plan is NULL");
    if (mu_out) std::memcpy(mu_out, p->mu, 256);
    if (table_out) {
        if (table_cap < p->table.size()) return fail(MAG_E_INVALID, "table_out too small");
        std::memcpy(table_out, p->table.data(), p->table.size());
    }
    return MAG_OK;
}

}  // extern "C"

namespace mag {
namespace {
// Enqueues counter reset, scan and finishing kernel; returns the key layout.
// fixed: scratch laid out in advance (the allocation-free entry point): the
// plan must already be resident on the current device, nothing is
// allocated, deferred starts beyond fixed->pending_cap are verified inline,
// SMAG plans compute their codes on the fly, and no profiling events are
// recorded.
mag_status scan_enqueue(mag_plan *p, const uint8_t *d_text, uint64_t n, mag_match *d_out,
                        uint64_t out_cap, uint64_t *d_count, mag_stats *d_stats, void *stream_,
                        bool device_sort, int *idbits_out, int *nbits_out, Scratch *fixed = nullptr) {
    if (!p) return fail(MAG_E_INVALID, "plan is NULL");
    if (!d_count) return fail(MAG_E_INVALID, "d_count is NULL");
    if (n && !d_text) return fail(MAG_E_INVALID, "d_text is NULL");
    if (out_cap && !d_out) return fail(MAG_E_INVALID, "d_out is NULL");
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    std::lock_guard<std::mutex> lock(p->mtx);
    mag_status s = MAG_OK;
    // without the host reading the count, large outputs are sorted by
    // kernels sized for the capacity
    const bool sort_on_device = device_sort && out_cap > small_sort_max();
    if (fixed) {
        int dev = 0;
        const hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
        if (p->device != dev)
            return fail(MAG_E_INVALID, "plan tables are not on this device (scan the plan once with "
                                       "mag_scan_async first)");
        if (out_cap > fixed->keys_cap)
            return fail(MAG_E_INVALID, "out_cap above the allocation-free scan's limit");
    } else {
        s = ensure_device(p);
        if (s != MAG_OK) return s;
        s = ensure_keys(p, out_cap, stream);
        if (s != MAG_OK) return s;
        if (sort_on_device) {
            s = ensure_radix_scratch(p->scratch, out_cap, stream);
            if (s != MAG_OK) return s;
        }
    }
    Scratch &sc = fixed ? *fixed : p->scratch;

    const int idbits = ceil_log2(p->r > 1 ? p->r : 2);
    const int posbits = ceil_log2(n + 1 > 2 ? n + 1 : 2);
    if (idbits + posbits > 64) return fail(MAG_E_UNSUPPORTED, "positions and ids need more than 64 key bits");
    const uint64_t kq = (uint64_t)p->k * p->q;
    // filter: q-grams read; dense: start positions tested
    const uint64_t samples = p->dense ? (n >= p->m && p->r ? n - p->m + 1 : 0)
                                      : (n >= (uint64_t)p->q ? (n - p->q) / kq + 1 : 0);

    // many expected verifications: the filter kernels defer them
    const bool slices = p->dense && p->slice_k > 0;
    const double expect = p->r == 0 ? 0.0
                          : p->dense ? (slices ? p->slice_fp : p->bloom_fp) * (double)samples
                          : p->est_verif < 0.0 ? -1.0 : p->est_verif * (double)n;
    uint64_t pcap = 0;
    // a grid of fewer workgroups than half the compute units verifies inline
    // with few waves: defer when each of them would face many starts
    const int ncu = device_compute_units();
    const int lane_pos = dense_lane_positions(p, samples, ncu);
    const uint64_t tile = slices ? (uint64_t)slice_scan_tile(lane_pos)
                          : p->dense ? (uint64_t)kDenseScanTile : kSmallGridTileSamples;
    const uint64_t tiles = (samples + tile - 1) / tile;
    const double vwaves = (double)std::max<uint64_t>(tiles, 1) *
                          (p->dense ? kDenseScanThreads / 64 : kScanConsumerLanes / 64);
    const bool small_grid = ncu > 0 && 2 * tiles < (uint64_t)ncu;
    const bool defer = p->verify == MAG_VERIFY_DEFERRED ||
                       (p->verify == MAG_VERIFY_AUTO &&
                        ((!p->dense && (expect < 0.0 || expect >= kDeferMinVerifications)) ||
                         (small_grid && expect >= kDeferPerWave * vwaves)));
    if (samples && defer)
        pcap = p->verify_buffer ? p->verify_buffer
                                : pending_capacity(expect < 0.0 ? expect : std::max(expect, (double)(1 << 20)));
    if (pcap && fixed) {
        pcap = std::min(pcap, fixed->pending_cap);
    } else if (pcap) {
        s = ensure_pending(p, pcap, stream);
        if (s != MAG_OK) return s;
    }

    ScanLaunch sl;
    sl.text = d_text;
    sl.n = n;
    sl.keys = sc.keys;
    sl.cap = out_cap;
    sl.counters = sc.counters;
    sl.idbits = idbits;
    sl.pending = pcap ? sc.pending : nullptr;
    sl.pending_cap = pcap ? (fixed ? pcap : sc.pending_cap) : 0;
    sl.seg_count = pcap ? sc.seg_count : nullptr;
    const bool smag = !fixed && p->encode && !p->dense && p->r && n >= (uint64_t)p->q;
    if (smag) {
        sl.csz = encoded_code_bytes(p);
        // 16 bytes of slack: phase A reads the 32-bit word holding each code
        s = ensure_codes(p, ((n - p->q) / p->q + 1) * (uint64_t)sl.csz + 16, stream);
        if (s != MAG_OK) return s;
        sl.codes = p->scratch.codes;
    }
    ProfileMarks prof;
    if (!fixed) {
        s = profile_start(prof, stream);
        if (s != MAG_OK) return s;
    }
    if (p->dense) {
        DenseArgs da{};
        const uintptr_t t = reinterpret_cast<uintptr_t>(d_text);
        da.tbase = reinterpret_cast<const uint8_t *>(t & ~(uintptr_t)15);
        da.delta = t & 15;
        da.n = n;
        da.last = (int64_t)n - (int64_t)p->m;
        da.bshift = 32u - (uint32_t)p->bloom_log2;
        da.counters = sc.counters;
        da.v = make_verify_args(p, sl);
        if (slices) {
            const uint64_t st = (uint64_t)slice_scan_tile(lane_pos);
            da.ntiles = samples ? (samples + st - 1) / st : 0;
            da.bloom_vec = (uint32_t)(p->slices.size() * 4 / 16);
            da.bloom = p->dev.slices;
            s = launch_dense_slices(da, p->slices.size() * 4, p->slice_k, lane_pos, stream);
        } else {
            da.ntiles = samples ? (samples + kDenseScanTile - 1) / kDenseScanTile : 0;
            da.bloom_vec = (uint32_t)(p->bloom.size() * 4 / 16);
            da.bloom = p->dev.bloom;
            s = launch_dense(da, p->bloom.size() * 4, stream);
        }
    } else {
        if (smag) s = launch_encode(p, d_text, n, p->scratch.codes, sl.csz, stream);
        if (s == MAG_OK) s = launch_scan(p, sl, stream);
    }
    if (s == MAG_OK && sl.pending) s = launch_verify(make_verify_args(p, sl), stream);
    if (s != MAG_OK) return s;
    profile_mark(prof, stream);
    if (idbits_out) *idbits_out = idbits;
    if (nbits_out) *nbits_out = idbits + posbits;
    StatsInfo info;
    info.q = p->q;
    info.k = p->k;
    info.sigma_prime = p->sigma_prime;
    info.m_prime = p->mprime;
    info.plan_ms = p->plan_ms;
    s = launch_finish(sc, out_cap, samples, d_count, d_stats, info, d_out, idbits, ~0ull, nullptr, stream);
    if (s != MAG_OK) return s;
    if (sort_on_device) {
        const int lo = sort_low_bit(p->var, idbits);
        // the last pass writes the records
        s = launch_radix_sort(sc, out_cap, out_cap, idbits + posbits, lo, stream, d_out, idbits, ~0ull);
        if (s == MAG_OK && radix_passes(idbits + posbits, lo) == 0)
            s = launch_expand(sc, out_cap, out_cap, idbits + posbits, lo, d_out, idbits, ~0ull, stream);
        if (s != MAG_OK) return s;
    }
    profile_commit(prof, stream);
    return MAG_OK;
}

}  // namespace

// ---- the allocation-free scan (mag_scan_noalloc) ----
// Its scratch is one static device array per GPU; `scratch` below is only a
// host-side stand-in for it, so host code uses the per-device address from
// hipGetSymbolAddress instead (noalloc_base).
constexpr uint64_t kNoAllocCap = 1ull << 20;       // largest out_cap
constexpr uint64_t kNoAllocPending = 1ull << 20;   // deferred starts it holds (more: inline)
constexpr uint64_t kNoAllocBytes = 28ull << 20;

}  // namespace mag

static __device__ __align__(256) uint8_t scratch[mag::kNoAllocBytes];

namespace mag {
namespace {

std::mutex g_noalloc_mtx;
std::map<int, uint8_t *> g_noalloc_base;

// The current device's copy of `scratch`, looked up once per device.
mag_status noalloc_base(int dev, uint8_t **out) {
    std::lock_guard<std::mutex> lock(g_noalloc_mtx);
    const auto it = g_noalloc_base.find(dev);
    if (it != g_noalloc_base.end()) {
        *out = it->second;
        return MAG_OK;
    }
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress of the allocation-free scratch");
    g_noalloc_base[dev] = static_cast<uint8_t *>(ptr);
    *out = static_cast<uint8_t *>(ptr);
    return MAG_OK;
}

uint64_t round256(uint64_t v) { return (v + 255) & ~255ull; }

// Lays the scan's scratch out in the static array at `base`: counters and
// segment counters, the two key buffers, the radix sort's counts and
// offsets, and the deferred-start buffer.
mag_status noalloc_layout(uint8_t *base, int dev, Scratch &sc) {
    const uint64_t C = radix_scratch_chunks(kNoAllocCap);
    const uint64_t o_cnt = 0;
    const uint64_t o_keys = round256((kCounterWords + kPendingSegments) * sizeof(uint64_t));
    const uint64_t o_hist = round256(o_keys + 2 * kNoAllocCap * sizeof(uint64_t));
    const uint64_t o_off = round256(o_hist + 256 * C * sizeof(uint32_t));
    const uint64_t o_pend = round256(o_off + (256 * C + 256) * sizeof(uint64_t));
    const uint64_t end = o_pend + kNoAllocPending * sizeof(uint64_t);
    if (end > kNoAllocBytes) return fail(MAG_E_UNSUPPORTED, "allocation-free scratch layout too large");
    sc.device = dev;
    sc.counters = reinterpret_cast<uint64_t *>(base + o_cnt);
    sc.seg_count = sc.counters + kCounterWords;
    sc.keys = reinterpret_cast<uint64_t *>(base + o_keys);
    sc.keys_cap = kNoAllocCap;
    sc.hist = reinterpret_cast<uint32_t *>(base + o_hist);
    sc.radix_off = reinterpret_cast<uint64_t *>(base + o_off);
    sc.radix_chunks = C;
    sc.pending = reinterpret_cast<uint64_t *>(base + o_pend);
    sc.pending_cap = kNoAllocPending;
    return MAG_OK;
}

}  // namespace
}  // namespace mag

extern "C" {

mag_status mag_scan_noalloc(mag_plan *p, const uint8_t *d_text, uint64_t n, mag_match *d_out,
                            uint64_t out_cap, uint64_t *d_count, mag_stats *d_stats, void *stream) {
    if (!p) return fail(MAG_E_INVALID, "plan is NULL");
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (out_cap > kNoAllocCap) return fail(MAG_E_INVALID, "out_cap above the allocation-free scan's limit (2^20)");
    uint8_t *base = nullptr;
    mag_status s = noalloc_base(dev, &base);
    if (s != MAG_OK) return s;
    Scratch sc;
    s = noalloc_layout(base, dev, sc);
    if (s != MAG_OK) return s;
    // the counters and segment counters start at zero, whatever an earlier
    // call left (a fill kernel, so that the call can be captured in a graph)
    s = launch_fill_u64(sc.counters, kCounterWords + kPendingSegments, 0, reinterpret_cast<hipStream_t>(stream));
    if (s != MAG_OK) return s;
    return scan_enqueue(p, d_text, n, d_out, out_cap, d_count, d_stats, stream, true, nullptr, nullptr, &sc);
}

mag_status mag_encode(mag_plan *p, const uint8_t *d_text, uint64_t n, uint32_t *d_codes,
                      uint64_t cap, uint64_t *n_codes, void *stream) {
    if (!p || !n_codes) return fail(MAG_E_INVALID, "NULL argument");
    const uint64_t G = n >= (uint64_t)p->q ? (n - p->q) / p->q + 1 : 0;
    *n_codes = G;
    if (G == 0) return MAG_OK;
    if (!d_text || !d_codes) return fail(MAG_E_INVALID, "d_text or d_codes is NULL");
    if (cap < G) return fail(MAG_E_INVALID, "d_codes holds fewer entries than there are q-grams");
    std::lock_guard<std::mutex> lock(p->mtx);
    mag_status s = ensure_device(p);
    if (s != MAG_OK) return s;
    return launch_encode(p, d_text, n, d_codes, 4, reinterpret_cast<hipStream_t>(stream));
}

mag_status mag_scan_async(mag_plan *p, const uint8_t *d_text, uint64_t n, mag_match *d_out,
                          uint64_t out_cap, uint64_t *d_count, mag_stats *d_stats, void *stream) {
    return scan_enqueue(p, d_text, n, d_out, out_cap, d_count, d_stats, stream, true, nullptr,
                        nullptr);
}

mag_status mag_scan(mag_plan *p, const uint8_t *d_text, uint64_t n, mag_match *d_out,
                    uint64_t out_cap, uint64_t *n_matches, mag_stats *stats, void *stream_) {
    if (!p) return fail(MAG_E_INVALID, "plan is NULL");
    if (!n_matches) return fail(MAG_E_INVALID, "n_matches is NULL");
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    {
        std::lock_guard<std::mutex> lock(p->mtx);
        mag_status s = ensure_device(p);
        if (s != MAG_OK) return s;
    }
    // the count and the counters land in the plan's own scratch words
    uint64_t *d_cnt = p->scratch.counters + 4;
    mag_stats *d_st = reinterpret_cast<mag_stats *>(p->scratch.counters + kStatsSlot);
    static_assert(kStatsSlot * 8 + sizeof(mag_stats) <= kCounterWords * 8, "stats fit the counter words");
    int idbits = 0, nbits = 0;
    // with stats, events around the scan's kernels give scan_ms
    hipEvent_t ev[2] = {nullptr, nullptr};
    if (stats) {
        ev[0] = make_event();
        ev[1] = make_event();
        if (ev[0] && ev[1]) (void)hipEventRecord(ev[0], stream);
    }
    mag_status s = scan_enqueue(p, d_text, n, d_out, out_cap, d_cnt, d_st, stream_, false, &idbits,
                                &nbits);
    if (ev[0] && ev[1] && s == MAG_OK) (void)hipEventRecord(ev[1], stream);
    uint64_t host[kCounterWords];
    hipError_t e = hipSuccess;
    if (s == MAG_OK) {
        e = hipMemcpyAsync(host, p->scratch.counters, kCounterWords * sizeof(uint64_t),
                           hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
    }
    float scan_ms = 0.0f;
    if (s == MAG_OK && e == hipSuccess && ev[0] && ev[1])
        (void)hipEventElapsedTime(&scan_ms, ev[0], ev[1]);
    for (auto x : ev)
        if (x) (void)hipEventDestroy(x);
    if (s != MAG_OK) return s;
    if (e != hipSuccess) return hip_fail(e, "reading the match count");
    *n_matches = host[4];
    if (stats) {
        std::memcpy(stats, &host[kStatsSlot], sizeof(mag_stats));
        stats->scan_ms = scan_ms;
    }
    if (host[4] > out_cap)
        return fail(MAG_E_OVERFLOW, "output capacity smaller than the match count");
    if (host[4] > small_sort_max()) {
        std::lock_guard<std::mutex> lock(p->mtx);
        s = ensure_radix_scratch(p->scratch, host[4], stream);
        const int lo = sort_low_bit(p->var, idbits);
        if (s == MAG_OK)
            s = launch_radix_sort(p->scratch, host[4], out_cap, nbits, lo, stream, d_out, idbits, ~0ull);
        if (s == MAG_OK && radix_passes(nbits, lo) == 0)
            s = launch_expand(p->scratch, host[4], out_cap, nbits, lo, d_out, idbits, ~0ull, stream);
    }
    return s;
}

}  // extern "C"
