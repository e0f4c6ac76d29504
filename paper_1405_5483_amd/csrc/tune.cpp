// Autotuner: chooses the mode, (q, k, sigma', map) and the tile shape (words
// per lane) for a pattern set by timing scans of a device-resident text
// sample, and, for batches, the same per job class plus the batched
// kernel's words per lane.
//
// Filter candidates: every q with 2q-1 <= m (q <= max_q), every k <=
// min(L, max_k), sigma' from 2 up to the number of distinct pattern bytes, and
// both alphabet maps, whose mask table fits the budget. They are ranked by an
// estimate of the scan cost per text byte: the sampling work (one gram every
// kq bytes) plus the expected verifications, q * sum_j prod_h p(j + hk) per
// sample, where p(b) is the probability that a text gram falls in the
// superimposed class C[b] (the class-density argument of Section 2), taking
// the pattern-set byte frequencies as the text's. The best-ranked ones are
// timed, always with the dense mode (every start position tested) beside
// them. The winner's tile shape is then timed over a few words-per-lane
// values.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "batch.hpp"
#include "mag_internal.hpp"

namespace mag {
namespace {

struct Candidate {
    int q, k, sp, map;
    double est;
};

int entry_bytes_of(int W) { return W <= 8 ? 1 : W <= 16 ? 2 : W <= 32 ? 4 : 8; }

// Estimated relative cost per text byte of a built plan.
double estimate(const mag_plan *p, const double *byte_freq) {
    const int sp = p->sigma_prime, q = p->q, W = p->W, k = p->k, esz = p->esz;
    std::vector<double> sym(sp, 0.0);
    for (int c = 0; c < 256; ++c) sym[p->mu[c]] += byte_freq[c];
    std::vector<double> pb(W, 0.0);
    const uint8_t *tb = p->table.data();
    for (uint64_t code = 0; code < p->n_codes; ++code) {
        double pr = 1.0;
        uint64_t c = code;
        for (int t = 0; t < q; ++t) {
            pr *= sym[c % sp];
            c /= sp;
        }
        if (pr == 0.0) continue;
        for (int b = 0; b < W; ++b)
            if (!(tb[code * esz + (b >> 3)] & (1u << (b & 7)))) pb[b] += pr;
    }
    double cand = 0.0;                      // candidate windows per sample
    for (int j = 0; j < k; ++j) {
        double prod = 1.0;
        for (int h = 0; h < p->mprime; ++h) prod *= std::min(1.0, pb[j + h * k]);
        cand += prod;
    }
    const double kq = (double)k * q;
    const double verif_per_byte = cand * q / kq;
    const double sample_cost = 1.0 + 0.25 * q;       // loads, q lookups, table lookup
    const double table_penalty = p->table.size() > 64 * 1024 ? 3.0 : 1.0;  // L2 vs LDS table
    return sample_cost * table_penalty / kq + 40.0 * verif_per_byte;
}

}  // namespace
}  // namespace mag

namespace mag {
namespace {

struct Timer {
    mag_match *d_out = nullptr;
    uint64_t cap = 0;
    uint64_t *d_cnt = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Timer() {
        (void)hipFree(d_out);
        (void)hipFree(d_cnt);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
    mag_status init() {
        hipError_t he = hipMalloc(&d_cnt, sizeof(uint64_t));
        if (he == hipSuccess) he = hipEventCreate(&e0);
        if (he == hipSuccess) he = hipEventCreate(&e1);
        return he == hipSuccess ? MAG_OK : hip_fail(he, "autotuner setup");
    }
    // Median device time (ms) of `repeats` scans of the sample with plan params
    // prm; +inf when the plan cannot be built.
    mag_status time(const uint8_t *patterns, uint32_t r, uint32_t m, const mag_params &prm,
                    const uint8_t *d_sample, uint64_t n_sample, int repeats, hipStream_t stream,
                    float &out) {
        out = INFINITY;
        mag_plan *pl = nullptr;
        if (mag_plan_create(patterns, r, m, &prm, &pl) != MAG_OK) return MAG_OK;
        hipError_t he = hipSuccess;
        if (!d_out) {
            cap = 1024;
            he = hipMalloc(&d_out, cap * sizeof(mag_match));
            if (he != hipSuccess) { d_out = nullptr; mag_plan_destroy(pl); return hip_fail(he, "autotuner output"); }
        }
        // the first scan sizes the output (every candidate finds the same occurrences)
        uint64_t z = 0;
        mag_status s = mag_scan(pl, d_sample, n_sample, d_out, cap, &z, nullptr, stream);
        if (s == MAG_E_OVERFLOW) {
            (void)hipStreamSynchronize(stream);
            (void)hipFree(d_out);
            cap = z + 1024;
            he = hipMalloc(&d_out, cap * sizeof(mag_match));
            if (he != hipSuccess) { d_out = nullptr; mag_plan_destroy(pl); return hip_fail(he, "autotuner output"); }
            s = mag_scan(pl, d_sample, n_sample, d_out, cap, &z, nullptr, stream);
        }
        std::vector<float> ts;
        for (int rep = 0; rep < repeats && s == MAG_OK; ++rep) {
            (void)hipEventRecord(e0, stream);
            s = mag_scan_async(pl, d_sample, n_sample, d_out, cap, d_cnt, nullptr, stream);
            (void)hipEventRecord(e1, stream);
            he = hipEventSynchronize(e1);
            float ms = 0;
            if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
            if (he != hipSuccess) { s = hip_fail(he, "autotuner timing"); break; }
            ts.push_back(ms);
        }
        mag_plan_destroy(pl);
        if (s != MAG_OK) return s;
        std::sort(ts.begin(), ts.end());
        out = ts[ts.size() / 2];
        return MAG_OK;
    }
};

mag_params explicit_params(int mode, int map, int q, int k, int sp) {
    mag_params prm;
    std::memset(&prm, 0, sizeof(prm));
    prm.select = MAG_SELECT_EXPLICIT;
    prm.mode = mode;
    prm.map_kind = map;
    prm.q = q;
    prm.k = k;
    prm.sigma_prime = sp;
    return prm;
}

}  // namespace
}  // namespace mag

using namespace mag;

extern "C" mag_status mag_autotune(const uint8_t *patterns, uint32_t r, uint32_t m,
                                   const mag_tune_opts *opts, const uint8_t *d_sample,
                                   uint64_t n_sample, mag_params *best, float *best_ms,
                                   void *stream_) {
    mag_tune_opts o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (o.reserved) return fail(MAG_E_INVALID, "mag_tune_opts.reserved must be zero");
    if (m == 0 || (r > 0 && !patterns)) return fail(MAG_E_INVALID, "bad pattern set");
    if (n_sample && !d_sample) return fail(MAG_E_INVALID, "d_sample is NULL");
    const int maps = o.map_kinds ? o.map_kinds : 3;
    const int modes = o.modes ? o.modes : 3;
    const int max_q = o.max_q > 0 ? std::min(o.max_q, kMaxQ) : kMaxQ;
    const int max_k = o.max_k > 0 ? std::min(o.max_k, kMaxK) : 8;
    const int64_t budget = o.table_budget > 0 ? o.table_budget : 64 * 1024;
    const int repeats = o.repeats > 0 ? o.repeats : 3;
    const int max_cand = o.max_candidates > 0 ? o.max_candidates : 64;
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);

    // pattern byte frequencies and sigma_P
    std::vector<uint64_t> hist(256, 0);
    for (uint64_t i = 0; i < (uint64_t)r * m; ++i) hist[patterns[i]]++;
    int sigma_p = 0;
    double byte_freq[256];
    for (int c = 0; c < 256; ++c) {
        sigma_p += hist[c] ? 1 : 0;
        byte_freq[c] = r ? (double)hist[c] / ((double)r * m) : 0.0;
    }
    sigma_p = std::max(sigma_p, 1);

    // enumerate and rank the filter candidates
    std::vector<Candidate> cands;
    if (modes & 1) {
        for (int q = 1; q <= max_q && 2 * q - 1 <= (int)m; ++q) {
            const int L = ((int)m - q + 1) / q;
            for (int k = 1; k <= std::min(L, max_k); ++k) {
                const int mp = std::min(L / k, kMaxW / k);
                if (o.batch_only && (k * mp > 32 || k >= 32)) continue;
                const int eb = entry_bytes_of(k * mp);
                for (int sp = std::min(sigma_p, 256); sp >= (sigma_p > 1 ? 2 : 1); --sp) {
                    if (std::pow((double)sp, q) * eb > (double)budget) continue;
                    for (int map = 0; map < 2; ++map) {
                        if (!(maps & (1 << map))) continue;
                        if (map == MAG_MAP_RANK && sp >= sigma_p) continue;  // same as greedy then
                        cands.push_back({q, k, sp, map, 0.0});
                    }
                }
            }
        }
    }
    for (auto &c : cands) {
        const mag_params prm = explicit_params(MAG_MODE_FILTER, c.map, c.q, c.k, c.sp);
        mag_plan *pl = nullptr;
        if (mag_plan_create(patterns, r, m, &prm, &pl) != MAG_OK) {
            c.est = INFINITY;
            continue;
        }
        c.est = estimate(pl, byte_freq);
        mag_plan_destroy(pl);
    }
    std::stable_sort(cands.begin(), cands.end(),
                     [](const Candidate &a, const Candidate &b) { return a.est < b.est; });
    if ((int)cands.size() > max_cand) cands.resize(max_cand);
    if (modes & 2) cands.push_back({0, 0, 0, -1, 0.0});      // the dense mode, always timed
    if (cands.empty()) return fail(MAG_E_INVALID, "no feasible parameters within the table budget");

    // time them on the sample
    Timer tm;
    mag_status st = tm.init();
    if (st != MAG_OK) return st;
    float best_t = INFINITY;
    mag_params best_p = explicit_params(MAG_MODE_DENSE, 0, 0, 0, 0);
    for (const auto &c : cands) {
        if (!std::isfinite(c.est)) continue;
        mag_params prm;
        if (c.map < 0) {
            // dense: q, k and sigma' only shape the unused filter; the heuristic's
            mag_plan *h = nullptr;
            if (mag_plan_create(patterns, r, m, nullptr, &h) != MAG_OK) continue;
            prm = explicit_params(MAG_MODE_DENSE, h->map_kind, h->q, h->k, h->sigma_prime);
            mag_plan_destroy(h);
        } else {
            prm = explicit_params(MAG_MODE_FILTER, c.map, c.q, c.k, c.sp);
        }
        float t = INFINITY;
        st = tm.time(patterns, r, m, prm, d_sample, n_sample, repeats, stream, t);
        if (st != MAG_OK) return st;
        if (t < best_t) {
            best_t = t;
            best_p = prm;
        }
    }
    if (!std::isfinite(best_t)) return fail(MAG_E_INVALID, "no candidate could be scanned");
    // the winner's tile shape: entries per lane of the filter kernel (around
    // its default 32 KiB entry buffer), or 16 / 32 positions per lane dense
    if (!o.fixed_tiles) {
        std::vector<int> wpl;
        if (best_p.mode == MAG_MODE_DENSE) {
            wpl = {32};
        } else {
            const int eb = entry_bytes_of(std::min(((int)m - best_p.q + 1) / best_p.q / best_p.k, kMaxW / best_p.k) *
                                          best_p.k);
            const int def = 32 * 1024 / (256 * eb);
            wpl = {def / 2, def * 3 / 2};
        }
        for (int w : wpl) {
            mag_params prm = best_p;
            prm.words_per_lane = w;
            float t = INFINITY;
            st = tm.time(patterns, r, m, prm, d_sample, n_sample, repeats, stream, t);
            if (st != MAG_OK) return st;
            if (t < 0.97f * best_t) {       // a clear gain over the default shape
                best_t = t;
                best_p = prm;
            }
        }
    }
    (void)hipStreamSynchronize(stream);
    if (best) *best = best_p;
    if (best_ms) *best_ms = best_t;
    return MAG_OK;
}

extern "C" mag_status mag_autotune_batch(const mag_job *jobs, const uint8_t *const *pat, const uint32_t *r,
                                         const uint32_t *m, uint32_t njobs, const mag_tune_opts *opts,
                                         uint64_t sample_bytes, mag_params *params, int32_t *words_per_lane,
                                         void *stream_) {
    if (!jobs || !pat || !r || !m || !params) return fail(MAG_E_INVALID, "NULL argument");
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    mag_tune_opts o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    o.batch_only = 1;
    const uint64_t sample = sample_bytes ? sample_bytes : (4ull << 20);
    // job classes: (m, distinct pattern bytes, floor(log2 r))
    std::map<std::tuple<uint32_t, int, int>, std::vector<uint32_t>> classes;
    for (uint32_t j = 0; j < njobs; ++j) {
        if (m[j] == 0 || (r[j] && !pat[j])) return fail(MAG_E_INVALID, "bad pattern set");
        if (jobs[j].n && !jobs[j].d_text) return fail(MAG_E_INVALID, "a job's text is NULL");
        bool seen[256] = {false};
        int sigma = 0;
        for (uint64_t i = 0; i < (uint64_t)r[j] * m[j]; ++i)
            if (!seen[pat[j][i]]) {
                seen[pat[j][i]] = true;
                ++sigma;
            }
        const int lr = r[j] ? 31 - __builtin_clz(r[j]) : -1;    // floor(log2 r)
        classes[std::make_tuple(m[j], sigma, lr)].push_back(j);
    }
    for (const auto &kv : classes) {
        uint32_t rep = kv.second[0];
        for (uint32_t j : kv.second)
            if (jobs[j].n > jobs[rep].n) rep = j;
        mag_params best;
        mag_status st;
        if (r[rep] == 0 || jobs[rep].n < m[rep]) {
            // nothing to time: the heuristic's parameters, explicitly
            mag_plan *h = nullptr;
            st = mag_plan_create(pat[rep], r[rep], m[rep], nullptr, &h);
            if (st != MAG_OK) return st;
            st = mag_plan_get_params(h, &best);
            mag_plan_destroy(h);
        } else {
            st = mag_autotune(pat[rep], r[rep], m[rep], &o, jobs[rep].d_text, std::min(jobs[rep].n, sample),
                              &best, nullptr, stream_);
        }
        if (st != MAG_OK) return st;
        for (uint32_t j : kv.second) params[j] = best;
    }
    if (!words_per_lane) return MAG_OK;
    *words_per_lane = kBatchWordsDefault;
    if (!njobs) return MAG_OK;

    // the batch's words per lane, timed on the whole batch
    std::vector<mag_plan *> plans(njobs, nullptr);
    auto release = [&]() {
        for (auto *p : plans) mag_plan_destroy(p);
    };
    for (uint32_t j = 0; j < njobs; ++j) {
        const mag_status st = mag_plan_create(pat[j], r[j], m[j], &params[j], &plans[j]);
        if (st != MAG_OK) {
            release();
            return st;
        }
    }
    std::vector<const uint8_t *> texts(njobs);
    std::vector<uint64_t> n(njobs);
    for (uint32_t j = 0; j < njobs; ++j) {
        texts[j] = jobs[j].d_text;
        n[j] = jobs[j].n;
    }
    mag_batch *b = nullptr;
    mag_status st = mag_batch_create(plans.data(), njobs, &b);
    mag_match *d_out = nullptr;
    uint64_t *d_aux = nullptr;   // offsets (njobs + 1), then the count
    hipEvent_t e0 = nullptr, e1 = nullptr;
    uint64_t cap = 1 << 16;
    hipError_t he = hipSuccess;
    if (st == MAG_OK) {
        he = hipMalloc(&d_aux, ((size_t)njobs + 2) * sizeof(uint64_t));
        if (he == hipSuccess) he = hipMalloc(&d_out, cap * sizeof(mag_match));
        if (he == hipSuccess) he = hipEventCreate(&e0);
        if (he == hipSuccess) he = hipEventCreate(&e1);
        if (he != hipSuccess) st = hip_fail(he, "batch autotuner setup");
    }
    float best_t = INFINITY;
    for (int w : {16, 8}) {
        if (st != MAG_OK) break;
        st = mag_batch_set_words_per_lane(b, w);
        if (st == MAG_OK) st = mag_batch_bind(b, texts.data(), n.data(), cap, stream_);
        if (st != MAG_OK) break;
        // one run to size the output, then the timed ones
        st = mag_batch_run_async(b, d_out, d_aux, d_aux + njobs + 1, stream_);
        uint64_t z = 0;
        if (st == MAG_OK) {
            he = hipMemcpyAsync(&z, d_aux + njobs + 1, sizeof(z), hipMemcpyDeviceToHost, stream);
            if (he == hipSuccess) he = hipStreamSynchronize(stream);
            if (he != hipSuccess) st = hip_fail(he, "batch autotuner count");
        }
        if (st == MAG_OK && z > cap) {
            (void)hipFree(d_out);
            d_out = nullptr;
            cap = z + 1024;
            he = hipMalloc(&d_out, cap * sizeof(mag_match));
            if (he != hipSuccess) {
                st = hip_fail(he, "batch autotuner output");
                break;
            }
            st = mag_batch_bind(b, texts.data(), n.data(), cap, stream_);
        }
        std::vector<float> ts;
        for (int rep = 0; rep < 3 && st == MAG_OK; ++rep) {
            (void)hipEventRecord(e0, stream);
            st = mag_batch_run_async(b, d_out, d_aux, d_aux + njobs + 1, stream_);
            (void)hipEventRecord(e1, stream);
            he = hipEventSynchronize(e1);
            float ms = 0;
            if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
            if (he != hipSuccess && st == MAG_OK) st = hip_fail(he, "batch autotuner timing");
            ts.push_back(ms);
        }
        if (st != MAG_OK) break;
        std::sort(ts.begin(), ts.end());
        if (ts[1] < 0.97f * best_t || !std::isfinite(best_t)) {
            best_t = ts[1];
            *words_per_lane = w;
        }
    }
    (void)hipStreamSynchronize(stream);
    mag_batch_destroy(b);
    (void)hipFree(d_out);
    (void)hipFree(d_aux);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    release();
    return st;
}
