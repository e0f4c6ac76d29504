// Autotuner: chooses (q, k, sigma', map) for a pattern set by timing scans of
// a device-resident text sample.
//
// Candidates: every q with 2q-1 <= m (q <= max_q), every k <= min(L, max_k),
// sigma' from 2 up to the number of distinct pattern bytes, and both alphabet
// maps, whose mask table fits the budget. They are ranked by an estimate of
// the scan cost per text byte: the sampling work (one gram every kq bytes)
// plus the expected verifications, q * sum_j prod_h p(j + hk) per sample,
// where p(b) is the probability that a text gram falls in the superimposed
// class C[b] (the class-density argument of Section 2), taking the pattern-set
// byte frequencies as the text's. The best-ranked candidates are then timed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

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

using namespace mag;

extern "C" mag_status mag_autotune(const uint8_t *patterns, uint32_t r, uint32_t m,
                                   const mag_tune_opts *opts, const uint8_t *d_sample,
                                   uint64_t n_sample, mag_params *best, float *best_ms,
                                   void *stream_) {
    mag_tune_opts o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    for (int v : o.reserved)
        if (v) return fail(MAG_E_INVALID, "mag_tune_opts.reserved must be zero");
    if (m == 0 || (r > 0 && !patterns)) return fail(MAG_E_INVALID, "bad pattern set");
    if (n_sample && !d_sample) return fail(MAG_E_INVALID, "d_sample is NULL");
    const int maps = o.map_kinds ? o.map_kinds : 3;
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

    // enumerate and rank
    std::vector<Candidate> cands;
    for (int q = 1; q <= max_q && 2 * q - 1 <= (int)m; ++q) {
        const int L = ((int)m - q + 1) / q;
        for (int k = 1; k <= std::min(L, max_k); ++k) {
            const int mp = std::min(L / k, kMaxW / k);
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
    if (cands.empty()) return fail(MAG_E_INVALID, "no feasible parameters within the table budget");
    for (auto &c : cands) {
        mag_params prm;
        std::memset(&prm, 0, sizeof(prm));
        prm.select = MAG_SELECT_EXPLICIT;
        prm.map_kind = c.map;
        prm.q = c.q;
        prm.k = c.k;
        prm.sigma_prime = c.sp;
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

    // time the best-ranked candidates on the sample
    uint64_t cap = 1024;
    mag_match *d_out = nullptr;
    uint64_t *d_cnt = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipMalloc(&d_cnt, sizeof(uint64_t));
    if (he == hipSuccess) he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    if (he != hipSuccess) return hip_fail(he, "autotuner setup");
    mag_status st = MAG_OK;
    float best_t = INFINITY;
    Candidate best_c = cands[0];
    for (const auto &c : cands) {
        if (!std::isfinite(c.est)) continue;
        mag_params prm;
        std::memset(&prm, 0, sizeof(prm));
        prm.select = MAG_SELECT_EXPLICIT;
        prm.map_kind = c.map;
        prm.q = c.q;
        prm.k = c.k;
        prm.sigma_prime = c.sp;
        mag_plan *pl = nullptr;
        if (mag_plan_create(patterns, r, m, &prm, &pl) != MAG_OK) continue;
        // first scan sizes the output (all candidates find the same occurrences)
        uint64_t z = 0;
        if (!d_out) {
            he = hipMalloc(&d_out, cap * sizeof(mag_match));
            if (he != hipSuccess) { st = hip_fail(he, "autotuner output"); mag_plan_destroy(pl); break; }
        }
        mag_status s = mag_scan(pl, d_sample, n_sample, d_out, cap, &z, nullptr, stream_);
        if (s == MAG_E_OVERFLOW) {
            (void)hipStreamSynchronize(stream);
            (void)hipFree(d_out);
            cap = z + 1024;
            he = hipMalloc(&d_out, cap * sizeof(mag_match));
            if (he != hipSuccess) { d_out = nullptr; st = hip_fail(he, "autotuner output"); mag_plan_destroy(pl); break; }
            s = mag_scan(pl, d_sample, n_sample, d_out, cap, &z, nullptr, stream_);
        }
        if (s != MAG_OK) { st = s; mag_plan_destroy(pl); break; }
        std::vector<float> ts;
        for (int rep = 0; rep < repeats && s == MAG_OK; ++rep) {
            (void)hipEventRecord(e0, stream);
            s = mag_scan_async(pl, d_sample, n_sample, d_out, cap, d_cnt, nullptr, stream_);
            (void)hipEventRecord(e1, stream);
            he = hipEventSynchronize(e1);
            float ms = 0;
            if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
            if (he != hipSuccess) { s = hip_fail(he, "autotuner timing"); break; }
            ts.push_back(ms);
        }
        mag_plan_destroy(pl);
        if (s != MAG_OK) { st = s; break; }
        std::sort(ts.begin(), ts.end());
        const float t = ts[ts.size() / 2];
        if (t < best_t) {
            best_t = t;
            best_c = c;
        }
    }
    (void)hipStreamSynchronize(stream);
    (void)hipFree(d_out);
    (void)hipFree(d_cnt);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != MAG_OK) return st;
    if (best) {
        std::memset(best, 0, sizeof(*best));
        best->select = MAG_SELECT_EXPLICIT;
        best->map_kind = best_c.map;
        best->q = best_c.q;
        best->k = best_c.k;
        best->sigma_prime = best_c.sp;
    }
    if (best_ms) *best_ms = best_t;
    return MAG_OK;
}
