// Learned parameter selection (include/mag.h): pattern-set features, the
// grid of candidate (q, k, sigma') triples, and the C ABI of the selector
// network whose kernels are in mlp.hip.
//
// The paper fixes q and k by formulas (Section 3.2) and lowers sigma' to keep
// sigma'^q tables small (Section 3.3). The selector instead predicts, for
// each of 32 choices (the dense mode, the alphabet mapping on q-grams, and 30
// (q, k, sigma') filter triples), the scan cost per text byte and the
// verifications per text byte from statistics of the pattern set, and takes
// the cheapest feasible choice; the fixed formulas remain the fallback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "mlp.hpp"

namespace mag {
namespace {

constexpr uint64_t kSelTableBudget = 64 * 1024;
constexpr int kSelMaxW = 32;      // batch-compatible state width

// Filter triples of choices 2..31: (q, k, level); level 0 takes sigma' = fit,
// level 1 sigma' = max(2, fit / 2).
struct GridEntry {
    int q, k, level;
};
GridEntry filter_entry(int c) {
    static const int qs[6] = {2, 3, 4, 5, 6, 8};
    if (c < 26) {
        const int i = c - 2;
        return {qs[i / 4], (i / 2) % 2 + 1, i % 2};
    }
    switch (c) {
        case 26: return {2, 3, 0};
        case 27: return {3, 3, 0};
        case 28: return {4, 3, 0};
        case 29: return {2, 4, 0};
        case 30: return {7, 1, 0};
        default: return {7, 1, 1};
    }
}

// D[q-1] = number of distinct q-byte substrings (q = 1..8) over every
// pattern and offset. Every window (pattern, offset) gets the key of its next
// up to 8 bytes, big-endian (bytes past the pattern end are 0) and the count
// of real bytes it holds; after one LSD radix sort of the keys, windows with
// equal q-byte prefixes are adjacent, so D_q is the number of prefix changes
// among the windows that hold at least q real bytes.
void distinct_substrings(const uint8_t *P, uint32_t r, uint32_t m, uint64_t D[8]) {
    const size_t count = (size_t)r * m;
    std::vector<uint64_t> key(count), key2(count);
    std::vector<uint8_t> len(count), len2(count);
    for (uint32_t i = 0; i < r; ++i) {
        const uint8_t *row = P + (size_t)i * m;
        for (uint32_t s = 0; s < m; ++s) {
            const uint32_t have = std::min<uint32_t>(8, m - s);
            uint64_t k = 0;
            for (uint32_t t = 0; t < 8; ++t) k = (k << 8) | (t < have ? row[s + t] : 0u);
            key[(size_t)i * m + s] = k;
            len[(size_t)i * m + s] = (uint8_t)have;
        }
    }
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = 8 * pass;
        size_t cnt[257] = {0};
        for (size_t i = 0; i < count; ++i) cnt[((key[i] >> shift) & 255u) + 1]++;
        for (int d = 0; d < 256; ++d) cnt[d + 1] += cnt[d];
        for (size_t i = 0; i < count; ++i) {
            const size_t at = cnt[(key[i] >> shift) & 255u]++;
            key2[at] = key[i];
            len2[at] = len[i];
        }
        key.swap(key2);
        len.swap(len2);
    }
    for (int q = 1; q <= 8; ++q) {
        const uint64_t mask = ~0ull << (64 - 8 * q);   // the first q bytes
        uint64_t d = 0, last = 0;
        bool any = false;
        for (size_t i = 0; i < count; ++i) {
            if (len[i] < q) continue;
            const uint64_t pre = key[i] & mask;
            if (!any || pre != last) ++d;
            last = pre;
            any = true;
        }
        D[q - 1] = d;
    }
}

int entry_bytes_w(int W) { return W <= 8 ? 1 : W <= 16 ? 2 : W <= 32 ? 4 : 8; }

}  // namespace
}  // namespace mag

struct mag_mlp {
    int device = -1;
    float *params = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *loss = nullptr;
    float *partials = nullptr;
    // one-set selection staging
    float *x1 = nullptr;
    uint8_t *f1 = nullptr;
    int32_t *pick1 = nullptr;
    uint64_t step = 0;
    bool has_params = false;
};

using namespace mag;

extern "C" {

mag_status mag_select_features(const uint8_t *patterns, uint32_t r, uint32_t m, float *out) {
    if (!out || !patterns || r == 0 || m == 0) return fail(MAG_E_INVALID, "features need a non-empty pattern set");
    const uint64_t N = (uint64_t)r * m;
    uint64_t hist[256] = {0};
    for (uint64_t i = 0; i < N; ++i) hist[patterns[i]]++;
    int sp = 0;
    double H = 0.0, pmax = 0.0;
    for (int c = 0; c < 256; ++c) {
        if (!hist[c]) continue;
        ++sp;
        const double p = (double)hist[c] / (double)N;
        H -= p * std::log2(p);
        pmax = std::max(pmax, p);
    }
    // distinct patterns: sort the rows, count changes
    std::vector<uint32_t> order(r);
    for (uint32_t i = 0; i < r; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        return std::memcmp(patterns + (size_t)a * m, patterns + (size_t)b * m, m) < 0;
    });
    uint32_t unique = r ? 1 : 0;
    for (uint32_t i = 1; i < r; ++i)
        if (std::memcmp(patterns + (size_t)order[i - 1] * m, patterns + (size_t)order[i] * m, m) != 0) ++unique;
    double f[16];
    f[0] = std::log2((double)sp) / 8.0;
    f[1] = m / 32.0;
    f[2] = std::log10((double)r) / 4.0;
    f[3] = H / 8.0;
    f[4] = pmax;
    f[5] = (double)unique / r;
    uint64_t D[8];
    distinct_substrings(patterns, r, m, D);
    for (int q = 1; q <= 8; ++q) {
        double v;
        if ((uint32_t)q > m) {
            v = 1.0;
        } else if (sp <= 1) {
            v = 0.0;
        } else {
            const double lg_cov = std::log2((double)D[q - 1]) - q * std::log2((double)sp);
            v = std::min(1.0, -lg_cov / 32.0);
        }
        f[5 + q] = v;
    }
    f[14] = heuristic_q(sp, r, m) / 8.0;
    f[15] = std::log2((double)N) / 20.0;
    for (int i = 0; i < 16; ++i) out[i] = (float)f[i];
    return MAG_OK;
}

mag_status mag_select_candidates(const uint8_t *patterns, uint32_t r, uint32_t m, mag_params *out,
                                 uint8_t *feasible) {
    if (!out || !feasible || m == 0 || (r && !patterns)) return fail(MAG_E_INVALID, "bad arguments");
    bool present[256] = {false};
    for (uint64_t i = 0; i < (uint64_t)r * m; ++i) present[patterns[i]] = true;
    int sp = 0;
    for (bool b : present) sp += b ? 1 : 0;
    sp = std::max(sp, 1);
    for (int c = 0; c < kSelOut; ++c) {
        std::memset(&out[c], 0, sizeof(out[c]));
        feasible[c] = 0;
    }
    // choice 0: every start position tested (the plan's heuristic q, k, sigma'
    // only shape the unused filter); choice 1: the alphabet mapping on
    // q-grams with its own heuristic
    out[0].select = MAG_SELECT_LEARNED;
    out[0].mode = MAG_MODE_DENSE;
    feasible[0] = 1;
    out[1].select = MAG_SELECT_LEARNED;
    out[1].mode = MAG_MODE_FILTER;
    out[1].map_kind = MAG_MAP_QGRAM;
    feasible[1] = r > 0 ? 1 : 0;
    for (int c = 2; c < kSelChoices; ++c) {
        mag_params &o = out[c];
        const GridEntry g = filter_entry(c);
        const int q = g.q, k = g.k;
        if (2 * q - 1 > (int)m) continue;
        const int L = ((int)m - q + 1) / q;
        if (k > L) continue;
        const int mprime = std::min(L / k, 64 / k);
        const int W = k * mprime;
        if (mprime < 1 || W > kSelMaxW) continue;
        const int e = entry_bytes_w(W);
        int fit = 1;
        for (int s = 1; s <= std::min(sp, 256); ++s) {
            const double codes = std::pow((double)s, q);
            if (codes * e <= (double)kSelTableBudget) fit = s;
        }
        int sig = fit;
        if (g.level == 1) {
            sig = std::max(2, fit / 2);
            if (sig >= fit) continue;
        }
        o.select = MAG_SELECT_EXPLICIT;
        o.mode = MAG_MODE_FILTER;
        o.map_kind = MAG_MAP_GREEDY;
        o.q = q;
        o.k = k;
        o.sigma_prime = sig;
        feasible[c] = 1;
    }
    return MAG_OK;
}

uint32_t mag_mlp_param_count(void) { return (uint32_t)kSelParams; }

mag_status mag_mlp_create(mag_mlp **out) {
    if (!out) return fail(MAG_E_INVALID, "out is NULL");
    *out = nullptr;
    mag_mlp *h = new (std::nothrow) mag_mlp();
    if (!h) return fail(MAG_E_NOMEM, "host allocation failed");
    hipError_t e = hipGetDevice(&h->device);
    const size_t P = (size_t)kSelParams * sizeof(float);
    if (e == hipSuccess) e = hipMalloc(&h->params, P);
    if (e == hipSuccess) e = hipMalloc(&h->m, P);
    if (e == hipSuccess) e = hipMalloc(&h->v, P);
    if (e == hipSuccess) e = hipMalloc(&h->grad, P);
    if (e == hipSuccess) e = hipMalloc(&h->loss, 16);
    if (e == hipSuccess) e = hipMalloc(&h->partials, (size_t)kSelGradGroups * (kSelParams + 2) * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&h->x1, kSelIn * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&h->f1, kSelOut);
    if (e == hipSuccess) e = hipMalloc(&h->pick1, 16);
    if (e == hipSuccess) e = hipMemset(h->params, 0, P);
    if (e == hipSuccess) e = hipMemset(h->m, 0, P);
    if (e == hipSuccess) e = hipMemset(h->v, 0, P);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipGetLastError();
        mag_mlp_destroy(h);
        return fail(MAG_E_NOMEM, "device allocation of the selector failed");
    }
    *out = h;
    return MAG_OK;
}

void mag_mlp_destroy(mag_mlp *h) {
    if (!h) return;
    for (void *p : {(void *)h->params, (void *)h->m, (void *)h->v, (void *)h->grad, (void *)h->loss,
                    (void *)h->partials, (void *)h->x1, (void *)h->f1, (void *)h->pick1})
        (void)hipFree(p);
    delete h;
}

mag_status mag_mlp_set_params(mag_mlp *h, const float *host_params) {
    if (!h || !host_params) return fail(MAG_E_INVALID, "NULL argument");
    const size_t P = (size_t)kSelParams * sizeof(float);
    hipError_t e = hipMemcpy(h->params, host_params, P, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(h->m, 0, P);
    if (e == hipSuccess) e = hipMemset(h->v, 0, P);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "setting selector parameters");
    h->step = 0;
    h->has_params = true;
    return MAG_OK;
}

mag_status mag_mlp_get_params(mag_mlp *h, float *host_params) {
    if (!h || !host_params) return fail(MAG_E_INVALID, "NULL argument");
    hipError_t e = hipMemcpy(host_params, h->params, (size_t)kSelParams * sizeof(float),
                             hipMemcpyDeviceToHost);
    return e == hipSuccess ? MAG_OK : hip_fail(e, "reading selector parameters");
}

mag_status mag_mlp_forward(mag_mlp *h, const float *d_x, uint32_t B, float *d_y, void *stream) {
    if (!h || (B && (!d_x || !d_y))) return fail(MAG_E_INVALID, "NULL argument");
    return launch_mlp_forward(h->params, d_x, B, d_y, reinterpret_cast<hipStream_t>(stream));
}

mag_status mag_mlp_grad(mag_mlp *h, const float *d_x, const float *d_t, const uint8_t *d_mask,
                        uint32_t B, float *d_grad, float *d_loss, void *stream) {
    if (!h || !d_grad || !d_loss || (B && (!d_x || !d_t || !d_mask))) return fail(MAG_E_INVALID, "NULL argument");
    return launch_mlp_grad(h->params, d_x, d_t, d_mask, B, h->partials, d_grad, d_loss,
                           reinterpret_cast<hipStream_t>(stream));
}

mag_status mag_mlp_adam(mag_mlp *h, const float *d_grad, float lr, void *stream) {
    if (!h || !d_grad) return fail(MAG_E_INVALID, "NULL argument");
    const double b1 = 0.9, b2 = 0.999;
    h->step += 1;
    const float bc1 = (float)(1.0 - std::pow(b1, (double)h->step));
    const float bc2 = (float)(1.0 - std::pow(b2, (double)h->step));
    return launch_mlp_adam(h->params, d_grad, h->m, h->v, lr, (float)b1, (float)b2, 1e-8f, bc1, bc2,
                           reinterpret_cast<hipStream_t>(stream));
}

mag_status mag_mlp_train_step(mag_mlp *h, const float *d_x, const float *d_t, const uint8_t *d_mask,
                              uint32_t B, float lr, float *d_loss, void *stream) {
    if (!h) return fail(MAG_E_INVALID, "NULL argument");
    mag_status s = mag_mlp_grad(h, d_x, d_t, d_mask, B, h->grad, d_loss ? d_loss : h->loss, stream);
    if (s != MAG_OK) return s;
    return mag_mlp_adam(h, h->grad, lr, stream);
}

mag_status mag_mlp_select(mag_mlp *h, const float *d_x, const uint8_t *d_feasible, uint32_t B,
                          int32_t *d_pick, void *stream) {
    if (!h || (B && (!d_x || !d_feasible || !d_pick))) return fail(MAG_E_INVALID, "NULL argument");
    return launch_mlp_select(h->params, d_x, d_feasible, B, d_pick, reinterpret_cast<hipStream_t>(stream));
}

mag_status mag_select_learned(mag_mlp *h, const uint8_t *patterns, uint32_t r, uint32_t m,
                              mag_params *out, void *stream_) {
    if (!out) return fail(MAG_E_INVALID, "out is NULL");
    std::memset(out, 0, sizeof(*out));
    out->select = MAG_SELECT_HEURISTIC;          // the fallback
    if (!h || !h->has_params || r == 0) return MAG_OK;
    float x[kSelIn];
    mag_params cand[kSelOut];
    uint8_t feas[kSelOut];
    mag_status s = mag_select_features(patterns, r, m, x);
    if (s == MAG_OK) s = mag_select_candidates(patterns, r, m, cand, feas);
    if (s != MAG_OK) return s;
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
    int32_t pick = -1;
    hipError_t e = hipMemcpyAsync(h->x1, x, sizeof(x), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h->f1, feas, sizeof(feas), hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_fail(e, "selector input upload");
    s = launch_mlp_select(h->params, h->x1, h->f1, 1, h->pick1, stream);
    if (s != MAG_OK) return s;
    e = hipMemcpyAsync(&pick, h->pick1, sizeof(pick), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "selector pick download");
    if (pick >= 0 && pick < kSelChoices && feas[pick]) {
        *out = cand[pick];
        out->select = MAG_SELECT_LEARNED;
    }
    return MAG_OK;
}

}  // extern "C"
