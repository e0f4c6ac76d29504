// Host side of a MAG plan: parameter choice, alphabet map, superimposed mask
// table and the verification set.
//
//  - fixed heuristic for (q, k, sigma')            Section 3.2 and 3.3
//  - alphabet map mu (frequency rank / greedy bins) Section 3.3
//  - q-gram classes over all q shifts, superimposed Section 2
//  - k interleaved sub-patterns, Shift-Or masks     Sections 3.1-3.2
//  - exact verification set                         Section 3.2
//  - alphabet mapping on whole q-grams (hashed)     Section 3.3
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "mag_internal.hpp"

namespace mag {
namespace {

int round_half_up(double v) { return (int)std::floor(v + 0.5); }

int entry_bytes_for(int W) {
    if (W <= 8) return 1;
    if (W <= 16) return 2;
    if (W <= 32) return 4;
    return 8;
}

// Byte histogram of the pattern set and the present bytes ordered by
// descending count, equal counts by ascending byte value.
void frequency_order(const mag_plan *p, uint64_t hist[256], std::vector<int> &order) {
    std::fill(hist, hist + 256, 0);
    for (uint8_t c : p->patterns) hist[c]++;
    order.clear();
    for (int c = 0; c < 256; ++c)
        if (hist[c]) order.push_back(c);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return hist[a] > hist[b]; });
}

// mu by frequency rank: rank i -> code i, ranks >= sigma'-1 and absent bytes
// -> sigma'-1.
void map_rank(mag_plan *p) {
    uint64_t hist[256];
    std::vector<int> order;
    frequency_order(p, hist, order);
    std::fill(p->mu, p->mu + 256, (uint8_t)(p->sigma_prime - 1));
    for (size_t i = 0; i < order.size(); ++i)
        p->mu[order[i]] = (uint8_t)std::min<size_t>(i, p->sigma_prime - 1);
}

// mu by equal-weight bins: each byte, heaviest first, joins the lightest bin
// (lowest index on ties); absent bytes -> sigma'-1.
void map_greedy(mag_plan *p) {
    uint64_t hist[256];
    std::vector<int> order;
    frequency_order(p, hist, order);
    std::fill(p->mu, p->mu + 256, (uint8_t)(p->sigma_prime - 1));
    std::vector<uint64_t> load(p->sigma_prime, 0);
    for (int c : order) {
        int best = 0;
        for (int b = 1; b < p->sigma_prime; ++b)
            if (load[b] < load[best]) best = b;
        p->mu[c] = (uint8_t)best;
        load[best] += hist[c];
    }
}

// mu(c) = (c >> s) & (sigma' - 1) for sigma' = 2^l, with the shift s in
// 0..8-l that leaves the heaviest code the least pattern-byte weight (ties to
// the smaller s).
void map_bits(mag_plan *p) {
    uint64_t hist[256] = {0};
    for (uint8_t c : p->patterns) hist[c]++;
    const int sp = p->sigma_prime;
    int l = 0;
    while ((1 << l) < sp) ++l;
    uint64_t best = UINT64_MAX;
    int best_s = 0;
    for (int sh = 0; sh <= 8 - l; ++sh) {
        std::vector<uint64_t> load(sp, 0);
        for (int c = 0; c < 256; ++c) load[(c >> sh) & (sp - 1)] += hist[c];
        const uint64_t mx = *std::max_element(load.begin(), load.end());
        if (mx < best) {
            best = mx;
            best_s = sh;
        }
    }
    p->bits_shift = best_s;
    for (int c = 0; c < 256; ++c) p->mu[c] = (uint8_t)((c >> best_s) & (sp - 1));
}

// MurmurHash3's 64-bit finalizer: the q-gram map's hash.
uint64_t fmix64(uint64_t x) {
    x ^= x >> 33;
    x *= 0xFF51AFD7ED558CCDull;
    x ^= x >> 33;
    x *= 0xC4CEB9FE1A85EC53ull;
    x ^= x >> 33;
    return x;
}

// Code of the q raw bytes at g under the q-gram map with sigma' = 2^qbits.
uint64_t qgram_code(const uint8_t *g, int q, int qbits) {
    if (qbits == 0) return 0;
    uint64_t key = 0;
    for (int t = 0; t < q; ++t) key |= (uint64_t)g[t] << (8 * t);
    return fmix64(key) >> (64 - qbits);
}

int packed_bits(int W) { return W <= 1 ? 1 : W <= 2 ? 2 : 4; }

// Distinct raw grams of class b (all q shifts), as 64-bit keys.
std::vector<uint64_t> class_keys(const mag_plan *p, int q, int b) {
    std::vector<uint64_t> keys;
    keys.reserve((size_t)p->r * q);
    for (uint32_t i = 0; i < p->r; ++i) {
        const uint8_t *pat = p->patterns.data() + (size_t)i * p->m;
        for (int s = 0; s < q; ++s) {
            uint64_t key = 0;
            for (int t = 0; t < q; ++t) key |= (uint64_t)pat[s + b * q + t] << (8 * t);
            keys.push_back(key);
        }
    }
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    return keys;
}

// (q, k, sigma') of the q-gram map: the largest q, k = 1, and the smallest
// sigma' = 2^b with kQgramLoad codes per distinct gram of the fullest class,
// halved while the table exceeds the budget.
void heuristic_qgram(const mag_plan *p, int budget, int &q, int &k, int &sp) {
    q = std::max(1, std::min<int>(kMaxQ, ((int)p->m + 1) / 2));
    k = 1;
    const int L = ((int)p->m - q + 1) / q;
    const int W = std::min(L, kMaxW);
    const int eb = W <= 4 ? packed_bits(W) : 8 * entry_bytes_for(W);
    uint64_t D = 0;
    for (int b = 0; p->r && b < W; ++b) D = std::max<uint64_t>(D, class_keys(p, q, b).size());
    uint64_t s = 2;
    while (s < (uint64_t)kQgramLoad * D && s < (1ull << kMaxQgramLog2)) s *= 2;
    while (s > 2 && s * (uint64_t)eb > 8ull * (uint64_t)budget) s /= 2;
    sp = (int)s;
}

void heuristic(const mag_plan *p, int budget, int &q, int &k, int &sp) {
    uint64_t hist[256];
    std::vector<int> order;
    frequency_order(p, hist, order);
    const int sigma = (int)order.size();
    if (p->r == 0) {        // nothing to find: the cheapest valid plan
        q = k = sp = 1;
        return;
    }
    const double s = std::max(sigma, 2);
    const double lg = std::log((double)p->r * p->m) / std::log(s);   // log_sigma(rm)
    q = heuristic_q(sigma, p->r, p->m);
    const int L = ((int)p->m - q + 1) / q;
    const double rho = lg / p->m;
    if (rho >= 1.0 || lg <= 0) {
        k = 1;
    } else {
        const double inv = std::log(1.0 / rho) / std::log(s);
        k = round_half_up((double)p->m / lg * inv / (lg + inv));
        k = std::max(1, std::min(k, std::max(L, 1)));
    }
    k = std::min(k, kMaxK);
    const int mprime = std::min(L / k, kMaxW / k);
    const int eb = entry_bytes_for(k * mprime);
    sp = std::max(sigma, 1);
    auto fits = [&](int sg) {
        double codes = std::pow((double)sg, q);
        return codes * eb <= (double)budget;
    };
    while (sp > 1 && !fits(sp)) --sp;
}

// Mask table of the q-gram map. Packed tables hold entry c in bits
// [c*eb, (c+1)*eb) of the little-endian bit stream, padded to 16 bytes.
void build_table_qgram(mag_plan *p) {
    const int q = p->q, W = p->W, eb = p->entry_bits;
    const uint64_t bytes = eb < 8 ? ((p->n_codes * (uint64_t)eb + 127) / 128) * 16
                                  : p->n_codes * (uint64_t)p->esz;
    p->table.assign(bytes, 0xFF);
    uint8_t *tb = p->table.data();
    for (int b = 0; b < W; ++b) {
        for (uint64_t key : class_keys(p, q, b)) {
            uint8_t g[8];
            for (int t = 0; t < 8; ++t) g[t] = (uint8_t)(key >> (8 * t));
            const uint64_t code = qgram_code(g, q, p->qbits);
            const uint64_t bit = eb < 8 ? code * (uint64_t)eb + (uint64_t)b
                                        : code * 8ull * (uint64_t)p->esz + (uint64_t)b;
            tb[bit >> 3] &= (uint8_t)~(1u << (bit & 7));
        }
    }
}

void build_table(mag_plan *p) {
    if (p->map_kind == MAG_MAP_QGRAM) return build_table_qgram(p);
    const int q = p->q, sp = p->sigma_prime, W = p->W, esz = p->esz;
    p->table.assign(p->n_codes * esz, 0xFF);
    uint8_t *tb = p->table.data();
    const uint8_t *mu = p->mu;
    for (uint32_t i = 0; i < p->r; ++i) {
        const uint8_t *pat = p->patterns.data() + (size_t)i * p->m;
        for (int s = 0; s < q; ++s) {
            for (int b = 0; b < W; ++b) {
                const uint8_t *g = pat + s + b * q;
                uint64_t code = 0;
                for (int t = q - 1; t >= 0; --t) code = code * sp + mu[g[t]];
                // clear bit b of entry `code` (little-endian storage)
                tb[code * esz + (b >> 3)] &= (uint8_t)~(1u << (b & 7));
            }
        }
    }
}

void build_verifier(mag_plan *p) {
    const uint32_t r = p->r, m = p->m, mw = p->mw;
    // ids ordered by (pattern bytes, id): equal patterns become one run
    std::vector<uint32_t> order(r);
    std::iota(order.begin(), order.end(), 0u);
    const uint8_t *P = p->patterns.data();
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        return std::memcmp(P + (size_t)a * m, P + (size_t)b * m, m) < 0;
    });
    p->ids = order;
    p->idstart.clear();
    p->pwords.clear();
    for (uint32_t i = 0; i < r; ++i) {
        if (i == 0 || std::memcmp(P + (size_t)order[i] * m, P + (size_t)order[i - 1] * m, m) != 0) {
            p->idstart.push_back(i);
            const uint8_t *src = P + (size_t)order[i] * m;
            for (uint32_t t = 0; t < mw; ++t) {
                uint32_t w = 0;
                for (uint32_t b = 0; b < 4; ++b)
                    if (4 * t + b < m) w |= (uint32_t)src[4 * t + b] << (8 * b);
                p->pwords.push_back(w);
            }
        }
    }
    p->n_unique = (uint32_t)p->idstart.size();
    p->idstart.push_back(r);

    uint32_t bits = 1;
    while ((1ull << bits) < 2ull * std::max<uint32_t>(p->n_unique, 1)) ++bits;
    p->slot_bits = bits;
    p->slots.assign(1ull << bits, 0);
    const uint64_t mask = (1ull << bits) - 1;
    const int hw = std::min<int>(mw, kHashWords);
    for (uint32_t u = 0; u < p->n_unique; ++u) {
        const uint32_t h = window_hash(&p->pwords[(size_t)u * mw], hw);
        uint64_t s = (uint64_t)(h >> (32 - bits));
        while (p->slots[s]) s = (s + 1) & mask;
        p->slots[s] = ((uint64_t)h << 32) | (uint64_t)(u + 1);
    }
}

// Bloom bitmaps of the dense mode: for every distinct pattern's first
// min(m, 16) bytes, bits bloom_bit(bloom_probe(prefilter_hash, j), B) for
// j < kBloomBits, for B = bloom_log2 and for the batched copy's smaller B.
void build_bloom(mag_plan *p) {
    int B = kBloomMinLog2;
    while (B < kBloomMaxLog2 && (1ull << B) < 64ull * std::max<uint32_t>(p->n_unique, 1)) ++B;
    p->bloom_log2 = B;
    // kBloomBits bits per distinct pattern: a random position passes with
    // the bitmap's fill to that power
    const double fill =
        1.0 - std::exp(-(double)kBloomBits * (double)p->n_unique / (double)(1ull << B));
    p->bloom_fp = std::pow(fill, (double)kBloomBits);
    const int Bb = std::min(B, kBloomBatchLog2);
    p->bloom.assign((1u << B) / 32, 0u);
    p->bloom_batch.assign((1u << Bb) / 32, 0u);
    const int hw = std::min<int>(p->mw, kHashWords);
    for (uint32_t u = 0; u < p->n_unique; ++u) {
        const uint32_t h = prefilter_hash(&p->pwords[(size_t)u * p->mw], hw);
        for (int j = 0; j < kBloomBits; ++j) {
            const uint32_t x = bloom_probe(h, j);
            const uint32_t i = bloom_bit(x, B), ib = bloom_bit(x, Bb);
            p->bloom[i >> 5] |= 1u << (i & 31);
            p->bloom_batch[ib >> 5] |= 1u << (ib & 31);
        }
    }
}

// Exact window codes for the batched dense scans (see mag_plan::code_shift):
// patterns of at most 8 bytes over at most four byte values that one 2-bit
// field (b >> s) & 3, s = 0..6, tells apart (the smallest such s).
void build_codes(mag_plan *p) {
    p->code_shift = -1;
    p->code_rep = 0;
    p->code_bits.clear();
    p->code_ids.clear();
    if (p->var || p->m > 8 || p->n_unique == 0) return;
    bool used[256] = {false};
    for (uint8_t c : p->patterns) used[c] = true;
    std::vector<int> alpha;
    for (int b = 0; b < 256; ++b)
        if (used[b]) alpha.push_back(b);
    if (alpha.size() > 4) return;
    for (int s = 0; s <= 6 && p->code_shift < 0; ++s) {
        int seen = 0;
        bool ok = true;
        for (int b : alpha) {
            const int c = (b >> s) & 3;
            if (seen & (1 << c)) ok = false;
            seen |= 1 << c;
        }
        if (!ok) continue;
        p->code_shift = s;
        uint32_t rep = 0;
        for (int c = 0; c < 4; ++c) {
            // an unused code gets a byte of another code: no byte with code c matches it
            uint32_t byte = (uint32_t)(((c ^ 1) & 3) << s);
            for (int b : alpha)
                if (((b >> s) & 3) == c) byte = (uint32_t)b;
            rep |= byte << (8 * c);
        }
        p->code_rep = rep;
    }
    if (p->code_shift < 0) return;
    const int bits = 2 * (int)p->m;
    p->code_bits.assign(std::max<size_t>((1ull << bits) / 32, 4), 0u);
    p->code_ids.assign(1ull << bits, 0u);
    for (uint32_t u = 0; u < p->n_unique; ++u) {
        const uint8_t *w = reinterpret_cast<const uint8_t *>(&p->pwords[(size_t)u * p->mw]);
        uint32_t code = 0;
        for (uint32_t t = 0; t < p->m; ++t) code |= (uint32_t)((w[t] >> p->code_shift) & 3) << (2 * t);
        p->code_bits[code >> 5] |= 1u << (code & 31);
        const bool one = p->idstart[u + 1] - p->idstart[u] == 1;
        p->code_ids[code] = one ? (p->ids[p->idstart[u]] | kCodeDirect) : u + 1;
    }
}

// One-probe dense bitmap (slice_hash): built when the patterns are at least
// kSliceBytes long and their bytes carry enough entropy that a 6-byte slice
// spreads over the bitmap (6 H >= B + 4 bits, H the byte entropy of the
// pattern set). k = ln 2 * 2^B / (distinct patterns) slices, the Bloom
// optimum, within [1, kSliceMaxK] and the slices that fit in m bytes.
void build_slices(mag_plan *p, int dense_probe) {
    p->slice_k = 0;
    p->slice_fp = 0.0;
    p->slices.clear();
    p->wf_bits = 0;
    p->wfilter.clear();
    if (dense_probe == MAG_DENSE_PROBE_BLOOM || p->m < (uint32_t)kSliceBytes || p->n_unique == 0)
        return;
    const int B = p->bloom_log2;
    if (dense_probe != MAG_DENSE_PROBE_SLICES) {
        double hist[256] = {0};
        for (uint8_t c : p->patterns) hist[c] += 1.0;
        double H = 0.0;
        for (double c : hist)
            if (c > 0) {
                const double f = c / (double)p->patterns.size();
                H -= f * std::log2(f);
            }
        if (kSliceBytes * H < B + 4.0) return;
    }
    const int kmax = std::min<int>(kSliceMaxK, ((int)p->m - kSliceBytes) / kSliceStride + 1);
    int k = (int)std::lround(std::log(2.0) * (double)(1ull << B) / (double)p->n_unique);
    k = std::max(1, std::min(k, kmax));
    p->slice_k = k;
    p->slices.assign((1u << B) / 32, 0u);
    uint8_t buf[kMaxM + 8];
    for (uint32_t u = 0; u < p->n_unique; ++u) {
        std::memset(buf, 0, sizeof(buf));
        std::memcpy(buf, &p->pwords[(size_t)u * p->mw], p->m);
        for (int j = 0; j < k; ++j) {
            const uint8_t *s = buf + kSliceStride * j;
            const uint32_t lo = s[0] | (uint32_t)s[1] << 8 | (uint32_t)s[2] << 16;
            const uint32_t hi = s[3] | (uint32_t)s[4] << 8 | (uint32_t)s[5] << 16;
            const uint32_t h = slice_hash(lo, hi);
            p->slices[h >> (37 - B)] |= 1u << ((h >> (32 - B)) & 31u);
        }
    }
    uint64_t set = 0;
    for (uint32_t w : p->slices) set += (uint64_t)__builtin_popcount(w);
    p->slice_fp = std::pow((double)set / (double)(1ull << B), (double)k);
    // the word filter over the window hashes: about one pattern per word
    int F = 6;
    while (F < 30 && (1ull << F) < p->n_unique) ++F;
    p->wf_bits = F;
    p->wfilter.assign(1ull << F, 0ull);
    const int hw = std::min<int>(p->mw, kHashWords);
    for (uint32_t u = 0; u < p->n_unique; ++u) {
        const uint32_t h = window_hash(&p->pwords[(size_t)u * p->mw], hw);
        p->wfilter[h >> (32 - F)] |= word_filter_mask(h);
    }
}

}  // namespace

namespace {

// p_b of the q-gram map: the probability that a text gram (bytes drawn
// independently by the pattern-set byte frequencies) is one of the class's
// grams, plus, for every other gram, the share of codes the class occupies.
double qgram_class_probability(const mag_plan *p, const double *freq, int b) {
    double exact = 0.0;
    std::vector<uint64_t> codes;
    for (uint64_t key : class_keys(p, p->q, b)) {
        double pr = 1.0;
        uint8_t g[8];
        for (int t = 0; t < p->q; ++t) {
            g[t] = (uint8_t)(key >> (8 * t));
            pr *= freq[g[t]];
        }
        exact += pr;
        codes.push_back(qgram_code(g, p->q, p->qbits));
    }
    std::sort(codes.begin(), codes.end());
    const double occupied = (double)(std::unique(codes.begin(), codes.end()) - codes.begin());
    const double share = occupied / (double)p->n_codes;
    return std::min(1.0, exact + (1.0 - std::min(exact, 1.0)) * share);
}

}  // namespace

double estimate_verifications(const mag_plan *p) {
    if (p->r == 0) return 0.0;
    if (p->map_kind == MAG_MAP_QGRAM) {
        double freq[256] = {0};
        for (uint8_t c : p->patterns) freq[c] += 1.0;
        for (double &f : freq) f /= (double)p->patterns.size();
        std::vector<double> pb(p->W);
        for (int b = 0; b < p->W; ++b) pb[b] = qgram_class_probability(p, freq, b);
        double cand = 0.0;
        for (int j = 0; j < p->k; ++j) {
            double prod = 1.0;
            for (int h = 0; h < p->mprime; ++h) prod *= pb[j + h * p->k];
            cand += prod;
        }
        return cand / (double)p->k;
    }
    if (p->n_codes > (1ull << 22)) return -1.0;
    const int sp = p->sigma_prime, q = p->q, W = p->W, k = p->k, esz = p->esz;
    double byte_freq[256] = {0};
    for (uint8_t c : p->patterns) byte_freq[c] += 1.0;
    for (double &f : byte_freq) f /= (double)p->patterns.size();
    std::vector<double> sym(sp, 0.0);
    for (int c = 0; c < 256; ++c) sym[p->mu[c]] += byte_freq[c];
    // p_b: probability that a text gram lies in class C[b]
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
    // candidate windows per sample (every j of k), q starts each, one sample per kq bytes
    double cand = 0.0;
    for (int j = 0; j < k; ++j) {
        double prod = 1.0;
        for (int h = 0; h < p->mprime; ++h) prod *= std::min(1.0, pb[j + h * k]);
        cand += prod;
    }
    return cand * q / ((double)k * q);
}

int heuristic_q_formula(int sigma, uint32_t r, uint32_t m) {
    if (r == 0 || m == 0) return 0;
    const double s = std::max(sigma, 2);
    const double lg = std::log((double)r * m) / std::log(s);   // log_sigma(rm)
    return std::max(1, std::min(round_half_up(lg), (int)(m + 1) / 2));
}

int heuristic_q(int sigma, uint32_t r, uint32_t m) {
    return std::min(heuristic_q_formula(sigma, r, m), kMaxQ);
}

mag_status build_plan(mag_plan *p, const uint8_t *patterns, uint32_t r, uint32_t m,
                      const mag_params *params) {
    mag_params prm;
    std::memset(&prm, 0, sizeof(prm));
    if (params) prm = *params;
    if (m == 0) return fail(MAG_E_INVALID, "pattern length m must be >= 1");
    if (m > (uint32_t)kMaxM) return fail(MAG_E_UNSUPPORTED, "pattern length above 64");
    if (r > 0 && !patterns) return fail(MAG_E_INVALID, "patterns is NULL");
    if (prm.map_kind < MAG_MAP_GREEDY || prm.map_kind > MAG_MAP_QGRAM)
        return fail(MAG_E_INVALID, "unknown map_kind");
    const bool qgram = prm.map_kind == MAG_MAP_QGRAM;
    if (prm.mode < MAG_MODE_AUTO || prm.mode > MAG_MODE_DENSE) return fail(MAG_E_INVALID, "unknown mode");
    if (prm.verify < MAG_VERIFY_AUTO || prm.verify > MAG_VERIFY_DEFERRED)
        return fail(MAG_E_INVALID, "unknown verify");
    if (prm.verify_buffer < 0) return fail(MAG_E_INVALID, "verify_buffer must be >= 0");
    if (prm.encode != 0 && prm.encode != 1) return fail(MAG_E_INVALID, "encode must be 0 or 1");
    if (prm.dense_probe < MAG_DENSE_PROBE_AUTO || prm.dense_probe > MAG_DENSE_PROBE_BLOOM)
        return fail(MAG_E_INVALID, "unknown dense_probe");
    if (prm.dense_probe == MAG_DENSE_PROBE_SLICES && m < (uint32_t)kSliceBytes)
        return fail(MAG_E_INVALID, "the one-probe dense bitmap needs m >= 6");
    if (prm.chunk_bytes < 0 || prm.words_per_lane < 0)
        return fail(MAG_E_INVALID, "chunk_bytes and words_per_lane must be >= 0");
    if (prm.chunk_bytes && prm.words_per_lane)
        return fail(MAG_E_INVALID, "give chunk_bytes or words_per_lane, not both");
    if (prm.words_per_lane > 256 || (prm.chunk_bytes && prm.chunk_bytes < 1024))
        return fail(MAG_E_INVALID, "words_per_lane above 256 or chunk_bytes below 1024");
    if (r >= (1u << 31)) return fail(MAG_E_UNSUPPORTED, "too many patterns");

    p->r = r;
    p->m = m;
    p->m_max = m;
    p->mw = (m + 3) / 4;
    p->patterns.assign(patterns, patterns + (size_t)r * m);
    p->map_kind = prm.map_kind;
    p->select = prm.select;

    {
        uint64_t hist[256];
        std::vector<int> order;
        frequency_order(p, hist, order);
        p->q_formula = heuristic_q_formula((int)order.size(), r, m);
    }
    int q, k, sp;
    const int budget = prm.table_budget > 0 ? prm.table_budget
                                            : (qgram ? kQgramTableBudget : kDefaultTableBudget);
    auto pick = [&]() {
        if (qgram) heuristic_qgram(p, budget, q, k, sp);
        else heuristic(p, budget, q, k, sp);
    };
    switch (prm.select) {
        case MAG_SELECT_LEARNED:    // a pick resolved by mag_select_learned
            if (prm.q > 0 && prm.k > 0 && prm.sigma_prime > 0) {
                q = prm.q;
                k = prm.k;
                sp = prm.sigma_prime;
                break;
            }
            pick();
            break;
        case MAG_SELECT_HEURISTIC:
        case MAG_SELECT_AUTOTUNE:   // mag_autotune returns its pick as explicit parameters
            pick();
            break;
        case MAG_SELECT_EXPLICIT:
            q = prm.q;
            k = prm.k;
            sp = prm.sigma_prime;
            break;
        default:
            return fail(MAG_E_INVALID, "unknown select");
    }
    if (q < 1 || 2 * q - 1 > (int)m) return fail(MAG_E_INVALID, "need 1 <= q and 2q-1 <= m");
    if (q > kMaxQ) return fail(MAG_E_UNSUPPORTED, "q above 8");
    const int L = ((int)m - q + 1) / q;
    if (k < 1 || k > L) return fail(MAG_E_INVALID, "need 1 <= k <= L = (m-q+1)/q");
    if (k > kMaxK) return fail(MAG_E_UNSUPPORTED, "k above 32");
    if (qgram) {
        if (sp < 1 || sp > (1 << kMaxQgramLog2) || (sp & (sp - 1)))
            return fail(MAG_E_INVALID, "the q-gram map needs sigma' = 2^b with b <= 28");
    } else if (sp < 1 || sp > 256) {
        return fail(MAG_E_INVALID, "sigma' must be in [1, 256]");
    }
    if (prm.map_kind == MAG_MAP_BITS && (sp & (sp - 1))) {
        // the bit-field map needs a power of two: the heuristic's sigma' is
        // lowered to one, an explicit one must be one
        if (prm.select == MAG_SELECT_EXPLICIT) return fail(MAG_E_INVALID, "the bit-field map needs sigma' = 2^l");
        while (sp & (sp - 1)) sp &= sp - 1;
    }
    double codes = qgram ? (double)sp : std::pow((double)sp, q);
    p->q = q;
    p->k = k;
    p->sigma_prime = sp;
    p->L = L;
    p->mprime = std::min(L / k, kMaxW / k);
    p->W = k * p->mprime;
    p->esz = entry_bytes_for(p->W);
    p->entry_bits = qgram && p->W <= 4 ? packed_bits(p->W) : 8 * p->esz;
    if (codes * p->entry_bits / 8.0 > (double)kMaxTableBytes)
        return fail(MAG_E_UNSUPPORTED, "mask table above 1 GiB");
    p->n_codes = 1;
    if (qgram) {
        p->n_codes = (uint64_t)sp;
        p->qbits = 0;
        while ((1 << p->qbits) < sp) ++p->qbits;
    } else {
        for (int t = 0; t < q; ++t) p->n_codes *= (uint64_t)sp;
    }

    if (p->map_kind == MAG_MAP_RANK) map_rank(p);
    else if (p->map_kind == MAG_MAP_BITS) map_bits(p);
    else if (qgram) std::memset(p->mu, 0, sizeof(p->mu));
    else map_greedy(p);
    build_table(p);
    build_verifier(p);
    build_bloom(p);
    build_slices(p, prm.dense_probe);
    build_codes(p);
    p->dense_probe = prm.dense_probe;
    p->chunk_bytes = prm.chunk_bytes;
    p->words_per_lane = prm.words_per_lane;
    p->mode = prm.mode;
    p->verify = prm.verify;
    p->verify_buffer = (uint64_t)prm.verify_buffer;
    p->encode = prm.encode;
    p->est_verif = estimate_verifications(p);
    // A learned pick with sigma' = 2^l: the bit-field map's codes need no map
    // lookups and scan faster; take it when its classes stay about as
    // selective (the selector's costs were measured with the greedy map).
    if (prm.select == MAG_SELECT_LEARNED && p->map_kind == MAG_MAP_GREEDY && p->r && sp > 1 &&
        (sp & (sp - 1)) == 0 && p->est_verif >= 0.0 && p->est_verif < kDenseVerifPerByte) {
        uint8_t mu_g[256];
        std::memcpy(mu_g, p->mu, 256);
        std::vector<uint8_t> table_g = p->table;
        const double est_g = p->est_verif;
        p->map_kind = MAG_MAP_BITS;
        map_bits(p);
        build_table(p);
        const double est_b = estimate_verifications(p);
        if (est_b >= 0.0 && est_b <= 1.25 * est_g + kLearnedBitsSlack) {
            p->est_verif = est_b;
        } else {
            p->map_kind = MAG_MAP_GREEDY;
            p->bits_shift = 0;
            std::memcpy(p->mu, mu_g, 256);
            p->table.swap(table_g);
        }
    }
    p->dense = prm.mode == MAG_MODE_DENSE ||
               (prm.mode == MAG_MODE_AUTO && p->est_verif >= kDenseVerifPerByte);
    return MAG_OK;
}

namespace {

// Verification set of a plan with unequal lengths. Ids are ordered by
// (first m bytes, length, bytes, id): equal patterns form one run of ids per
// distinct pattern u, and distinct patterns sharing their first m bytes form
// one group, which the probe table indexes by the hash of those bytes.
void build_verifier_var(mag_plan *p) {
    const uint32_t r = p->r, m = p->m;
    const uint8_t *B = p->fbytes.data();
    auto len = [&](uint32_t i) { return (uint32_t)(p->foff[i + 1] - p->foff[i]); };
    auto at = [&](uint32_t i) { return B + p->foff[i]; };
    std::vector<uint32_t> order(r);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        const int c = std::memcmp(at(a), at(b), m);
        if (c) return c < 0;
        if (len(a) != len(b)) return len(a) < len(b);
        return std::memcmp(at(a), at(b), len(a)) < 0;
    });
    p->ids = order;
    p->idstart.clear();
    p->pwords.clear();
    p->pwoff.clear();
    p->plen.clear();
    p->gstart.clear();
    for (uint32_t i = 0; i < r; ++i) {
        const uint32_t a = order[i];
        const bool new_u = i == 0 || len(a) != len(order[i - 1]) ||
                           std::memcmp(at(a), at(order[i - 1]), len(a)) != 0;
        if (!new_u) continue;
        const bool new_g = i == 0 || std::memcmp(at(a), at(order[i - 1]), m) != 0;
        if (new_g) p->gstart.push_back((uint32_t)p->idstart.size());
        p->idstart.push_back(i);
        p->pwoff.push_back((uint32_t)p->pwords.size());
        p->plen.push_back(len(a));
        for (uint32_t t = 0; t < (len(a) + 3) / 4; ++t) {
            uint32_t w = 0;
            for (uint32_t b = 0; b < 4; ++b)
                if (4 * t + b < len(a)) w |= (uint32_t)at(a)[4 * t + b] << (8 * b);
            p->pwords.push_back(w);
        }
    }
    p->n_unique = (uint32_t)p->idstart.size();
    p->idstart.push_back(r);
    const uint32_t groups = (uint32_t)p->gstart.size();
    p->gstart.push_back(p->n_unique);

    uint32_t bits = 1;
    while ((1ull << bits) < 2ull * std::max<uint32_t>(groups, 1)) ++bits;
    p->slot_bits = bits;
    p->slots.assign(1ull << bits, 0);
    const uint64_t mask = (1ull << bits) - 1;
    const int hw = std::min<int>(p->mw, kHashWords);
    const uint32_t lastmask = (m & 3) ? ((1u << (8 * (m & 3))) - 1u) : 0xFFFFFFFFu;
    for (uint32_t g = 0; g < groups; ++g) {
        uint32_t hv[kHashWords] = {0};
        const uint32_t *pw = &p->pwords[p->pwoff[p->gstart[g]]];
        for (int t = 0; t < hw; ++t) hv[t] = (t == (int)p->mw - 1) ? (pw[t] & lastmask) : pw[t];
        const uint32_t h = window_hash(hv, hw);
        uint64_t s = (uint64_t)(h >> (32 - bits));
        while (p->slots[s]) s = (s + 1) & mask;
        p->slots[s] = ((uint64_t)h << 32) | (uint64_t)(g + 1);
    }
}

}  // namespace

mag_status build_plan_var(mag_plan *p, const uint8_t *bytes, const uint64_t *offsets, uint32_t r,
                          const mag_params *params) {
    if (r == 0) return fail(MAG_E_INVALID, "unequal-length plans need at least one pattern");
    if (!bytes || !offsets) return fail(MAG_E_INVALID, "bytes or offsets is NULL");
    uint32_t m_min = UINT32_MAX, m_max = 0;
    for (uint32_t i = 0; i < r; ++i) {
        if (offsets[i + 1] < offsets[i]) return fail(MAG_E_INVALID, "offsets must not decrease");
        const uint64_t L = offsets[i + 1] - offsets[i];
        if (L == 0) return fail(MAG_E_INVALID, "pattern length must be >= 1");
        if (L > (uint64_t)kMaxM) return fail(MAG_E_UNSUPPORTED, "pattern length above 64");
        m_min = std::min<uint32_t>(m_min, (uint32_t)L);
        m_max = std::max<uint32_t>(m_max, (uint32_t)L);
    }
    // the filter's view: every pattern's first m_min bytes
    std::vector<uint8_t> prefixes((size_t)r * m_min);
    for (uint32_t i = 0; i < r; ++i)
        std::memcpy(&prefixes[(size_t)i * m_min], bytes + offsets[i], m_min);
    mag_status s = build_plan(p, prefixes.data(), r, m_min, params);
    if (s != MAG_OK) return s;
    p->var = 1;
    p->m_max = m_max;
    p->fbytes.assign(bytes + offsets[0], bytes + offsets[r]);
    p->foff.resize(r + 1);
    for (uint32_t i = 0; i <= r; ++i) p->foff[i] = offsets[i] - offsets[0];
    build_verifier_var(p);
    return MAG_OK;
}

}  // namespace mag
