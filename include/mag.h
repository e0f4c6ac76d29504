/*
 * mag.h - C ABI of the MAG multiple-pattern-matching scan on MI355X (gfx950).
 *
 * Problem (Section 1 of Susik, Grabowski, Fredriksson, "Multiple pattern
 * matching revisited"): given a text T of n bytes and r patterns P_0..P_{r-1},
 * all of the same length m, report every occurrence
 *
 *     (i, id)  with  0 <= i <= n-m  and  T[i..i+m) == P_id.
 *
 * Method (Sections 2-3, "MAG"): bytes are reduced to sigma' codes (Section 3.3),
 * the patterns are cut into non-overlapping q-grams for all q shifts and
 * superimposed into character classes (Section 2), the classes are split into
 * k interleaved sub-patterns searched with one bit-parallel Shift-Or automaton
 * that reads every k-th q-gram of the text (Sections 3.1-3.2), and each window
 * that survives is verified exactly (Section 3.2). The filter only prunes, so
 * the output is exactly the occurrence set above.
 *
 * Conventions shared by every call:
 *  - Pointers named d_* are device pointers (HIP, current device); all others
 *    are host pointers. The library never frees caller memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream). Work
 *    is enqueued in stream order; device outputs are valid once the stream
 *    has reached that point.
 *  - Every call returns mag_status; on failure mag_last_error() holds a
 *    thread-local description. Calls are thread-compatible: one plan may be
 *    scanned by one stream at a time (its scratch buffers are shared).
 *  - A match record is 16 bytes {u64 pos, u32 pattern_id, u32 reserved=0}.
 *    Records are sorted ascending by (pos, pattern_id); positions are
 *    0-based starts; overlapping matches are all reported and every id of a
 *    repeated pattern is reported.
 */
#ifndef MAG_H
#define MAG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MAG_OK = 0,
    MAG_E_INVALID = -1,     /* bad argument or parameter combination           */
    MAG_E_UNSUPPORTED = -2, /* valid but outside the library's limits         */
    MAG_E_NOMEM = -3,       /* host or device allocation failed                */
    MAG_E_DEVICE = -4,      /* a HIP call failed (detail in mag_last_error)    */
    MAG_E_OVERFLOW = -5     /* output capacity too small; count still returned */
} mag_status;

/* How the filter parameters (q, k, sigma') are chosen. */
typedef enum {
    MAG_SELECT_HEURISTIC = 0, /* q = log_sigma(rm), k from Section 3.2, sigma'
                                 lowered until the mask table fits the budget */
    MAG_SELECT_EXPLICIT = 1,  /* q, k, sigma_prime taken from mag_params       */
    MAG_SELECT_LEARNED = 2,   /* a pick of mag_select_learned: q, k, sigma_prime
                                 as it filled them; all zero = the heuristic.
                                 With the greedy map and sigma' = 2^l the plan
                                 takes the bit-field map instead when its
                                 expected verifications per byte are at most
                                 1.25x the greedy map's + 1e-5                */
    MAG_SELECT_AUTOTUNE = 3   /* measured on the device over a small grid      */
} mag_select;

/* How start positions reach exact verification. */
typedef enum {
    MAG_MODE_AUTO = 0,   /* dense when the filter is expected to pass more than
                            0.1 start positions per text byte                  */
    MAG_MODE_FILTER = 1, /* the q-gram Shift-Or filter of Sections 2-3         */
    MAG_MODE_DENSE = 2   /* every start position, through a Bloom bitmap of the
                            patterns' first min(m, 16) bytes (the degenerate
                            filter that passes every window, Section 3.2)      */
} mag_mode;

/* Where filter survivors are verified (Section 3.2's exact check). */
typedef enum {
    MAG_VERIFY_AUTO = 0,     /* deferred when a filter scan is expected to
                                verify at least 2^24 start positions, else
                                inline (the dense mode always inline)          */
    MAG_VERIFY_INLINE = 1,   /* by the filter kernel's own waves               */
    MAG_VERIFY_DEFERRED = 2  /* the filter kernel appends the start positions
                                to a device buffer and a verification kernel
                                with a full-occupancy grid checks them; starts
                                past the buffer's capacity are verified inline,
                                so the result never depends on it              */
} mag_verify;

/* Alphabet reduction mu: byte -> [0, sigma') (Section 3.3). */
typedef enum {
    MAG_MAP_GREEDY = 0, /* equal-weight bins by longest-processing-time greedy */
    MAG_MAP_RANK = 1,   /* frequency rank; ranks >= sigma'-1 share the last code */
    MAG_MAP_BITS = 2,   /* bit fields (combined alphabet mapping and q-gram
                           generation): sigma' = 2^l, mu(c) = (c >> s) & (2^l-1)
                           with the shift s that spreads the pattern bytes most
                           evenly; the scan computes codes without a map table */
    MAG_MAP_QGRAM = 3   /* alphabet mapping on q-grams (Section 3.3): the whole
                           gram (its q <= 8 raw bytes, S[0] in the low byte of a
                           64-bit key) is mapped to the top log2(sigma') bits of
                           MurmurHash3's 64-bit finalizer. sigma' is a power of
                           two in [1, 2^28] and counts table entries directly
                           (not sigma'^q); tables with W <= 4 are packed at 1, 2
                           or 4 bits per entry. The heuristic takes the largest
                           q, k = 1 and sigma' >= 32 codes per distinct gram of
                           the fullest class within table_budget (0 = 8 MiB).
                           Not accepted by mag_batch_create unless dense.      */
} mag_map_kind;

/* How the dense mode tests a start position before exact verification. */
typedef enum {
    MAG_DENSE_PROBE_AUTO = 0,   /* slices when the patterns have m >= 6 and their
                                   bytes carry enough entropy (6 H >= B + 4 bits,
                                   H the pattern bytes' entropy, 2^B the bitmap's
                                   bits), else the Bloom bitmap                 */
    MAG_DENSE_PROBE_SLICES = 1, /* one bitmap word per position: every distinct
                                   pattern sets the bits of its 6-byte slices at
                                   offsets 0, 2, .., 2(k-1) (k <= 8, the Bloom
                                   optimum for the pattern count), and a position
                                   passes when its own slices' bits are all set;
                                   neighbouring positions share the probes.
                                   Needs m >= 6                                  */
    MAG_DENSE_PROBE_BLOOM = 2   /* three probes per position into a Bloom bitmap
                                   of the first min(m, 16) bytes                */
} mag_dense_probe;

typedef struct {
    int32_t select;       /* mag_select                                         */
    int32_t map_kind;     /* mag_map_kind                                       */
    int32_t q;            /* q-gram length (explicit selection)                 */
    int32_t k;            /* sampling parameter (explicit selection)            */
    int32_t sigma_prime;  /* reduced alphabet size (explicit selection)         */
    int32_t table_budget; /* bytes the heuristic allows for the mask table;
                             0 = 96 KiB (8 MiB for MAG_MAP_QGRAM)                */
    int32_t mode;         /* mag_mode                                           */
    int32_t verify;       /* mag_verify                                         */
    int32_t verify_buffer;/* entries of the deferred-start buffer; 0 = sized
                             from the expected verifications (2^20 .. 2^26)     */
    int32_t encode;       /* 0: MAG, q-gram codes computed on the fly while
                             scanning; 1: SMAG, each scan first encodes the
                             whole text (mag_encode's codes, kept in 16 bits
                             when sigma'^q <= 2^16) and the filter reads them
                             (Section 3.2, "Implementation"). Same results;
                             the dense mode and batches always compute on the
                             fly                                               */
    int32_t chunk_bytes;  /* reserved for the tile size; must be 0 (auto)       */
    int32_t words_per_lane; /* reserved for the lane run length; must be 0      */
    int32_t dense_probe;  /* mag_dense_probe                                    */
    int32_t reserved[3];  /* must be zero                                       */
} mag_params;

typedef struct {
    uint64_t pos;
    uint32_t pattern_id;
    uint32_t reserved;
} mag_match;

/* Resolved shape of a plan (filled by mag_plan_info). */
typedef struct {
    int32_t q, k, sigma_prime;
    int32_t L;            /* gram positions shared by all shifts: (m-q+1)/q     */
    int32_t m_prime;      /* sub-pattern length: min(L/k, 64/k)                 */
    int32_t W;            /* automaton bits: k * m_prime                        */
    int32_t entry_bytes;  /* bytes per mask-table entry (1, 2, 4 or 8)          */
    int32_t map_kind;
    int32_t select;       /* how the parameters were chosen                     */
    uint32_t r, m;
    uint32_t n_unique;    /* distinct patterns                                  */
    int32_t dense;        /* 1: scans test every start position (mag_mode)      */
    int32_t bloom_log2;   /* bits of the dense mode's Bloom bitmap (log2)       */
    int32_t bits_shift;   /* s of the bit-field map (MAG_MAP_BITS), else 0      */
    int32_t entry_bits;   /* bits a stored table entry takes: 1, 2 or 4 when
                             packed (MAG_MAP_QGRAM with W <= 4), else
                             8 * entry_bytes                                    */
    uint64_t n_codes;     /* mask-table entries: sigma'^q (sigma' for QGRAM)    */
    uint64_t table_bytes; /* n_codes * entry_bits / 8, padded to 16 bytes       */
    double est_verif;     /* estimated verifications per text byte of the
                             filter (-1: not evaluated)                        */
    uint32_t m_max;       /* longest pattern (m for equal lengths)             */
    uint32_t var;         /* 1: built by mag_plan_create_var; m is the shortest
                             length and the filter sees every pattern's first
                             m bytes                                           */
    int32_t q_formula;    /* q by Section 3.2's formula for this pattern set:
                             log_sigma(r*m), sigma the number of distinct
                             pattern bytes (at least 2), rounded half up and
                             clamped to [1, (m+1)/2]; 0 when r == 0. The
                             heuristic runs min(q_formula, 8): the scan kernels
                             are built for grams of at most 8 bytes          */
    int32_t dense_slices; /* one-probe dense bitmap: slices per pattern (k of
                             MAG_DENSE_PROBE_SLICES); 0 when dense scans use the
                             Bloom bitmap                                      */
    double dense_pass;    /* estimated share of start positions the dense
                             mode's bitmap passes to exact verification        */
} mag_plan_desc;

/* Work counters of one scan (integers; equal to the oracle's counts) and
 * the plan's resolved parameters. mag_scan fills every field; the device
 * copy that mag_scan_async and mag_scan_noalloc write holds all of them but
 * scan_ms (0: only mag_scan, which waits, times the scan). */
typedef struct {
    uint64_t samples;        /* text q-grams read by the filter (dense mode:
                                start positions tested)                        */
    uint64_t cand_windows;   /* (x, j) windows that passed the filter (dense
                                mode: positions that passed its bitmap)        */
    uint64_t verifications;  /* start positions verified exactly                */
    uint64_t matches;        /* occurrences found                               */
    int32_t q, k, sigma_prime, m_prime;   /* the plan's filter parameters       */
    float plan_ms;           /* host time mag_plan_create took for the plan     */
    float scan_ms;           /* device time of the scan and finishing kernels
                                (mag_scan only, else 0)                         */
} mag_stats;

typedef struct mag_plan mag_plan;

/* Builds a plan for the pattern set of Section 1's problem: r patterns of
 * length m (host array, row-major r*m bytes; copied, so the caller may free
 * it on return), preprocessed by Sections 2-3 (alphabet map, superimposed
 * q-gram classes, Shift-Or masks, verification set). params may be NULL (heuristic,
 * greedy map). Host-only work: device tables are uploaded on first use.
 * Errors: m == 0 or m > 64, explicit q with 2q-1 > m, k outside [1, L],
 * sigma' outside [1, 256] (for MAG_MAP_QGRAM: not a power of two in
 * [1, 2^28]) or a mask table above 1 GiB -> MAG_E_INVALID /
 * MAG_E_UNSUPPORTED. r == 0 is valid (every scan returns no match). */
mag_status mag_plan_create(const uint8_t *patterns, uint32_t r, uint32_t m,
                           const mag_params *params, mag_plan **out);

/* Builds a plan for r patterns of unequal lengths (the introduction notes
 * the equal-length requirement may be removed): pattern i is
 * bytes[offsets[i] .. offsets[i+1]) (host arrays, copied), 1 to 64 bytes.
 * The filter is the one mag_plan_create builds for the patterns' first m_min
 * bytes (m_min = the shortest length; every occurrence contains an
 * occurrence of its prefix, so none is lost); verification checks each
 * candidate start against every distinct pattern with that prefix over its
 * full length, and a pattern only matches where it ends inside the text.
 * Results: every (i, id) with T[i .. i + len_id) == P_id, sorted. Equal
 * lengths give the same plan as mag_plan_create. Errors: r == 0, NULL
 * arrays, decreasing offsets, an empty pattern -> MAG_E_INVALID; a pattern
 * above 64 bytes -> MAG_E_UNSUPPORTED; params as for mag_plan_create. Such
 * plans are rejected by mag_batch_create. */
mag_status mag_plan_create_var(const uint8_t *bytes, const uint64_t *offsets, uint32_t r,
                               const mag_params *params, mag_plan **out);

/* Releases the plan and its device tables. NULL is ignored. The caller must
 * not destroy a plan while a stream still runs work that uses it. */
void mag_plan_destroy(mag_plan *plan);

/* Resolved parameters and table sizes of a plan. */
mag_status mag_plan_info(const mag_plan *plan, mag_plan_desc *desc);

/* The plan's resolved choices as creation parameters: select = explicit,
 * map_kind, q, k and sigma' as chosen (Section 3.2's formulas and Section
 * 3.3's table fit for the heuristic, the selector's pick for learned plans),
 * mode = filter or dense as resolved, and the plan's verify, verify_buffer
 * and encode settings; table_budget 0. mag_plan_create with the same
 * patterns and these parameters builds the same filter and tables. Errors:
 * NULL arguments -> MAG_E_INVALID. */
mag_status mag_plan_get_params(const mag_plan *plan, mag_params *resolved);

/* Host copies of the plan's alphabet map (256 bytes; all zero for
 * MAG_MAP_QGRAM, which has none) and mask table (desc.table_bytes bytes,
 * little-endian entries of desc.entry_bytes; packed tables hold entry c in
 * bits [c * entry_bits, (c + 1) * entry_bits) of the little-endian bit
 * stream). Either output may be NULL. table_cap is the capacity of table_out
 * in bytes. */
mag_status mag_plan_export(const mag_plan *plan, uint8_t *mu_out, void *table_out,
                           uint64_t table_cap);

/* SMAG's encoding pass on its own (Section 3.2, "Implementation"): writes to
 * d_codes (device, capacity cap entries) the plan's code of every complete
 * non-overlapping q-gram d_text[y*q .. y*q+q), y = 0 .. (n-q)/q, and their
 * number to *n_codes (host). The codes are those the filter looks up: the
 * Horner value of the mapped bytes, sigma'^t weighting byte t, or the q-gram
 * map's hash. Enqueued on `stream`; no wait. n < q writes nothing. Errors:
 * NULL arguments, cap below the count -> MAG_E_INVALID. */
mag_status mag_encode(mag_plan *plan, const uint8_t *d_text, uint64_t n, uint32_t *d_codes,
                      uint64_t cap, uint64_t *n_codes, void *stream);

/* Section 1's problem for one text: every occurrence (i, id) of the plan's
 * patterns in d_text[0..n). Enqueues everything on `stream` without waiting:
 * filter, verification and the final sort. Writes min(z, out_cap) sorted
 * records to d_out and z, the exact number of occurrences, to *d_count (a
 * device uint64). If z > out_cap the records are unspecified (never written
 * past out_cap) and the caller should retry with a larger buffer. d_stats may
 * be NULL or a device mag_stats that receives the work counters. Any d_text
 * alignment is accepted. The plan's device scratch holds about 17 bytes per
 * unit of out_cap; a call that needs more scratch than earlier ones allocates
 * it and waits for the stream first, while a call within the capacity of an
 * earlier one only enqueues kernels (and can be captured in a hipGraph). */
mag_status mag_scan_async(mag_plan *plan, const uint8_t *d_text, uint64_t n,
                          mag_match *d_out, uint64_t out_cap, uint64_t *d_count,
                          mag_stats *d_stats, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * scan as mag_scan_async, with every scratch buffer (counters, sort keys,
 * radix-sort counts, deferred-start buffer) in one static device array of
 * 28 MiB per GPU instead of the plan's own scratch. It calls no hipMalloc,
 * hipFree or other allocating routine. Limits: out_cap <= 2^20 records
 * (else MAG_E_INVALID); at most 2^20 deferred starts are buffered (the rest
 * are verified inline, so results never depend on it); SMAG plans compute
 * their codes on the fly (same results). The plan's tables must already be
 * on the current device: a plan is uploaded by its first mag_scan or
 * mag_scan_async there (MAG_E_INVALID otherwise). The first call on a device
 * looks up that device's copy of the array. Every call on a GPU shares that
 * GPU's array and clears its counters first: calls that overlap on one GPU
 * (other streams, other threads) race and must be serialized by the caller.
 * Enqueued on `stream` without waiting; outputs as for mag_scan_async. */
mag_status mag_scan_noalloc(mag_plan *plan, const uint8_t *d_text, uint64_t n, mag_match *d_out,
                            uint64_t out_cap, uint64_t *d_count, mag_stats *d_stats, void *stream);

/* Section 1's problem for one text, as mag_scan_async, then waits for the
 * stream and returns the count in
 * *n_matches (host) and the counters in *stats (host, may be NULL). Returns
 * MAG_E_OVERFLOW when z > out_cap (with *n_matches = z). */
mag_status mag_scan(mag_plan *plan, const uint8_t *d_text, uint64_t n, mag_match *d_out,
                    uint64_t out_cap, uint64_t *n_matches, mag_stats *stats, void *stream);

/* ---- batched scans: many independent (text, pattern set) jobs at once ---- */

typedef struct mag_batch mag_batch;

/* A batch over njobs plans (plans[j] is job j's pattern set and parameters;
 * each needs W = k*m' <= 32). The batch keeps the plan pointers: the plans
 * must outlive it and not be scanned concurrently with it. */
mag_status mag_batch_create(mag_plan *const *plans, uint32_t njobs, mag_batch **out);
void mag_batch_destroy(mag_batch *batch);

/* Binds the jobs' texts: d_texts[j] (device pointer) of n[j] bytes (both host
 * arrays). Uploads the job table and sizes the device scratch for outputs of
 * up to out_cap occurrences in total; waits for the upload. Rebinding
 * replaces the previous texts. */
mag_status mag_batch_bind(mag_batch *batch, const uint8_t *const *d_texts, const uint64_t *n,
                          uint64_t out_cap, void *stream);

/* The filter jobs' tile shape (the batch autotuner's knob): each lane's
 * Shift-Or run takes words_per_lane samples (8 or 16), so filter jobs are
 * cut into tiles of 1024 * words_per_lane samples (a tile is one workgroup's
 * unit of work in the filter jobs' persistent launch); dense jobs run in a
 * launch of their own with tiles of 1 to 8 times the single-job dense
 * kernels' (16,128 start positions with a slice bitmap, else 16,384), fewer
 * for jobs whose positions pass the dense test more often.
 * Default 16. Takes effect at the next mag_batch_bind.
 * Errors: other values -> MAG_E_INVALID. */
mag_status mag_batch_set_words_per_lane(mag_batch *batch, int32_t words_per_lane);

/* Scans every bound job (two persistent launches: the filter jobs, then the
 * dense jobs) and sorts the output, all
 * enqueued on `stream` without host synchronization or allocation (so the
 * sequence can be captured in a hipGraph and replayed). Occurrences land in
 * d_out job by job, each job's records sorted by (pos, id) with positions
 * relative to that job's text; d_offsets (device, njobs + 1 uint64) receives
 * the first record of each job and the total, and *d_count (device) the total
 * count. If the total exceeds the bound out_cap, d_offsets[njobs] and
 * *d_count still hold the exact total and the records are unspecified. */
mag_status mag_batch_run_async(mag_batch *batch, mag_match *d_out, uint64_t *d_offsets,
                               uint64_t *d_count, void *stream);

/* One job of mag_scan_batch: a plan and its text (device pointer). */
typedef struct {
    mag_plan *plan;
    const uint8_t *d_text;
    uint64_t n;
} mag_job;

/* One-shot batched scan (Section 1's problem for many independent (text,
 * pattern set) instances): builds a batch over the jobs (a plan may serve
 * several), binds their texts, runs it on `stream`, waits, and writes the
 * first record of each job and the total to offsets (host, njobs + 1
 * uint64). Records land in d_out as for mag_batch_run_async (job by job,
 * each job's sorted by (pos, id), positions relative to its text). Allocates
 * and frees its own device scratch, so it is not for graph capture (use the
 * mag_batch_* calls there). Returns MAG_E_OVERFLOW when the total exceeds
 * out_cap (offsets[njobs] = the total, the other offsets and the records
 * unspecified). Errors: NULL arrays, a NULL plan or text (n > 0) ->
 * MAG_E_INVALID; plans mag_batch_create rejects -> its error. */
mag_status mag_scan_batch(const mag_job *jobs, uint32_t njobs, mag_match *d_out, uint64_t out_cap,
                          uint64_t *offsets, void *stream);

/* ---- learned parameter selection ----
 *
 * The paper fixes q and k by formulas (Section 3.2) and lowers sigma' until
 * the sigma'^q table fits (Section 3.3). The selector predicts instead, from
 * 16 statistics of the pattern set, the scan cost per text byte (outputs
 * 0..31) and the verifications per text byte (outputs 32..63) of each of 32
 * choices, with a small network (16 -> 64 ReLU -> 64 ReLU -> 64, FP32) whose
 * forward, gradient, Adam and selection kernels run on the device; it takes
 * the choice of lowest predicted cost among the feasible ones and falls back
 * to the heuristic. Both output groups are trained on what the scans
 * themselves measure: their kernel time and their verification count.
 *
 * Features (host floats): f0 log2(sigma_P)/8, f1 m/32, f2 log10(r)/4, f3 byte
 * entropy/8, f4 largest byte frequency, f5 distinct patterns / r, f5+q for
 * q = 1..8 min(1, -log2(D_q / sigma_P^q)/32) with D_q the distinct q-byte
 * substrings of the patterns (1 if q > m, 0 if sigma_P = 1), f14 the
 * heuristic's q (at most 8) / 8, f15 log2(r*m)/20.
 *
 * Choices: 0 = the dense mode (mode MAG_MODE_DENSE; q, k, sigma' from the
 * heuristic), 1 = the alphabet mapping on q-grams (MAG_MAP_QGRAM with its
 * heuristic; feasible when r > 0; batches reject it), 2..31 = filter triples
 * (mode MAG_MODE_FILTER, greedy map): c = 2..25 take q = (2, 3, 4, 5, 6, 8)[i/4],
 * k = (i/2)%2 + 1, level i%2 for i = c - 2; 26..29 take (q, k) = (2, 3),
 * (3, 3), (4, 3), (2, 4) at level 0; 30 and 31 take q = 7, k = 1 at levels 0
 * and 1. A triple is feasible iff 2q-1 <= m, k <= L and W = k*m' <= 32;
 * sigma' = fit (level 0) or max(2, fit/2) (level 1, infeasible when equal to
 * fit), fit = the largest s <= sigma_P with s^q * entry_bytes(W) <= 64 KiB.
 * Feasible filter picks also run in batches (W <= 32). Slots 32..63 are never
 * feasible (they are the verification outputs). */

/* out: 16 floats. Errors: r == 0 or m == 0 -> MAG_E_INVALID. */
mag_status mag_select_features(const uint8_t *patterns, uint32_t r, uint32_t m, float *out);

/* out[64] parameters of the choices (filter triples: select = explicit; the
 * dense and q-gram choices: select = learned with q, k, sigma' left to the
 * plan's heuristics) and feasible[64] (1 or 0; slots 32..63 always 0). */
mag_status mag_select_candidates(const uint8_t *patterns, uint32_t r, uint32_t m,
                                 mag_params *out, uint8_t *feasible);

typedef struct mag_mlp mag_mlp;

/* Number of FP32 parameters: W1[64][16], b1[64], W2[64][64], b2[64],
 * W3[64][64], b3[64], rows are output units. */
uint32_t mag_mlp_param_count(void);

/* A network on the current device, parameters zero. */
mag_status mag_mlp_create(mag_mlp **out);
void mag_mlp_destroy(mag_mlp *mlp);

/* Host copies of the parameters; setting them also clears the Adam state. */
mag_status mag_mlp_set_params(mag_mlp *mlp, const float *params);
mag_status mag_mlp_get_params(mag_mlp *mlp, float *params);

/* d_y[B][64] = network(d_x[B][16]). */
mag_status mag_mlp_forward(mag_mlp *mlp, const float *d_x, uint32_t B, float *d_y, void *stream);

/* Gradient of the masked mean squared error sum M (y - t)^2 / sum M over
 * the batch (d_t [B][64] targets, d_mask [B][64] of 0/1) into d_grad
 * (param_count floats) and the loss into *d_loss (device float); zero when
 * nothing is labelled. */
mag_status mag_mlp_grad(mag_mlp *mlp, const float *d_x, const float *d_t, const uint8_t *d_mask,
                        uint32_t B, float *d_grad, float *d_loss, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected with the
 * network's own step counter) with gradient d_grad. */
mag_status mag_mlp_adam(mag_mlp *mlp, const float *d_grad, float lr, void *stream);

/* mag_mlp_grad into the network's own buffer, then mag_mlp_adam. d_loss may
 * be NULL. */
mag_status mag_mlp_train_step(mag_mlp *mlp, const float *d_x, const float *d_t,
                              const uint8_t *d_mask, uint32_t B, float lr, float *d_loss,
                              void *stream);

/* d_pick[b] = the feasible candidate (d_feasible [B][64] of 0/1) with the
 * smallest predicted cost, lowest index on ties; -1 if none is feasible. */
mag_status mag_mlp_select(mag_mlp *mlp, const float *d_x, const uint8_t *d_feasible, uint32_t B,
                          int32_t *d_pick, void *stream);

/* Features, candidates and one selection for a pattern set (waits for the
 * stream). *out receives the pick with select = MAG_SELECT_LEARNED, or the
 * heuristic (select = MAG_SELECT_HEURISTIC) when mlp is NULL or has no
 * parameters, r == 0 or no candidate is feasible. Pass *out to
 * mag_plan_create. */
mag_status mag_select_learned(mag_mlp *mlp, const uint8_t *patterns, uint32_t r, uint32_t m,
                              mag_params *out, void *stream);

/* Options of mag_autotune (NULL = defaults). */
typedef struct {
    int32_t map_kinds;    /* bit 0: greedy, bit 1: rank; 0 = both                   */
    int32_t max_q;        /* largest q tried; 0 = 8                                  */
    int32_t max_k;        /* largest k tried; 0 = 8                                  */
    int64_t table_budget; /* largest mask table in bytes; 0 = 64 KiB (LDS-resident)  */
    int32_t repeats;      /* timed scans per candidate (median); 0 = 3               */
    int32_t max_candidates; /* cap on filter candidates timed, best predicted
                               first; 0 = 64                                        */
    int32_t modes;        /* bit 0: filter, bit 1: dense (timed beside the filter
                             candidates); 0 = both                                  */
    int32_t fixed_tiles;  /* 1: keep the default tile shape (no words-per-lane
                             timing)                                                */
    int32_t batch_only;   /* 1: only parameters batches accept (W = k*m' <= 32)      */
    int32_t reserved;     /* must be zero                                            */
} mag_tune_opts;

/* Autotuner: picks the mode, (q, k, sigma', map) and the tile shape for a
 * pattern set by timing the scan on a device-resident text sample
 * d_sample[0..n_sample) (the choice of q and k is Section 3.2's trade-off,
 * settled by measurement instead of its formulas). Filter candidates are
 * every q with 2q-1 <= m, k <= L, reduced alphabet sizes from 2 to sigma_P
 * and both maps whose mask table fits the budget; they are ranked by a
 * density estimate (superimposed classes of Section 2: expected
 * verifications per sample) plus the sampling cost, and the best-ranked ones
 * are timed with mode = MAG_MODE_FILTER, beside the dense mode. The winner's
 * words_per_lane is then timed at half and 1.5 times its default (filter)
 * or at 32 (dense) and kept on a gain of 3% or more. Any choice returns
 * exactly the same occurrences (the filter only prunes); the pick only
 * changes the time. *best receives explicit parameters (select =
 * MAG_SELECT_EXPLICIT, mode filter or dense) and *best_ms the median scan
 * time of the sample (either may be NULL). Uses the device and stream like
 * mag_scan. */
mag_status mag_autotune(const uint8_t *patterns, uint32_t r, uint32_t m,
                        const mag_tune_opts *opts, const uint8_t *d_sample, uint64_t n_sample,
                        mag_params *best, float *best_ms, void *stream);

/* Batch autotuner (the batched scans' "chunk size, q and k"): jobs are
 * grouped into classes by pattern length, distinct pattern bytes and
 * log2(r), and mag_autotune (with opts) times candidates for each class on a
 * sample of its largest job's text (at most sample_bytes, 0 = 4 MiB);
 * params[j] (host, njobs entries) receives the pick for job j's class. Then
 * the whole batch, planned with those parameters, is timed with 8 and 16
 * words per lane (filter tiles of 1024 times that many samples) and the fastest goes
 * to *words_per_lane. jobs[j].plan is ignored (may be NULL); the patterns
 * come from pat[j] (host, r[j] * m[j] bytes). Allocates and waits; not for
 * graph capture. Errors: NULL arrays -> MAG_E_INVALID; errors of
 * mag_autotune or the batch calls. */
mag_status mag_autotune_batch(const mag_job *jobs, const uint8_t *const *pat, const uint32_t *r,
                              const uint32_t *m, uint32_t njobs, const mag_tune_opts *opts,
                              uint64_t sample_bytes, mag_params *params, int32_t *words_per_lane,
                              void *stream);

/* Kernel timing for benchmarks. While enabled (process-wide), every scan and
 * every mag_batch_run_async records HIP events on its own stream: before its
 * scan kernel (the filter or dense kernel with fused exact verification; the
 * batched kernel), after it, and after the scan's last kernel (deferred
 * verification, finishing kernel, sort, batch offsets). mag_profile_read
 * waits for the recorded events, stores their summed elapsed times in
 * milliseconds (scan kernel; the rest), sets *launches to the number of scans
 * measured, and clears the record. Nothing is recorded on a stream that is
 * being captured. Enabling adds three event records per scan; disabled by
 * default. */
mag_status mag_profile_enable(int enable);
mag_status mag_profile_read(double *scan_ms, double *finish_ms, uint64_t *launches);

const char *mag_status_string(mag_status s);
const char *mag_last_error(void);

/* Measurement aid, not part of the method: a plain streaming read of
 * d[0..n) (device, 16-byte aligned) with 16-byte loads, one 1024-thread
 * workgroup per compute unit reading 32 KiB tiles in turn (the fastest plain
 * read layout measured), each word folded into an xor written to d_sink
 * (device, at least mag_stream_read_sink_words() words: word b is block b's
 * xor of the 32-bit words, the bytes past the last whole 16-byte vector
 * shifted in by position mod 4), so the read cannot be skipped. Time it on
 * `stream` to get the read bandwidth a plain stream reaches on the device,
 * the ceiling the scan is compared with besides the HBM specification.
 * Enqueued only; no wait. d not 16-byte aligned -> MAG_E_INVALID. */
mag_status mag_stream_read(const uint8_t *d, uint64_t n, uint32_t *d_sink, void *stream);
uint32_t mag_stream_read_sink_words(void);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int32_t mag_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MAG_H */
