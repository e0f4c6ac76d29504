/*
 * Oracle for exact multiple pattern matching. TEST INFRASTRUCTURE ONLY: only
 * the tests, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code with the HIP library.
 *
 * It computes the plain definition of the problem statement (Section 1):
 *
 *   Occ(T, P) = { (i, id) : 0 <= i <= n - m, 0 <= id < r, T[i..i+m) == P_id }
 *
 * as a list sorted by (i, id). Positions are 0-based starts, overlapping
 * occurrences are all reported, and every id of a repeated pattern is listed.
 * The paper's filter only prunes text windows and then verifies exactly
 * (Section 3), so the method must return exactly this set.
 *
 * Two matchers:
 *   occ_brute  - every (i, id) pair compared with memcmp: O(n r m);
 *   occ_hashed - a chained hash table keyed by the whole pattern (FNV-1a
 *                64-bit), every text window looked up; start positions are
 *                split into contiguous blocks across POSIX threads and the
 *                per-thread lists are concatenated in block order.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t *pos;
    uint32_t *id;
    uint64_t size, cap;
    int failed;
} occ_list;

static int list_push(occ_list *L, uint64_t pos, uint32_t id) {
    if (L->size == L->cap) {
        uint64_t nc = L->cap ? 2 * L->cap : 1024;
        uint64_t *np = (uint64_t *)realloc(L->pos, nc * sizeof(uint64_t));
        if (!np) { L->failed = 1; return -1; }
        L->pos = np;
        uint32_t *ni = (uint32_t *)realloc(L->id, nc * sizeof(uint32_t));
        if (!ni) { L->failed = 1; return -1; }
        L->id = ni;
        L->cap = nc;
    }
    L->pos[L->size] = pos;
    L->id[L->size] = id;
    L->size++;
    return 0;
}

/* Result handle returned to the caller. */
typedef struct {
    occ_list all;
} occ_result;

uint64_t occ_size(const occ_result *h) { return h ? h->all.size : 0; }

int occ_failed(const occ_result *h) { return h == NULL || h->all.failed; }

void occ_copy(const occ_result *h, uint64_t *pos, uint32_t *id) {
    if (!h || !h->all.size) return;
    memcpy(pos, h->all.pos, h->all.size * sizeof(uint64_t));
    memcpy(id, h->all.id, h->all.size * sizeof(uint32_t));
}

void occ_free(occ_result *h) {
    if (!h) return;
    free(h->all.pos);
    free(h->all.id);
    free(h);
}

/* ---------------------------------------------------------------- brute */

occ_result *occ_brute(const uint8_t *T, uint64_t n, const uint8_t *P, uint32_t r,
                      uint32_t m) {
    occ_result *h = (occ_result *)calloc(1, sizeof(occ_result));
    if (!h) return NULL;
    if (m == 0 || n < m) return h;
    for (uint64_t i = 0; i + m <= n; i++)
        for (uint32_t id = 0; id < r; id++)
            if (memcmp(T + i, P + (uint64_t)id * m, m) == 0)
                list_push(&h->all, i, id);
    return h;
}

/* --------------------------------------------------------------- hashed */

static uint64_t fnv1a(const uint8_t *s, uint32_t len) {
    uint64_t x = 0xcbf29ce484222325ull;
    for (uint32_t t = 0; t < len; t++) {
        x ^= s[t];
        x *= 0x100000001b3ull;
    }
    return x;
}

typedef struct {
    const uint8_t *T, *P;
    uint32_t m;
    uint64_t begin, end; /* start positions [begin, end) */
    uint64_t mask;
    const int64_t *head;
    const int64_t *next;
    occ_list out;
} occ_task;

static void *occ_worker(void *arg) {
    occ_task *t = (occ_task *)arg;
    for (uint64_t i = t->begin; i < t->end; i++) {
        const uint8_t *w = t->T + i;
        int64_t id = t->head[fnv1a(w, t->m) & t->mask];
        /* chains hold ids in ascending order, so each position's ids come out sorted */
        for (; id >= 0; id = t->next[id])
            if (memcmp(w, t->P + (uint64_t)id * t->m, t->m) == 0)
                if (list_push(&t->out, i, (uint32_t)id)) return NULL;
    }
    return NULL;
}

occ_result *occ_hashed(const uint8_t *T, uint64_t n, const uint8_t *P, uint32_t r,
                       uint32_t m, int nthreads) {
    occ_result *h = (occ_result *)calloc(1, sizeof(occ_result));
    if (!h) return NULL;
    if (m == 0 || r == 0 || n < m) return h;
    if (nthreads < 1) nthreads = 1;

    uint64_t nb = 1;
    while (nb < 2ull * r) nb <<= 1;
    int64_t *head = (int64_t *)malloc(nb * sizeof(int64_t));
    int64_t *tail = (int64_t *)malloc(nb * sizeof(int64_t));
    int64_t *next = (int64_t *)malloc((uint64_t)r * sizeof(int64_t));
    if (!head || !tail || !next) {
        free(head); free(tail); free(next);
        h->all.failed = 1;
        return h;
    }
    for (uint64_t b = 0; b < nb; b++) head[b] = tail[b] = -1;
    for (uint32_t id = 0; id < r; id++) {
        uint64_t b = fnv1a(P + (uint64_t)id * m, m) & (nb - 1);
        next[id] = -1;
        if (tail[b] < 0) head[b] = id; else next[tail[b]] = id;
        tail[b] = id;
    }

    uint64_t npos = n - m + 1;
    if ((uint64_t)nthreads > npos) nthreads = (int)npos;
    occ_task *tasks = (occ_task *)calloc((size_t)nthreads, sizeof(occ_task));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!tasks || !th) {
        free(tasks); free(th); free(head); free(tail); free(next);
        h->all.failed = 1;
        return h;
    }
    for (int t = 0; t < nthreads; t++) {
        tasks[t].T = T;
        tasks[t].P = P;
        tasks[t].m = m;
        tasks[t].begin = npos * (uint64_t)t / (uint64_t)nthreads;
        tasks[t].end = npos * (uint64_t)(t + 1) / (uint64_t)nthreads;
        tasks[t].mask = nb - 1;
        tasks[t].head = head;
        tasks[t].next = next;
    }
    int spawned = 0;
    for (int t = 1; t < nthreads; t++) {
        if (pthread_create(&th[t], NULL, occ_worker, &tasks[t]) != 0) break;
        spawned = t;
    }
    occ_worker(&tasks[0]);
    for (int t = 1; t <= spawned; t++) pthread_join(th[t], NULL);
    /* threads that could not be spawned run here, in order */
    for (int t = spawned + 1; t < nthreads; t++) occ_worker(&tasks[t]);

    uint64_t total = 0;
    int failed = 0;
    for (int t = 0; t < nthreads; t++) {
        total += tasks[t].out.size;
        failed |= tasks[t].out.failed;
    }
    if (!failed && total) {
        h->all.pos = (uint64_t *)malloc(total * sizeof(uint64_t));
        h->all.id = (uint32_t *)malloc(total * sizeof(uint32_t));
        if (!h->all.pos || !h->all.id) failed = 1;
    }
    if (!failed) {
        uint64_t at = 0;
        for (int t = 0; t < nthreads; t++) {
            if (!tasks[t].out.size) continue;
            memcpy(h->all.pos + at, tasks[t].out.pos, tasks[t].out.size * sizeof(uint64_t));
            memcpy(h->all.id + at, tasks[t].out.id, tasks[t].out.size * sizeof(uint32_t));
            at += tasks[t].out.size;
        }
        h->all.size = h->all.cap = total;
    }
    h->all.failed = failed;
    for (int t = 0; t < nthreads; t++) {
        free(tasks[t].out.pos);
        free(tasks[t].out.id);
    }
    free(tasks); free(th); free(head); free(tail); free(next);
    return h;
}
