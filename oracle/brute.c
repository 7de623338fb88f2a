/*
 * BRUTE-FORCE CHECKERS -- test infrastructure that pins the CPU oracle.
 *
 * Nothing here uses an index.  Each function restates a definition
 * directly over the text:
 *
 *  - brute_sa: the suffix array of T$ by sorting all suffixes with a plain
 *    symbol-by-symbol comparison ($ smallest).
 *  - brute_align: every valid transcript of the read (both strands)
 *    starting at every text position, enumerated left to right; the result
 *    is the set of (strand, position, reference length) it reaches, each
 *    with the smallest (score, diffs, n_gapo, n_mm) -- the ALL set of the
 *    oracle, keyed by position instead of by suffix-array interval.
 *  - brute_hamming: the same set when only mismatches are allowed, by
 *    counting mismatches at every position.
 *  - brute_hamming_many: brute_hamming for a whole batch of reads on
 *    several threads, the mismatches of 64 positions at a time counted with
 *    XOR and popcount over bit-sliced text words.
 *  - brute_exact_many: every occurrence of every pattern of a batch, by one
 *    pass over the text that looks each position's 16-base prefix up in a
 *    hash of the patterns' prefixes and compares the rest base by base.
 *  - brute_edit_many: the gapped ALL set of a batch at sizes where
 *    brute_align over the whole text is too slow.  A transcript of d
 *    differences (mismatches plus gap bases) is an alignment of unit edit
 *    cost d, so every valid hit ends at a text position where the smallest
 *    edit distance of W_s against a substring ending there is at most
 *    max_diff.  A Myers bit-vector scan (Myers, J. ACM 46(3), 1999; the
 *    multi-word form of Hyyro) finds those end positions; brute_align's
 *    enumeration then runs on the window of at most m + max_diff bases
 *    that ends at each of them.  The filter drops no valid hit, so the
 *    result equals brute_align over the whole text.
 *
 * The transcript rules are those of the oracle's header: gap = maximal run
 * of I or of D; I at read index i needs s <= i < m - s; D at boundary b
 * needs max(s,1) <= b <= m - max(s,1); diffs touching the seed (first
 * seed_len bases as sequenced, a D counting when strictly inside) are at
 * most seed_diff.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint32_t pos;
    uint16_t len, score;
    uint8_t strand, n_mm, n_gapo, n_gape;
} brute_rec;

typedef struct {
    int32_t max_diff, max_gapo, max_gape, seed_len, seed_diff, indel_end_skip;
    int32_t s_mm, s_gapo, s_gape;
} brute_params;

static const uint8_t *g_t;
static int64_t g_n;

static int cmp_suffix(const void *x, const void *y)
{
    int64_t i = *(const uint32_t *)x, j = *(const uint32_t *)y;
    for (;;) {
        /* symbol value: $ (past the end) = 0, A..T = 1..4 */
        int a = i < g_n ? g_t[i] + 1 : 0, b = j < g_n ? g_t[j] + 1 : 0;
        if (a != b) return a < b ? -1 : 1;
        if (a == 0) return 0;
        i++;
        j++;
    }
}

void brute_sa(const uint8_t *t, int64_t n, uint32_t *sa)
{
    g_t = t;
    g_n = n;
    for (int64_t i = 0; i <= n; i++) sa[i] = (uint32_t)i;
    qsort(sa, (size_t)(n + 1), sizeof(uint32_t), cmp_suffix);
}

typedef struct {
    const uint8_t *t;
    int64_t n, p;
    const uint8_t *w;
    int m, strand, seed_lo, seed_hi, s, s1;
    const brute_params *pr;
    brute_rec *out;
    int64_t nout, cap;
    int oom;
} en_t;

static void push(en_t *e, int64_t len, int nmm, int ngo, int nge)
{
    if (e->nout == e->cap) {
        int64_t nc = e->cap ? e->cap * 2 : 256;
        brute_rec *nb = (brute_rec *)realloc(e->out, sizeof(brute_rec) * (size_t)nc);
        if (!nb) { e->oom = 1; return; }
        e->out = nb;
        e->cap = nc;
    }
    brute_rec *r = &e->out[e->nout++];
    r->pos = (uint32_t)e->p;
    r->len = (uint16_t)len;
    r->score = (uint16_t)(e->pr->s_mm * nmm + e->pr->s_gapo * ngo + e->pr->s_gape * nge);
    r->strand = (uint8_t)e->strand;
    r->n_mm = (uint8_t)nmm;
    r->n_gapo = (uint8_t)ngo;
    r->n_gape = (uint8_t)nge;
}

/* gs: 0 none, 1 inside an I run, 2 inside a D run.  i: next read index,
 * j: next text index. */
static void enumerate(en_t *e, int i, int64_t j, int nmm, int ngo, int nge, int gs, int sd)
{
    const brute_params *p = e->pr;
    if (nmm + ngo + nge > p->max_diff || ngo > p->max_gapo || (p->max_gape >= 0 && nge > p->max_gape) ||
        (p->seed_len > 0 && sd > p->seed_diff) || e->oom)
        return;
    if (i == e->m) {
        if (j > e->p) push(e, j - e->p, nmm, ngo, nge);
        return;
    }
    int in_seed = i >= e->seed_lo && i < e->seed_hi;
    if (j < e->n) {
        int mm = e->w[i] > 3 || e->w[i] != e->t[j];
        enumerate(e, i + 1, j + 1, nmm + mm, ngo, nge, 0, sd + (mm && in_seed));
    }
    if (i >= e->s && i < e->m - e->s) {
        if (gs == 1) enumerate(e, i + 1, j, nmm, ngo, nge + 1, 1, sd + in_seed);
        else enumerate(e, i + 1, j, nmm, ngo + 1, nge, 1, sd + in_seed);
    }
    if (j < e->n && i >= e->s1 && i <= e->m - e->s1) {
        int inside = i > e->seed_lo && i < e->seed_hi;
        if (gs == 2) enumerate(e, i, j + 1, nmm, ngo, nge + 1, 2, sd + inside);
        else enumerate(e, i, j + 1, nmm, ngo + 1, nge, 2, sd + inside);
    }
}

static int cmp_rec(const void *x, const void *y)
{
    const brute_rec *a = (const brute_rec *)x, *b = (const brute_rec *)y;
    if (a->strand != b->strand) return a->strand < b->strand ? -1 : 1;
    if (a->pos != b->pos) return a->pos < b->pos ? -1 : 1;
    if (a->len != b->len) return a->len < b->len ? -1 : 1;
    if (a->score != b->score) return a->score < b->score ? -1 : 1;
    int da = a->n_mm + a->n_gapo + a->n_gape, db = b->n_mm + b->n_gapo + b->n_gape;
    if (da != db) return da < db ? -1 : 1;
    if (a->n_gapo != b->n_gapo) return a->n_gapo < b->n_gapo ? -1 : 1;
    if (a->n_mm != b->n_mm) return a->n_mm < b->n_mm ? -1 : 1;
    return 0;
}

static int64_t dedup(brute_rec *r, int64_t n)
{
    if (n == 0) return 0;
    qsort(r, (size_t)n, sizeof(brute_rec), cmp_rec);
    int64_t u = 0;
    for (int64_t i = 0; i < n; i++) {
        if (u && r[u - 1].strand == r[i].strand && r[u - 1].pos == r[i].pos && r[u - 1].len == r[i].len) continue;
        r[u++] = r[i];
    }
    return u;
}

static void strand_pattern(const uint8_t *W, int m, int strand, uint8_t *w)
{
    for (int i = 0; i < m; i++)
        w[i] = strand == 0 ? W[i] : (W[m - 1 - i] > 3 ? 4 : (uint8_t)(3 - W[m - 1 - i]));
}

/* All (strand, pos, len) reached by a valid transcript of read W; returns
 * the count and a malloc'ed array in *out (free with brute_free), or -1. */
int64_t brute_align(const uint8_t *t, int64_t n, const uint8_t *W, int m, const brute_params *p, brute_rec **out)
{
    en_t e;
    memset(&e, 0, sizeof(e));
    e.t = t;
    e.n = n;
    e.m = m;
    e.pr = p;
    e.s = p->indel_end_skip;
    e.s1 = p->indel_end_skip > 1 ? p->indel_end_skip : 1;
    uint8_t *w = (uint8_t *)malloc((size_t)m + 1);
    if (!w) return -1;
    int sl = p->seed_len > 0 ? (p->seed_len < m ? p->seed_len : m) : 0;
    for (int strand = 0; strand < 2; strand++) {
        strand_pattern(W, m, strand, w);
        e.w = w;
        e.strand = strand;
        e.seed_lo = strand == 0 ? 0 : m - sl;
        e.seed_hi = strand == 0 ? sl : (sl ? m : 0);
        for (int64_t pos = 0; pos < n; pos++) {
            e.p = pos;
            enumerate(&e, 0, pos, 0, 0, 0, 0, 0);
        }
    }
    free(w);
    if (e.oom) { free(e.out); return -1; }
    *out = e.out;
    return dedup(e.out, e.nout);
}

/* Mismatch-only variant: every position where W_s fits with at most
 * max_diff mismatches (and at most seed_diff of them in the seed). */
int64_t brute_hamming(const uint8_t *t, int64_t n, const uint8_t *W, int m, const brute_params *p,
                      brute_rec **out)
{
    int64_t cap = 256, cnt = 0;
    brute_rec *r = (brute_rec *)malloc(sizeof(brute_rec) * (size_t)cap);
    uint8_t *w = (uint8_t *)malloc((size_t)m + 1);
    if (!r || !w) { free(r); free(w); return -1; }
    int sl = p->seed_len > 0 ? (p->seed_len < m ? p->seed_len : m) : 0;
    for (int strand = 0; strand < 2; strand++) {
        strand_pattern(W, m, strand, w);
        int slo = strand == 0 ? 0 : m - sl, shi = strand == 0 ? sl : (sl ? m : 0);
        for (int64_t pos = 0; pos + m <= n; pos++) {
            int mm = 0, sd = 0, ok = 1;
            for (int i = 0; i < m; i++) {
                if (w[i] > 3 || w[i] != t[pos + i]) {
                    mm++;
                    if (i >= slo && i < shi) sd++;
                    if (mm > p->max_diff || (p->seed_len > 0 && sd > p->seed_diff)) { ok = 0; break; }
                }
            }
            if (!ok) continue;
            if (cnt == cap) {
                cap *= 2;
                brute_rec *nb = (brute_rec *)realloc(r, sizeof(brute_rec) * (size_t)cap);
                if (!nb) { free(r); free(w); return -1; }
                r = nb;
            }
            r[cnt].pos = (uint32_t)pos;
            r[cnt].len = (uint16_t)m;
            r[cnt].score = (uint16_t)(p->s_mm * mm);
            r[cnt].strand = (uint8_t)strand;
            r[cnt].n_mm = (uint8_t)mm;
            r[cnt].n_gapo = 0;
            r[cnt].n_gape = 0;
            cnt++;
        }
    }
    free(w);
    *out = r;
    return cnt;
}

/* ------------------------------------------------------------ batches */

/* Run fn(arg, i) for i in [0, n) on up to `threads` threads, items taken
 * from a shared counter. */
typedef struct {
    void (*fn)(void *, int64_t);
    void *arg;
    int64_t n, next;
    pthread_mutex_t mu;
} pool_t;

static void *pool_worker(void *a)
{
    pool_t *P = (pool_t *)a;
    for (;;) {
        pthread_mutex_lock(&P->mu);
        int64_t i = P->next++;
        pthread_mutex_unlock(&P->mu);
        if (i >= P->n) return NULL;
        P->fn(P->arg, i);
    }
}

static void pool_run(void (*fn)(void *, int64_t), void *arg, int64_t n, int threads)
{
    pool_t P;
    P.fn = fn;
    P.arg = arg;
    P.n = n;
    P.next = 0;
    pthread_mutex_init(&P.mu, NULL);
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    pthread_t th[256];
    int started = 0;
    for (int i = 1; i < threads; i++)
        if (pthread_create(&th[started], NULL, pool_worker, &P) == 0) started++;
    pool_worker(&P);
    for (int i = 0; i < started; i++) pthread_join(th[i], NULL);
    pthread_mutex_destroy(&P.mu);
}

/* Per-read record lists of a batch, concatenated in read order. */
typedef struct {
    brute_rec **recs;
    int64_t *cnt;
    int fail;
} lists_t;

static int64_t lists_join(lists_t *L, int64_t n_reads, uint64_t *rec_off, brute_rec **out)
{
    int64_t tot = 0;
    for (int64_t r = 0; r < n_reads; r++) {
        if (L->cnt[r] < 0) L->fail = 1;
        else tot += L->cnt[r];
    }
    brute_rec *o = L->fail ? NULL : (brute_rec *)malloc(sizeof(brute_rec) * (size_t)(tot ? tot : 1));
    if (!o) L->fail = 1;
    int64_t k = 0;
    rec_off[0] = 0;
    for (int64_t r = 0; r < n_reads; r++) {
        if (!L->fail && L->cnt[r] > 0) memcpy(o + k, L->recs[r], sizeof(brute_rec) * (size_t)L->cnt[r]);
        if (!L->fail) k += L->cnt[r];
        rec_off[r + 1] = (uint64_t)k;
        free(L->recs[r]);
    }
    free(L->recs);
    free(L->cnt);
    if (L->fail) { free(o); return -1; }
    *out = o;
    return tot;
}

static int lists_init(lists_t *L, int64_t n_reads)
{
    L->recs = (brute_rec **)calloc((size_t)(n_reads ? n_reads : 1), sizeof(brute_rec *));
    L->cnt = (int64_t *)calloc((size_t)(n_reads ? n_reads : 1), sizeof(int64_t));
    L->fail = !L->recs || !L->cnt;
    if (L->fail) { free(L->recs); free(L->cnt); }
    return L->fail ? -1 : 0;
}

/* ------------------------------------------------ Hamming scan, batched */

/* bit-sliced text: bit j of H[p] (of L[p]) is the high (low) bit of the
 * code of T[p + j], zero past the end */
typedef struct {
    const uint8_t *t;
    int64_t n;
    uint64_t *H, *L;
    const uint8_t *bases;
    const uint64_t *offs;
    const brute_params *p;
    lists_t lists;
} ham_t;

__attribute__((target("popcnt"))) static void ham_read(void *a, int64_t r)
{
    ham_t *A = (ham_t *)a;
    const brute_params *p = A->p;
    const uint8_t *W = A->bases + A->offs[r];
    const int m = (int)(A->offs[r + 1] - A->offs[r]);
    const int nw = (m + 63) / 64;
    uint64_t wh[8], wl[8], wn[8], wm[8], ws[8];
    uint8_t w[512];
    int64_t cap = 0, cnt = 0;
    brute_rec *out = NULL;
    if (m == 0 || m > 512 || (int64_t)m > A->n) { A->lists.cnt[r] = 0; return; }
    const int sl = p->seed_len > 0 ? (p->seed_len < m ? p->seed_len : m) : 0;
    for (int strand = 0; strand < 2; strand++) {
        strand_pattern(W, m, strand, w);
        const int slo = strand == 0 ? 0 : m - sl, shi = strand == 0 ? sl : (sl ? m : 0);
        for (int k = 0; k < nw; k++) wh[k] = wl[k] = wn[k] = wm[k] = ws[k] = 0;
        for (int i = 0; i < m; i++) {
            const uint64_t b = 1ULL << (i & 63);
            const int k = i >> 6;
            wm[k] |= b;
            if (w[i] > 3) wn[k] |= b;
            else {
                if (w[i] & 2) wh[k] |= b;
                if (w[i] & 1) wl[k] |= b;
            }
            if (i >= slo && i < shi) ws[k] |= b;
        }
        for (int64_t pos = 0; pos + m <= A->n; pos++) {
            if (nw == 1 &&
                __builtin_popcountll(((A->H[pos] ^ wh[0]) | (A->L[pos] ^ wl[0]) | wn[0]) & wm[0]) > p->max_diff)
                continue;  /* the common case of one word, decided at once */
            int mm = 0, sd = 0;
            for (int k = 0; k < nw && mm <= p->max_diff; k++) {
                const uint64_t x = ((A->H[pos + 64 * k] ^ wh[k]) | (A->L[pos + 64 * k] ^ wl[k]) | wn[k]) & wm[k];
                mm += __builtin_popcountll(x);
                sd += __builtin_popcountll(x & ws[k]);
            }
            if (mm > p->max_diff || (p->seed_len > 0 && sd > p->seed_diff)) continue;
            if (cnt == cap) {
                cap = cap ? 2 * cap : 16;
                brute_rec *nb = (brute_rec *)realloc(out, sizeof(brute_rec) * (size_t)cap);
                if (!nb) { free(out); A->lists.cnt[r] = -1; return; }
                out = nb;
            }
            brute_rec *o = &out[cnt++];
            o->pos = (uint32_t)pos;
            o->len = (uint16_t)m;
            o->score = (uint16_t)(p->s_mm * mm);
            o->strand = (uint8_t)strand;
            o->n_mm = (uint8_t)mm;
            o->n_gapo = o->n_gape = 0;
        }
    }
    A->lists.recs[r] = out;
    A->lists.cnt[r] = cnt;
}

/* brute_hamming for reads r of a batch (bases, offsets[n_reads + 1], at
 * most 512 bases each): the records of read r are out[rec_off[r] ..
 * rec_off[r + 1]), in strand then position order.  Returns the total or -1. */
int64_t brute_hamming_many(const uint8_t *t, int64_t n, const uint8_t *bases, const uint64_t *offs, int64_t n_reads,
                           const brute_params *p, int threads, uint64_t *rec_off, brute_rec **out)
{
    ham_t A;
    memset(&A, 0, sizeof(A));
    A.t = t;
    A.n = n;
    A.bases = bases;
    A.offs = offs;
    A.p = p;
    const int64_t pad = n + 8 * 64;
    A.H = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)pad);
    A.L = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)pad);
    if (!A.H || !A.L || lists_init(&A.lists, n_reads)) { free(A.H); free(A.L); return -1; }
    uint64_t h = 0, l = 0;
    for (int64_t q = pad - 1; q >= 0; q--) {
        const int c = q < n ? t[q] : 0;
        h = (h << 1) | (uint64_t)((c >> 1) & 1);
        l = (l << 1) | (uint64_t)(c & 1);
        A.H[q] = h;
        A.L[q] = l;
    }
    pool_run(ham_read, &A, n_reads, threads);
    free(A.H);
    free(A.L);
    return lists_join(&A.lists, n_reads, rec_off, out);
}

/* ------------------------------------------------ exact occurrences, batched */

typedef struct {
    const uint8_t *t;
    int64_t n;
    const uint8_t *pats;
    const uint64_t *poff;
    int64_t n_pats;
    uint32_t *slot_key;   /* 16-base prefix code */
    int64_t *slot_head;   /* first pattern of the prefix, -1 = empty */
    int64_t *next;        /* next pattern of the same prefix */
    uint32_t mask;        /* slots - 1 */
    int64_t chunk;
    /* per chunk: found (pattern, position) pairs */
    uint64_t **found;
    int64_t *nfound;
    int fail;
} exact_t;

static uint32_t code16(const uint8_t *x)
{
    uint32_t c = 0;
    for (int i = 0; i < 16; i++) c = (c << 2) | x[i];
    return c;
}

static uint32_t slot_of(uint32_t code, uint32_t mask) { return (uint32_t)((code * 2654435761u) >> 7) & mask; }

static void exact_chunk(void *a, int64_t ci)
{
    exact_t *E = (exact_t *)a;
    const int64_t lo = ci * E->chunk, hi = lo + E->chunk < E->n ? lo + E->chunk : E->n;
    int64_t cap = 0, cnt = 0;
    uint64_t *f = NULL;
    uint32_t c = 0;
    for (int64_t q = lo; q < hi && q + 16 <= E->n; q++) {
        c = q == lo ? code16(E->t + q) : (c << 2) | E->t[q + 15];
        uint32_t s = slot_of(c, E->mask);
        while (E->slot_head[s] >= 0 && E->slot_key[s] != c) s = (s + 1) & E->mask;
        for (int64_t k = E->slot_head[s]; k >= 0; k = E->next[k]) {
            const int64_t m = (int64_t)(E->poff[k + 1] - E->poff[k]);
            if (q + m > E->n || memcmp(E->t + q, E->pats + E->poff[k], (size_t)m) != 0) continue;
            if (cnt + 2 > cap) {
                cap = cap ? 2 * cap : 64;
                uint64_t *nb = (uint64_t *)realloc(f, sizeof(uint64_t) * (size_t)cap);
                if (!nb) { free(f); E->fail = 1; E->nfound[ci] = 0; E->found[ci] = NULL; return; }
                f = nb;
            }
            f[cnt++] = (uint64_t)k;
            f[cnt++] = (uint64_t)q;
        }
    }
    E->found[ci] = f;
    E->nfound[ci] = cnt / 2;
}

static int cmp_u64pair(const void *x, const void *y)
{
    const uint64_t *a = (const uint64_t *)x, *b = (const uint64_t *)y;
    if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;
    if (a[1] != b[1]) return a[1] < b[1] ? -1 : 1;
    return 0;
}

/* Every occurrence of every pattern (codes 0..3, at least 16 bases each) in
 * T: the positions of pattern k, ascending, are out[occ_off[k] ..
 * occ_off[k + 1]).  Returns the total or -1. */
int64_t brute_exact_many(const uint8_t *t, int64_t n, const uint8_t *pats, const uint64_t *poff, int64_t n_pats,
                         int threads, uint64_t *occ_off, uint32_t **out)
{
    exact_t E;
    memset(&E, 0, sizeof(E));
    E.t = t;
    E.n = n;
    E.pats = pats;
    E.poff = poff;
    E.n_pats = n_pats;
    uint32_t slots = 64;
    while (slots < 4 * (uint64_t)n_pats) slots *= 2;
    E.mask = slots - 1;
    E.slot_key = (uint32_t *)calloc(slots, sizeof(uint32_t));
    E.slot_head = (int64_t *)malloc(sizeof(int64_t) * slots);
    E.next = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_pats ? n_pats : 1));
    E.chunk = 1 << 22;
    const int64_t nch = (n + E.chunk - 1) / E.chunk;
    E.found = (uint64_t **)calloc((size_t)(nch ? nch : 1), sizeof(uint64_t *));
    E.nfound = (int64_t *)calloc((size_t)(nch ? nch : 1), sizeof(int64_t));
    int64_t tot = -1;
    if (!E.slot_key || !E.slot_head || !E.next || !E.found || !E.nfound) goto done;
    for (uint32_t s = 0; s < slots; s++) E.slot_head[s] = -1;
    for (int64_t k = n_pats - 1; k >= 0; k--) {
        const int64_t m = (int64_t)(poff[k + 1] - poff[k]);
        if (m < 16) goto done;
        for (int64_t i = 0; i < m; i++)
            if (pats[poff[k] + i] > 3) goto done;
        const uint32_t c = code16(pats + poff[k]);
        uint32_t s = slot_of(c, E.mask);
        while (E.slot_head[s] >= 0 && E.slot_key[s] != c) s = (s + 1) & E.mask;
        E.slot_key[s] = c;
        E.next[k] = E.slot_head[s];
        E.slot_head[s] = k;
    }
    pool_run(exact_chunk, &E, nch, threads);
    if (E.fail) goto done;
    {
        int64_t all = 0;
        for (int64_t ci = 0; ci < nch; ci++) all += E.nfound[ci];
        uint64_t *pr = (uint64_t *)malloc(sizeof(uint64_t) * 2 * (size_t)(all ? all : 1));
        uint32_t *o = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(all ? all : 1));
        if (!pr || !o) { free(pr); free(o); goto done; }
        int64_t k = 0;
        for (int64_t ci = 0; ci < nch; ci++) {
            memcpy(pr + 2 * k, E.found[ci], sizeof(uint64_t) * 2 * (size_t)E.nfound[ci]);
            k += E.nfound[ci];
        }
        qsort(pr, (size_t)all, 2 * sizeof(uint64_t), cmp_u64pair);
        for (int64_t j = 0; j <= n_pats; j++) occ_off[j] = 0;
        for (int64_t j = 0; j < all; j++) {
            occ_off[pr[2 * j] + 1]++;
            o[j] = (uint32_t)pr[2 * j + 1];
        }
        for (int64_t j = 0; j < n_pats; j++) occ_off[j + 1] += occ_off[j];
        free(pr);
        *out = o;
        tot = all;
    }
done:
    for (int64_t ci = 0; E.found && ci < nch; ci++) free(E.found[ci]);
    free(E.found);
    free(E.nfound);
    free(E.slot_key);
    free(E.slot_head);
    free(E.next);
    return tot;
}

/* ------------------------------------------------ gapped ALL set, batched */

/* End positions e (exclusive) at which some substring T[s, e) has unit edit
 * distance at most k from pattern w (m <= 512 bases, codes 0..3 or N, which
 * equals nothing): Myers' bit-parallel column recurrence over 64-bit words,
 * the pattern's first base in bit 0 of word 0; a free start in the text
 * means nothing is shifted into bit 0.  Calls hit(ctx, e) per end. */
static void myers_ends(const uint8_t *t, int64_t n, const uint8_t *w, int m, int k,
                       void (*hit)(void *, int64_t), void *ctx)
{
    const int nw = (m + 63) / 64;
    uint64_t peq[4][8], Pv[8], Mv[8];
    memset(peq, 0, sizeof(peq));
    for (int i = 0; i < m; i++)
        if (w[i] <= 3) peq[w[i]][i >> 6] |= 1ULL << (i & 63);
    for (int j = 0; j < nw; j++) {
        Pv[j] = ~0ULL;
        Mv[j] = 0;
    }
    const int top = (m - 1) & 63;
    int score = m;
    for (int64_t e = 0; e < n; e++) {
        const int c = t[e];
        uint64_t carry = 0, ph_in = 0, mh_in = 0;
        for (int j = 0; j < nw; j++) {
            const uint64_t eq = peq[c][j], pv = Pv[j], mv = Mv[j];
            const uint64_t xv = eq | mv;
            const uint64_t a = eq & pv;
            const uint64_t s1 = a + pv;
            const uint64_t c1 = s1 < a;
            const uint64_t s2 = s1 + carry;
            const uint64_t c2 = s2 < s1;
            carry = c1 | c2;
            const uint64_t xh = (s2 ^ pv) | eq;
            uint64_t ph = mv | ~(xh | pv);
            uint64_t mh = pv & xh;
            if (j == nw - 1) {
                if ((ph >> top) & 1) score++;
                if ((mh >> top) & 1) score--;
            }
            const uint64_t po = ph >> 63, mo = mh >> 63;
            ph = (ph << 1) | ph_in;
            mh = (mh << 1) | mh_in;
            ph_in = po;
            mh_in = mo;
            Pv[j] = mh | ~(xv | ph);
            Mv[j] = ph & xv;
        }
        if (score <= k) hit(ctx, e + 1);
    }
}

typedef struct {
    int64_t *e;
    int64_t n, cap;
    int oom;
} ends_t;

static void ends_push(void *a, int64_t e)
{
    ends_t *E = (ends_t *)a;
    if (E->n == E->cap) {
        int64_t nc = E->cap ? 2 * E->cap : 64;
        int64_t *nb = (int64_t *)realloc(E->e, sizeof(int64_t) * (size_t)nc);
        if (!nb) { E->oom = 1; return; }
        E->e = nb;
        E->cap = nc;
    }
    E->e[E->n++] = e;
}

typedef struct {
    const uint8_t *t;
    int64_t n;
    const uint8_t *bases;
    const uint64_t *offs;
    const brute_params *p;
    lists_t lists;
    int64_t *n_ends;  /* per read: candidate end positions, both strands */
} edit_t;

static void edit_read(void *a, int64_t r)
{
    edit_t *A = (edit_t *)a;
    const brute_params *p = A->p;
    const uint8_t *W = A->bases + A->offs[r];
    const int m = (int)(A->offs[r + 1] - A->offs[r]);
    A->lists.cnt[r] = 0;
    A->n_ends[r] = 0;
    if (m == 0 || m > 512) return;
    const int k = p->max_diff;
    uint8_t w[512];
    en_t e;
    memset(&e, 0, sizeof(e));
    e.t = A->t;
    e.n = A->n;
    e.m = m;
    e.pr = p;
    e.s = p->indel_end_skip;
    e.s1 = p->indel_end_skip > 1 ? p->indel_end_skip : 1;
    const int sl = p->seed_len > 0 ? (p->seed_len < m ? p->seed_len : m) : 0;
    for (int strand = 0; strand < 2; strand++) {
        strand_pattern(W, m, strand, w);
        ends_t E;
        memset(&E, 0, sizeof(E));
        myers_ends(A->t, A->n, w, m, k, ends_push, &E);
        if (E.oom) { free(E.e); free(e.out); A->lists.cnt[r] = -1; return; }
        A->n_ends[r] += E.n;
        e.w = w;
        e.strand = strand;
        e.seed_lo = strand == 0 ? 0 : m - sl;
        e.seed_hi = strand == 0 ? sl : (sl ? m : 0);
        /* every start of a substring ending at a candidate end, each start
         * once: a transcript of X = T[s, s + len) ends at s + len, which is a
         * candidate, and len <= m + k */
        int64_t done_to = 0;  /* starts below this were enumerated */
        for (int64_t j = 0; j < E.n; j++) {
            int64_t s0 = E.e[j] - m - k, s1 = E.e[j] - (m > k ? m - k : 0);
            if (s0 < done_to) s0 = done_to;
            if (s0 < 0) s0 = 0;
            for (int64_t s = s0; s <= s1 && s < A->n; s++) {
                e.p = s;
                enumerate(&e, 0, s, 0, 0, 0, 0, 0);
            }
            if (s1 + 1 > done_to) done_to = s1 + 1;
        }
        free(E.e);
        if (e.oom) { free(e.out); A->lists.cnt[r] = -1; return; }
    }
    A->lists.recs[r] = e.out;
    A->lists.cnt[r] = dedup(e.out, e.nout);
}

/* The ALL set of brute_align for reads r of a batch (at most 512 bases
 * each): records of read r at out[rec_off[r] .. rec_off[r + 1]), sorted by
 * (strand, pos, len); n_ends[r] = candidate end positions the filter passed.
 * Returns the total or -1. */
int64_t brute_edit_many(const uint8_t *t, int64_t n, const uint8_t *bases, const uint64_t *offs, int64_t n_reads,
                        const brute_params *p, int threads, uint64_t *rec_off, int64_t *n_ends, brute_rec **out)
{
    edit_t A;
    memset(&A, 0, sizeof(A));
    A.t = t;
    A.n = n;
    A.bases = bases;
    A.offs = offs;
    A.p = p;
    A.n_ends = n_ends;
    if (lists_init(&A.lists, n_reads)) return -1;
    pool_run(edit_read, &A, n_reads, threads);
    return lists_join(&A.lists, n_reads, rec_off, out);
}

void brute_free(void *p) { free(p); }
