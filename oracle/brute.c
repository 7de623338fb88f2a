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
 *
 * The transcript rules are those of the oracle's header: gap = maximal run
 * of I or of D; I at read index i needs s <= i < m - s; D at boundary b
 * needs max(s,1) <= b <= m - max(s,1); diffs touching the seed (first
 * seed_len bases as sequenced, a D counting when strictly inside) are at
 * most seed_diff.
 */
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

void brute_free(void *p) { free(p); }
