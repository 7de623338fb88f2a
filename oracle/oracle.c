/*
 * CPU ORACLE -- test infrastructure, not the product.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this code.  It shares nothing with the GPU library: its own
 * suffix-array algorithm, its own index layout (one byte per BWT symbol,
 * rank checkpoints every 64 rows, the full suffix array), its own recursive
 * search.  It is written to be read against the method, not to be fast.
 *
 * What it computes (Genetically Improved BarraCUDA, section 2, and the
 * BWA short-read backtracking method that BarraCUDA's aln derives from):
 *
 *  - FM-index of T$ (symbols $ < A < C < G < T): suffix array SA, BWT,
 *    C[a] = 1 + #symbols of T smaller than a, Occ(a, i) = #a in BWT[0, i).
 *    A string X has the SA interval [k, l] of the rows whose suffix starts
 *    with X; it is empty iff k > l (the two pointers have passed each other) and its width
 *    l - k + 1 is the number of occurrences of X (section 2, the upper and
 *    lower pointer description).  Backward step for aX:
 *        k' = C[a] + Occ(a, k),  l' = C[a] + Occ(a, l + 1) - 1,
 *    from the root [0, n].  The same index is built for reverse(T).
 *    Both strands are searched 5' end (seed) first: strand + searches
 *    reverse(W) on the index of reverse(T), so its hit intervals are those
 *    of reverse(X) there; strand - searches revcomp(W) on the index of T.
 *    Each search takes its D-array bound from the other index.
 *
 *  - Inexact search by backtracking (section 2: the search backs up and
 *    tries alternatives when the read does not match exactly).  A transcript
 *    of read W (length m) against a reference string X uses match/mismatch,
 *    I (read base only) and D (reference base only); a gap is a maximal run
 *    of I or of D.  n_mm = #mismatches, n_gapo = #gaps, n_gape = sum of
 *    (gap length - 1), diffs = n_mm + n_gapo + n_gape, score = s_mm n_mm +
 *    s_gapo n_gapo + s_gape n_gape.  A read base N (code 4) mismatches every
 *    reference base.  A transcript is valid iff diffs <= max_diff, n_gapo <=
 *    max_gapo, n_gape <= max_gape (when max_gape >= 0), every I sits at a
 *    read index i with s <= i < m - s, every D sits at a boundary b (between
 *    read bases b-1 and b) with max(s,1) <= b <= m - max(s,1), where s is
 *    indel_end_skip, and the diffs touching the seed (the first seed_len
 *    bases of the read as sequenced; a D counts when strictly inside) number
 *    at most seed_diff.
 *
 *    ALL(W) = {(strand, X) : X occurs in T and a valid transcript of W_s
 *    against X exists}, W_+ = W, W_- = revcomp(W).  Each hit carries the
 *    lexicographically smallest (score, diffs, n_gapo, n_mm) over its valid
 *    transcripts.  BEST(W): S* = min score; tier 1 = hits of score S*,
 *    tier 2 = hits with S* < score <= S* + s_mm; c1, c2 = summed widths of
 *    the tiers; tier 2 is reported iff c1 <= max_best.  A read whose
 *    candidate set (both tiers in BEST mode, every hit in ALL mode) has more
 *    than max_hits members reports nothing and is flagged.  Reported hits
 *    are ordered by (score, strand, k, len).
 *
 *  - Locate: the positions of a reported hit of width <= max_occ are the
 *    sorted 0-based leftmost forward coordinates of X: SA values of its rows
 *    for strand -, n - SA_rev - |X| for strand +.
 *
 *  - Pairing (section 2: the approximate fragment length lets far-apart
 *    matches of the two ends be discarded).  A proper pair puts the two
 *    ends on opposite strands; with (pf) the + end's position and (pr, lr)
 *    the - end's position and length, pf <= pr and lo <= pr + lr - pf <= hi.
 *    The chosen pair minimises (score1 + score2, |insert - mu|, pf,
 *    strand1, pos1, len1, pos2, len2).  Without one, each end takes its
 *    single-end primary, the minimum (score, diffs, strand, pos, len).
 *
 *  - Mate rescue and mapping quality, the rest of the pairing step that
 *    closes the pipeline (section 3.7); the paper gives no details, so both
 *    are readings, stated where they are computed (orc_rescue_mates,
 *    orc_mapq).
 *
 * The search visits children in a fixed order -- match, mismatches by base,
 * insertion, deletions by base -- and, in BEST mode, drops a state whose
 * score plus min(s_mm, s_gapo, s_gape) * D[i] exceeds best-so-far + s_mm.
 * The result is order independent; the order only fixes the counters of
 * index lines touched, which the benchmark reports as algorithmic bytes.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define CK 64          /* rank checkpoint spacing, in rows */
#define MAX_READ 512   /* longest read accepted */
#define MAX_DIFF 15    /* largest per-read difference budget accepted */
#define INF_SCORE 0x7fffffff

enum { GAP_NONE = 0, GAP_INS = 1, GAP_DEL = 2 };
enum { MODE_ALL = 0, MODE_BEST = 1 };
enum { ST_HIT = 1, ST_OVERFLOW = 2, ST_INVALID = 4 };

/* ------------------------------------------------------------------ */
/* FM-index                                                             */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t n;       /* text length; rows 0..n */
    uint32_t *sa;    /* n + 1 */
    uint8_t *bwt;    /* n + 1, code 4 = $ */
    uint32_t *ck;    /* ((n + 1) / CK + 1) x 4 */
    uint64_t C[4];
    int64_t primary; /* row whose SA value is 0 */
} fm_t;

typedef struct {
    int64_t n;
    fm_t fwd, rev;
} orc_index;

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/* Stable LSD radix sort of 64-bit words, 16 bits per pass. */
static int radix_u64(uint64_t *a, int64_t N)
{
    uint64_t *b = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)N);
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * 65536);
    if (!b || !cnt) { free(b); free(cnt); return -1; }
    for (int pass = 0; pass < 4; pass++) {
        int sh = 16 * pass;
        memset(cnt, 0, sizeof(int64_t) * 65536);
        for (int64_t i = 0; i < N; i++) cnt[(a[i] >> sh) & 0xffff]++;
        int64_t s = 0;
        for (int d = 0; d < 65536; d++) { int64_t c = cnt[d]; cnt[d] = s; s += c; }
        for (int64_t i = 0; i < N; i++) b[cnt[(a[i] >> sh) & 0xffff]++] = a[i];
        uint64_t *t = a; a = b; b = t;
    }
    /* four passes: the data is back in the caller's array */
    free(b);
    free(cnt);
    return 0;
}

/*
 * Suffix array of T$ by prefix doubling (Manber and Myers, with the
 * group refinement of Larsson and Sadakane): suffixes are first ordered
 * by their first H0 symbols, then every group of suffixes that still tie
 * on their first h symbols is re-ordered by the rank of the suffix h
 * positions later, which orders them by their first 2h symbols.  The loop
 * ends when every group holds one suffix.
 */
static int sa_doubling(const uint8_t *t, int64_t n, uint32_t *sa)
{
    const int H0 = 13; /* 5^13 < 2^31: a 13-symbol key and the position fit one word */
    int64_t N = n + 1;
    uint64_t *a = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)N);
    uint32_t *rank = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)N);
    uint32_t *nrank = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)N);
    uint8_t *head = (uint8_t *)malloc((size_t)N + 1);
    uint64_t *tmp = NULL;
    int64_t tmp_cap = 0;
    int rc = -1;
    if (!a || !rank || !nrank || !head) goto out;
    for (int64_t i = 0; i < N; i++) {
        uint64_t key = 0;
        for (int j = 0; j < H0; j++) {
            int64_t p = i + j;
            key = key * 5 + (p < n ? (uint64_t)t[p] + 1 : 0);
        }
        a[i] = (key << 32) | (uint64_t)i;
    }
    if (radix_u64(a, N)) goto out;
    for (int64_t j = 0; j < N; j++) {
        sa[j] = (uint32_t)(a[j] & 0xffffffffu);
        head[j] = (uint8_t)(j == 0 || (a[j] >> 32) != (a[j - 1] >> 32));
    }
    head[N] = 1;
    {
        int64_t h0 = 0;
        for (int64_t j = 0; j < N; j++) {
            if (head[j]) h0 = j;
            rank[sa[j]] = (uint32_t)h0;
        }
    }
    free(a);
    a = NULL;

    for (int64_t h = H0;; h *= 2) {
        int any = 0;
        memcpy(nrank, rank, sizeof(uint32_t) * (size_t)N);
        int64_t j = 0;
        while (j < N) {
            int64_t e = j + 1;
            while (!head[e]) e++;
            int64_t g = e - j;
            if (g > 1) {
                any = 1;
                if (g > tmp_cap) {
                    free(tmp);
                    tmp_cap = g * 2;
                    tmp = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)tmp_cap);
                    if (!tmp) goto out;
                }
                /* members of a tied group have at least h symbols before $ */
                for (int64_t x = 0; x < g; x++)
                    tmp[x] = ((uint64_t)rank[sa[j + x] + h] << 32) | sa[j + x];
                if (g <= 16) {
                    for (int64_t x = 1; x < g; x++) {
                        uint64_t v = tmp[x];
                        int64_t y = x - 1;
                        while (y >= 0 && tmp[y] > v) { tmp[y + 1] = tmp[y]; y--; }
                        tmp[y + 1] = v;
                    }
                } else {
                    qsort(tmp, (size_t)g, sizeof(uint64_t), cmp_u64);
                }
                int64_t hd = j;
                for (int64_t x = 0; x < g; x++) {
                    sa[j + x] = (uint32_t)(tmp[x] & 0xffffffffu);
                    if (x > 0 && (tmp[x] >> 32) != (tmp[x - 1] >> 32)) { hd = j + x; head[j + x] = 1; }
                    nrank[sa[j + x]] = (uint32_t)hd;
                }
            }
            j = e;
        }
        uint32_t *sw = rank; rank = nrank; nrank = sw;
        if (!any) break;
    }
    rc = 0;
out:
    free(a); free(rank); free(nrank); free(head); free(tmp);
    return rc;
}

static int fm_build(fm_t *f, const uint8_t *t, int64_t n)
{
    memset(f, 0, sizeof(*f));
    int64_t N = n + 1;
    f->n = n;
    f->sa = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)N);
    f->bwt = (uint8_t *)malloc((size_t)N);
    int64_t nck = N / CK + 1;
    f->ck = (uint32_t *)calloc((size_t)nck * 4, sizeof(uint32_t));
    if (!f->sa || !f->bwt || !f->ck) return -1;
    if (sa_doubling(t, n, f->sa)) return -1;
    uint64_t cnt[4] = {0, 0, 0, 0};
    for (int64_t j = 0; j < N; j++) {
        if (j % CK == 0)
            for (int a = 0; a < 4; a++) f->ck[(j / CK) * 4 + a] = (uint32_t)cnt[a];
        uint32_t s = f->sa[j];
        uint8_t c = s == 0 ? 4 : t[s - 1];
        if (s == 0) f->primary = j;
        f->bwt[j] = c;
        if (c < 4) cnt[c]++;
    }
    if (N % CK == 0)
        for (int a = 0; a < 4; a++) f->ck[(N / CK) * 4 + a] = (uint32_t)cnt[a];
    f->C[0] = 1;
    for (int a = 1; a < 4; a++) f->C[a] = f->C[a - 1] + cnt[a - 1];
    return 0;
}

static void fm_free(fm_t *f)
{
    free(f->sa); free(f->bwt); free(f->ck);
    memset(f, 0, sizeof(*f));
}

/* Occ(a, i) = number of symbol a in BWT[0, i), 0 <= i <= n + 1. */
static inline uint64_t occ(const fm_t *f, int a, uint64_t i)
{
    uint64_t c = f->ck[(i / CK) * 4 + a];
    for (uint64_t r = (i / CK) * CK; r < i; r++) c += f->bwt[r] == a;
    return c;
}

void orc_index_free(void *h)
{
    orc_index *x = (orc_index *)h;
    if (!x) return;
    fm_free(&x->fwd);
    fm_free(&x->rev);
    free(x);
}

typedef struct {
    fm_t *f;
    const uint8_t *t;
    int64_t n;
    int rc;
} build_job;

static void *build_worker(void *arg)
{
    build_job *b = (build_job *)arg;
    b->rc = fm_build(b->f, b->t, b->n);
    return NULL;
}

/* Build the index of T (codes 0..3) and of reverse(T), the two in parallel.
 * NULL on failure, when T holds a code outside 0..3, or when n + 1 does not
 * fit 32 bits. */
void *orc_index_build(const uint8_t *t, int64_t n)
{
    if (n < 1 || n + 1 > (int64_t)0xffffffffLL) return NULL;
    for (int64_t i = 0; i < n; i++)
        if (t[i] > 3) return NULL;
    orc_index *x = (orc_index *)calloc(1, sizeof(orc_index));
    uint8_t *r = (uint8_t *)malloc((size_t)n);
    if (!x || !r) { free(x); free(r); return NULL; }
    x->n = n;
    for (int64_t i = 0; i < n; i++) r[i] = t[n - 1 - i];
    build_job jf = {&x->fwd, t, n, -1}, jr = {&x->rev, r, n, -1};
    pthread_t th;
    int threaded = pthread_create(&th, NULL, build_worker, &jr) == 0;
    build_worker(&jf);
    if (threaded) pthread_join(th, NULL);
    else build_worker(&jr);
    free(r);
    if (jf.rc || jr.rc) { orc_index_free(x); return NULL; }
    return x;
}

int64_t orc_index_n(void *h) { return ((orc_index *)h)->n; }

/* Copy out one direction (0 = forward, 1 = reverse): SA (n + 1), BWT with
 * $ as 4 (n + 1), C (4), primary. */
void orc_index_get(void *h, int which, uint32_t *sa, uint8_t *bwt, uint64_t *C, int64_t *primary)
{
    const fm_t *f = which ? &((orc_index *)h)->rev : &((orc_index *)h)->fwd;
    if (sa) memcpy(sa, f->sa, sizeof(uint32_t) * (size_t)(f->n + 1));
    if (bwt) memcpy(bwt, f->bwt, (size_t)(f->n + 1));
    if (C) memcpy(C, f->C, sizeof(f->C));
    if (primary) *primary = f->primary;
}

void orc_occ4(void *h, int which, uint64_t i, uint64_t *out)
{
    const fm_t *f = which ? &((orc_index *)h)->rev : &((orc_index *)h)->fwd;
    for (int a = 0; a < 4; a++) out[a] = occ(f, a, i);
}

/* Exact backward search of p[0, m) on the chosen index; returns 1 when the
 * interval is non-empty.  *steps counts backward steps taken. */
int orc_exact(void *h, int which, const uint8_t *p, int m, uint64_t *k_out, uint64_t *l_out, int *steps)
{
    const fm_t *f = which ? &((orc_index *)h)->rev : &((orc_index *)h)->fwd;
    uint64_t k = 0, l = (uint64_t)f->n;
    int s = 0;
    for (int i = m - 1; i >= 0; i--) {
        int a = p[i];
        if (a > 3) { k = 1; l = 0; break; }
        k = f->C[a] + occ(f, a, k);
        l = f->C[a] + occ(f, a, l + 1) - 1;
        s++;
        if (k > l) break;
    }
    *k_out = k;
    *l_out = l;
    if (steps) *steps = s;
    return k <= l;
}

/* ------------------------------------------------------------------ */
/* D-array                                                              */
/* ------------------------------------------------------------------ */

/*
 * D[i] is a lower bound on the diffs needed to place w[0..i] in the text S
 * that the search runs on: scan w left to right, extending w[j..i] on the
 * index of reverse(S) (prepending w[i] to reverse(w[j..i-1])); whenever the
 * interval empties, w[j..i] is not a substring of S, so it holds at least
 * one difference; count it and start a fresh segment at i + 1.  The
 * segments are disjoint, so the count is a lower bound on the differences
 * of any transcript of w[0..i].
 */
static void darray(const fm_t *rv, const uint8_t *w, int m, uint8_t *D, uint64_t *touch, int bpl, int maxd)
{
    uint64_t k = 0, l = (uint64_t)rv->n;
    int z = 0;
    for (int i = 0; i < m; i++) {
        int a = w[i];
        if (a > 3) {
            k = 1; l = 0;
        } else {
            if (touch) *touch += (k / (uint64_t)bpl == (l + 1) / (uint64_t)bpl) ? 1 : 2;
            k = rv->C[a] + occ(rv, a, k);
            l = rv->C[a] + occ(rv, a, l + 1) - 1;
        }
        if (k > l) {
            z++;
            k = 0;
            l = (uint64_t)rv->n;
            if (z > maxd) {
                /* the strand is already out of budget at the root; the rest
                 * of the scan cannot change any decision */
                for (int j = i; j < m; j++) D[j] = (uint8_t)(z > 255 ? 255 : z);
                return;
            }
        }
        D[i] = (uint8_t)(z > 255 ? 255 : z);
    }
}

/* D-array of pattern w for a search on index `which` (0 = T, 1 = reverse(T));
 * the scan runs on the other index. */
void orc_darray(void *h, int which, const uint8_t *w, int m, uint8_t *D)
{
    const orc_index *ix = (const orc_index *)h;
    darray(which ? &ix->fwd : &ix->rev, w, m, D, NULL, 1, 255);
}

/* ------------------------------------------------------------------ */
/* Search                                                               */
/* ------------------------------------------------------------------ */

typedef struct {
    int32_t max_diff, max_gapo, max_gape, seed_len, seed_diff, indel_end_skip;
    int32_t s_mm, s_gapo, s_gape, mode, max_best;
    uint32_t max_hits;
    int32_t use_d;          /* 1 = prune with the D-array bound (0 only for testing) */
    int32_t bases_per_line; /* rows per index line, for the line-touch counters */
    int32_t sa_sample;      /* row sampling interval, for the locate counters */
    int32_t pad;
} orc_params;

typedef struct {
    uint32_t k, l;
    uint16_t len, score;
    uint8_t strand, n_mm, n_gapo, n_gape;
} orc_hit;

typedef struct {
    uint64_t expand;  /* states expanded (each issues rank queries at k and l + 1) */
    uint64_t touch_s; /* index lines touched by the search */
    uint64_t touch_d; /* index lines touched by the D-array scans */
    uint64_t max_stack; /* deepest pending-sibling stack of a depth-first search
                           that keeps the first surviving child current and
                           stacks the others (the GPU kernel's scheme) */
} orc_count;

typedef struct {
    const fm_t *fm;
    const orc_params *p;
    const uint8_t *w;
    int m, strand, maxd, seed_lo, seed_hi, s1, minc;
    const uint8_t *D;
    int best;
    orc_hit *cand;
    int64_t ncand, cap;
    orc_count *cnt;
    int oom;
} dfs_t;

static void record(dfs_t *c, uint64_t k, uint64_t l, int len, int nmm, int ngo, int nge, int score)
{
    if (c->ncand == c->cap) {
        int64_t nc = c->cap ? c->cap * 2 : 64;
        orc_hit *nb = (orc_hit *)realloc(c->cand, sizeof(orc_hit) * (size_t)nc);
        if (!nb) { c->oom = 1; return; }
        c->cand = nb;
        c->cap = nc;
    }
    orc_hit *h = &c->cand[c->ncand++];
    h->k = (uint32_t)k;
    h->l = (uint32_t)l;
    h->len = (uint16_t)len;
    h->score = (uint16_t)score;
    h->strand = (uint8_t)c->strand;
    h->n_mm = (uint8_t)nmm;
    h->n_gapo = (uint8_t)ngo;
    h->n_gape = (uint8_t)nge;
    if (score < c->best) c->best = score;
}

static inline int in_seed(const dfs_t *c, int i) { return i >= c->seed_lo && i < c->seed_hi; }
static inline int in_seed_gap(const dfs_t *c, int b) { return b > c->seed_lo && b < c->seed_hi; }

/* One child of an expanded state. */
typedef struct {
    int i;
    uint64_t k, l;
    int nmm, ngo, nge, gs, sd, len, score;
} kid_t;

static void visit(dfs_t *c, int i, uint64_t k, uint64_t l, int nmm, int ngo, int nge, int gs, int sd, int len,
                  int score, int sp);

/* The static validity constraints of a child. */
static int child_ok(const dfs_t *c, const kid_t *x)
{
    const orc_params *p = c->p;
    int diffs = x->nmm + x->ngo + x->nge;
    if (diffs > c->maxd) return 0;
    if (x->ngo > p->max_gapo) return 0;
    if (p->max_gape >= 0 && x->nge > p->max_gape) return 0;
    if (p->seed_len > 0 && x->sd > p->seed_diff) return 0;
    if (p->use_d && x->i >= 0 && diffs + c->D[x->i] > c->maxd) return 0;
    return 1;
}

/* Would the BEST bound drop this child right now? */
static int child_bound_ok(const dfs_t *c, const kid_t *x)
{
    const orc_params *p = c->p;
    if (p->mode != MODE_BEST || c->best == INF_SCORE) return 1;
    int lb = x->score + (p->use_d && x->i >= 0 ? c->minc * c->D[x->i] : 0);
    return lb <= c->best + p->s_mm;
}

static void visit(dfs_t *c, int i, uint64_t k, uint64_t l, int nmm, int ngo, int nge, int gs, int sd, int len,
                  int score, int sp)
{
    const orc_params *p = c->p;
    const fm_t *f = c->fm;
    if (c->oom) return;
    if (p->mode == MODE_BEST && c->best != INF_SCORE) {
        int lb = score + (p->use_d && i >= 0 ? c->minc * c->D[i] : 0);
        if (lb > c->best + p->s_mm) return;
    }
    if (sp > (int)c->cnt->max_stack) c->cnt->max_stack = (uint64_t)sp;
    if (i < 0) {
        record(c, k, l, len, nmm, ngo, nge, score);
        return;
    }
    c->cnt->expand++;
    c->cnt->touch_s += (k / (uint64_t)p->bases_per_line == (l + 1) / (uint64_t)p->bases_per_line) ? 1 : 2;
    uint64_t ka[4], la[4];
    for (int a = 0; a < 4; a++) {
        ka[a] = f->C[a] + occ(f, a, k);
        la[a] = f->C[a] + occ(f, a, l + 1) - 1;
    }
    int b = c->w[i];
    /* children in the fixed order: match, mismatches by base, insertion,
     * deletions by base */
    kid_t kids[9];
    int nk = 0;
#define KID(I, K, L, NMM, NGO, NGE, GS, SD, LEN, SC)                                                     \
    do {                                                                                              \
        kid_t x_ = {(I), (K), (L), (NMM), (NGO), (NGE), (GS), (SD), (LEN), (SC)};                     \
        if (child_ok(c, &x_)) kids[nk++] = x_;                                                        \
    } while (0)
    /* match */
    if (b < 4 && ka[b] <= la[b]) KID(i - 1, ka[b], la[b], nmm, ngo, nge, GAP_NONE, sd, len + 1, score);
    /* mismatches */
    for (int a = 0; a < 4; a++)
        if (a != b && ka[a] <= la[a])
            KID(i - 1, ka[a], la[a], nmm + 1, ngo, nge, GAP_NONE, sd + in_seed(c, i), len + 1, score + p->s_mm);
    /* insertion: read base w[i] has no reference base */
    if (i >= p->indel_end_skip && i < c->m - p->indel_end_skip) {
        if (gs == GAP_INS)
            KID(i - 1, k, l, nmm, ngo, nge + 1, GAP_INS, sd + in_seed(c, i), len, score + p->s_gape);
        else
            KID(i - 1, k, l, nmm, ngo + 1, nge, GAP_INS, sd + in_seed(c, i), len, score + p->s_gapo);
    }
    /* deletion: reference base a between read bases i and i + 1 */
    int bd = i + 1;
    if (bd >= c->s1 && bd <= c->m - c->s1) {
        for (int a = 0; a < 4; a++) {
            if (ka[a] > la[a]) continue;
            if (gs == GAP_DEL)
                KID(i, ka[a], la[a], nmm, ngo, nge + 1, GAP_DEL, sd + in_seed_gap(c, bd), len + 1, score + p->s_gape);
            else
                KID(i, ka[a], la[a], nmm, ngo + 1, nge, GAP_DEL, sd + in_seed_gap(c, bd), len + 1, score + p->s_gapo);
        }
    }
#undef KID
    /* stack depth bookkeeping: the kernel keeps the first child that the
     * bound lets through current and stacks the others above sp */
    int v = 0;
    int pos_[9];
    for (int j = 0; j < nk; j++) pos_[j] = child_bound_ok(c, &kids[j]) ? v++ : -1;
    for (int j = 0; j < nk; j++) {
        int csp = pos_[j] < 0 ? sp : sp + v - 1 - pos_[j];
        visit(c, kids[j].i, kids[j].k, kids[j].l, kids[j].nmm, kids[j].ngo, kids[j].nge, kids[j].gs, kids[j].sd,
              kids[j].len, kids[j].score, csp);
    }
}

static int cmp_dedup(const void *x, const void *y)
{
    const orc_hit *a = (const orc_hit *)x, *b = (const orc_hit *)y;
    if (a->strand != b->strand) return a->strand < b->strand ? -1 : 1;
    if (a->k != b->k) return a->k < b->k ? -1 : 1;
    if (a->len != b->len) return a->len < b->len ? -1 : 1;
    if (a->score != b->score) return a->score < b->score ? -1 : 1;
    int da = a->n_mm + a->n_gapo + a->n_gape, db = b->n_mm + b->n_gapo + b->n_gape;
    if (da != db) return da < db ? -1 : 1;
    if (a->n_gapo != b->n_gapo) return a->n_gapo < b->n_gapo ? -1 : 1;
    if (a->n_mm != b->n_mm) return a->n_mm < b->n_mm ? -1 : 1;
    return 0;
}

static int cmp_report(const void *x, const void *y)
{
    const orc_hit *a = (const orc_hit *)x, *b = (const orc_hit *)y;
    if (a->score != b->score) return a->score < b->score ? -1 : 1;
    if (a->strand != b->strand) return a->strand < b->strand ? -1 : 1;
    if (a->k != b->k) return a->k < b->k ? -1 : 1;
    if (a->len != b->len) return a->len < b->len ? -1 : 1;
    return 0;
}

typedef struct {
    orc_hit *hits;
    int64_t n;
    uint32_t c1, c2;
    uint8_t status;
} read_out;

/* Align one read (both strands) and canonicalise its hits. */
static void align_one(const orc_index *ix, const uint8_t *W, int m, int maxd, const orc_params *p, read_out *ro,
                      orc_count *cnt)
{
    memset(ro, 0, sizeof(*ro));
    if (m > MAX_READ || maxd > MAX_DIFF || maxd < 0) { ro->status = ST_INVALID; return; }
    if (m == 0) return;
    uint8_t ws[MAX_READ], D[MAX_READ];
    dfs_t c;
    memset(&c, 0, sizeof(c));
    c.p = p;
    c.m = m;
    c.maxd = maxd;
    c.best = INF_SCORE;
    c.cnt = cnt;
    c.s1 = p->indel_end_skip > 1 ? p->indel_end_skip : 1;
    c.minc = p->s_mm;
    if (p->s_gapo < c.minc) c.minc = p->s_gapo;
    if (p->s_gape < c.minc) c.minc = p->s_gape;
    int sl = p->seed_len > 0 ? (p->seed_len < m ? p->seed_len : m) : 0;
    /* Both strands are searched seed first.  Strand +: pattern reverse(W)
     * on the index of reverse(T) (finds reverse(X)); strand -: pattern
     * revcomp(W) on the index of T.  In either pattern the read's 5' end is
     * at the right, so the seed is w[m - sl, m), consumed first. */
    c.seed_lo = m - sl;
    c.seed_hi = sl ? m : 0;
    for (int strand = 0; strand < 2; strand++) {
        const fm_t *srch = strand == 0 ? &ix->rev : &ix->fwd;
        const fm_t *other = strand == 0 ? &ix->fwd : &ix->rev;
        for (int i = 0; i < m; i++) {
            uint8_t b = W[m - 1 - i];
            ws[i] = strand == 0 ? b : (b > 3 ? 4 : (uint8_t)(3 - b));
        }
        c.fm = srch;
        c.w = ws;
        c.strand = strand;
        darray(other, ws, m, D, &cnt->touch_d, p->bases_per_line, maxd);
        c.D = D;
        /* the root: nothing consumed, interval of the empty string */
        if (!p->use_d || D[m - 1] <= maxd) visit(&c, m - 1, 0, (uint64_t)ix->n, 0, 0, 0, GAP_NONE, 0, 0, 0, 0);
    }
    if (c.oom) { free(c.cand); ro->status = ST_INVALID; return; }
    /* deduplicate by (strand, k, len), keeping the smallest (score, diffs, n_gapo, n_mm) */
    int64_t nu = 0;
    if (c.ncand) {
        qsort(c.cand, (size_t)c.ncand, sizeof(orc_hit), cmp_dedup);
        for (int64_t i = 0; i < c.ncand; i++) {
            if (nu > 0 && c.cand[nu - 1].strand == c.cand[i].strand && c.cand[nu - 1].k == c.cand[i].k &&
                c.cand[nu - 1].len == c.cand[i].len)
                continue;
            c.cand[nu++] = c.cand[i];
        }
    }
    if (nu == 0) { free(c.cand); return; }
    int smin = INF_SCORE;
    for (int64_t i = 0; i < nu; i++)
        if (c.cand[i].score < smin) smin = c.cand[i].score;
    uint64_t c1 = 0, c2 = 0;
    int64_t nc = 0;
    for (int64_t i = 0; i < nu; i++) {
        const orc_hit *h = &c.cand[i];
        uint64_t w = (uint64_t)h->l - h->k + 1;
        if (h->score == smin) c1 += w;
        else if (h->score <= smin + p->s_mm) c2 += w;
        if (p->mode == MODE_ALL || h->score <= smin + p->s_mm) nc++;
    }
    if ((uint64_t)nc > p->max_hits) {
        ro->status = ST_OVERFLOW;
        ro->c1 = ro->c2 = 0xffffffffu;
        free(c.cand);
        return;
    }
    ro->c1 = c1 > 0xffffffffu ? 0xffffffffu : (uint32_t)c1;
    ro->c2 = c2 > 0xffffffffu ? 0xffffffffu : (uint32_t)c2;
    int keep2 = c1 <= (uint64_t)p->max_best;
    int64_t nr = 0;
    for (int64_t i = 0; i < nu; i++) {
        const orc_hit *h = &c.cand[i];
        int keep = p->mode == MODE_ALL || h->score == smin || (keep2 && h->score <= smin + p->s_mm);
        if (keep) c.cand[nr++] = *h;
    }
    qsort(c.cand, (size_t)nr, sizeof(orc_hit), cmp_report);
    ro->hits = c.cand;
    ro->n = nr;
    ro->status = nr ? ST_HIT : 0;
}

typedef struct {
    const orc_index *ix;
    const uint8_t *bases;
    const uint64_t *off;
    const uint8_t *maxd;
    const orc_params *p;
    int64_t lo, hi;
    read_out *ro;
    orc_count *cnt;
} job_t;

static void *align_worker(void *arg)
{
    job_t *j = (job_t *)arg;
    for (int64_t r = j->lo; r < j->hi; r++) {
        int m = (int)(j->off[r + 1] - j->off[r]);
        int md = j->maxd ? j->maxd[r] : j->p->max_diff;
        align_one(j->ix, j->bases + j->off[r], m, md, j->p, &j->ro[r], &j->cnt[r]);
    }
    return NULL;
}

/*
 * Align n_reads reads (CSR bases/offsets; optional per-read budgets maxd)
 * with n_threads threads.  Fills hit_off (n_reads + 1), c1, c2, status and
 * the per-read counters, and returns a malloc'ed array of the reported hits
 * in *hits_out (release with orc_free).  Returns the total hit count, or -1.
 */
int64_t orc_align(void *h, const uint8_t *bases, const uint64_t *off, const uint8_t *maxd, int64_t n_reads,
                  const orc_params *p, int n_threads, uint64_t *hit_off, orc_hit **hits_out, uint32_t *c1,
                  uint32_t *c2, uint8_t *status, orc_count *cnt)
{
    const orc_index *ix = (const orc_index *)h;
    if (p->bases_per_line <= 0) return -1;
    read_out *ro = (read_out *)calloc((size_t)(n_reads > 0 ? n_reads : 1), sizeof(read_out));
    if (!ro) return -1;
    memset(cnt, 0, sizeof(orc_count) * (size_t)n_reads);
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    pthread_t th[256];
    job_t jobs[256];
    int joinable[256];
    int64_t per = (n_reads + n_threads - 1) / n_threads;
    for (int t = 0; t < n_threads; t++) {
        jobs[t].ix = ix;
        jobs[t].bases = bases;
        jobs[t].off = off;
        jobs[t].maxd = maxd;
        jobs[t].p = p;
        jobs[t].lo = t * per < n_reads ? t * per : n_reads;
        jobs[t].hi = (t + 1) * per < n_reads ? (t + 1) * per : n_reads;
        jobs[t].ro = ro;
        jobs[t].cnt = cnt;
        joinable[t] = 0;
        if (n_threads > 1 && pthread_create(&th[t], NULL, align_worker, &jobs[t]) == 0) joinable[t] = 1;
        else align_worker(&jobs[t]);
    }
    for (int t = 0; t < n_threads; t++)
        if (joinable[t]) pthread_join(th[t], NULL);
    int64_t total = 0;
    for (int64_t r = 0; r < n_reads; r++) total += ro[r].n;
    orc_hit *all = (orc_hit *)malloc(sizeof(orc_hit) * (size_t)(total > 0 ? total : 1));
    if (!all) { for (int64_t r = 0; r < n_reads; r++) free(ro[r].hits); free(ro); return -1; }
    int64_t w = 0;
    hit_off[0] = 0;
    for (int64_t r = 0; r < n_reads; r++) {
        if (ro[r].n) memcpy(all + w, ro[r].hits, sizeof(orc_hit) * (size_t)ro[r].n);
        w += ro[r].n;
        hit_off[r + 1] = (uint64_t)w;
        c1[r] = ro[r].c1;
        c2[r] = ro[r].c2;
        status[r] = ro[r].status;
        free(ro[r].hits);
    }
    free(ro);
    *hits_out = all;
    return total;
}

void orc_free(void *p) { free(p); }

/* ------------------------------------------------------------------ */
/* Locate                                                               */
/* ------------------------------------------------------------------ */

static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

/* Number of LF steps a row-sampled walk takes from row j to a sampled row
 * (row % sample == 0, or the row holding position 0). */
static uint64_t lf_steps(const fm_t *f, uint64_t j, uint64_t sample)
{
    uint64_t s = 0;
    while (j % sample != 0 && j != (uint64_t)f->primary) {
        int a = f->bwt[j];
        j = f->C[a] + occ(f, a, j);
        s++;
    }
    return s;
}

/*
 * Positions of every hit with width <= max_occ: pos_off (n_hits + 1) gets
 * the CSR offsets, *pos_out a malloc'ed array of sorted positions.  If
 * steps is not NULL it receives, per hit, the LF steps a row-sampled walk
 * needs (sample rows apart) summed over the hit's rows.  Returns the total
 * number of positions, or -1.
 */
int64_t orc_locate(void *h, const orc_hit *hits, int64_t n_hits, uint32_t max_occ, uint64_t *pos_off,
                   uint32_t **pos_out, uint64_t *steps, uint32_t sample)
{
    const orc_index *ix = (const orc_index *)h;
    int64_t total = 0;
    pos_off[0] = 0;
    for (int64_t i = 0; i < n_hits; i++) {
        uint64_t w = (uint64_t)hits[i].l - hits[i].k + 1;
        if (hits[i].k <= hits[i].l && w <= max_occ) total += (int64_t)w;
        pos_off[i + 1] = (uint64_t)total;
    }
    uint32_t *pos = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(total > 0 ? total : 1));
    if (!pos) return -1;
    for (int64_t i = 0; i < n_hits; i++) {
        uint64_t o = pos_off[i], w = pos_off[i + 1] - o;
        uint64_t st = 0;
        /* strand + hits are intervals of reverse(X) in the index of
         * reverse(T): reverse(X) at q there is X at n - q - |X| in T */
        const fm_t *f = hits[i].strand == 0 ? &ix->rev : &ix->fwd;
        for (uint64_t x = 0; x < w; x++) {
            uint64_t q = f->sa[hits[i].k + x];
            pos[o + x] = hits[i].strand == 0 ? (uint32_t)((uint64_t)ix->n - q - hits[i].len) : (uint32_t)q;
            if (steps) st += lf_steps(f, hits[i].k + x, sample);
        }
        qsort(pos + o, (size_t)w, sizeof(uint32_t), cmp_u32);
        if (steps) steps[i] = st;
    }
    *pos_out = pos;
    return total;
}

/* ------------------------------------------------------------------ */
/* Pairing                                                              */
/* ------------------------------------------------------------------ */

typedef struct {
    uint32_t pos1, pos2;
    int32_t insert;
    uint16_t len1, len2;
    uint16_t score1, score2;
    uint8_t strand1, strand2, flags, pad;
} orc_pair;

enum { PF_PAIRED = 1, PF_MAPPED1 = 2, PF_MAPPED2 = 4, PF_REP1 = 8, PF_REP2 = 16 };

/* Single-end primary of one read: smallest (score, diffs, strand, pos, len)
 * over the located positions of its reported hits.  Returns 1 if found;
 * *rep is set when some reported hit was wider than max_occ. */
static int se_primary(const orc_hit *h, int64_t nh, const uint64_t *po, const uint32_t *pos, uint32_t *p_out,
                      const orc_hit **h_out, int *rep)
{
    int found = 0;
    *rep = 0;
    for (int64_t i = 0; i < nh; i++) {
        if (po[i + 1] == po[i]) { *rep = 1; continue; }
        for (uint64_t x = po[i]; x < po[i + 1]; x++) {
            int better = 0;
            if (!found) better = 1;
            else {
                const orc_hit *b = *h_out;
                int da = h[i].n_mm + h[i].n_gapo + h[i].n_gape, db = b->n_mm + b->n_gapo + b->n_gape;
                if (h[i].score != b->score) better = h[i].score < b->score;
                else if (da != db) better = da < db;
                else if (h[i].strand != b->strand) better = h[i].strand < b->strand;
                else if (pos[x] != *p_out) better = pos[x] < *p_out;
                else better = h[i].len < b->len;
            }
            if (better) { found = 1; *p_out = pos[x]; *h_out = &h[i]; }
        }
    }
    return found;
}

/*
 * Pair n_pairs read pairs from their reported hits (hits1/hits2 with CSR
 * offsets) and their located positions (pos_off*, pos*, per hit).  With
 * hits2 == NULL every record holds end 1's single-end primary only.
 */
void orc_pair_reads(int64_t n_pairs, const uint64_t *hoff1, const orc_hit *hits1, const uint64_t *poff1,
                    const uint32_t *pos1, const uint64_t *hoff2, const orc_hit *hits2, const uint64_t *poff2,
                    const uint32_t *pos2, int32_t lo, int32_t hi, int32_t mu, orc_pair *out)
{
    for (int64_t q = 0; q < n_pairs; q++) {
        orc_pair o;
        memset(&o, 0, sizeof(o));
        o.pos1 = o.pos2 = 0xffffffffu;
        const orc_hit *H1 = hits1 + hoff1[q];
        int64_t n1 = (int64_t)(hoff1[q + 1] - hoff1[q]);
        const uint64_t *P1 = poff1 + hoff1[q];
        int found = 0;
        int64_t bs = 0, bd = 0, bpf = 0;
        if (hits2) {
            const orc_hit *H2 = hits2 + hoff2[q];
            int64_t n2 = (int64_t)(hoff2[q + 1] - hoff2[q]);
            const uint64_t *P2 = poff2 + hoff2[q];
            for (int64_t i = 0; i < n1; i++)
                for (uint64_t x = P1[i]; x < P1[i + 1]; x++)
                    for (int64_t j = 0; j < n2; j++) {
                        if (H1[i].strand == H2[j].strand) continue;
                        for (uint64_t y = P2[j]; y < P2[j + 1]; y++) {
                            int64_t pf, pr, lr;
                            if (H1[i].strand == 0) { pf = pos1[x]; pr = pos2[y]; lr = H2[j].len; }
                            else { pf = pos2[y]; pr = pos1[x]; lr = H1[i].len; }
                            if (pf > pr) continue;
                            int64_t ins = pr + lr - pf;
                            if (ins < lo || ins > hi) continue;
                            int64_t s = (int64_t)H1[i].score + H2[j].score;
                            int64_t d = ins > mu ? ins - mu : mu - ins;
                            int better;
                            if (!found) better = 1;
                            else if (s != bs) better = s < bs;
                            else if (d != bd) better = d < bd;
                            else if (pf != bpf) better = pf < bpf;
                            else if (H1[i].strand != o.strand1) better = H1[i].strand < o.strand1;
                            else if (pos1[x] != o.pos1) better = pos1[x] < o.pos1;
                            else if (H1[i].len != o.len1) better = H1[i].len < o.len1;
                            else if (pos2[y] != o.pos2) better = pos2[y] < o.pos2;
                            else better = H2[j].len < o.len2;
                            if (better) {
                                found = 1;
                                bs = s; bd = d; bpf = pf;
                                o.pos1 = pos1[x]; o.pos2 = pos2[y];
                                o.len1 = H1[i].len; o.len2 = H2[j].len;
                                o.score1 = H1[i].score; o.score2 = H2[j].score;
                                o.strand1 = H1[i].strand; o.strand2 = H2[j].strand;
                                o.insert = (int32_t)ins;
                            }
                        }
                    }
            int rep1 = 0, rep2 = 0;
            uint32_t pp1 = 0, pp2 = 0;
            const orc_hit *hp1 = NULL, *hp2 = NULL;
            int f1 = se_primary(H1, n1, P1, pos1, &pp1, &hp1, &rep1);
            int f2 = se_primary(H2, n2, P2, pos2, &pp2, &hp2, &rep2);
            if (found) {
                o.flags = PF_PAIRED | PF_MAPPED1 | PF_MAPPED2;
            } else {
                if (f1) {
                    o.pos1 = pp1; o.len1 = hp1->len; o.score1 = hp1->score; o.strand1 = hp1->strand;
                    o.flags |= PF_MAPPED1;
                }
                if (f2) {
                    o.pos2 = pp2; o.len2 = hp2->len; o.score2 = hp2->score; o.strand2 = hp2->strand;
                    o.flags |= PF_MAPPED2;
                }
            }
            if (rep1) o.flags |= PF_REP1;
            if (rep2) o.flags |= PF_REP2;
        } else {
            int rep1 = 0;
            uint32_t pp;
            const orc_hit *hp;
            if (se_primary(H1, n1, P1, pos1, &pp, &hp, &rep1)) {
                o.pos1 = pp; o.len1 = hp->len; o.score1 = hp->score; o.strand1 = hp->strand;
                o.flags |= PF_MAPPED1;
            }
            if (rep1) o.flags |= PF_REP1;
        }
        out[q] = o;
    }
}

/* ------------------------------------------------------------------ */
/* Host helpers                                                         */
/* ------------------------------------------------------------------ */

/*
 * Difference budget for a read of length L: the smallest k >= 0 with
 * P[Poisson(err L) > k] < thres (the rule BWA documents for its
 * fractional -n option, with err = 0.02 and thres = 0.04).
 */
int orc_max_diff_rule(int L, double err, double thres)
{
    double lam = err * L, term = exp(-lam), cdf = term;
    for (int k = 0; k < 1000; k++) {
        if (1.0 - cdf < thres) return k;
        term *= lam / (double)(k + 1);
        cdf += term;
    }
    return 1000;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/*
 * Insert-size window from the inserts of uniquely placed proper pairs:
 * sort; quartiles at index floor(q (N - 1)); keep inserts within
 * [p25 - 2 IQR, p75 + 2 IQR]; mu = their mean, sigma = population standard
 * deviation (summed in ascending order); lo = max(0, floor(mu - 4 sigma)),
 * hi = ceil(mu + 4 sigma), mu rounded half to even.  Fewer than 100
 * inserts give [0, 500] and mu = 250.  out = {lo, hi, mu}.
 */
int orc_estimate_insert(const int32_t *ins, int64_t N, int32_t *out)
{
    if (N < 100) { out[0] = 0; out[1] = 500; out[2] = 250; return 0; }
    int32_t *s = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    if (!s) return -1;
    memcpy(s, ins, sizeof(int32_t) * (size_t)N);
    qsort(s, (size_t)N, sizeof(int32_t), cmp_i32);
    double p25 = s[(int64_t)floor(0.25 * (double)(N - 1))];
    double p75 = s[(int64_t)floor(0.75 * (double)(N - 1))];
    double iqr = p75 - p25, lo_k = p25 - 2 * iqr, hi_k = p75 + 2 * iqr;
    double sum = 0;
    int64_t c = 0;
    for (int64_t i = 0; i < N; i++)
        if (s[i] >= lo_k && s[i] <= hi_k) { sum += s[i]; c++; }
    double mu = sum / (double)c, v = 0;
    for (int64_t i = 0; i < N; i++)
        if (s[i] >= lo_k && s[i] <= hi_k) v += ((double)s[i] - mu) * ((double)s[i] - mu);
    double sd = sqrt(v / (double)c);
    double lo = floor(mu - 4 * sd), hi = ceil(mu + 4 * sd);
    out[0] = (int32_t)(lo < 0 ? 0 : lo);
    out[1] = (int32_t)hi;
    out[2] = (int32_t)nearbyint(mu);
    free(s);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Mate rescue                                                          */
/* ------------------------------------------------------------------ */

/*
 * A pair left without a proper pair, with a primary for at least one end,
 * gets a second chance for the other end (the mate): the best local
 * alignment of the mate inside the reference window that the fragment
 * length allows around the primary (the anchor; with primaries for both
 * ends, the one of lower score, end 1 on ties).  This is the sampe step the
 * paper's pipeline ends with (section 3.7), here a reading: affine-gap local
 * alignment (match +a, mismatch -b, a gap of g bases -(o + e g); a read N
 * mismatches everything), kept only when its score reaches min_score.
 *
 *  anchor on +, at pf: the mate is on - (revcomp(mate) aligns), window
 *    [pf, pf + hi) clipped to the reference; the alignment must end at
 *    window column >= lo - 1, so that insert = pr + lr - pf lies in [lo, hi].
 *  anchor on -, at pr with length lr: the mate is on + and must start at
 *    pf <= pr + lr - lo inside [pr + lr - hi, pr + lr).  Reversing both the
 *    mate and the window turns this into the first case's constraint on the
 *    end column, so one routine serves both.
 *
 * The routine fills a column of the local-alignment matrices per reference
 * base, carrying with every cell the window column where its alignment
 * starts.  Ties: a cell prefers the diagonal move, then the gap along the
 * reference, then the gap along the read, over 0 (no alignment); a gap
 * prefers opening over extending.  The reported alignment is the first
 * cell of highest score in column order (smallest end column, then
 * smallest read row) among the columns allowed.
 */

typedef struct {
    uint32_t pos;    /* leftmost reference base of the rescued alignment */
    uint16_t len;    /* reference bases it spans */
    int16_t score;   /* its local alignment score */
    int32_t insert;  /* pr + lr - pf of the rescued pair */
    uint8_t end;     /* 0: nothing rescued, else the rescued end (1 or 2) */
    uint8_t strand;  /* strand of the rescued end */
    uint8_t pad[2];
} orc_rescue;

#define RESCUE_NEG (-1000000000)

/* best local alignment of q (m) in r (w) ending at column >= e_min:
 * returns the score (0: none), sets *jend and *jstart */
static int local_best(const uint8_t *q, int m, const uint8_t *r, int w, int e_min, int a, int b, int o, int e,
                      int *jend, int *jstart)
{
    int *Hp = malloc(sizeof(int) * (m + 1) * 4);
    int *Ep = Hp + (m + 1), *HpO = Ep + (m + 1), *EpO = HpO + (m + 1);
    for (int i = 0; i <= m; i++) {
        Hp[i] = 0;
        Ep[i] = RESCUE_NEG;
        HpO[i] = EpO[i] = 0;
    }
    int best = 0;
    *jend = *jstart = -1;
    for (int j = 0; j < w; j++) {
        int F = RESCUE_NEG, FO = 0;
        int Hdiag = 0, HdiagO = 0; /* H[i-1][j-1] */
        int Hup = 0, HupO = 0;     /* H[i-1][j] */
        for (int i = 1; i <= m; i++) {
            /* gap along the reference (E), from the previous column */
            int eo = Hp[i] - (o + e), ee = Ep[i] - e, E, EO;
            if (eo >= ee) {
                E = eo;
                EO = HpO[i];
            } else {
                E = ee;
                EO = EpO[i];
            }
            /* gap along the read (F), from the row above */
            int fo = Hup - (o + e), fe = F - e;
            if (fo >= fe) {
                F = fo;
                FO = HupO;
            } else {
                F = fe;
            }
            int s = (q[i - 1] < 4 && q[i - 1] == r[j]) ? a : -b;
            int diag = Hdiag + s, diagO = Hdiag > 0 ? HdiagO : j;
            int H = 0, HO = 0;
            if (diag > H) {
                H = diag;
                HO = diagO;
            }
            if (E > H) {
                H = E;
                HO = EO;
            }
            if (F > H) {
                H = F;
                HO = FO;
            }
            Hdiag = Hp[i];
            HdiagO = HpO[i];
            Hp[i] = H;
            HpO[i] = HO;
            Ep[i] = E;
            EpO[i] = EO;
            Hup = H;
            HupO = HO;
            if (j >= e_min && H > best) {
                best = H;
                *jend = j;
                *jstart = HO;
            }
        }
    }
    free(Hp);
    return best;
}

void orc_rescue_mates(int64_t n_pairs, const uint8_t *ref, int64_t n, const uint8_t *b1, const uint64_t *o1,
                      const uint8_t *b2, const uint64_t *o2, const orc_pair *pairs, int32_t lo, int32_t hi,
                      int32_t a, int32_t b, int32_t o, int32_t e, int32_t min_score, orc_rescue *out)
{
    uint8_t *q = malloc(MAX_READ), *win = malloc(hi > 0 ? (size_t)hi : 1);
    for (int64_t p = 0; p < n_pairs; p++) {
        orc_rescue *res = &out[p];
        memset(res, 0, sizeof(*res));
        const orc_pair *pr = &pairs[p];
        const int m1 = (pr->flags & 2) != 0, m2 = (pr->flags & 4) != 0;
        if ((pr->flags & 1) || (!m1 && !m2)) continue;
        const int anchor = (m1 && m2) ? (pr->score1 <= pr->score2 ? 1 : 2) : (m1 ? 1 : 2);
        const int mate = 3 - anchor;
        const int64_t pa = anchor == 1 ? pr->pos1 : pr->pos2;
        const int la = anchor == 1 ? pr->len1 : pr->len2;
        const int sa = anchor == 1 ? pr->strand1 : pr->strand2;
        const uint8_t *W = mate == 1 ? b1 + o1[p] : b2 + o2[p];
        const int m = (int)(mate == 1 ? o1[p + 1] - o1[p] : o2[p + 1] - o2[p]);
        if (m == 0 || m > MAX_READ) continue;
        int64_t w0, w1;
        if (sa == 0) {
            w0 = pa;
            w1 = pa + hi < n ? pa + hi : n;
            for (int i = 0; i < m; i++) { /* revcomp(mate) */
                uint8_t c = W[m - 1 - i];
                q[i] = c < 4 ? (uint8_t)(3 - c) : c;
            }
        } else {
            w1 = pa + la;
            w0 = w1 - hi > 0 ? w1 - hi : 0;
            for (int i = 0; i < m; i++) q[i] = W[m - 1 - i]; /* reverse(mate) */
        }
        const int w = (int)(w1 - w0);
        if (w <= 0) continue;
        for (int j = 0; j < w; j++) win[j] = sa == 0 ? ref[w0 + j] : ref[w1 - 1 - j];
        int jend, jstart;
        const int sc = local_best(q, m, win, w, lo - 1, a, b, o, e, &jend, &jstart);
        if (sc <= 0 || sc < min_score) continue;
        res->end = (uint8_t)mate;
        res->score = (int16_t)sc;
        res->len = (uint16_t)(jend - jstart + 1);
        if (sa == 0) {
            res->strand = 1;
            res->pos = (uint32_t)(w0 + jstart);
            res->insert = jend + 1;
        } else {
            res->strand = 0;
            res->pos = (uint32_t)(w1 - 1 - jend);
            res->insert = jend + 1;
        }
    }
    free(q);
    free(win);
}

/* the local alignment routine alone, for the tests that pin it */
int orc_local_best(const uint8_t *q, int m, const uint8_t *r, int w, int e_min, int a, int b, int o, int e, int *jend,
                   int *jstart)
{
    return local_best(q, m, r, w, e_min, a, b, o, e, jend, jstart);
}

/* ------------------------------------------------------------------ */
/* Mapping quality                                                      */
/* ------------------------------------------------------------------ */

/*
 * MAPQ, phred-scaled confidence that an end's reported placement is right
 * (a reading: the paper has no such output).  Each placement the search
 * reported weighs 1 when it is in tier 1 and r = 10^(-q_tier / 10) when it is
 * in tier 2 (one mismatch-penalty step worse); the chosen placement's share
 * of the total weight c1 + c2 r is the probability it is right:
 *
 *     P = w / (c1 + c2 r),  w = 1 (its score is the read's best) or r,
 *     Q_se = round(-10 log10(1 - P)), at most q_unique; q_unique when P = 1;
 *
 * with Q_se at most q_budget when every tier-1 hit spends the read's whole
 * difference budget (a placement just past the budget was not searched),
 * and 0 for an end that is not placed or whose candidate set overflowed.
 * An end of a proper pair is wrong only if both placements are, so both
 * ends of a proper pair get min(q_pair, Q_se(end 1) + Q_se(end 2)).  A
 * rescued mate is placed relative to its anchor and takes the anchor's
 * Q_se.  Rounding is half up, in double precision.
 */
static int mapq_se(const orc_pair *pr, int e, const uint64_t *hoff, const orc_hit *hits, const uint32_t *c1,
                   const uint32_t *c2, const uint8_t *st, int64_t p, int budget, double r, int q_unique,
                   int q_budget)
{
    const uint32_t pos = e == 1 ? pr->pos1 : pr->pos2;
    const int score = e == 1 ? pr->score1 : pr->score2;
    if (pos == 0xFFFFFFFFu || (st[p] & 2) || c1[p] == 0 || hoff[p + 1] == hoff[p]) return 0;
    const orc_hit *h = hits + hoff[p];
    const int64_t nh = (int64_t)(hoff[p + 1] - hoff[p]);
    /* tier 1: the leading hits of the best score (hits are ordered by score first) */
    int dmin = 1 << 30;
    for (int64_t i = 0; i < nh && h[i].score == h[0].score; i++) {
        const int d = h[i].n_mm + h[i].n_gapo + h[i].n_gape;
        if (d < dmin) dmin = d;
    }
    const double w = score == h[0].score ? 1.0 : r;
    const double den = (double)c1[p] + (double)c2[p] * r;
    int q;
    if (den - w <= 0.0) {
        q = q_unique;
    } else {
        q = (int)floor(-10.0 * log10((den - w) / den) + 0.5);
        if (q > q_unique) q = q_unique;
        if (q < 0) q = 0;
    }
    if (dmin >= budget && q > q_budget) q = q_budget;
    return q;
}

void orc_mapq(int64_t n_pairs, const uint64_t *hoff1, const orc_hit *hits1, const uint32_t *c1_1,
              const uint32_t *c2_1, const uint8_t *st1, const uint8_t *bud1, const uint64_t *hoff2,
              const orc_hit *hits2, const uint32_t *c1_2, const uint32_t *c2_2, const uint8_t *st2,
              const uint8_t *bud2, int32_t max_diff, const orc_pair *pairs, const orc_rescue *rescue,
              int32_t q_tier, int32_t q_unique, int32_t q_budget, int32_t q_pair, uint8_t *out)
{
    const double r = pow(10.0, -q_tier / 10.0);
    for (int64_t p = 0; p < n_pairs; p++) {
        const orc_pair *pr = &pairs[p];
        int q1 = mapq_se(pr, 1, hoff1, hits1, c1_1, c2_1, st1, p, bud1 ? bud1[p] : max_diff, r, q_unique, q_budget);
        int q2 = hoff2 ? mapq_se(pr, 2, hoff2, hits2, c1_2, c2_2, st2, p, bud2 ? bud2[p] : max_diff, r, q_unique,
                                 q_budget)
                       : 0;
        int o1 = q1, o2 = q2;
        if (pr->flags & 1) {
            const int s = q1 + q2 < q_pair ? q1 + q2 : q_pair;
            o1 = o2 = s;
        } else if (rescue && rescue[p].end == 2) {
            o2 = q1;
        } else if (rescue && rescue[p].end == 1) {
            o1 = q2;
        }
        out[2 * p] = (uint8_t)o1;
        out[2 * p + 1] = (uint8_t)o2;
    }
}
