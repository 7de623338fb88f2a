/*
 * Seeded synthetic inputs: reference genomes and sequencing reads.
 *
 * This file draws random data only.  It holds none of the alignment
 * method's arithmetic (no suffix arrays, no rank queries, no scoring), and
 * it is the one module that both the CPU oracle's tests and the GPU
 * library's tests and benchmark use to obtain inputs.
 *
 * Randomness is counter based: every draw is splitmix64's output function
 * applied to (stream key + (counter + 1) * golden gamma), following Steele,
 * Lea and Flood, "Fast splittable pseudorandom number generators" (OOPSLA
 * 2014).  A draw therefore depends only on (seed, stream, item, counter),
 * never on thread scheduling or on the order in which items are produced.
 *
 * Base codes: A=0, C=1, G=2, T=3 (complement of x is 3-x).
 *
 * Truth records: for every read the generator reports where it came from
 * (strand, leftmost forward coordinate of the consumed template, number of
 * template bases consumed) and its edit script in read coordinates, 5' to 3'
 * as sequenced: type 0 = substitution at read index e, 1 = inserted read
 * base at read index e, 2 = one deleted template base at boundary e (between
 * read bases e-1 and e).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL
#define MAX_EDITS 64

static inline uint64_t sm_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Key of one random stream: (seed, stream id, item index). */
static inline uint64_t skey(uint64_t seed, uint64_t stream, uint64_t item)
{
    return sm_mix(sm_mix(seed * GOLDEN + stream) ^ (item * 0xD1B54A32D192ED03ULL));
}

static inline uint64_t rnd(uint64_t key, uint64_t ctr) { return sm_mix(key + (ctr + 1) * GOLDEN); }

/* Uniform double in [0, 1) from the top 53 bits. */
static inline double unif(uint64_t key, uint64_t ctr)
{
    return (double)(rnd(key, ctr) >> 11) * (1.0 / 9007199254740992.0);
}

/* Uniform integer in [0, m), m > 0 (modulo bias below 2^-30 for the ranges used). */
static inline uint64_t below(uint64_t key, uint64_t ctr, uint64_t m) { return rnd(key, ctr) % m; }

/* Standard normal by Box-Muller from two draws. */
static inline double gauss(uint64_t key, uint64_t ctr)
{
    double u1 = unif(key, ctr), u2 = unif(key, ctr + 1);
    if (u1 < 1e-300) u1 = 1e-300;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

/* One base with P(C)=P(G)=gc/2 and P(A)=P(T)=(1-gc)/2. */
static inline uint8_t draw_base(double u, double gc)
{
    double at = 0.5 * (1.0 - gc);
    if (u < at) return 0;
    if (u < 0.5) return 1;
    if (u < 0.5 + 0.5 * gc) return 2;
    return 3;
}

enum {
    ST_REF = 1,
    ST_CONS = 2,
    ST_COPY = 3,
    ST_CUT = 4,
    ST_SE = 5,
    ST_PAIR = 6,
    ST_END1 = 7,
    ST_END2 = 8,
    ST_LEN = 9,
    ST_UNIQ = 10,
};

int gen_max_edits(void) { return MAX_EDITS; }

/* i.i.d. reference of n bases at the given GC fraction (0.5 = uniform). */
void gen_ref_iid(uint64_t seed, uint64_t n, double gc, uint8_t *out)
{
    uint64_t key = skey(seed, ST_REF, 0);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)n; i++) out[i] = draw_base(unif(key, (uint64_t)i), gc);
}

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/*
 * Reference with repeat families.  n_fam consensus sequences of log-uniform
 * length in [min_len, max_len] are drawn i.i.d. at GC fraction gc.  Copies
 * are then drawn (family uniform, divergence d ~ U[div_lo, div_hi]; each
 * consensus base is substituted with probability 0.9 d, or starts an indel
 * event of 1-3 bases with probability 0.1 d, insertion or deletion with
 * probability 1/2; the copy is reverse-complemented with probability 1/2)
 * until they cover repeat_frac of n.  The rest is i.i.d. sequence at GC
 * fraction gc, cut at uniform points into one more segment than there are
 * copies; the copies sit between those segments in the order drawn.
 *
 * spans receives (start, end, family, reversed) per copy, 4 uint64 each, for
 * at most max_copies copies.  Returns the number of copies, -1 when
 * max_copies is too small or the arguments are bad, -2 when out of memory.
 */
int64_t gen_ref_repeats(uint64_t seed, uint64_t n, double gc, double repeat_frac, int32_t n_fam,
                        int32_t min_len, int32_t max_len, double div_lo, double div_hi, uint8_t *out,
                        uint64_t *spans, int64_t max_copies)
{
    if (n_fam <= 0 || min_len <= 0 || max_len < min_len || max_copies <= 0) return -1;
    int64_t rc = -2;
    uint64_t *cons_off = NULL, *copy_len = NULL, *cuts = NULL;
    uint8_t *cons = NULL, *stage = NULL, *tmp = NULL;

    cons_off = (uint64_t *)malloc(sizeof(uint64_t) * ((size_t)n_fam + 1));
    if (!cons_off) goto done;
    cons_off[0] = 0;
    double lmin = log((double)min_len), lmax = log((double)max_len);
    for (int32_t f = 0; f < n_fam; f++) {
        uint64_t k = skey(seed, ST_CONS, (uint64_t)f);
        uint64_t len = (uint64_t)floor(exp(lmin + unif(k, 0) * (lmax - lmin)));
        if (len < (uint64_t)min_len) len = (uint64_t)min_len;
        if (len > (uint64_t)max_len) len = (uint64_t)max_len;
        cons_off[f + 1] = cons_off[f] + len;
    }
    cons = (uint8_t *)malloc(cons_off[n_fam] + 1);
    if (!cons) goto done;
    for (int32_t f = 0; f < n_fam; f++) {
        uint64_t k = skey(seed, ST_CONS, (uint64_t)f);
        for (uint64_t j = cons_off[f]; j < cons_off[f + 1]; j++)
            cons[j] = draw_base(unif(k, 1 + (j - cons_off[f])), gc);
    }

    uint64_t target = (uint64_t)floor(repeat_frac * (double)n);
    if (target > n) target = n;
    stage = (uint8_t *)malloc(target + 4 * (size_t)max_len + 64);
    copy_len = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)max_copies);
    tmp = (uint8_t *)malloc(4 * (size_t)max_len + 64);
    if (!stage || !copy_len || !tmp) goto done;

    uint64_t total = 0;
    int64_t c = 0;
    while (total < target) {
        if (c >= max_copies) { rc = -1; goto done; }
        uint64_t k = skey(seed, ST_COPY, (uint64_t)c);
        uint64_t ctr = 0;
        int32_t f = (int32_t)below(k, ctr++, (uint64_t)n_fam);
        double d = div_lo + unif(k, ctr++) * (div_hi - div_lo);
        int rev = unif(k, ctr++) < 0.5;
        const uint8_t *src = cons + cons_off[f];
        uint64_t slen = cons_off[f + 1] - cons_off[f];
        uint64_t tl = 0, j = 0;
        while (j < slen) {
            double u = unif(k, ctr++);
            if (u < 0.9 * d) {
                tmp[tl++] = (uint8_t)((src[j] + 1 + below(k, ctr++, 3)) & 3);
                j++;
            } else if (u < d) {
                int ins = unif(k, ctr++) < 0.5;
                uint64_t L = 1 + below(k, ctr++, 3);
                if (ins) {
                    for (uint64_t t = 0; t < L; t++) tmp[tl++] = (uint8_t)below(k, ctr++, 4);
                    tmp[tl++] = src[j];
                    j++;
                } else {
                    j += L;
                }
            } else {
                tmp[tl++] = src[j];
                j++;
            }
        }
        if (total + tl > n) tl = n - total;
        for (uint64_t t = 0; t < tl; t++) stage[total + t] = rev ? (uint8_t)(3 - tmp[tl - 1 - t]) : tmp[t];
        copy_len[c] = tl;
        spans[4 * c + 2] = (uint64_t)f;
        spans[4 * c + 3] = (uint64_t)rev;
        total += tl;
        c++;
    }

    /* unique sequence: U = n - total bases, cut at c uniform points */
    uint64_t U = n - total;
    cuts = (uint64_t *)malloc(sizeof(uint64_t) * ((size_t)c + 2));
    if (!cuts) goto done;
    uint64_t kc = skey(seed, ST_CUT, 0);
    for (int64_t i = 0; i < c; i++) cuts[i] = below(kc, (uint64_t)i, U + 1);
    qsort(cuts, (size_t)c, sizeof(uint64_t), cmp_u64);
    cuts[c] = U;

    uint64_t ku = skey(seed, ST_UNIQ, 0);
    uint64_t w = 0, u_done = 0, s_done = 0;
    for (int64_t i = 0; i <= c; i++) {
        uint64_t seg = cuts[i] - u_done;
        for (uint64_t t = 0; t < seg; t++) out[w + t] = draw_base(unif(ku, u_done + t), gc);
        w += seg;
        u_done = cuts[i];
        if (i < c) {
            memcpy(out + w, stage + s_done, copy_len[i]);
            spans[4 * i + 0] = w;
            spans[4 * i + 1] = w + copy_len[i];
            w += copy_len[i];
            s_done += copy_len[i];
        }
    }
    rc = c;
done:
    free(cons_off); free(cons); free(stage); free(copy_len); free(tmp); free(cuts);
    return rc;
}

/*
 * Emit one read of length L from a template.  The template is the forward
 * reference from tstart on (tstrand 0) or the reverse complement of the
 * reference read leftwards from tstart, exclusive (tstrand 1).  Per emitted
 * base: with probability pi an indel event (insertion or deletion with
 * probability 1/2, length uniform in 1..3), with probability ps a
 * substitution (uniform among the other three bases), else a copy.  The
 * caller guarantees that the template holds at least L + 3 * L bases on the
 * chosen side of tstart.
 */
static void emit_read(uint64_t key, const uint8_t *ref, uint64_t tstart, int tstrand, int32_t L, double ps,
                      double pi, uint8_t *out, uint32_t *o_pos, uint32_t *o_len, uint8_t *o_strand,
                      uint8_t *e_type, uint16_t *e_idx, uint8_t *n_ed)
{
    uint64_t ctr = 0;
    int32_t e = 0;
    uint64_t j = 0;
    int ne = 0, over = 0;
#define TB(jj) (tstrand == 0 ? ref[tstart + (jj)] : (uint8_t)(3 - ref[tstart - 1 - (jj)]))
#define REC(t, ix)                                                                                        \
    do {                                                                                                  \
        if (ne < MAX_EDITS) { e_type[ne] = (uint8_t)(t); e_idx[ne] = (uint16_t)(ix); ne++; }              \
        else over = 1;                                                                                    \
    } while (0)
    while (e < L) {
        double u = unif(key, ctr++);
        if (u < pi) {
            int ins = unif(key, ctr++) < 0.5;
            int len = 1 + (int)below(key, ctr++, 3);
            if (ins) {
                for (int t = 0; t < len && e < L; t++) {
                    out[e] = (uint8_t)below(key, ctr++, 4);
                    REC(1, e);
                    e++;
                }
            } else {
                for (int t = 0; t < len; t++) REC(2, e);
                j += (uint64_t)len;
            }
        } else if (u < pi + ps) {
            out[e] = (uint8_t)((TB(j) + 1 + below(key, ctr++, 3)) & 3);
            REC(0, e);
            e++;
            j++;
        } else {
            out[e] = TB(j);
            e++;
            j++;
        }
    }
#undef TB
#undef REC
    *o_len = (uint32_t)j;
    *o_strand = (uint8_t)tstrand;
    *o_pos = (uint32_t)(tstrand == 0 ? tstart : tstart - j);
    *n_ed = over ? 255 : (uint8_t)ne;
}

/*
 * Single-end reads.  Read r has length lens[r] and is written to
 * bases[offsets[r] ..).  Per read the substitution rate ps ~ U[ps_lo, ps_hi]
 * and the indel event rate is indel_ratio * ps.  With probability rep_frac
 * (when n_spans > 0) the read starts inside a repeat copy span chosen
 * uniformly, otherwise uniformly in the genome; the strand is + or - with
 * probability 1/2.  Truth arrays are per read; e_type/e_idx hold MAX_EDITS
 * entries per read.  Returns 0, or -1 when the genome is too short.
 */
int gen_reads_se(uint64_t seed, const uint8_t *ref, uint64_t n, uint64_t n_reads, const int32_t *lens,
                 const uint64_t *offsets, double ps_lo, double ps_hi, double indel_ratio,
                 const uint64_t *spans, int64_t n_spans, double rep_frac, uint8_t *bases, uint32_t *o_pos,
                 uint32_t *o_len, uint8_t *o_strand, uint8_t *e_type, uint16_t *e_idx, uint8_t *n_ed)
{
    int32_t maxL = 0;
    for (uint64_t r = 0; r < n_reads; r++)
        if (lens[r] > maxL) maxL = lens[r];
    uint64_t margin = 4 * (uint64_t)maxL + 8;
    if (n < 2 * margin + 2) return -1;
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t r = 0; r < (int64_t)n_reads; r++) {
        uint64_t k = skey(seed, ST_SE, (uint64_t)r);
        uint64_t ctr = 0;
        int32_t L = lens[r];
        uint64_t need = 4 * (uint64_t)L + 8;
        int strand = unif(k, ctr++) < 0.5;
        double ps = ps_lo + unif(k, ctr++) * (ps_hi - ps_lo);
        double pi = indel_ratio * ps;
        int in_rep = n_spans > 0 && unif(k, ctr++) < rep_frac;
        uint64_t lo, hi; /* range of tstart */
        if (strand == 0) { lo = 0; hi = n - need; }
        else { lo = need; hi = n; }
        if (in_rep) {
            uint64_t s = below(k, ctr++, (uint64_t)n_spans);
            uint64_t cs = spans[4 * s], ce = spans[4 * s + 1];
            uint64_t a, b;
            if (strand == 0) { a = cs; b = ce > cs + (uint64_t)L ? ce - (uint64_t)L : cs; }
            else { a = cs + (uint64_t)L < ce ? cs + (uint64_t)L : ce; b = ce; }
            if (a < lo) a = lo;
            if (b > hi) b = hi;
            if (a <= b) { lo = a; hi = b; }
        }
        uint64_t tstart = lo + below(k, ctr++, hi - lo + 1);
        emit_read(skey(seed, ST_SE + 100, (uint64_t)r), ref, tstart, strand, L, ps, pi, bases + offsets[r],
                  o_pos + r, o_len + r, o_strand + r, e_type + (size_t)r * MAX_EDITS,
                  e_idx + (size_t)r * MAX_EDITS, n_ed + r);
    }
    return 0;
}

/* Per-pair read length drawn uniformly from choices[0..n_choices). */
void gen_pair_lengths(uint64_t seed, uint64_t n_pairs, const int32_t *choices, int32_t n_choices,
                      int32_t *lens)
{
    for (uint64_t p = 0; p < n_pairs; p++) {
        uint64_t k = skey(seed, ST_LEN, p);
        lens[p] = choices[below(k, 0, (uint64_t)n_choices)];
    }
}

/*
 * Paired-end reads.  Pair p has read length lens[p] (both ends).  The
 * fragment length is round(N(frag_mu, frag_sd)), at least max(frag_min,
 * L + 24); the fragment start is uniform; the fragment is taken from the +
 * or - strand with probability 1/2.  End 1 is the first L bases of the
 * fragment, end 2 the first L bases of its reverse complement (forward-
 * reverse orientation).  Each read's substitution rate ps ~ U[ps_lo, ps_hi],
 * indel event rate indel_ratio * ps.  Reads of end 1 are written to
 * bases1[offsets[p] ..), end 2 to bases2[offsets[p] ..).  frag receives
 * (start, length, strand) per pair.  Returns 0, or -1 when the genome is too
 * short.
 */
int gen_reads_pe(uint64_t seed, const uint8_t *ref, uint64_t n, uint64_t n_pairs, const int32_t *lens,
                 const uint64_t *offsets, double frag_mu, double frag_sd, int32_t frag_min, double ps_lo,
                 double ps_hi, double indel_ratio, uint8_t *bases1, uint8_t *bases2, uint32_t *frag,
                 uint32_t *o_pos, uint32_t *o_len, uint8_t *o_strand, uint8_t *e_type, uint16_t *e_idx,
                 uint8_t *n_ed)
{
    int32_t maxL = 0;
    for (uint64_t p = 0; p < n_pairs; p++)
        if (lens[p] > maxL) maxL = lens[p];
    uint64_t fmax = (uint64_t)(frag_mu + 8.0 * frag_sd) + 4 * (uint64_t)maxL + 64;
    if (n < 2 * fmax) return -1;
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t p = 0; p < (int64_t)n_pairs; p++) {
        uint64_t k = skey(seed, ST_PAIR, (uint64_t)p);
        int32_t L = lens[p];
        double g = gauss(k, 0);
        int64_t fl = (int64_t)llround(frag_mu + frag_sd * g);
        int64_t fmin = frag_min > L + 24 ? frag_min : L + 24;
        if (fl < fmin) fl = fmin;
        if ((uint64_t)fl > fmax - 4 * (uint64_t)L - 16) fl = (int64_t)(fmax - 4 * (uint64_t)L - 16);
        int fstrand = unif(k, 2) < 0.5;
        /* keep 4L bases of slack on both sides for deletions */
        uint64_t slack = 4 * (uint64_t)L + 8;
        uint64_t f = slack + below(k, 3, n - 2 * slack - (uint64_t)fl + 1);
        frag[3 * p + 0] = (uint32_t)f;
        frag[3 * p + 1] = (uint32_t)fl;
        frag[3 * p + 2] = (uint32_t)fstrand;
        double ps1 = ps_lo + unif(k, 4) * (ps_hi - ps_lo);
        double ps2 = ps_lo + unif(k, 5) * (ps_hi - ps_lo);
        /* end 1 template: fragment from its own start */
        uint64_t t1 = fstrand == 0 ? f : f + (uint64_t)fl;
        uint64_t t2 = fstrand == 0 ? f + (uint64_t)fl : f;
        size_t r1 = 2 * (size_t)p, r2 = 2 * (size_t)p + 1;
        emit_read(skey(seed, ST_END1, (uint64_t)p), ref, t1, fstrand, L, ps1, indel_ratio * ps1,
                  bases1 + offsets[p], o_pos + r1, o_len + r1, o_strand + r1, e_type + r1 * MAX_EDITS,
                  e_idx + r1 * MAX_EDITS, n_ed + r1);
        emit_read(skey(seed, ST_END2, (uint64_t)p), ref, t2, 1 - fstrand, L, ps2, indel_ratio * ps2,
                  bases2 + offsets[p], o_pos + r2, o_len + r2, o_strand + r2, e_type + r2 * MAX_EDITS,
                  e_idx + r2 * MAX_EDITS, n_ed + r2);
    }
    return 0;
}
