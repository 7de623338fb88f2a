// bwfm: GPU side of the FM-index short-read alignment path and its C ABI.
//
// Method: Genetically Improved BarraCUDA, section 2 (backward search with an
// upper and a lower pointer per read, backtracking over alternatives for
// inexact reads, the whole index resident in GPU memory), with the search
// rules of the BWA short-read backtracking method that BarraCUDA derives
// from; locate and pairing as in "sampe" (sections 2 and 3.7).  The exact
// definitions are stated in include/bwfm.h.
//
// Layout.  Each direction of the index is an array of rank lines (64 or
// 128 bytes): four uint32 counts of A, C, G, T before the line ($ counted as
// A), then the line's BWT rows as bit planes -- per 32 rows a word of the
// codes' high bits and a word of their low bits -- so one rank query is one
// line fetch plus three popcounts per 32 rows.  Row-sampled suffix array values
// serve locate.
//
// Search.  One lane per read, both strands in turn, each strand 5' end
// first (strand +: reverse(read) on the index of reverse(T); strand -:
// revcomp(read) on the index of T).  Per strand the lane first builds the
// D-array lower bound on the other index, then runs a depth-first search
// whose current state lives in registers; the first surviving child becomes
// the next current state and its siblings go to a lane-private stack in
// device memory, so the common one-child step touches no stack.  Children are
// taken in a fixed order (match, mismatches by base, insertion, deletions by
// base), and in BEST mode a state is dropped when its score plus the least
// cost of its remaining D[i] differences exceeds best + s_mm.  Distinct hits
// collect in a lane-private buffer.  Reads whose stack or hit buffer fills up
// are searched again in a second pass with buffers of the worst-case size.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "bwfm_internal.h"

using namespace bwfm;

namespace {

// ------------------------------------------------------------------ constants

constexpr int GAP_INS = 1, GAP_DEL = 2;  // gap state of a search state (0: not in a gap)
constexpr uint32_t ST_RESEARCH = 8;  // status bit: needed the second pass
constexpr int PH_FAST = 0, PH_BEST = 1, PH_COLLECT = 2;
constexpr int INF_SCORE = 0x7fffffff;
constexpr uint32_t PLAIN_STACK = 320;  // stack entries per lane, plain form first pass
// Tuning constants a variant build may override with -D (results do not
// depend on them; paper_1505_07855_amd/variants.py searches over them).
// First-pass hit slots per lane: 128 keeps reads with up to that many
// candidate hits, common on repeat-rich references, out of the second pass,
// at no cost on reads with few hits.
#ifndef BWFM_FAST_CAND
#define BWFM_FAST_CAND 128
#endif
#ifndef BWFM_POPS_PER_STEP
#define BWFM_POPS_PER_STEP 1
#endif
#ifndef BWFM_SLOW_LANES
#define BWFM_SLOW_LANES 16384
#endif
// Alternative implementations of single code sites ("genes"), chosen at
// compile time; every alternative computes the same results, only its cost
// differs.  0 is the shipped one.  paper_1505_07855_amd/variants.py
// searches over them.
//   ROWMASK:  row masks of a 32-row group by compare and select (0) or by
//             one 64-bit shift (1).
//   PAIRLINE: the paired rank query of planar lines shares a line that
//             holds both rows (0) or always fetches two (1).
//   REFILL:   idle lanes take new reads every iteration (0) or only once a
//             quarter of the wave is idle or no lane is busy (1).
//   SUBHDR:   with SUBLOAD 0, a 128-byte sub-counted query reads the
//             boundary words only for rows past 128 (0) or always (1).
#ifndef BWFM_GENE_ROWMASK
#define BWFM_GENE_ROWMASK 0
#endif
#ifndef BWFM_GENE_PAIRLINE
#define BWFM_GENE_PAIRLINE 0
#endif
#ifndef BWFM_GENE_REFILL
#define BWFM_GENE_REFILL 0
#endif
#ifndef BWFM_GENE_SUBHDR
#define BWFM_GENE_SUBHDR 0
#endif
//   DPREPASS: the batched form scans each read's D-arrays inside the
//             persistent loop, one rank query per iteration, unless its
//             reads may be DPRE_MIN_LEN bases or longer (0), or always (1)
//             in a pre-pass kernel of its own, one lane per read, so the
//             loop only searches.
#ifndef BWFM_GENE_DPREPASS
#define BWFM_GENE_DPREPASS 0
#endif
// Batches whose max_len reaches this scan their D-arrays in the pre-pass:
// on 250 bp reads the pre-pass and a loop that only searches take 5-6% less
// time than the loop's own scans, on 100 bp reads 7% more.
constexpr uint32_t DPRE_MIN_LEN = 200;
//   TWOSTATE: a searching lane expands one state per iteration (0), or two
//             (1): besides its current state it keeps a second one, taken
//             from the top of its stack, whose rank query is issued with
//             the first, so two expansions share one round trip (before the
//             batch runs dry; in the endgame the second state goes back on
//             the stack for the sharing).
#ifndef BWFM_GENE_TWOSTATE
#define BWFM_GENE_TWOSTATE 0
#endif
//   SUBLOAD:  a 128-byte sub-counted query loads the line's first 16 bytes
//             and, past row 128, its next 16 (0), or 12 bytes of counts and
//             the one boundary word its row needs (1, shipped: fewer
//             registers hold line data, 1.5% faster on the benchmark batch).
#ifndef BWFM_GENE_SUBLOAD
#define BWFM_GENE_SUBLOAD 1
#endif
//   KTLOOP:   the batched form's persistent loop ignores the short-string
//             table (0), or reads it, like the plain form, for states and
//             D-array steps whose string is shorter than its levels (1):
//             with a few levels the table sits in L2, where those rank
//             queries' line fills from the Infinity Cache do not.
#ifndef BWFM_GENE_KTLOOP
#define BWFM_GENE_KTLOOP 0
#endif
constexpr bool KT_LOOP = BWFM_GENE_KTLOOP == 1;
constexpr uint32_t FAST_CAND = BWFM_FAST_CAND;  // hit slots per lane, first pass
constexpr int BLOCK = 256;
constexpr int POPS_PER_STEP = BWFM_POPS_PER_STEP;  // stack pops per lane per persistent iteration (more costs the
                                  // whole wave a pass of the pop code; measured best at 1)

struct Params {
    int max_diff, max_gapo, max_gape, seed_len, seed_diff, ies, s_mm, s_gapo, s_gape, mode, max_best;
    uint32_t max_hits;
    int minc, s1;
};

struct ReadsView {
    const uint8_t *bases;
    const uint64_t *off;
    const uint32_t *len;  // per-read lengths, or NULL: read r ends where read r + 1 starts
    const uint8_t *maxd;
    uint32_t n, max_len;
    const uint64_t *n_dev;  // or NULL; else the batch holds min(*n_dev, n) reads (set on the device)
};

// number of reads in the batch
__device__ __forceinline__ uint32_t reads_n(const ReadsView &rd) {
    return rd.n_dev ? (uint32_t)min(*rd.n_dev, (uint64_t)rd.n) : rd.n;
}

// a count known on the host (n) or, when n_dev is set, on the device (at most n)
__device__ __forceinline__ uint64_t count_of(uint64_t n, const uint64_t *n_dev) {
    return n_dev ? min(*n_dev, n) : n;
}

// start and length of read r
__device__ __forceinline__ void read_span(const ReadsView &rd, uint32_t r, uint64_t &o0, uint64_t &len, bool &bad) {
    o0 = rd.off[r];
    if (rd.len) {
        len = rd.len[r];
        bad = false;
    } else {
        const uint64_t o1 = rd.off[r + 1];
        bad = o1 < o0;
        len = bad ? 0 : o1 - o0;
    }
}

// Lane-private buffers in device memory.  Element e of lane t sits at
// base[t * lane_step + e * stride]: interleaved (lane_step 1, stride = lanes)
// when a wave's lanes move in step, contiguous (lane_step = cap, stride 1)
// when they do not.  Each lane's strand pattern and D-array live in LDS,
// lds_stride bytes per lane.
struct LaneBufs {
    uint4 *stack;
    uint4 *cand;
    uint32_t stack_lane_step, stack_stride, stack_cap;
    uint32_t cand_lane_step, cand_stride, cand_cap;
    uint32_t lds_stride;
};

// ------------------------------------------------------------------ rank queries

// element b of a four-element register array without dynamic indexing
__device__ __forceinline__ uint32_t sel4(const uint32_t (&v)[4], int b) {
    return b == 0 ? v[0] : (b == 1 ? v[1] : (b == 2 ? v[2] : v[3]));
}

// direction 0 or 1 of the index without dynamic indexing into the argument
__device__ __forceinline__ DevDir pick_dir(const DevIndex &ix, int which) {
    DevDir d;
    d.lines = which ? ix.dir[1].lines : ix.dir[0].lines;
    d.sa = which ? ix.dir[1].sa : ix.dir[0].sa;
#pragma unroll
    for (int a = 0; a < 4; a++) d.C[a] = which ? ix.dir[1].C[a] : ix.dir[0].C[a];
    d.primary = which ? ix.dir[1].primary : ix.dir[0].primary;
    d.pad = 0;
    d.kt = which ? ix.dir[1].kt : ix.dir[0].kt;
    return d;
}

__device__ __forceinline__ uint32_t line_of(const DevIndex &ix, uint32_t i) {
    return (uint32_t)__umul64hi((uint64_t)i, ix.magic);
}

// Rank-line format as a template tag: 8, 16 or 32 = lines of that many
// uint32 words with counts then bit planes; LW_SUB = 64-byte sub-counted
// lines of 160 rows (counts of C, G, T, then per base the counts at the
// first four 32-row boundaries as bytes, then the bit planes).
constexpr int LW_SUB = 17;
// LW_SUB128 = 128-byte sub-counted lines of 384 rows: counts of C, G, T
// before the line (words 0-2); the counts within the line before rows 64,
// 128, 192, 256 and 320, each as C | G << 9 | T << 18 (words 3-7); the bit
// planes (words 8-31), per 32 rows a word of high bits then one of low bits,
// so the four plane words of a 64-row group are one aligned 16-byte load.
// A rank query reads the line's first 16 bytes, its boundary word and one
// group: an L2 fill brings 128 bytes the query can use.
constexpr int LW_SUB128 = 33;
template <int LW> constexpr int line_words() { return LW == LW_SUB ? 16 : (LW == LW_SUB128 ? 32 : LW); }
constexpr uint32_t SUB128_ROWS = 384;

// The four (k, l) pairs of a string's one-base extensions, read from the
// short-string table as two 16-byte words (p: A and C, q: G and T), in the
// rank-query form the search consumes: o1[a] = k_a - C[a],
// o2[a] = l_a + 1 - C[a].
__device__ __forceinline__ void kt_pick(const DevDir &d, uint4 p, uint4 q, uint32_t o1[4], uint32_t o2[4]) {
    o1[0] = p.x - d.C[0];
    o2[0] = p.y + 1 - d.C[0];
    o1[1] = p.z - d.C[1];
    o2[1] = p.w + 1 - d.C[1];
    o1[2] = q.x - d.C[2];
    o2[2] = q.y + 1 - d.C[2];
    o1[3] = q.z - d.C[3];
    o2[3] = q.w + 1 - d.C[3];
}
// entry of the first child of the string of d < 15 bases with code c:
// level d + 1 starts at (4^(d+1) + 8) / 3, and every entry below level 16
// has an index under 2^32
__device__ __forceinline__ uint32_t kt_children(int d, uint32_t c) {
    return ((1u << (2 * d + 2)) + 8u) / 3u + 4u * c;
}

// Occ of all four bases at row i of a sub-counted line: the counts before
// the line, the count at the boundary of row i's 32-row group, and a count
// of bits in that one group.  A is what the rows leave ($ excluded).
__device__ __forceinline__ void occ4_sub(const DevIndex &ix, const DevDir &d, uint32_t i, uint32_t o[4]) {
    const uint32_t line = line_of(ix, i);
    const uint32_t r = i - line * 160u, g = r >> 5;
    const uint32_t *L = d.lines + (size_t)line * 16;
    const uint4 h = *reinterpret_cast<const uint4 *>(L);       // C, G, T before the line; C boundaries
    const uint2 b = *reinterpret_cast<const uint2 *>(L + 4);   // G, T boundaries
    const uint2 w = *reinterpret_cast<const uint2 *>(L + 6 + 2 * g);
    const uint32_t m = (1u << (r & 31)) - 1u;
    uint32_t cC = __popc(~w.x & w.y & m), cG = __popc(w.x & ~w.y & m), cT = __popc(w.x & w.y & m);
    if (g) {
        const uint32_t sh = 8 * (g - 1);
        cC += (h.w >> sh) & 255u;
        cG += (b.x >> sh) & 255u;
        cT += (b.y >> sh) & 255u;
    }
    o[1] = h.x + cC;
    o[2] = h.y + cG;
    o[3] = h.z + cT;
    o[0] = i - o[1] - o[2] - o[3] - (i > d.primary ? 1u : 0u);
}

// Occ at rows i1 and i2 of sub-counted lines, for the search loop, where
// line requests cost more than bit counting: whole lines are fetched (four
// 16-byte loads, once when both rows fall in one line) and each row's
// group is picked from registers.
__device__ __forceinline__ void occ4_sub_pair(const DevIndex &ix, const DevDir &d, uint32_t i1, uint32_t i2,
                                              uint32_t o1[4], uint32_t o2[4]) {
    const uint32_t l1 = line_of(ix, i1), l2 = line_of(ix, i2);
    const uint4 *L1 = reinterpret_cast<const uint4 *>(d.lines) + (size_t)l1 * 4;
    const uint4 *L2 = reinterpret_cast<const uint4 *>(d.lines) + (size_t)l2 * 4;
    uint4 a[4], b[4];
#pragma unroll
    for (int q = 0; q < 4; q++) a[q] = L1[q];
    if (l1 != l2) {
#pragma unroll
        for (int q = 0; q < 4; q++) b[q] = L2[q];
    } else {
#pragma unroll
        for (int q = 0; q < 4; q++) b[q] = a[q];
    }
    auto count = [&](const uint4(&v)[4], uint32_t i, uint32_t line, uint32_t o[4]) {
        const uint32_t r = i - line * 160u, g = r >> 5;
        // the group's two plane words: words 6 + 2 g and 7 + 2 g of the line
        const uint32_t hi = g == 0 ? v[1].z : g == 1 ? v[2].x : g == 2 ? v[2].z : g == 3 ? v[3].x : v[3].z;
        const uint32_t lo = g == 0 ? v[1].w : g == 1 ? v[2].y : g == 2 ? v[2].w : g == 3 ? v[3].y : v[3].w;
        const uint32_t m = (1u << (r & 31)) - 1u;
        uint32_t cC = __popc(~hi & lo & m), cG = __popc(hi & ~lo & m), cT = __popc(hi & lo & m);
        if (g) {
            const uint32_t sh = 8 * (g - 1);
            cC += (v[0].w >> sh) & 255u;
            cG += (v[1].x >> sh) & 255u;
            cT += (v[1].y >> sh) & 255u;
        }
        o[1] = v[0].x + cC;
        o[2] = v[0].y + cG;
        o[3] = v[0].z + cT;
        o[0] = i - o[1] - o[2] - o[3] - (i > d.primary ? 1u : 0u);
    };
    count(a, i1, l1, o1);
    count(b, i2, l2, o2);
}

// Occ of all four bases at row i from the pieces of its 128-byte
// sub-counted line: h = words 0-3 (C, G, T before the line, boundary word
// of row 64), b = words 4-7 (boundary words of rows 128 .. 320; read only
// when the row's group needs one of them), p = the four plane words of the
// row's 64-row group; r = i's row within the line.
__device__ __forceinline__ void sub128_count(uint4 h, uint4 b, uint4 p, uint32_t r, uint32_t i, uint32_t primary,
                                             uint32_t o[4]) {
    const uint32_t g = r >> 6, t = r & 63;
    const uint32_t m0 = t >= 32 ? 0xffffffffu : (1u << t) - 1u;
    const uint32_t m1 = t > 32 ? (1u << (t - 32)) - 1u : 0u;
    // high plane set: G or T; low plane set: C or T; both: T
    const uint32_t cT = __popc(p.x & p.y & m0) + __popc(p.z & p.w & m1);
    const uint32_t cH = __popc(p.x & m0) + __popc(p.z & m1);
    const uint32_t cL = __popc(p.y & m0) + __popc(p.w & m1);
    const uint32_t bw = g == 0 ? 0u : (g == 1 ? h.w : (g == 2 ? b.x : (g == 3 ? b.y : (g == 4 ? b.z : b.w))));
    o[1] = h.x + (bw & 511u) + cL - cT;
    o[2] = h.y + ((bw >> 9) & 511u) + cH - cT;
    o[3] = h.z + (bw >> 18) + cT;
    o[0] = i - o[1] - o[2] - o[3] - (i > primary ? 1u : 0u);
}

// The same count from the counts before the line (C, G, T), the row's
// boundary word (0 for the first 64 rows) and its group's plane words.
__device__ __forceinline__ void sub128_count3(uint3 h, uint32_t bw, uint4 p, uint32_t r, uint32_t i,
                                              uint32_t primary, uint32_t o[4]) {
    const uint32_t t = r & 63;
    const uint32_t m0 = t >= 32 ? 0xffffffffu : (1u << t) - 1u;
    const uint32_t m1 = t > 32 ? (1u << (t - 32)) - 1u : 0u;
    const uint32_t cT = __popc(p.x & p.y & m0) + __popc(p.z & p.w & m1);
    const uint32_t cH = __popc(p.x & m0) + __popc(p.z & m1);
    const uint32_t cL = __popc(p.y & m0) + __popc(p.w & m1);
    o[1] = h.x + (bw & 511u) + cL - cT;
    o[2] = h.y + ((bw >> 9) & 511u) + cH - cT;
    o[3] = h.z + (bw >> 18) + cT;
    o[0] = i - o[1] - o[2] - o[3] - (i > primary ? 1u : 0u);
}

// One row's pieces of its line: counts, boundary word, group planes.
__device__ __forceinline__ void sub128_load(const uint32_t *L, uint32_t r, uint3 &h, uint32_t &bw, uint4 &p) {
    h = *reinterpret_cast<const uint3 *>(L);
    const uint32_t g = r >> 6;
    bw = 0;
    if (g) bw = L[2 + g];
    p = reinterpret_cast<const uint4 *>(L)[2 + g];
}

__device__ __forceinline__ void occ4_sub128(const DevIndex &ix, const DevDir &d, uint32_t i, uint32_t o[4]) {
#if BWFM_GENE_SUBLOAD == 1
    {
        const uint32_t line = line_of(ix, i);
        const uint32_t r = i - line * SUB128_ROWS;
        uint3 h;
        uint32_t bw;
        uint4 p;
        sub128_load(d.lines + (size_t)line * 32, r, h, bw, p);
        sub128_count3(h, bw, p, r, i, d.primary, o);
        return;
    }
#endif
    const uint32_t line = line_of(ix, i);
    const uint32_t r = i - line * SUB128_ROWS;
    const uint4 *L = reinterpret_cast<const uint4 *>(d.lines) + (size_t)line * 8;
    const uint4 h = L[0];
    uint4 b = make_uint4(0, 0, 0, 0);
    if (BWFM_GENE_SUBHDR == 1 || r >= 128) b = L[1];
    const uint4 p = L[2 + (r >> 6)];
    sub128_count(h, b, p, r, i, d.primary, o);
}

// Occ at rows i1 and i2 (k and l + 1 of an interval) on 128-byte
// sub-counted lines: the shared parts of one line are read once.
__device__ __forceinline__ void occ4_sub128_pair(const DevIndex &ix, const DevDir &d, uint32_t i1, uint32_t i2,
                                                 uint32_t o1[4], uint32_t o2[4]) {
#if BWFM_GENE_SUBLOAD == 1
    {
        const uint32_t l1 = line_of(ix, i1), l2 = line_of(ix, i2);
        const uint32_t r1 = i1 - l1 * SUB128_ROWS, r2 = i2 - l2 * SUB128_ROWS;
        uint3 h1, h2;
        uint32_t b1, b2;
        uint4 p1, p2;
        sub128_load(d.lines + (size_t)l1 * 32, r1, h1, b1, p1);
        if (l1 != l2 || (r1 >> 6) != (r2 >> 6)) {
            sub128_load(d.lines + (size_t)l2 * 32, r2, h2, b2, p2);
        } else {
            h2 = h1;
            b2 = b1;
            p2 = p1;
        }
        sub128_count3(h1, b1, p1, r1, i1, d.primary, o1);
        sub128_count3(h2, b2, p2, r2, i2, d.primary, o2);
        return;
    }
#endif
    const uint32_t l1 = line_of(ix, i1), l2 = line_of(ix, i2);
    const uint32_t r1 = i1 - l1 * SUB128_ROWS, r2 = i2 - l2 * SUB128_ROWS;
    const uint4 *L1 = reinterpret_cast<const uint4 *>(d.lines) + (size_t)l1 * 8;
    const uint4 *L2 = reinterpret_cast<const uint4 *>(d.lines) + (size_t)l2 * 8;
    const bool same = l1 == l2;
    const uint4 h1 = L1[0];
    uint4 b1 = make_uint4(0, 0, 0, 0), h2 = h1, b2 = b1;
    if (BWFM_GENE_SUBHDR == 1 || r1 >= 128 || (same && r2 >= 128)) b1 = L1[1];
    const uint4 p1 = L1[2 + (r1 >> 6)];
    if (!same) {
        h2 = L2[0];
        if (BWFM_GENE_SUBHDR == 1 || r2 >= 128) b2 = L2[1];
    } else {
        b2 = b1;
    }
    uint4 p2 = p1;
    if (!same || (r1 >> 6) != (r2 >> 6)) p2 = L2[2 + (r2 >> 6)];
    sub128_count(h1, b1, p1, r1, i1, d.primary, o1);
    sub128_count(h2, b2, p2, r2, i2, d.primary, o2);
}

// mask of the first t rows of a 32-row group (t may be <= 0 or >= 32)
__device__ __forceinline__ uint32_t rows_mask(int t) {
#if BWFM_GENE_ROWMASK == 1
    // the low t bits of a 64-bit all-ones word shifted right by 64 - t,
    // clamped to [0, 32] rows
    const int c = t < 0 ? 0 : (t > 32 ? 32 : t);
    return (uint32_t)(c == 0 ? 0ull : (~0ull >> (64 - c)));
#else
    return t >= 32 ? 0xffffffffu : (t <= 0 ? 0u : ((1u << t) - 1u));
#endif
}

// Occ(a, i) for all four bases (i <= n + 1).  Per 32-row group: one word of
// high bits (h) and one of low bits (l); T = h & l, G = h & ~l, C = ~h & l.
template <int LW>
__device__ __forceinline__ void occ4(const DevIndex &ix, const DevDir &d, uint32_t i, uint32_t o[4]) {
    if constexpr (LW == LW_SUB) {
        occ4_sub(ix, d, i, o);
        return;
    }
    if constexpr (LW == LW_SUB128) {
        occ4_sub128(ix, d, i, o);
        return;
    }
    uint32_t line = line_of(ix, i);
    int r = (int)(i - line * ix.bpl);
    const uint4 *L = reinterpret_cast<const uint4 *>(d.lines) + (size_t)line * (LW / 4);
    uint4 h = L[0];
    uint32_t cC = 0, cG = 0, cT = 0;
#pragma unroll
    for (int q = 0; q < LW / 4 - 1; q++) {
        uint4 v = L[1 + q];
        uint32_t m0 = rows_mask(r - q * 64), m1 = rows_mask(r - q * 64 - 32);
        cT += __popc(v.x & v.y & m0) + __popc(v.z & v.w & m1);
        cG += __popc(v.x & ~v.y & m0) + __popc(v.z & ~v.w & m1);
        cC += __popc(~v.x & v.y & m0) + __popc(~v.z & v.w & m1);
    }
    uint32_t cA = (uint32_t)r - cC - cG - cT;
    o[0] = h.x + cA - (i > d.primary ? 1u : 0u);
    o[1] = h.y + cC;
    o[2] = h.z + cG;
    o[3] = h.w + cT;
}

// Occ(., i1) and Occ(., i2) on one direction, as occ4 twice, except that a
// lane whose two rows fall in one rank line (k and l + 1 of a narrow
// interval: two thirds of the expansions on the benchmark) fetches that
// line once.  The search is bound by line requests more than by their
// bytes, so the skipped request is the saving.
template <int LW>
__device__ __forceinline__ void occ4_pair(const DevIndex &ix, const DevDir &d, uint32_t i1, uint32_t i2, uint32_t o1[4],
                                          uint32_t o2[4]) {
    if constexpr (LW == LW_SUB) {
        occ4_sub_pair(ix, d, i1, i2, o1, o2);
        return;
    }
    if constexpr (LW == LW_SUB128) {
        occ4_sub128_pair(ix, d, i1, i2, o1, o2);
        return;
    }
    const uint32_t l1 = line_of(ix, i1), l2 = line_of(ix, i2);
    const uint4 *L1 = reinterpret_cast<const uint4 *>(d.lines) + (size_t)l1 * (LW / 4);
    const uint4 *L2 = reinterpret_cast<const uint4 *>(d.lines) + (size_t)l2 * (LW / 4);
    const bool same = BWFM_GENE_PAIRLINE == 0 && l1 == l2;
    uint4 a[LW / 4], b[LW / 4];
#pragma unroll
    for (int q = 0; q < LW / 4; q++) a[q] = L1[q];
    if (!same) {
#pragma unroll
        for (int q = 0; q < LW / 4; q++) b[q] = L2[q];
    } else {
#pragma unroll
        for (int q = 0; q < LW / 4; q++) b[q] = a[q];
    }
    const uint4(&A)[LW / 4] = a;
    const uint4(&B)[LW / 4] = b;
    auto count = [&](const uint4(&v)[LW / 4], uint32_t i, uint32_t line, uint32_t o[4]) {
        const int r = (int)(i - line * ix.bpl);
        uint32_t cC = 0, cG = 0, cT = 0;
#pragma unroll
        for (int q = 0; q < LW / 4 - 1; q++) {
            const uint4 w = v[1 + q];
            const uint32_t m0 = rows_mask(r - q * 64), m1 = rows_mask(r - q * 64 - 32);
            cT += __popc(w.x & w.y & m0) + __popc(w.z & w.w & m1);
            cG += __popc(w.x & ~w.y & m0) + __popc(w.z & ~w.w & m1);
            cC += __popc(~w.x & w.y & m0) + __popc(~w.z & w.w & m1);
        }
        const uint32_t cA = (uint32_t)r - cC - cG - cT;
        o[0] = v[0].x + cA - (i > d.primary ? 1u : 0u);
        o[1] = v[0].y + cC;
        o[2] = v[0].z + cG;
        o[3] = v[0].w + cT;
    };
    count(A, i1, l1, o1);
    count(B, i2, l2, o2);
}

// Occ(a, i) for one base a.
template <int LW>
__device__ __forceinline__ uint32_t occ1(const DevIndex &ix, const DevDir &d, int a, uint32_t i) {
    if constexpr (LW == LW_SUB || LW == LW_SUB128) {
        uint32_t o[4];
        occ4<LW>(ix, d, i, o);
        return sel4(o, a);
    }
    uint32_t line = line_of(ix, i);
    int r = (int)(i - line * ix.bpl);
    const uint4 *L = reinterpret_cast<const uint4 *>(d.lines) + (size_t)line * (LW / 4);
    uint4 h = L[0];
    // rows of base a have high bit (a >> 1) and low bit (a & 1)
    const uint32_t fh = (a & 2) ? 0u : 0xffffffffu, fl = (a & 1) ? 0u : 0xffffffffu;
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < LW / 4 - 1; q++) {
        uint4 v = L[1 + q];
        c += __popc((v.x ^ fh) & (v.y ^ fl) & rows_mask(r - q * 64));
        c += __popc((v.z ^ fh) & (v.w ^ fl) & rows_mask(r - q * 64 - 32));
    }
    uint32_t base = a == 0 ? h.x : (a == 1 ? h.y : (a == 2 ? h.z : h.w));
    return base + c - ((a == 0 && i > d.primary) ? 1u : 0u);
}

// BWT symbol at row j (j != primary) and Occ(that symbol, j): one line.
template <int LW>
__device__ __forceinline__ uint32_t lf_step(const DevIndex &ix, const DevDir &d, uint32_t j) {
    if constexpr (LW == LW_SUB128) {
        const uint32_t line = line_of(ix, j);
        const uint32_t r = j - line * SUB128_ROWS;
        const uint4 *L = reinterpret_cast<const uint4 *>(d.lines) + (size_t)line * 8;
        const uint4 h = L[0];
        uint4 b = make_uint4(0, 0, 0, 0);
        if (r >= 128) b = L[1];
        const uint4 p = L[2 + (r >> 6)];
        const uint32_t hi = (r & 32) ? p.z : p.x, lo = (r & 32) ? p.w : p.y, s = r & 31;
        const int a = (int)((((hi >> s) & 1u) << 1) | ((lo >> s) & 1u));
        uint32_t o[4];
        sub128_count(h, b, p, r, j, d.primary, o);
        return sel4(d.C, a) + sel4(o, a);
    }
    uint32_t line = line_of(ix, j);
    uint32_t r = j - line * ix.bpl;
    const uint32_t *L = d.lines + (size_t)line * line_words<LW>();
    constexpr int po = LW == LW_SUB ? 6 : 4;  // first word of the bit planes
    int a = (int)((((L[po + 2 * (r >> 5)] >> (r & 31)) & 1) << 1) | ((L[po + 1 + 2 * (r >> 5)] >> (r & 31)) & 1));
    return sel4(d.C, a) + occ1<LW>(ix, d, a, j);
}

// ------------------------------------------------------------------ search state

// Search states are packed in 16 bytes: x = k (or, while |X| is below the
// index's short-string levels, the code of X: see state_k), y = l,
// z = (i + 1) | gap state << 10 | n_mm << 12 | n_gapo << 16 | n_gape << 20 | seed diffs << 24,
// w = score | |X| << 10 | lb << 20, where lb = score + minc * D[i] is the
// state's lower bound on its final score, fixed once the D-array is built.
// Every field fits: diffs <= 15, score <= 15 * 63, |X| <= 512 + 15.
__device__ __forceinline__ int entry_lb(uint4 v) { return (int)(v.w >> 20); }

// hit record, same bytes as bwfm_hit
__device__ __forceinline__ uint4 make_hit(int strand, uint32_t k, uint32_t l, int len, int score, int nmm, int ngo,
                                          int nge) {
    return make_uint4(k, l, (uint32_t)len | ((uint32_t)score << 16),
                      (uint32_t)strand | ((uint32_t)nmm << 8) | ((uint32_t)ngo << 16) | ((uint32_t)nge << 24));
}
__device__ __forceinline__ int h_strand(uint4 h) { return h.w & 255; }
__device__ __forceinline__ int h_score(uint4 h) { return h.z >> 16; }
__device__ __forceinline__ int h_len(uint4 h) { return h.z & 0xffff; }
__device__ __forceinline__ int h_nmm(uint4 h) { return (h.w >> 8) & 255; }
__device__ __forceinline__ int h_ngo(uint4 h) { return (h.w >> 16) & 255; }
__device__ __forceinline__ int h_nge(uint4 h) { return (h.w >> 24) & 255; }
__device__ __forceinline__ int h_diffs(uint4 h) { return h_nmm(h) + h_ngo(h) + h_nge(h); }

// (score, diffs, n_gapo, n_mm) of a is smaller than b's
__device__ __forceinline__ bool better(uint4 a, uint4 b) {
    if (h_score(a) != h_score(b)) return h_score(a) < h_score(b);
    if (h_diffs(a) != h_diffs(b)) return h_diffs(a) < h_diffs(b);
    if (h_ngo(a) != h_ngo(b)) return h_ngo(a) < h_ngo(b);
    return h_nmm(a) < h_nmm(b);
}

// report order (score, strand, k, len)
__device__ __forceinline__ bool before(uint4 a, uint4 b) {
    if (h_score(a) != h_score(b)) return h_score(a) < h_score(b);
    if (h_strand(a) != h_strand(b)) return h_strand(a) < h_strand(b);
    if (a.x != b.x) return a.x < b.x;
    return h_len(a) < h_len(b);
}

struct LaneCtx {
    uint4 *stack, *cand;
    uint8_t *pd;  // LDS, per pattern position i: base code | D[i] << 3
    uint32_t sstride, cstride, stack_cap, cand_cap;
    uint32_t sp, sbase;  // stack entries [sbase, sp) are this lane's pending states
    uint32_t ncand;
    int best;
    uint32_t expand;
};

extern __shared__ __align__(16) uint8_t lds_bytes[];

__device__ __forceinline__ void init_ctx(LaneCtx &c, const LaneBufs &B, uint32_t lane) {
    c.stack = B.stack + (size_t)lane * B.stack_lane_step;
    c.cand = B.cand + (size_t)lane * B.cand_lane_step;
    c.pd = lds_bytes + (size_t)threadIdx.x * B.lds_stride;
    c.sstride = B.stack_stride;
    c.cstride = B.cand_stride;
    c.stack_cap = B.stack_cap;
    c.cand_cap = B.cand_cap;
    c.sp = 0;
    c.sbase = 0;
    c.ncand = 0;
    c.best = INF_SCORE;
    c.expand = 0;
}

__device__ __forceinline__ int pd_base(const LaneCtx &c, int i) { return c.pd[i] & 7; }
__device__ __forceinline__ int pd_d(const LaneCtx &c, int i) { return i >= 0 ? (c.pd[i] >> 3) : 0; }

enum { R_OK = 0, R_STACK = 1, R_CAND = 2 };

// Insert a hit: merge with an equal (strand, k, len), else append.  In the
// first pass a full buffer is first cleared of hits above best + s_mm.
__device__ int record(LaneCtx &c, const Params &P, uint4 h, int phase) {
    if (phase == PH_BEST) return R_OK;
    for (uint32_t j = 0; j < c.ncand; j++) {
        uint4 o = c.cand[(size_t)j * c.cstride];
        if (h_strand(o) == h_strand(h) && o.x == h.x && h_len(o) == h_len(h)) {
            if (better(h, o)) c.cand[(size_t)j * c.cstride] = h;
            return R_OK;
        }
    }
    if (c.ncand == c.cand_cap && phase == PH_FAST && P.mode == BWFM_MODE_BEST) {
        uint32_t w = 0;
        for (uint32_t j = 0; j < c.ncand; j++) {
            uint4 o = c.cand[(size_t)j * c.cstride];
            if (h_score(o) <= c.best + P.s_mm) c.cand[(size_t)(w++) * c.cstride] = o;
        }
        c.ncand = w;
    }
    if (c.ncand == c.cand_cap) return R_CAND;
    c.cand[(size_t)(c.ncand++) * c.cstride] = h;
    return R_OK;
}

// pattern base w[i] of the strand: strand + reads the read backwards,
// strand - reads its complement backwards
__device__ __forceinline__ int pat(const uint8_t *W, int m, int strand, int i) {
    int b = W[m - 1 - i];
    return (strand == 0 || b > 3) ? b : 3 - b;
}

// Copy read W (m bases) into an LDS row reversed, row[i] = W[m - 1 - i]:
// the strand + pattern, whose D-array scan then rewrites each byte in place
// as base | D << 3 (strand -: the complement of the same low bits).  Whole
// aligned dwords are loaded 8 at a time, so a read costs a few memory round
// trips instead of one per D-array step; only dwords holding read bases are
// touched.
__device__ __forceinline__ void stage_read(uint8_t *row, const uint8_t *W, int m) {
    const uint32_t *A = reinterpret_cast<const uint32_t *>(reinterpret_cast<uintptr_t>(W) & ~uintptr_t(3));
    const int off = (int)(reinterpret_cast<uintptr_t>(W) & 3);
    const int ndw = (off + m + 3) >> 2;
    for (int k0 = 0; k0 < ndw; k0 += 8) {
        uint32_t v[8];
#pragma unroll
        for (int j = 0; j < 8; j++) v[j] = k0 + j < ndw ? A[k0 + j] : 0u;
#pragma unroll
        for (int j = 0; j < 8; j++)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int i = 4 * (k0 + j) + q - off;
                if (i >= 0 && i < m) row[m - 1 - i] = (uint8_t)(v[j] >> (8 * q));
            }
    }
}

// seed window of the strand pattern: the read's 5' end, consumed first
struct Seed {
    int sl, lo, hi;
};
__device__ __forceinline__ Seed seed_of(const Params &P, int m) {
    Seed s;
    s.sl = P.seed_len > 0 ? (P.seed_len < m ? P.seed_len : m) : 0;
    s.lo = m - s.sl;
    s.hi = s.sl ? m : 0;
    return s;
}

// fields of a packed state (see pack)
__device__ __forceinline__ int s_i(uint4 s) { return (int)(s.z & 1023) - 1; }
__device__ __forceinline__ int s_gs(uint4 s) { return (s.z >> 10) & 3; }
__device__ __forceinline__ int s_nmm(uint4 s) { return (s.z >> 12) & 15; }
__device__ __forceinline__ int s_ngo(uint4 s) { return (s.z >> 16) & 15; }
__device__ __forceinline__ int s_nge(uint4 s) { return (s.z >> 20) & 15; }
__device__ __forceinline__ int s_sd(uint4 s) { return (s.z >> 24) & 15; }
__device__ __forceinline__ int s_score(uint4 s) { return s.w & 1023; }
__device__ __forceinline__ int s_len(uint4 s) { return (s.w >> 10) & 1023; }

// k of a state: x itself, or, for a state whose X is shorter than the
// short-string levels (x holds the code of X), k from X's table entry on
// the strand's search index.  Only completed hits need it.
__device__ __forceinline__ uint32_t state_k(const DevIndex &ix, int strand, uint4 s) {
    const int len = s_len(s);
    if (len >= (int)ix.kt_levels) return s.x;
    const uint32_t *kt = strand == 0 ? ix.dir[1].kt : ix.dir[0].kt;
    return kt[2 * (kt_level_start(len) + s.x)];
}

// the empty string's interval, nothing consumed, lower bound minc * D[m - 1]
__device__ __forceinline__ uint4 root_state(const DevIndex &ix, int m, int lb) {
    return make_uint4(0u, ix.n, (uint32_t)m, (uint32_t)lb << 20);
}

// Advance the search until the current state needs expanding: pop, drop
// states whose stored lower bound exceeds the BEST bound, record completed
// hits.  At most max_pops entries are popped.  Returns 1 when cur must be
// expanded, 0 when the lane's part of the strand's search is over, 2 when
// the pop limit was reached first, 3 when cur is a completed hit left for
// the caller to record (only with defer), or -R_CAND when the hit buffer
// overflowed.
template <bool KT = true>
__device__ int resolve(uint4 &cur, bool &valid, int strand, const Params &P, LaneCtx &c, int phase, int max_pops,
                       const DevIndex &ix, bool defer = false) {
    for (int pops = 0;;) {
        const int bound = (P.mode == BWFM_MODE_BEST && c.best != INF_SCORE) ? c.best + P.s_mm : INF_SCORE;
        if (!valid) {
            if (c.sp == c.sbase) return 0;
            if (pops == max_pops) return 2;
            pops++;
            c.sp--;
            cur = c.stack[(size_t)c.sp * c.sstride];
            valid = true;
        }
        if (entry_lb(cur) > bound) {
            valid = false;
            continue;
        }
        if (s_i(cur) < 0) {
            if (defer) return 3;
            const int score = s_score(cur);
            if (score < c.best) c.best = score;
            int rc = record(c, P,
                            make_hit(strand, KT ? state_k(ix, strand, cur) : cur.x, cur.y, s_len(cur), score,
                                     s_nmm(cur), s_ngo(cur), s_nge(cur)),
                            phase);
            if (rc) return -rc;
            valid = false;
            continue;
        }
        return 1;
    }
}

// Children of an expanded state, from the rank counts at k (ok) and l + 1
// (ol) on the search index, built directly in packed form: each differs
// from the parent by a few field increments.  They are taken in reverse of
// the fixed order (match, mismatches by base, insertion, deletions by base);
// the first surviving one becomes cur, the others are pushed with their
// lower bounds.  Returns R_OK or R_STACK.
__device__ int expand_children(uint4 &cur, bool &valid, const uint32_t (&ok)[4], const uint32_t (&ol)[4],
                               const DevDir &sd_, int b, int m, int maxd, int Di, int Dn, const Seed &S,
                               const Params &P, LaneCtx &c, uint32_t K) {
    const int i = s_i(cur), gs = s_gs(cur), ngo = s_ngo(cur), nge = s_nge(cur), sd = s_sd(cur);
    const int score = s_score(cur), len = s_len(cur);
    // x of the children that consume a base: k, or their code while
    // shorter than the short-string levels
    const bool coded = (uint32_t)(len + 1) < K;
    uint32_t kx[4];
#pragma unroll
    for (int a = 0; a < 4; a++) kx[a] = coded ? (cur.x << 2) | (uint32_t)a : sd_.C[a] + ok[a];
    const int diffs = s_nmm(cur) + ngo + nge;
    const int bound = (P.mode == BWFM_MODE_BEST && c.best != INF_SCORE) ? c.best + P.s_mm : INF_SCORE;
    const uint32_t z0 = cur.z & ~(3u << 10);  // gap state cleared
    // room for the at most 8 states pushed below: checked once per
    // expansion.  Entries below sbase were handed to other lanes; sliding
    // the pending ones down makes room when the top of the stack is reached.
    if (c.sp + 8 > c.stack_cap && c.sbase > 0) {
        for (uint32_t j = c.sbase; j < c.sp; j++)
            c.stack[(size_t)(j - c.sbase) * c.sstride] = c.stack[(size_t)j * c.sstride];
        c.sp -= c.sbase;
        c.sbase = 0;
    }
    if (c.sp + 8 > c.stack_cap) {
        valid = false;
        return R_STACK;
    }
    uint4 pend = cur;
    bool have = false;
    const int rc = R_OK;
    auto offer = [&](uint32_t k, uint32_t l, uint32_t z, uint32_t w) {
        if (have) {
            c.stack[(size_t)c.sp * c.sstride] = pend;
            c.sp++;
        }
        pend = make_uint4(k, l, z, w);
        have = true;
    };
    // deletions: reference base a between read bases i and i + 1 (same i)
    {
        const int bd = i + 1;
        const bool ext = gs == GAP_DEL;
        const int nd = diffs + 1, ngo2 = ngo + (ext ? 0 : 1), nge2 = nge + (ext ? 1 : 0);
        const int in = (bd > S.lo && bd < S.hi) ? 1 : 0;
        const int nsc = score + (ext ? P.s_gape : P.s_gapo);
        const int lb = nsc + P.minc * Di;
        if (bd >= P.s1 && bd <= m - P.s1 && nd <= maxd && ngo2 <= P.max_gapo && (P.max_gape < 0 || nge2 <= P.max_gape) &&
            (S.sl == 0 || sd + in <= P.seed_diff) && nd + Di <= maxd && lb <= bound) {
            const uint32_t z = (z0 | ((uint32_t)GAP_DEL << 10)) + (ext ? (1u << 20) : (1u << 16)) + ((uint32_t)in << 24);
            const uint32_t w = (uint32_t)nsc | ((uint32_t)(len + 1) << 10) | ((uint32_t)lb << 20);
#pragma unroll
            for (int a = 3; a >= 0; a--)
                if (ok[a] < ol[a]) offer(kx[a], sd_.C[a] + ol[a] - 1, z, w);
        }
    }
    const int in_i = (i >= S.lo && i < S.hi) ? 1 : 0;
    // insertion: read base w[i] without a reference base (same interval)
    if (i >= P.ies && i < m - P.ies) {
        const bool ext = gs == GAP_INS;
        const int nd = diffs + 1, ngo2 = ngo + (ext ? 0 : 1), nge2 = nge + (ext ? 1 : 0);
        const int nsc = score + (ext ? P.s_gape : P.s_gapo);
        const int lb = nsc + P.minc * Dn;
        if (nd <= maxd && ngo2 <= P.max_gapo && (P.max_gape < 0 || nge2 <= P.max_gape) &&
            (S.sl == 0 || sd + in_i <= P.seed_diff) && nd + Dn <= maxd && lb <= bound) {
            const uint32_t z =
                (z0 | ((uint32_t)GAP_INS << 10)) - 1u + (ext ? (1u << 20) : (1u << 16)) + ((uint32_t)in_i << 24);
            offer(cur.x, cur.y, z, (uint32_t)nsc | ((uint32_t)len << 10) | ((uint32_t)lb << 20));
        }
    }
    // mismatches, then the match (offered last, so it becomes current)
    {
        const int nsc = score + P.s_mm;
        const int lb = nsc + P.minc * Dn;
        if (diffs + 1 <= maxd && (S.sl == 0 || sd + in_i <= P.seed_diff) && diffs + 1 + Dn <= maxd && lb <= bound) {
            const uint32_t z = z0 - 1u + (1u << 12) + ((uint32_t)in_i << 24);
            const uint32_t w = (uint32_t)nsc | ((uint32_t)(len + 1) << 10) | ((uint32_t)lb << 20);
#pragma unroll
            for (int a = 3; a >= 0; a--)
                if (a != b && ok[a] < ol[a]) offer(kx[a], sd_.C[a] + ol[a] - 1, z, w);
        }
        const int lbm = score + P.minc * Dn;
        if (b < 4 && sel4(ok, b) < sel4(ol, b) && diffs + Dn <= maxd && lbm <= bound)
            offer(sel4(kx, b), sel4(sd_.C, b) + sel4(ol, b) - 1, z0 - 1u,
                  (uint32_t)score | ((uint32_t)(len + 1) << 10) | ((uint32_t)lbm << 20));
    }
    if (have) cur = pend;
    valid = have;
    return rc;
}

// D-array of one strand on the other index.  Returns false when the bound
// already exceeds the budget at the root (the strand cannot match).
template <int LW>
__device__ bool build_d(const DevIndex &ix, const DevDir &od, const uint8_t *W, int m, int strand, int maxd,
                        LaneCtx &c) {
    uint32_t k = 0, l = ix.n;
    uint32_t code = 0, len = 0;  // the current segment, while shorter than the short-string levels
    int z = 0;
    for (int i = 0; i < m; i++) {
        int a = pat(W, m, strand, i);
        bool empty = true;
        if (a < 4 && len < ix.kt_levels) {
            const uint2 e = reinterpret_cast<const uint2 *>(od.kt)[kt_children((int)len, code) + a];
            empty = e.x > e.y;
            k = e.x;
            l = e.y;
            code = (code << 2) | (uint32_t)a;
            len++;
        } else if (a < 4) {
            uint32_t ok = occ1<LW>(ix, od, a, k), ol = occ1<LW>(ix, od, a, l + 1);
            empty = ok >= ol;
            k = sel4(od.C, a) + ok;
            l = sel4(od.C, a) + ol - 1;
        }
        if (empty) {
            z++;
            k = 0;
            l = ix.n;
            code = len = 0;
            if (z > maxd) return false;
        }
        c.pd[i] = (uint8_t)(a | (z << 3));
    }
    return true;
}

// Depth-first search of one strand, one lane, start to end.
template <int LW>
__device__ int search_strand(const DevIndex &ix, const DevDir &sd_, const uint8_t *W, int m, int strand, int maxd,
                             const Params &P, LaneCtx &c, int phase) {
    const Seed S = seed_of(P, m);
    uint4 cur = root_state(ix, m, P.minc * pd_d(c, m - 1));
    bool valid = true;
    c.sp = 0;
    for (;;) {
        int rr = resolve(cur, valid, strand, P, c, phase, 0x7fffffff, ix);
        if (rr == 0) return R_OK;
        if (rr < 0) return -rr;
        c.expand++;
        uint32_t ok[4], ol[4];
        if ((uint32_t)s_len(cur) < ix.kt_levels) {
            const uint4 *e = reinterpret_cast<const uint4 *>(sd_.kt + 2 * kt_children(s_len(cur), cur.x));
            kt_pick(sd_, e[0], e[1], ok, ol);
        } else {
            occ4<LW>(ix, sd_, cur.x, ok);
            occ4<LW>(ix, sd_, cur.y + 1, ol);
        }
        const int i = s_i(cur);
        const int b = pd_base(c, i);
        const int Di = pd_d(c, i), Dn = pd_d(c, i - 1);
        int rc = expand_children(cur, valid, ok, ol, sd_, b, m, maxd, Di, Dn, S, P, c, ix.kt_levels);
        if (rc) return rc;
    }
}

// Canonicalise the lane's hit buffer: tiers, c1/c2, the max_hits rule, the
// report order.  Returns the number of reported hits (at the front of the
// buffer); sets status, c1, c2.
__device__ uint32_t finish(LaneCtx &c, const Params &P, uint8_t &status, uint32_t &c1o, uint32_t &c2o) {
    status = 0;
    c1o = c2o = 0;
    if (c.ncand == 0) return 0;
    const int S = c.best;
    uint32_t n = 0;
    uint64_t c1 = 0, c2 = 0;
    for (uint32_t j = 0; j < c.ncand; j++) {
        uint4 h = c.cand[(size_t)j * c.cstride];
        int sc = h_score(h);
        if (P.mode == BWFM_MODE_ALL || sc <= S + P.s_mm) c.cand[(size_t)(n++) * c.cstride] = h;
        uint64_t w = (uint64_t)h.y - h.x + 1;
        if (sc == S) c1 += w;
        else if (sc <= S + P.s_mm) c2 += w;
    }
    if (n > P.max_hits) {
        status = BWFM_ST_OVERFLOW;
        c1o = c2o = 0xffffffffu;
        return 0;
    }
    c1o = c1 > 0xffffffffULL ? 0xffffffffu : (uint32_t)c1;
    c2o = c2 > 0xffffffffULL ? 0xffffffffu : (uint32_t)c2;
    const bool keep2 = c1 <= (uint64_t)P.max_best;
    uint32_t r = 0;
    for (uint32_t j = 0; j < n; j++) {
        uint4 h = c.cand[(size_t)j * c.cstride];
        if (P.mode == BWFM_MODE_ALL || h_score(h) == S || keep2) c.cand[(size_t)(r++) * c.cstride] = h;
    }
    for (uint32_t j = 1; j < r; j++) {  // insertion sort by (score, strand, k, len)
        uint4 v = c.cand[(size_t)j * c.cstride];
        uint32_t q = j;
        while (q > 0) {
            uint4 u = c.cand[(size_t)(q - 1) * c.cstride];
            if (!before(v, u)) break;
            c.cand[(size_t)q * c.cstride] = u;
            q--;
        }
        c.cand[(size_t)q * c.cstride] = v;
    }
    status = r ? BWFM_ST_HIT : 0;
    return r;
}

template <int LW>
__device__ int align_read(const DevIndex &ix, const uint8_t *W, int m, int maxd, const Params &P, LaneCtx &c,
                          int phase) {
    c.ncand = 0;
    for (int strand = 0; strand < 2; strand++) {
        const DevDir sdir = pick_dir(ix, strand == 0 ? 1 : 0);
        const DevDir odir = pick_dir(ix, strand == 0 ? 0 : 1);
        if (!build_d<LW>(ix, odir, W, m, strand, maxd, c)) continue;
        int rc = search_strand<LW>(ix, sdir, W, m, strand, maxd, P, c, phase);
        if (rc) return rc;
    }
    return R_OK;
}

// Per-read outputs shared by the kernels.
struct ReadOut {
    uint32_t *n_rep, *c1, *c2;
    uint8_t *status;
    uint32_t *slow_list, *n_slow;
    uint4 *stage;                    // reported hits, a block per read
    unsigned long long *stage_used;  // staging slots taken
    uint64_t stage_cap;
    uint64_t *stage_off;             // per read: first staging slot
    uint32_t *expand;                // per read work counter, or NULL
    unsigned long long *work;        // or NULL: [0] wave iterations, [1] lane iterations with a read,
                                     // [2] lane iterations that issued a rank query
};

__device__ __forceinline__ void send_to_second_pass(const ReadOut &O, uint32_t r) {
    O.status[r] = ST_RESEARCH;
    O.n_rep[r] = 0;
    O.slow_list[atomicAdd(O.n_slow, 1u)] = r;
}

// Move a read's nr reported hits (the front of its hit buffer) to the
// staging arena.  The arena holds as many hits as the caller's output, so
// running out of it means the output is too small: the count is kept (the
// offsets scan then reports what is needed) and nothing is copied.
__device__ void stage_hits(const LaneCtx &c, const ReadOut &O, uint32_t r, uint32_t nr) {
    if (!nr) return;
    const unsigned long long off = atomicAdd(O.stage_used, (unsigned long long)nr);
    if (off + nr > O.stage_cap) return;
    for (uint32_t j = 0; j < nr; j++) O.stage[off + j] = c.cand[(size_t)j * c.cstride];
    O.stage_off[r] = off;
}

// Canonicalise a finished read and move its reported hits to the staging
// arena.
__device__ void publish(LaneCtx &c, const Params &P, const ReadOut &O, uint32_t r, uint8_t extra = 0) {
    uint8_t st;
    uint32_t a, b;
    uint32_t nr = finish(c, P, st, a, b);
    if (O.expand) O.expand[r] = c.expand;
    stage_hits(c, O, r, nr);
    O.n_rep[r] = nr;
    O.status[r] = st | extra;
    O.c1[r] = a;
    O.c2[r] = b;
}

// validity of read r: 0 = search it, 1 = done (empty or invalid, outputs written)
__device__ __forceinline__ int check_read(const ReadsView &rd, const Params &P, const ReadOut &O, uint32_t r, int &m,
                                          int &maxd, uint64_t &o0) {
    uint64_t len;
    bool bad;
    read_span(rd, r, o0, len, bad);
    m = (int)len;
    maxd = rd.maxd ? rd.maxd[r] : P.max_diff;
    O.n_rep[r] = 0;
    O.c1[r] = O.c2[r] = 0;
    if (O.expand) O.expand[r] = 0;
    if (bad || len > rd.max_len || len > BWFM_MAX_READ || maxd > BWFM_MAX_DIFF) {
        O.status[r] = BWFM_ST_INVALID;
        return 1;
    }
    if (m == 0) {
        O.status[r] = 0;
        return 1;
    }
    return 0;
}

// Copy n dwords, the loads of eight issued before their stores: through
// generic pointers the compiler must assume a store may alias the next
// load, so a plain loop waits one memory round trip per dword.
__device__ __forceinline__ void copy_dwords(uint32_t *dst, const uint32_t *src, int n) {
    for (int k0 = 0; k0 < n; k0 += 8) {
        uint32_t v[8];
#pragma unroll
        for (int j = 0; j < 8; j++) v[j] = k0 + j < n ? src[k0 + j] : 0u;
#pragma unroll
        for (int j = 0; j < 8; j++)
            if (k0 + j < n) dst[k0 + j] = v[j];
    }
}

// ------------------------------------------------------------------ split searches

// Batched form: a read whose search outgrows a budget of expansions is
// split.  Its pending states become tasks that any lane of the grid may
// take, in rounds of one launch each, so that the largest trees of a batch
// are searched by the whole device rather than by one lane or one wave.
// The read's slot holds what a task needs (the strand's pattern and D-array
// row, the read's length and budget, the best score found so far) and
// collects the hits of every part; after the rounds each slot's read is
// canonicalised like any other, duplicates merged first.  The reported hits
// do not depend on how the tree was cut: each part prunes with a bound that
// is never below the final one, so every hit within the final bound is
// found by the part that holds it.
constexpr int SPLIT_ROUNDS = 8;               // task rounds; the last one runs every task to its end
constexpr uint32_t TASK_EMPTY = 0xffffffffu;  // a reserved task entry left unused
// hits a slot collects: those of the read's first-pass lane (at most
// FAST_CAND), then at most as many again from its tasks
constexpr uint32_t SLOT_HITS = 2 * FAST_CAND;
// control words: [0] slots taken; [1 + g] task entries reserved in
// generation g (0: by the first pass, k: by round k); [2 + SPLIT_ROUNDS + g]
// entries of generation g taken by round g + 1
constexpr uint32_t SPLIT_CTL = 2 * (SPLIT_ROUNDS + 1) + 2;

struct SplitBufs {
    uint32_t *slot_read;    // the slot's read
    uint32_t *slot_meta;    // m | budget << 10
    int *slot_best;         // best score found by any part
    uint32_t *slot_nhit;    // hits delivered (above SLOT_HITS: the slot failed)
    uint32_t *slot_fail;    // nonzero: the read goes to the second pass
    uint32_t *slot_exp;     // states expanded by the read's parts
    uint32_t *slot_owner;   // the first-pass lane that owns the read (its hit buffer)
    uint32_t *slot_own;     // hits in that buffer when the first pass finished the read
    int *slot_obest;        // and its best score then
    uint8_t *slot_rows;     // per slot and strand: the pattern and D-array row, dstride bytes
    uint4 *slot_hits;       // per slot: SLOT_HITS hits
    uint4 *tasks[2];        // task states, by generation parity
    uint32_t *task_ref[2];  // slot | strand << 31, or TASK_EMPTY
    uint32_t *ctl;          // SPLIT_CTL control words
    uint4 *lane_cand;       // the first pass's hit buffers, FAST_CAND per lane
    uint32_t slot_cap, task_cap, dstride;
    uint32_t budget;  // expansions of a lane's part of a read before it is split (endgame); 0: off
    uint32_t count;   // nonzero: the parts' expansions are summed (per-read work counters)
};

__device__ __forceinline__ uint32_t ld_agent(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Reserve cnt task entries of generation g at off.  False when they do not
// all fit; reserved entries inside the array are then marked unused.
__device__ bool take_tasks(const SplitBufs &X, uint32_t g, uint32_t cnt, uint32_t &off) {
    // a full generation is not reserved from again, which also keeps the
    // counter far from wrapping
    if (ld_agent(&X.ctl[1 + g]) >= X.task_cap) return false;
    off = atomicAdd(&X.ctl[1 + g], cnt);
    if (off + cnt <= X.task_cap) return true;
    for (uint32_t j = off; j < X.task_cap; j++) X.task_ref[g & 1][j] = TASK_EMPTY;
    return false;
}

// Write cur when has_cur, then the lane's pending stack entries, to the
// entries reserved at off in generation g; the lane's stack is left empty.
__device__ void put_tasks(const SplitBufs &X, uint32_t g, uint32_t off, uint32_t ref, LaneCtx &c, uint4 cur,
                          bool has_cur) {
    uint4 *T = X.tasks[g & 1];
    uint32_t *R = X.task_ref[g & 1];
    if (has_cur) {
        T[off] = cur;
        R[off] = ref;
        off++;
    }
    for (uint32_t j = c.sbase; j < c.sp; j++, off++) {
        T[off] = c.stack[(size_t)j * c.sstride];
        R[off] = ref;
    }
    c.sp = c.sbase = 0;
}

// Copy an m-byte pattern and D-array row from the lane's LDS row to the
// slot: whole dwords, within both rows.
// (A plain loop on purpose: this runs once per split read, in the endgame of
// the batched kernel, and a batched copy there changed the code of that
// kernel's whole loop and cost it about 3% on 100-base reads.)
__device__ __forceinline__ void save_row(const SplitBufs &X, uint32_t s, int strand, const uint8_t *pd, int m) {
    const uint32_t *src = reinterpret_cast<const uint32_t *>(pd);
    uint32_t *dst = reinterpret_cast<uint32_t *>(X.slot_rows + ((size_t)s * 2 + (size_t)strand) * X.dstride);
    for (int k = 0; k < (m + 3) / 4; k++) dst[k] = src[k];
}
// Deliver the lane's hits to slot s -- those within the bound of the best
// score known -- with its expansions; the lane's hit buffer is emptied.
__device__ void flush_slot(const SplitBufs &X, const Params &P, uint32_t s, LaneCtx &c) {
    if (X.count && c.expand) atomicAdd(&X.slot_exp[s], c.expand);
    c.expand = 0;
    // a lane's best score changes only with a hit it holds: without hits
    // there is nothing to deliver
    if (c.ncand == 0) return;
    const int old = atomicMin(&X.slot_best[s], c.best);
    const int best = old < c.best ? old : c.best;
    const int bound = (P.mode == BWFM_MODE_BEST && best != INF_SCORE) ? best + P.s_mm : INF_SCORE;
    uint32_t keep = 0;
    for (uint32_t j = 0; j < c.ncand; j++) keep += h_score(c.cand[(size_t)j * c.cstride]) <= bound ? 1u : 0u;
    if (keep) {
        uint32_t off = atomicAdd(&X.slot_nhit[s], keep);
        if (off + keep > SLOT_HITS) {  // the collection left room for FAST_CAND of them
            atomicOr(&X.slot_fail[s], 1u);
        } else {
            uint4 *dst = X.slot_hits + (size_t)s * SLOT_HITS;
            for (uint32_t j = 0; j < c.ncand; j++) {
                const uint4 h = c.cand[(size_t)j * c.cstride];
                if (h_score(h) <= bound) dst[off++] = h;
            }
        }
    }
    c.ncand = 0;
}

// Flag word of a read in its wave's sharing block: SH_FAIL, SH_HELPED, the
// strands whose rows the read's slot holds, SH_NOSPLIT once a split found
// no room, and the slot plus one above SH_SLOT_SHIFT (0: none yet).
enum { SH_FAIL = 1, SH_HELPED = 2, SH_ROW0 = 4, SH_NOSPLIT = 16 };
constexpr int SH_SLOT_SHIFT = 5;

// Endgame of the first pass: hand this lane's part of read r on `strand`
// -- cur when valid, then the pending stack entries -- to the tasks of
// generation 0, taking the read's slot at its first split (fl is the
// read's flag word; best its best score so far; owner the global index of
// the lane that owns the read).  The caller runs one lane of a wave at a
// time.  False, with the lane's search unchanged, when no slot or task room
// is left.
__device__ bool split_part(const SplitBufs &X, uint32_t r, uint32_t owner, int strand, int m, int maxd, int best,
                           LaneCtx &c, uint4 cur, bool valid, int &fl) {
    const uint32_t cnt = (valid ? 1u : 0u) + (c.sp - c.sbase);
    const bool had = (fl >> SH_SLOT_SHIFT) != 0;
    if (!had && ld_agent(&X.ctl[0]) >= X.slot_cap) return false;
    uint32_t off = 0;
    if (!take_tasks(X, 0, cnt, off)) return false;
    uint32_t s;
    if (had) {
        s = (uint32_t)(fl >> SH_SLOT_SHIFT) - 1;
    } else {
        s = atomicAdd(&X.ctl[0], 1u);
        if (s >= X.slot_cap) {
            for (uint32_t j = 0; j < cnt; j++) X.task_ref[0][off + j] = TASK_EMPTY;
            return false;
        }
        X.slot_read[s] = r;
        X.slot_meta[s] = (uint32_t)m | ((uint32_t)maxd << 10);
        X.slot_best[s] = best;
        X.slot_nhit[s] = 0;
        X.slot_fail[s] = 0;
        X.slot_exp[s] = 0;
        X.slot_owner[s] = owner;
        X.slot_own[s] = 0;
        X.slot_obest[s] = INF_SCORE;
        fl |= (int)((s + 1) << SH_SLOT_SHIFT);
    }
    if (!(fl & (SH_ROW0 << strand))) {
        save_row(X, s, strand, c.pd, m);
        fl |= SH_ROW0 << strand;
    }
    put_tasks(X, 0, off, s | ((uint32_t)strand << 31), c, cur, valid);
    return true;
}

// The first pass's end of a split read (fl: its flag word, with the slot):
// the owner's hits stay in its hit buffer -- a lane whose wave has reached
// the endgame takes no further read -- and the slot records their number
// and the best score, for the collection before the rounds.  A failed read
// goes to the second pass through its slot.
__device__ __forceinline__ void end_split_read(const SplitBufs &X, const LaneCtx &c, int fl) {
    const uint32_t s = (uint32_t)(fl >> SH_SLOT_SHIFT) - 1;
    if (fl & SH_FAIL) {
        X.slot_fail[s] = 1;
        return;
    }
    X.slot_own[s] = c.ncand;
    X.slot_obest[s] = c.best;
    if (X.count) X.slot_exp[s] += c.expand;
}

// Before the rounds: each split read's first-pass hits join its slot's
// list, and the slot's best score takes theirs.  One thread per slot.
__global__ void k_split_collect(SplitBufs X) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= min(X.ctl[0], X.slot_cap) || X.slot_fail[s]) return;
    const uint32_t n = X.slot_own[s];
    const uint4 *src = X.lane_cand + (size_t)X.slot_owner[s] * FAST_CAND;
    uint4 *dst = X.slot_hits + (size_t)s * SLOT_HITS;
    for (uint32_t j = 0; j < n; j++) dst[j] = src[j];
    X.slot_nhit[s] = n;
    if (X.slot_obest[s] < X.slot_best[s]) X.slot_best[s] = X.slot_obest[s];
}

// After the rounds: each split read's hits, duplicates merged as a lane's
// buffer merges them, are canonicalised and published; a failed slot's
// read goes to the second pass.
__global__ void k_split_publish(Params P, SplitBufs X, ReadOut O) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t ns = min(X.ctl[0], X.slot_cap);
    if (s >= ns) return;
    const uint32_t r = X.slot_read[s];
    const uint32_t nh = X.slot_nhit[s];
    if (X.slot_fail[s] || nh > SLOT_HITS) {
        if (O.expand) O.expand[r] = X.slot_exp[s];
        send_to_second_pass(O, r);
        return;
    }
    LaneCtx c;
    c.cand = X.slot_hits + (size_t)s * SLOT_HITS;
    c.cstride = 1;
    uint32_t w = 0;
    for (uint32_t j = 0; j < nh; j++) {
        const uint4 h = c.cand[j];
        uint32_t q = 0;
        while (q < w && !(h_strand(c.cand[q]) == h_strand(h) && c.cand[q].x == h.x && h_len(c.cand[q]) == h_len(h))) q++;
        if (q == w)
            c.cand[w++] = h;
        else if (better(h, c.cand[q]))
            c.cand[q] = h;
    }
    c.ncand = w;
    c.best = X.slot_best[s];
    c.expand = X.slot_exp[s];
    publish(c, P, O, r, (uint8_t)BWFM_ST_SPLIT);
}

// ------------------------------------------------------------------ kernels

// Plain form: one lane per read, one launch per batch.
template <int LW>
__global__ __launch_bounds__(BLOCK) void k_align_plain(DevIndex ix, ReadsView rd, Params P, LaneBufs B, ReadOut O) {
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= reads_n(rd)) return;
    int m, maxd;
    uint64_t o0;
    if (check_read(rd, P, O, r, m, maxd, o0)) return;
    LaneCtx c;
    init_ctx(c, B, r);
    int rc = align_read<LW>(ix, rd.bases + o0, m, maxd, P, c, PH_FAST);
    if (rc) {
        if (O.expand) O.expand[r] = c.expand;
        send_to_second_pass(O, r);
        return;
    }
    publish(c, P, O, r);
}

enum { PZ_IDLE = 0, PZ_DSCAN = 1, PZ_SEARCH = 2, PZ_HELP = 3, PZ_WAIT = 4 };
enum { ACT_NONE = 0, ACT_DSTEP = 1, ACT_EXPAND = 2 };

// Per-wave block in LDS through which the lanes of a wave share one read's
// search once the batch's reads are all taken: an idle lane receives the
// oldest pending state of a busy lane's stack (the root of the largest
// untouched subtree) and searches it on the owner's pattern, D-array, bound
// and hit buffer.  Arrays are indexed by the owner lane, the lane that took
// the read; box and meta pass the donated states, by donor rank.
struct WaveShare {
    int best[64];       // best score found so far for the owner's read
    int ncand[64];      // hits in the owner's hit buffer
    int pending[64];    // helper lanes still searching donated subtrees
    int flags[64];      // SH_FAIL: the hit buffer overflowed; SH_HELPED; the read's slot
    int hexp[64];       // states expanded by helpers
    uint4 box[64];      // donated states
    uint32_t meta[64];  // owner lane | strand << 6 | budget << 7 | m << 11
};

__device__ __forceinline__ int sh_ld(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void sh_st(int *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// order this wave's earlier LDS and global accesses before its later ones,
// as seen by the other lanes of the wave
__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// Batched form: a persistent grid whose lanes pull reads from a shared
// counter.  Each loop iteration performs one rank-query pair per busy lane --
// a D-array step or a search expansion -- so lanes at different stages of
// different reads still share the expensive part, and a lane whose read is
// done takes the next one at once (wave-wide ballot, one atomic per wave).
// When the counter runs past the batch, idle lanes help the busy lanes of
// their wave through WaveShare instead of waiting for the slowest one.
// Arguments of the batched kernel that are used only at read boundaries:
// kept in device memory and loaded where used, so that they do not occupy
// scalar registers across the loop (the spills of a full argument list
// cost more vector instructions than the loop's own work).
struct PersistentArgs {
    ReadsView rd;
    LaneBufs B;
    ReadOut O;
    uint32_t *next_read;
    // the D-array pre-pass's output: per read, one row per strand of
    // dstride bytes (base | D << 3 per pattern position) and a byte whose
    // bit s is set when strand s is pruned at the root
    const uint8_t *drows;
    const uint8_t *dflag;
    uint32_t dstride;
    // split searches (X.budget 0: off), and per lane the read it owns
    // (helpers of a read find its index there)
    SplitBufs X;
    uint32_t *lane_read;
};

// Row of read r, strand s, in the pre-pass's output.
__device__ __forceinline__ const uint8_t *drow_of(const uint8_t *drows, uint32_t dstride, uint32_t r, int s) {
    return drows + ((size_t)r * 2 + (size_t)s) * dstride;
}

// D-array pre-pass of the batched form: one lane per read, both strands in
// turn on the other index (the same scan as the plain form's, with the
// short-string table when the index has one), each strand's row staged in
// LDS and then copied out whole.
template <int LW>
__global__ __launch_bounds__(BLOCK) void k_dscan(DevIndex ix, ReadsView rd, Params P, uint8_t *drows, uint8_t *dflag,
                                                 uint32_t dstride, uint32_t lstride) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= reads_n(rd)) return;
    uint64_t o0, len;
    bool bad;
    read_span(rd, r, o0, len, bad);
    const int maxd = rd.maxd ? rd.maxd[r] : P.max_diff;
    // reads the search will not take (invalid or empty) get no rows
    if (bad || len == 0 || len > rd.max_len || len > BWFM_MAX_READ || maxd > BWFM_MAX_DIFF) return;
    const int m = (int)len;
    LaneCtx c;
    c.pd = lds_bytes + (size_t)threadIdx.x * lstride;
    uint8_t fl = 0;
    for (int strand = 0; strand < 2; strand++) {
        const DevDir odir = pick_dir(ix, strand == 0 ? 0 : 1);
        if (!build_d<LW>(ix, odir, rd.bases + o0, m, strand, maxd, c)) {
            fl |= (uint8_t)(1 << strand);
            continue;
        }
        copy_dwords(reinterpret_cast<uint32_t *>(drows + ((size_t)r * 2 + (size_t)strand) * dstride),
                    reinterpret_cast<const uint32_t *>(c.pd), (m + 3) / 4);
    }
    dflag[r] = fl;
}

// Copy a pre-pass row (m bytes) into the lane's LDS row.  The rows start
// 16-byte aligned and their stride is a multiple of 16, so whole 16-byte
// blocks are read, four of them before any store: a row costs a few memory
// round trips (one per dword when each load waits for the store before it,
// which the compiler must assume may alias it).
__device__ __forceinline__ void load_drow(uint8_t *pd, const uint8_t *row, int m) {
    const uint4 *src = reinterpret_cast<const uint4 *>(row);
    uint32_t *dst = reinterpret_cast<uint32_t *>(pd);
    const int ndw = (m + 3) >> 2;
    for (int q0 = 0; 4 * q0 < ndw; q0 += 4) {
        uint4 v[4];
#pragma unroll
        for (int j = 0; j < 4; j++) v[j] = 4 * (q0 + j) < ndw ? src[q0 + j] : make_uint4(0, 0, 0, 0);
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int k = 4 * (q0 + j);
            if (k < ndw) dst[k] = v[j].x;
            if (k + 1 < ndw) dst[k + 1] = v[j].y;
            if (k + 2 < ndw) dst[k + 2] = v[j].z;
            if (k + 3 < ndw) dst[k + 3] = v[j].w;
        }
    }
}

__global__ void k_set_args(PersistentArgs *dst, PersistentArgs a) {
    if (threadIdx.x == 0) *dst = a;
}

// DP: the D-arrays come from the pre-pass (k_dscan); otherwise the loop
// scans them itself.
template <int LW, bool DP>
__device__ __forceinline__ void persistent_body(const DevIndex &ix, const Params &P, const PersistentArgs *A) {
    const uint32_t gl = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const uint32_t wave0 = threadIdx.x & ~63u;  // the wave's first thread in the block
    const uint32_t n_reads = reads_n(A->rd);
    const uint32_t lds_stride = A->B.lds_stride;
    WaveShare &ws = reinterpret_cast<WaveShare *>(lds_bytes + (size_t)blockDim.x * lds_stride)[threadIdx.x >> 6];
    LaneCtx c;
    init_ctx(c, A->B, gl);
    c.sstride = 1;  // persistent lanes own contiguous runs
    c.cstride = 1;
    uint4 *const own_cand = c.cand;
    uint8_t *const own_pd = c.pd;

    int phase = PZ_IDLE;
    bool exhausted = false;
    bool endgame = false;  // wave-uniform: the batch's reads are all taken
    int ow = lane;         // owner lane of the read this lane works on
    uint32_t r = 0;
    int m = 0, maxd = 0, strand = 0;
    // D scan state
    int di = 0, dz = 0;
    uint32_t dk = 0, dl = 0;
    uint32_t dcode = 0, dlen = 0;  // the current segment while the table covers it (KTLOOP)
    // search state
    uint4 cur = make_uint4(0, 0, 0, 0);
    bool valid = false;
#if BWFM_GENE_TWOSTATE == 1
    uint4 cur2 = make_uint4(0, 0, 0, 0);  // the second state (valid2), same read and strand
    bool valid2 = false;
#endif
    Seed S{0, 0, 0};
    // work statistics (measurement only)
    uint32_t w_iters = 0, w_busy = 0, w_query = 0;  // per lane: far below 2^32 per launch

    for (;;) {
        // an opaque step on the pointer keeps the argument loads inside the
        // loop, next to their uses
        asm volatile("" : "+s"(A));
        const ReadsView &rd = A->rd;
        const ReadOut &O = A->O;
        uint32_t *const next_read = A->next_read;
        // refill idle lanes, one atomic per wave
        const bool want = phase == PZ_IDLE && !exhausted;
        const unsigned long long wm = __ballot(want);
#if BWFM_GENE_REFILL == 1
        // refill in bulk: a quarter of the wave idle, or nothing left running
        if (wm && (__popcll(wm) >= 16 || __ballot(phase != PZ_IDLE) == 0)) {
#else
        if (wm) {
#endif
            const int leader = __ffsll(wm) - 1;
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(next_read, (uint32_t)__popcll(wm));
            base = __shfl(base, leader);
            if (want) {
                const uint32_t rr = base + (uint32_t)__popcll(wm & ((1ULL << lane) - 1));
                if (rr >= n_reads) {
                    exhausted = true;
                } else {
                    r = rr;
                    uint64_t o0;
                    if (!check_read(rd, P, O, r, m, maxd, o0)) {
                        ow = lane;
                        c.pd = own_pd;
                        c.cand = own_cand;
                        c.ncand = 0;
                        c.best = INF_SCORE;
                        c.expand = 0;
                        if (DP) {
                            // the first strand the pre-pass left searchable,
                            // or nothing to search
                            const int dfl = A->dflag[r];
                            strand = (dfl & 1) ? 1 : 0;
                            if ((dfl & 3) == 3) {
                                publish(c, P, O, r);
                                phase = PZ_IDLE;
                            } else {
                                load_drow(own_pd, drow_of(A->drows, A->dstride, r, strand), m);
                                phase = PZ_SEARCH;
                                cur = root_state(ix, m, P.minc * pd_d(c, m - 1));
                                valid = true;
                                c.sp = c.sbase = 0;
                            }
                        } else {
                            stage_read(own_pd, rd.bases + o0, m);
                            strand = 0;
                            phase = PZ_DSCAN;
                            di = 0;
                            dz = 0;
                            dk = 0;
                            dl = ix.n;
                            dcode = dlen = 0;
                        }
                        S = seed_of(P, m);
                        sh_st(&ws.best[lane], INF_SCORE);
                        sh_st(&ws.ncand[lane], 0);
                        sh_st(&ws.pending[lane], 0);
                        sh_st(&ws.flags[lane], 0);
                        sh_st(&ws.hexp[lane], 0);
                        if (A->X.budget) A->lane_read[gl] = r;
                    }
                }
            }
        }
        if (__ballot(phase != PZ_IDLE) == 0) {
            if (__ballot(!exhausted) == 0) break;
            continue;
        }
        endgame = endgame || __ballot(exhausted) != 0;
#if BWFM_GENE_TWOSTATE == 1
        if (endgame && valid2) {
            // the sharing below works on single states: the second one goes
            // back on the stack; with the stack full the read (still this
            // lane's alone: nothing is shared before the endgame) goes to
            // the second pass
            if (c.sp < c.stack_cap) {
                c.stack[(size_t)c.sp * c.sstride] = cur2;
                c.sp++;
            } else {
                send_to_second_pass(A->O, r);
                if (A->O.expand) A->O.expand[r] = c.expand;
                phase = PZ_IDLE;
                valid = false;
                c.sp = c.sbase = 0;
            }
            valid2 = false;
        }
#endif
        if (O.work) {
            w_iters++;
            w_busy += phase != PZ_IDLE && phase != PZ_WAIT;
        }

        if (endgame) {
            wave_fence();
            const bool searching = phase == PZ_SEARCH || phase == PZ_HELP;
            if (searching) {
                const int sb = sh_ld(&ws.best[ow]);
                if (sb < c.best) c.best = sb;
                if (sh_ld(&ws.flags[ow]) & SH_FAIL) {
                    // the read goes to the second pass: drop this lane's part
                    valid = false;
                    c.sp = c.sbase = 0;
                }
            }
            // hand the oldest pending state of busy lanes to idle lanes
            const int avail = searching ? (int)(c.sp - c.sbase) - (valid ? 0 : 1) : 0;
            const bool give = avail >= 1;
            const bool recv = phase == PZ_IDLE;
            const unsigned long long R = __ballot(recv), G = __ballot(give);
            if (R && G) {
                const int n = min(__popcll(R), __popcll(G));
                const unsigned long long lt = (1ULL << lane) - 1;
                if (give) {
                    const int gi = __popcll(G & lt);
                    if (gi < n) {
                        ws.box[gi] = c.stack[(size_t)c.sbase * c.sstride];
                        ws.meta[gi] = (uint32_t)ow | ((uint32_t)strand << 6) | ((uint32_t)maxd << 7) | ((uint32_t)m << 11);
                        c.sbase++;
                        atomicAdd(&ws.pending[ow], 1);
                        atomicOr(&ws.flags[ow], SH_HELPED);
                    }
                }
                wave_fence();
                if (recv) {
                    const int ri = __popcll(R & lt);
                    if (ri < n) {
                        cur = ws.box[ri];
                        const uint32_t mt = ws.meta[ri];
                        ow = (int)(mt & 63);
                        strand = (int)((mt >> 6) & 1);
                        maxd = (int)((mt >> 7) & 15);
                        m = (int)(mt >> 11);
                        S = seed_of(P, m);
                        valid = true;
                        c.sp = c.sbase = 0;
                        c.pd = lds_bytes + (size_t)(wave0 + ow) * lds_stride;
                        c.cand = own_cand + ((int)ow - lane) * (ptrdiff_t)FAST_CAND;
                        c.best = sh_ld(&ws.best[ow]);
                        c.expand = 0;
                        phase = PZ_HELP;
                    }
                }
                wave_fence();
            }
            // a part past the budget goes to the split searches, one lane
            // of the wave at a time (a read's slot is taken once); a part's
            // expansions count from the read's start for its owner and from
            // the hand-over for a helper
            const uint32_t bud = A->X.budget;
            if (bud) {
                const bool want = (phase == PZ_SEARCH || phase == PZ_HELP) && c.sp > c.sbase && c.expand >= bud &&
                                  !(sh_ld(&ws.flags[ow]) & (SH_FAIL | SH_NOSPLIT));
                unsigned long long sm = __ballot(want);
                while (sm) {
                    const int L = __ffsll(sm) - 1;
                    if (lane == L) {
                        int fl = sh_ld(&ws.flags[ow]);
                        const uint32_t og = gl - (uint32_t)lane + (uint32_t)ow;  // the owner's global lane
                        const uint32_t rr = ow == lane ? r : A->lane_read[og];
                        if (split_part(A->X, rr, og, strand, m, maxd, sh_ld(&ws.best[ow]), c, cur, valid, fl))
                            valid = false;  // the lane's part is over
                        else
                            fl |= SH_NOSPLIT;  // no room: the read's parts go on in the wave
                        sh_st(&ws.flags[ow], fl);
                    }
                    wave_fence();
                    sm &= sm - 1;
                }
            }
        }

        // decide this lane's action and rank queries; a lane that changes
        // phase here acts in its new phase from the next iteration on
        int act = ACT_NONE;
        bool query = false;
        bool hit = false;
        int qdir = 0;  // index queried: 0 = T, 1 = reverse(T)
        uint32_t q1 = 0, q2 = 0;
        int da = 4;
        bool part_done = false;  // this lane's part of the strand's search is over
        if (!DP && phase == PZ_DSCAN) {
            act = ACT_DSTEP;
            {
                const int b = own_pd[di] & 7;  // the staged base (strand +)
                da = (strand == 0 || b > 3) ? b : 3 - b;
            }
            if (da < 4) {
                query = true;
                qdir = strand == 0 ? 0 : 1;
                q1 = dk;
                q2 = dl + 1;
            }
        } else if (phase == PZ_SEARCH || phase == PZ_HELP) {
            int rr = resolve<KT_LOOP>(cur, valid, strand, P, c, PH_FAST, POPS_PER_STEP, ix, endgame);
            if (rr == 2) {
                // pop limit reached: keep popping next iteration
            } else if (rr == 3) {
                hit = true;
            } else if (rr < 0) {
                // only without endgame, so the lane owns its read alone
                send_to_second_pass(O, r);
                if (O.expand) O.expand[r] = c.expand;
                phase = PZ_IDLE;
            } else if (rr == 0) {
                part_done = true;
            }
            if (rr == 1) {
                act = ACT_EXPAND;
                query = true;
                qdir = strand == 0 ? 1 : 0;
                q1 = cur.x;
                q2 = cur.y + 1;
            }
#if BWFM_GENE_TWOSTATE == 1
            if (!endgame && phase == PZ_SEARCH) {
                const int bound = (P.mode == BWFM_MODE_BEST && c.best != INF_SCORE) ? c.best + P.s_mm : INF_SCORE;
                // the second state: dropped once the bound passes it,
                // recorded when it is a completed hit
                if (valid2 && entry_lb(cur2) > bound) valid2 = false;
                if (valid2 && s_i(cur2) < 0) {
                    valid2 = false;
                    const int score = s_score(cur2);
                    if (score < c.best) c.best = score;
                    if (record(c, P, make_hit(strand, KT_LOOP ? state_k(ix, strand, cur2) : cur2.x, cur2.y,
                                              s_len(cur2), score, s_nmm(cur2), s_ngo(cur2), s_nge(cur2)),
                               PH_FAST)) {
                        send_to_second_pass(O, r);
                        if (O.expand) O.expand[r] = c.expand;
                        phase = PZ_IDLE;
                        act = ACT_NONE;
                        query = false;
                        part_done = false;
                    }
                }
                // else the next state on the stack, unless it is a completed
                // hit (left for resolve) or already beaten by the bound
                if (phase == PZ_SEARCH && !valid2 && c.sp > c.sbase) {
                    const uint4 t = c.stack[(size_t)(c.sp - 1) * c.sstride];
                    if (entry_lb(t) > bound) {
                        c.sp--;
                    } else if (s_i(t) >= 0) {
                        c.sp--;
                        cur2 = t;
                        valid2 = true;
                    }
                }
                // the lane's part is not over while the second state is left:
                // it becomes the current one (already resolved above)
                if (part_done && valid2) {
                    part_done = false;
                    cur = cur2;
                    valid = true;
                    valid2 = false;
                    act = ACT_EXPAND;
                    query = true;
                    q1 = cur.x;
                    q2 = cur.y + 1;
                }
                // a searching lane queries the strand's search index, for
                // either state
                qdir = strand == 0 ? 1 : 0;
            }
#endif
            if (!endgame && phase == PZ_SEARCH) {
                sh_st(&ws.best[lane], c.best);
                sh_st(&ws.ncand[lane], (int)c.ncand);
            }
        }

        // completed hits found in the endgame, one lane at a time: lanes of
        // one read share its hit buffer
        if (endgame) {
            unsigned long long hm = __ballot(hit);
            while (hm) {
                const int L = __ffsll(hm) - 1;
                if (lane == L) {
                    c.ncand = (uint32_t)sh_ld(&ws.ncand[ow]);
                    const int sb = sh_ld(&ws.best[ow]);
                    if (sb < c.best) c.best = sb;
                    const int score = s_score(cur);
                    if (score < c.best) c.best = score;
                    const int rc = record(c, P,
                                          make_hit(strand, KT_LOOP ? state_k(ix, strand, cur) : cur.x, cur.y,
                                                   s_len(cur), score, s_nmm(cur), s_ngo(cur), s_nge(cur)),
                                          PH_FAST);
                    sh_st(&ws.best[ow], c.best);
                    sh_st(&ws.ncand[ow], (int)c.ncand);
                    if (rc) {
                        atomicOr(&ws.flags[ow], SH_FAIL);
                        c.sp = c.sbase = 0;
                        part_done = true;
                    }
                    valid = false;
                }
                wave_fence();
                hm &= hm - 1;
            }
        }

        // the end of a lane's part: a helper reports back; an owner waits
        // for its helpers before the next strand or the publication
        if (part_done) {
            valid = false;
            c.sp = c.sbase = 0;
            if (phase == PZ_HELP) {
                atomicAdd(&ws.hexp[ow], (int)c.expand);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                atomicSub(&ws.pending[ow], 1);
                phase = PZ_IDLE;
            } else {
                phase = PZ_WAIT;
            }
        }
        if (phase == PZ_WAIT && sh_ld(&ws.pending[lane]) == 0) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            const int fl = sh_ld(&ws.flags[lane]);
            if (fl & SH_FAIL) {
                if (fl >> SH_SLOT_SHIFT)
                    end_split_read(A->X, c, fl);
                else
                    send_to_second_pass(O, r);
                if (O.expand) O.expand[r] = c.expand + (uint32_t)sh_ld(&ws.hexp[lane]);
                phase = PZ_IDLE;
            } else if (strand == 0 && (!DP || !(A->dflag[r] & 2))) {
                strand = 1;
                if (DP) {
                    load_drow(own_pd, drow_of(A->drows, A->dstride, r, 1), m);
                    phase = PZ_SEARCH;
                    cur = root_state(ix, m, P.minc * pd_d(c, m - 1));
                    valid = true;
                    c.sp = c.sbase = 0;
                } else {
                    phase = PZ_DSCAN;
                    di = 0;
                    dz = 0;
                    dk = 0;
                    dl = ix.n;
                    dcode = dlen = 0;
                }
            } else {
                c.ncand = (uint32_t)sh_ld(&ws.ncand[lane]);
                const int sb = sh_ld(&ws.best[lane]);
                if (sb < c.best) c.best = sb;
                c.cand = own_cand;
                c.expand += (uint32_t)sh_ld(&ws.hexp[lane]);
                if (fl >> SH_SLOT_SHIFT)
                    end_split_read(A->X, c, fl);
                else
                    publish(c, P, O, r, (fl & SH_HELPED) ? (uint8_t)BWFM_ST_SHARED : (uint8_t)0);
                phase = PZ_IDLE;
            }
        }

        // the shared part: rank counts at q1 and q2 on one index
        uint32_t ok[4] = {0, 0, 0, 0}, ol[4] = {0, 0, 0, 0};
        const DevDir qd = pick_dir(ix, qdir);
        if (O.work) w_query += query;
        if (query) {
            // a D-array step or an expansion whose string the table covers
            // reads the children's intervals there
            const uint32_t qlen = act == ACT_DSTEP ? dlen : (uint32_t)s_len(cur);
            if (KT_LOOP && qlen < ix.kt_levels) {
                const uint32_t code = act == ACT_DSTEP ? dcode : cur.x;
                const uint4 *e = reinterpret_cast<const uint4 *>(qd.kt + 2 * kt_children((int)qlen, code));
                kt_pick(qd, e[0], e[1], ok, ol);
            } else {
                occ4_pair<LW>(ix, qd, q1, q2, ok, ol);
            }
        }
#if BWFM_GENE_TWOSTATE == 1
        const bool act2 = valid2 && phase == PZ_SEARCH && !endgame;
        uint32_t ok2[4] = {0, 0, 0, 0}, ol2[4] = {0, 0, 0, 0};
        if (act2) {
            if (KT_LOOP && (uint32_t)s_len(cur2) < ix.kt_levels) {
                const uint4 *e = reinterpret_cast<const uint4 *>(qd.kt + 2 * kt_children(s_len(cur2), cur2.x));
                kt_pick(qd, e[0], e[1], ok2, ol2);
            } else {
                occ4_pair<LW>(ix, qd, cur2.x, cur2.y + 1, ok2, ol2);
            }
        }
        if (O.work) w_query += act2;
#endif

        // consume
        if (!DP && act == ACT_DSTEP) {
            bool empty = true;
            if (da < 4) {
                const uint32_t a1 = sel4(ok, da), a2 = sel4(ol, da);
                empty = a1 >= a2;
                dk = sel4(qd.C, da) + a1;
                dl = sel4(qd.C, da) + a2 - 1;
                if (KT_LOOP) {
                    dcode = (dcode << 2) | (uint32_t)da;
                    dlen++;
                }
            }
            bool skip = false;
            if (empty) {
                dz++;
                dk = 0;
                dl = ix.n;
                dcode = dlen = 0;
                skip = dz > maxd;
            }
            if (!skip) {
                c.pd[di] = (uint8_t)(da | (dz << 3));
                di++;
            }
            if (skip || di == m) {
                if (!skip) {
                    phase = PZ_SEARCH;
                    cur = root_state(ix, m, P.minc * dz);
                    valid = true;
                    c.sp = c.sbase = 0;
                } else if (strand == 0) {
                    strand = 1;
                    di = 0;
                    dz = 0;
                    dk = 0;
                    dl = ix.n;
                    dcode = dlen = 0;
                } else {
                    // strand - cannot match; the read's helpers, if any,
                    // were all done before this D scan began
                    c.ncand = (uint32_t)sh_ld(&ws.ncand[lane]);
                    const int sb = sh_ld(&ws.best[lane]);
                    if (sb < c.best) c.best = sb;
                    c.expand += (uint32_t)sh_ld(&ws.hexp[lane]);
                    const int fl = sh_ld(&ws.flags[lane]);
                    if (fl >> SH_SLOT_SHIFT)
                        end_split_read(A->X, c, fl);
                    else
                        publish(c, P, O, r, (fl & SH_HELPED) ? (uint8_t)BWFM_ST_SHARED : (uint8_t)0);
                    phase = PZ_IDLE;
                }
            }
        } else if (act == ACT_EXPAND) {
            c.expand++;
            const int i = s_i(cur);
            const int b = pd_base(c, i);
            const int Di = pd_d(c, i), Dn = pd_d(c, i - 1);
            int rc = expand_children(cur, valid, ok, ol, qd, b, m, maxd, Di, Dn, S, P, c, KT_LOOP ? ix.kt_levels : 0);
            if (rc) {
                // cannot happen with worst-case stacks; kept as a guard
                if (endgame) {
                    atomicOr(&ws.flags[ow], SH_FAIL);  // every lane of the read drops out
                } else {
                    send_to_second_pass(O, r);
                    if (O.expand) O.expand[r] = c.expand;
                    phase = PZ_IDLE;
                }
            }
        }
#if BWFM_GENE_TWOSTATE == 1
        if (act2 && phase == PZ_SEARCH) {
            c.expand++;
            const int i2 = s_i(cur2);
            const int b2 = pd_base(c, i2);
            const int Di2 = pd_d(c, i2), Dn2 = pd_d(c, i2 - 1);
            // with two states in flight the stack can outgrow its one-path
            // worst case; the read then goes to the second pass
            if (expand_children(cur2, valid2, ok2, ol2, qd, b2, m, maxd, Di2, Dn2, S, P, c,
                                KT_LOOP ? ix.kt_levels : 0)) {
                send_to_second_pass(O, r);
                if (O.expand) O.expand[r] = c.expand;
                phase = PZ_IDLE;
            }
        }
        if (phase == PZ_IDLE) valid2 = false;
#endif
    }
    if (A->O.work) {
        if (lane == 0) atomicAdd(&A->O.work[0], (unsigned long long)w_iters);
        atomicAdd(&A->O.work[1], (unsigned long long)w_busy);
        atomicAdd(&A->O.work[2], (unsigned long long)w_query);
    }
}

// Two builds of the batched kernel: the compiler's own register budget
// (about 144 VGPRs: 3 waves per SIMD) and one held to 128 VGPRs so that 4
// waves stay resident per SIMD.  The search is latency-bound, so the second
// is faster on the benchmark batch (122 ms against 134); a build held to 96
// VGPRs spills to scratch and is slower still (205 ms).  The autotuner picks.
template <int LW, bool DP = false>
__global__ __launch_bounds__(BLOCK) void k_align_persistent(DevIndex ix, Params P, const PersistentArgs *A) {
    persistent_body<LW, DP>(ix, P, A);
}
template <int LW, bool DP = false>
__global__ __launch_bounds__(BLOCK, 4) void k_align_persistent4(DevIndex ix, Params P, const PersistentArgs *A) {
    persistent_body<LW, DP>(ix, P, A);
}

using PersistentKernel = void (*)(DevIndex, Params, const PersistentArgs *);

// the build serving a waves_per_simd setting: 0 and >= 4 take the 4-wave
// build, 1-3 the compiler's own; dp: D-arrays from the pre-pass
template <int LW>
PersistentKernel persistent_kernel(int waves_per_simd, bool dp = false) {
    if (dp)
        return (waves_per_simd == 0 || waves_per_simd >= 4) ? k_align_persistent4<LW, true>
                                                              : k_align_persistent<LW, true>;
    return (waves_per_simd == 0 || waves_per_simd >= 4) ? k_align_persistent4<LW> : k_align_persistent<LW>;
}

// Arguments of the task rounds, kept in device memory like PersistentArgs.
struct TaskArgs {
    LaneBufs B;
    SplitBufs X;
};

__global__ void k_set_task_args(TaskArgs *dst, TaskArgs a) {
    if (threadIdx.x == 0) *dst = a;
}

// One round of split searches: a persistent grid whose lanes take the
// tasks of generation g from a counter, one atomic per wave as the batched
// kernel takes reads.  A task is one state of a split read: its subtree is
// searched depth-first on the lane's own stack with the slot's row (read in
// place, so the kernel needs no LDS and as many lanes as its registers
// allow), budget and best score, one rank-query pair per lane and
// iteration.  Once the
// round's tasks are all taken (drain set), a lane that has expanded at
// least DRAIN_MIN states of its task hands its pending states to
// generation g + 1, so that the round ends soon and the next one spreads
// them over the grid; the last round has no drain.  At a task's end its
// hits go to the slot.
constexpr uint32_t DRAIN_MIN = 256;
constexpr int TASK_REFILL = 32;  // idle lanes of a wave that make it take new tasks
template <int LW>
__global__ __launch_bounds__(BLOCK) void k_align_tasks(DevIndex ix, Params P, const TaskArgs *A, uint32_t g,
                                                       uint32_t drain) {
    const uint32_t ntask = min(ld_agent(&A->X.ctl[1 + g]), A->X.task_cap);
    if (ntask == 0) return;  // the whole grid: nothing was split
    const int lane = threadIdx.x & 63;
    LaneCtx c;
    init_ctx(c, A->B, blockIdx.x * blockDim.x + threadIdx.x);
    c.sstride = 1;
    c.cstride = 1;
    bool busy = false, exhausted = false, valid = false;
    bool drained = false;  // wave-uniform: the round's tasks are all taken
    uint32_t s = 0, texp = 0, witer = 0;
    int strand = 0, m = 0, maxd = 0;
    uint4 cur = make_uint4(0, 0, 0, 0);
    Seed S{0, 0, 0};
    for (;;) {
        asm volatile("" : "+s"(A));
        const SplitBufs &X = A->X;
        witer++;
        // a wave learns that the round's tasks are all taken when one of
        // its lanes finds none left, else from one load of the counter
        // every 64 iterations (the same address for the whole wave)
        if (drain && !drained && (witer & 63) == 0) drained = ld_agent(&X.ctl[2 + SPLIT_ROUNDS + g]) >= ntask;
        // every 64 iterations, at once for the wave (lanes on one read share
        // the load), the bound takes the best score any part has found
        if ((witer & 63) == 32 && busy) {
            const int sb = (int)ld_agent(reinterpret_cast<const uint32_t *>(&X.slot_best[s]));
            if (sb < c.best) c.best = sb;
        }
        // idle lanes take the next tasks, one atomic per wave, once
        // TASK_REFILL lanes of the wave are idle (or none is busy): tasks
        // end every few hundred expansions, and one counter taken by every
        // wave at that rate held the rounds to half their speed
        const bool idle = !busy && !exhausted;
        const unsigned long long im = __ballot(idle);
        const bool bulk = __popcll(im) >= TASK_REFILL || __ballot(busy) == 0;
        const bool want = idle && bulk;
        const unsigned long long wm = bulk ? im : 0ull;
        uint32_t t = 0;
        if (wm) {
            const int leader = __ffsll(wm) - 1;
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(&X.ctl[2 + SPLIT_ROUNDS + g], (uint32_t)__popcll(wm));
            base = __shfl(base, leader);
            t = base + (uint32_t)__popcll(wm & ((1ULL << lane) - 1));
            if (want && t >= ntask) exhausted = true;
        }
        if (want && !exhausted) {
            const uint32_t ref = X.task_ref[g & 1][t];
            // unused entries and the parts of failed reads are skipped (a
            // stale flag only costs the work)
            if (ref != TASK_EMPTY && !X.slot_fail[ref & 0x7fffffffu]) {
                s = ref & 0x7fffffffu;
                strand = (int)(ref >> 31);
                const uint32_t meta = X.slot_meta[s];
                m = (int)(meta & 1023);
                maxd = (int)(meta >> 10);
                // the slot's row, read in place: the tasks of one read share
                // it in the caches
                c.pd = X.slot_rows + ((size_t)s * 2 + (size_t)strand) * X.dstride;
                cur = X.tasks[g & 1][t];
                valid = true;
                c.sp = c.sbase = 0;
                c.ncand = 0;
                c.best = X.slot_best[s];  // a stale value only prunes less
                c.expand = 0;
                texp = 0;
                S = seed_of(P, m);
                busy = true;
            }
        }
        if (__ballot(busy) == 0) {
            if (__ballot(!exhausted) == 0) break;
            continue;
        }
        drained = drained || __ballot(exhausted) != 0;
        bool query = false, done = false;
        if (busy) {
            const int rr = resolve<KT_LOOP>(cur, valid, strand, P, c, PH_FAST, POPS_PER_STEP, ix, true);
            if (rr == 3) {
                // a completed hit; a better score is shared with the read's
                // other parts at once, a full buffer is first delivered
                const int score = s_score(cur);
                if (score < c.best) {
                    c.best = score;
                    atomicMin(&X.slot_best[s], score);
                }
                const uint4 h = make_hit(strand, KT_LOOP ? state_k(ix, strand, cur) : cur.x, cur.y, s_len(cur), score,
                                         s_nmm(cur), s_ngo(cur), s_nge(cur));
                if (record(c, P, h, PH_FAST)) {
                    flush_slot(X, P, s, c);
                    if (record(c, P, h, PH_FAST)) {
                        atomicOr(&X.slot_fail[s], 1u);
                        done = true;
                    }
                }
                valid = false;
            } else if (rr == 0) {
                done = true;
            } else if (rr == 1) {
                if (drain && drained && texp >= DRAIN_MIN && c.sp > c.sbase) {
                    uint32_t off = 0;
                    if (take_tasks(X, g + 1, 1 + (c.sp - c.sbase), off)) {
                        put_tasks(X, g + 1, off, s | ((uint32_t)strand << 31), c, cur, true);
                        valid = false;
                        done = true;
                    }
                }
                query = !done;
            }
            // rr == 2: the pop limit; popping goes on next iteration
        }
        uint32_t ok[4] = {0, 0, 0, 0}, ol[4] = {0, 0, 0, 0};
        const DevDir qd = pick_dir(ix, strand == 0 ? 1 : 0);
        if (query) {
            if (KT_LOOP && (uint32_t)s_len(cur) < ix.kt_levels) {
                const uint4 *e = reinterpret_cast<const uint4 *>(qd.kt + 2 * kt_children(s_len(cur), cur.x));
                kt_pick(qd, e[0], e[1], ok, ol);
            } else {
                occ4_pair<LW>(ix, qd, cur.x, cur.y + 1, ok, ol);
            }
            c.expand++;
            texp++;
            const int i = s_i(cur);
            if (expand_children(cur, valid, ok, ol, qd, pd_base(c, i), m, maxd, pd_d(c, i), pd_d(c, i - 1), S, P, c,
                                KT_LOOP ? ix.kt_levels : 0)) {
                atomicOr(&X.slot_fail[s], 1u);  // cannot happen with worst-case stacks; kept as a guard
                done = true;
            }
        }
        if (done) {
            flush_slot(X, P, s, c);
            busy = false;
            valid = false;
        }
    }
}

// Totals of the split searches for the work counters (work[3..5] start at
// zero): reads split, task entries handed out over all generations, split
// reads sent on to the second pass; then per generation the entries asked
// for (above the room when some found none).  One thread per slot.
__global__ void k_split_stats(SplitBufs X, unsigned long long *work) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t ns = min(X.ctl[0], X.slot_cap);
    if (s == 0) {
        unsigned long long t = 0;
        for (int g = 0; g <= SPLIT_ROUNDS; g++) t += min(X.ctl[1 + g], X.task_cap);
        work[3] = ns;
        work[4] = t;
        for (int g = 0; g < SPLIT_ROUNDS; g++) work[6 + g] = X.ctl[1 + g];
    }
    if (s < ns && (X.slot_fail[s] || X.slot_nhit[s] > SLOT_HITS)) atomicAdd(&work[5], 1ull);
}

// Second pass for the reads listed in slow_list (*O.n_slow of them, set by
// the first pass): a fixed grid pulls them from a counter.  Each read gets
// the worst-case stack; first the best score S*, then the hits with the
// bound fixed at S* + s_mm.  The reported hits go to the staging arena like
// the first pass's.
template <int LW>
__global__ __launch_bounds__(BLOCK) void k_align_slow(DevIndex ix, ReadsView rd, Params P, LaneBufs B, ReadOut O,
                                                      uint32_t *slow_next) {
    const uint32_t gl = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t ns = *O.n_slow;
    if (blockIdx.x * blockDim.x >= ns) return;  // the whole block has nothing to take
    LaneCtx c;
    init_ctx(c, B, gl);
    for (;;) {
        const uint32_t t = atomicAdd(slow_next, 1u);
        if (t >= ns) break;
        const uint32_t r = O.slow_list[t];
        uint64_t o0, len;
        bool bad;
        read_span(rd, r, o0, len, bad);
        const int m = (int)len;
        const int maxd = rd.maxd ? rd.maxd[r] : P.max_diff;
        c.expand = 0;
        c.best = INF_SCORE;
        align_read<LW>(ix, rd.bases + o0, m, maxd, P, c, PH_BEST);
        uint8_t st = 0;
        uint32_t a = 0, b = 0, nr = 0;
        if (c.best != INF_SCORE) {
            const int rc = align_read<LW>(ix, rd.bases + o0, m, maxd, P, c, PH_COLLECT);
            if (rc == R_CAND) {
                st = BWFM_ST_OVERFLOW;
                a = b = 0xffffffffu;
            } else {
                nr = finish(c, P, st, a, b);
            }
        }
        stage_hits(c, O, r, nr);
        O.n_rep[r] = nr;
        O.status[r] = st | ST_RESEARCH;
        O.c1[r] = a;
        O.c2[r] = b;
        if (O.expand) O.expand[r] += c.expand;
    }
}

// Copy each read's reported hits from the staging arena to the CSR output.
// Launched only when the output holds them all.
__global__ void k_compact(uint32_t n, const uint64_t *hoff, const uint4 *stage, const uint64_t *stage_off,
                          uint4 *hits, const uint64_t *n_dev, const uint32_t *err) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (err && *err) return;  // the output cannot hold the hits
    if (r >= count_of(n, n_dev)) return;
    const uint64_t o = hoff[r], e = hoff[r + 1];
    if (e == o) return;
    const uint4 *src = stage + stage_off[r];
    for (uint64_t j = 0; j < e - o; j++) hits[o + j] = src[j];
}

// Fill n words with v (used instead of a memset node, so that a captured
// sequence replays it reliably).
__global__ void k_fill_u32(uint32_t *p, uint32_t n, uint32_t v) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ exclusive scan (u32 counts -> u64 offsets)

constexpr int SCAN_BLOCK = 1024;

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_reduce(const uint32_t *in, uint64_t n, uint64_t *part,
                                                            const uint64_t *n_dev) {
    __shared__ uint64_t s[SCAN_BLOCK / 64];
    n = count_of(n, n_dev);
    uint64_t i = (uint64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x;
    uint64_t v = i < n ? in[i] : 0;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int w = 0; w < SCAN_BLOCK / 64; w++) t += s[w];
        part[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_parts(uint64_t *part, uint64_t nb) {
    // exclusive scan of nb block sums by one workgroup, in chunks
    __shared__ uint64_t s[SCAN_BLOCK];
    __shared__ uint64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint64_t base = 0; base < nb; base += SCAN_BLOCK) {
        uint64_t i = base + threadIdx.x;
        uint64_t v = i < nb ? part[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < SCAN_BLOCK; o <<= 1) {
            uint64_t t = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        uint64_t incl = s[threadIdx.x];
        if (i < nb) part[i] = carry + incl - v;
        __syncthreads();
        if (threadIdx.x == SCAN_BLOCK - 1) carry += incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) part[nb] = carry;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_apply(const uint32_t *in, uint64_t n, const uint64_t *part,
                                                           uint64_t *out, const uint64_t *n_dev) {
    __shared__ uint64_t s[SCAN_BLOCK];
    n = count_of(n, n_dev);
    uint64_t i = (uint64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x;
    if (n == 0) {
        if (i == 0) out[0] = 0;
        return;
    }
    uint64_t v = i < n ? in[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < SCAN_BLOCK; o <<= 1) {
        uint64_t t = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    if (i < n) out[i] = part[blockIdx.x] + s[threadIdx.x] - v;
    if (i == n - 1) out[n] = part[blockIdx.x] + s[threadIdx.x];
}

// ------------------------------------------------------------------ locate

// per hit: number of positions to locate (width if <= max_occ, else 0)
__global__ void k_loc_count(uint64_t n_hits, const uint4 *hits, uint32_t max_occ, uint32_t *cnt,
                            const uint64_t *n_dev) {
    uint64_t h = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= count_of(n_hits, n_dev)) return;
    uint4 x = hits[h];
    uint64_t w = (uint64_t)x.y - x.x + 1;
    cnt[h] = (x.x <= x.y && w <= max_occ) ? (uint32_t)w : 0;
}

// position p of the located hits: its hit is the last h with poff[h] <= p
template <int LW>
__device__ void locate_one(const DevIndex &ix, uint64_t n_hits, const uint4 *hits, const uint64_t *poff, uint64_t p,
                           uint32_t *pos) {
    uint64_t lo = 0, hi = n_hits;
    while (hi - lo > 1) {
        uint64_t mid = (lo + hi) / 2;
        if (poff[mid] <= p) lo = mid;
        else hi = mid;
    }
    uint4 x = hits[lo];
    int strand = h_strand(x);
    const DevDir d = pick_dir(ix, strand == 0 ? 1 : 0);
    uint32_t j = x.x + (uint32_t)(p - poff[lo]);
    uint32_t steps = 0;
    const uint32_t smask = (1u << ix.sa_shift) - 1;
    uint32_t q;
    for (;;) {
        if (j == d.primary) { q = steps; break; }
        if ((j & smask) == 0) { q = d.sa[j >> ix.sa_shift] + steps; break; }
        j = lf_step<LW>(ix, d, j);
        steps++;
    }
    pos[p] = strand == 0 ? ix.n - q - (uint32_t)h_len(x) : q;
}

// one lane per position (grid-stride): find its hit, walk LF to a sampled row
template <int LW>
__global__ void k_loc_rows(DevIndex ix, uint64_t n_hits, const uint4 *hits, const uint64_t *poff, uint64_t total,
                           uint32_t *pos, const uint64_t *n_hits_dev, const uint64_t *total_dev) {
    n_hits = count_of(n_hits, n_hits_dev);
    total = count_of(total, total_dev);
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total;
         p += (uint64_t)gridDim.x * blockDim.x)
        locate_one<LW>(ix, n_hits, hits, poff, p, pos);
}
// sort each hit's positions: short segments by one lane, long ones by a
// workgroup running a bitonic network (pairs past the end count as +inf)
__global__ void k_sort_small(uint64_t n_hits, const uint64_t *poff, uint32_t *pos, uint32_t *big, uint32_t *n_big,
                             const uint64_t *n_dev) {
    uint64_t h = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= count_of(n_hits, n_dev)) return;
    uint64_t o = poff[h], w = poff[h + 1] - o;
    if (w <= 1) return;
    if (w > 32) {
        big[atomicAdd(n_big, 1u)] = (uint32_t)h;
        return;
    }
    uint32_t *a = pos + o;
    for (uint64_t i = 1; i < w; i++) {
        uint32_t v = a[i];
        uint64_t q = i;
        while (q > 0 && a[q - 1] > v) { a[q] = a[q - 1]; q--; }
        a[q] = v;
    }
}

__global__ __launch_bounds__(256) void k_sort_big(const uint64_t *poff, uint32_t *pos, const uint32_t *big,
                                                  const uint32_t *n_big) {
    __shared__ uint32_t s[4096];
    const uint32_t nb = *n_big;
    for (uint32_t b = blockIdx.x; b < nb; b += gridDim.x) {
        uint32_t h = big[b];
        uint64_t o = poff[h], n = poff[h + 1] - o;
        uint32_t *a = pos + o;
        const bool lds = n <= 4096;
        if (lds) {
            for (uint64_t i = threadIdx.x; i < n; i += blockDim.x) s[i] = a[i];
            __syncthreads();
        }
        uint32_t *x = lds ? s : a;
        for (uint64_t k = 2; k < 2 * n; k <<= 1) {
            for (uint64_t j = k >> 1; j > 0; j >>= 1) {
                for (uint64_t i = threadIdx.x; i < n; i += blockDim.x) {
                    uint64_t q = (j == (k >> 1)) ? (i ^ (k - 1)) : (i ^ j);
                    if (q > i && q < n && x[i] > x[q]) {
                        uint32_t t = x[i];
                        x[i] = x[q];
                        x[q] = t;
                    }
                }
                __syncthreads();
            }
        }
        if (lds) {
            for (uint64_t i = threadIdx.x; i < n; i += blockDim.x) a[i] = s[i];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ pairing

struct EndView {
    const uint64_t *hoff;
    const uint4 *hits;
    const uint64_t *poff;  // per hit, indexed by (hit index - hbase)
    const uint32_t *pos;
    uint64_t hbase;        // hoff[0]
};

__device__ __forceinline__ uint64_t lower_bound(const uint32_t *a, uint64_t n, uint64_t v) {
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        uint64_t mid = (lo + hi) / 2;
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// single-end primary: smallest (score, diffs, strand, pos, len)
__device__ bool se_primary(const EndView &e, uint32_t q, uint32_t &pos, uint4 &hit, bool &rep) {
    bool found = false;
    rep = false;
    for (uint64_t i = e.hoff[q]; i < e.hoff[q + 1]; i++) {
        uint64_t o = e.poff[i - e.hbase], w = e.poff[i - e.hbase + 1] - o;
        if (w == 0) { rep = true; continue; }
        uint4 h = e.hits[i];
        uint32_t p = e.pos[o];  // sorted: the first is the smallest
        bool b;
        if (!found) b = true;
        else if (h_score(h) != h_score(hit)) b = h_score(h) < h_score(hit);
        else if (h_diffs(h) != h_diffs(hit)) b = h_diffs(h) < h_diffs(hit);
        else if (h_strand(h) != h_strand(hit)) b = h_strand(h) < h_strand(hit);
        else if (p != pos) b = p < pos;
        else b = h_len(h) < h_len(hit);
        if (b) { found = true; pos = p; hit = h; }
    }
    return found;
}

// One lane per pair.  With n_dev, the pair count is read on the device and
// end 2's reads follow end 1's in one batch (its offsets start at
// e1.hoff + n); a nonzero *err (an output was too small) writes nothing.
__global__ void k_pair(uint32_t n_pairs, EndView e1, EndView e2, int paired, int32_t lo, int32_t hi, int32_t mu,
                       bwfm_pair *out, const uint64_t *n_dev, const uint32_t *err) {
    uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (err && *err) return;
    if (n_dev) {
        n_pairs = (uint32_t)count_of(n_pairs, n_dev);
        e2.hoff = e1.hoff + n_pairs;
    }
    if (q >= n_pairs) return;
    bwfm_pair o;
    memset(&o, 0, sizeof(o));
    o.pos1 = o.pos2 = 0xffffffffu;
    bool found = false;
    int64_t bs = 0, bd = 0, bpf = 0;
    if (paired) {
        for (uint64_t i = e1.hoff[q]; i < e1.hoff[q + 1]; i++) {
            uint4 h1 = e1.hits[i];
            const uint32_t *P1 = e1.pos + e1.poff[i - e1.hbase];
            uint64_t n1 = e1.poff[i - e1.hbase + 1] - e1.poff[i - e1.hbase];
            for (uint64_t j = e2.hoff[q]; j < e2.hoff[q + 1]; j++) {
                uint4 h2 = e2.hits[j];
                if (h_strand(h1) == h_strand(h2)) continue;
                const uint32_t *P2 = e2.pos + e2.poff[j - e2.hbase];
                uint64_t n2 = e2.poff[j - e2.hbase + 1] - e2.poff[j - e2.hbase];
                int64_t s = (int64_t)h_score(h1) + h_score(h2);
                for (uint64_t x = 0; x < n1; x++) {
                    int64_t p1 = P1[x];
                    // range of end-2 positions forming a proper pair with p1
                    int64_t a, b;
                    if (h_strand(h1) == 0) {  // end 1 is +: pf = p1, pr = p2, lr = len2
                        int64_t lr = h_len(h2);
                        a = p1 + lo - lr > p1 ? p1 + lo - lr : p1;
                        b = p1 + hi - lr;
                    } else {  // end 1 is -: pr = p1, lr = len1, pf = p2
                        int64_t lr = h_len(h1);
                        a = p1 + lr - hi;
                        b = p1 + lr - lo < p1 ? p1 + lr - lo : p1;
                    }
                    if (b < a || b < 0) continue;
                    uint64_t y = lower_bound(P2, n2, (uint64_t)(a < 0 ? 0 : a));
                    for (; y < n2 && (int64_t)P2[y] <= b; y++) {
                        int64_t p2 = P2[y];
                        int64_t pf = h_strand(h1) == 0 ? p1 : p2;
                        int64_t pr = h_strand(h1) == 0 ? p2 : p1;
                        int64_t lr = h_strand(h1) == 0 ? h_len(h2) : h_len(h1);
                        int64_t ins = pr + lr - pf;
                        int64_t d = ins > mu ? ins - mu : mu - ins;
                        bool bt;
                        if (!found) bt = true;
                        else if (s != bs) bt = s < bs;
                        else if (d != bd) bt = d < bd;
                        else if (pf != bpf) bt = pf < bpf;
                        else if ((uint32_t)h_strand(h1) != o.strand1) bt = (uint32_t)h_strand(h1) < o.strand1;
                        else if ((uint32_t)p1 != o.pos1) bt = (uint32_t)p1 < o.pos1;
                        else if ((uint32_t)h_len(h1) != o.len1) bt = (uint32_t)h_len(h1) < o.len1;
                        else if ((uint32_t)p2 != o.pos2) bt = (uint32_t)p2 < o.pos2;
                        else bt = (uint32_t)h_len(h2) < o.len2;
                        if (bt) {
                            found = true;
                            bs = s;
                            bd = d;
                            bpf = pf;
                            o.pos1 = (uint32_t)p1;
                            o.pos2 = (uint32_t)p2;
                            o.len1 = (uint16_t)h_len(h1);
                            o.len2 = (uint16_t)h_len(h2);
                            o.score1 = (uint16_t)h_score(h1);
                            o.score2 = (uint16_t)h_score(h2);
                            o.strand1 = (uint8_t)h_strand(h1);
                            o.strand2 = (uint8_t)h_strand(h2);
                            o.insert = (int32_t)ins;
                        }
                    }
                }
            }
        }
    }
    uint32_t pp;
    uint4 hp;
    bool rep1 = false, rep2 = false;
    bool f1 = se_primary(e1, q, pp, hp, rep1);
    if (found) {
        o.flags = BWFM_PF_PAIRED | BWFM_PF_MAPPED1 | BWFM_PF_MAPPED2;
    } else if (f1) {
        o.pos1 = pp;
        o.len1 = (uint16_t)h_len(hp);
        o.score1 = (uint16_t)h_score(hp);
        o.strand1 = (uint8_t)h_strand(hp);
        o.flags |= BWFM_PF_MAPPED1;
    }
    if (paired) {
        bool f2 = se_primary(e2, q, pp, hp, rep2);
        if (!found && f2) {
            o.pos2 = pp;
            o.len2 = (uint16_t)h_len(hp);
            o.score2 = (uint16_t)h_score(hp);
            o.strand2 = (uint8_t)h_strand(hp);
            o.flags |= BWFM_PF_MAPPED2;
        }
    }
    if (rep1) o.flags |= BWFM_PF_REP1;
    if (rep2) o.flags |= BWFM_PF_REP2;
    out[q] = o;
}


// ------------------------------------------------------------------ short-string table

// Level d of direction `which`'s table from level d - 1: one thread per
// string S of d - 1 bases writes the intervals of aS, a = 0..3, from the
// rank counts at S's k and l + 1 (the same step the search takes).
template <int LW>
__global__ __launch_bounds__(256) void k_kt_level(DevIndex ix, int which, int d) {
    const uint64_t p = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (p >= ((uint64_t)1 << (2 * (d - 1)))) return;
    const DevDir dd = pick_dir(ix, which);
    uint32_t *kt = const_cast<uint32_t *>(dd.kt);
    const uint64_t pe = kt_level_start(d - 1) + p;
    const uint32_t k = kt[2 * pe], l = kt[2 * pe + 1];
    uint32_t ok[4], ol[4];
    occ4<LW>(ix, dd, k, ok);
    occ4<LW>(ix, dd, l + 1, ol);
    uint4 *dst = reinterpret_cast<uint4 *>(kt + 2 * kt_children(d - 1, (uint32_t)p));
    dst[0] = make_uint4(dd.C[0] + ok[0], dd.C[0] + ol[0] - 1, dd.C[1] + ok[1], dd.C[1] + ol[1] - 1);
    dst[1] = make_uint4(dd.C[2] + ok[2], dd.C[2] + ol[2] - 1, dd.C[3] + ok[3], dd.C[3] + ol[3] - 1);
}

// level 0: the empty string's interval (0, n)
__global__ void k_kt_root(uint32_t *kt, uint32_t n) {
    if (threadIdx.x == 0) {
        kt[0] = 0;
        kt[1] = n;
    }
}

// ------------------------------------------------------------------ random-line probe

// Each lane performs `iters` dependent fetches of whole lines at
// pseudo-random line indices; the next index depends on the data just read,
// as in the search's pointer chase.  Every index is reduced into
// [0, n_lines), so any buffer contents are safe.
template <int LW>
__global__ __launch_bounds__(256) void k_probe_gather(const uint4 *buf, uint64_t n_lines, uint32_t iters,
                                                      uint32_t *sink) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t x = 0x9E3779B97F4A7C15ULL * (t + 1);
    uint32_t acc = 0;
    for (uint32_t it = 0; it < iters; it++) {
        x ^= x >> 31;
        x *= 0xBF58476D1CE4E5B9ULL;
        x ^= x >> 29;
        const uint64_t line = __umul64hi(x, n_lines);
        const uint4 *L = buf + line * (LW / 4);
#pragma unroll
        for (int q = 0; q < LW / 4; q++) {
            uint4 v = L[q];
            acc += v.x ^ v.y ^ v.z ^ v.w;
        }
        x += acc;
    }
    sink[t] = acc;
}

// ------------------------------------------------------------------ host helpers

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(BWFM_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

inline uint32_t blocks(uint64_t n, uint32_t b) { return (uint32_t)((n + b - 1) / b); }

// ------------------------------------------------------------------ kernel timing

struct TimingStore {
    std::mutex mu;
    bool on = false;
    std::map<std::string, std::pair<double, uint64_t>> acc;
};
TimingStore &timing() {
    static TimingStore t;
    return t;
}

// Events around the launches of one API call; resolved when the call has
// synchronised its stream.
struct CallTimer {
    struct Rec {
        const char *name;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    bool on;
    hipStream_t st;
    explicit CallTimer(hipStream_t s, bool allowed = true) : on(false), st(s) {
        if (!allowed) return;  // callers that must not create events
        std::lock_guard<std::mutex> g(timing().mu);
        on = timing().on;
    }
    int begin(const char *name) {
        if (!on) return -1;
        Rec r{name, nullptr, nullptr};
        if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return -1;
        (void)hipEventRecord(r.a, st);
        recs.push_back(r);
        return (int)recs.size() - 1;
    }
    void end(int i) {
        if (i >= 0) (void)hipEventRecord(recs[i].b, st);
    }
    ~CallTimer() {
        if (recs.empty()) return;
        (void)hipStreamSynchronize(st);
        std::lock_guard<std::mutex> g(timing().mu);
        for (auto &r : recs) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                auto &e = timing().acc[r.name];
                e.first += ms;
                e.second += 1;
            }
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
    }
};

DevIndex dev_index(const bwfm_index *ix) {
    DevIndex d;
    memset(&d, 0, sizeof(d));
    for (int k = 0; k < 2; k++) {
        d.dir[k].lines = (const uint32_t *)ix->d_lines[k];
        d.dir[k].sa = (const uint32_t *)ix->d_sa[k];
        for (int a = 0; a < 4; a++) d.dir[k].C[a] = (uint32_t)ix->dir[k].C[a];
        d.dir[k].primary = (uint32_t)ix->dir[k].primary;
        d.dir[k].kt = (const uint32_t *)ix->d_kt[k];
    }
    d.kt_levels = ix->kt_levels;
    d.magic = (uint64_t)(((unsigned __int128)1 << 64) / ix->bpl) + 1;
    d.n = (uint32_t)ix->n;
    d.bpl = ix->bpl;
    uint32_t s = 0;
    while ((1u << s) < ix->sa_sample) s++;
    d.sa_shift = s;
    d.line_words = ix->line_bytes / 4;
    return d;
}

Params make_params(const bwfm_aln_params &p) {
    Params P;
    P.max_diff = p.max_diff;
    P.max_gapo = p.max_gapo;
    P.max_gape = p.max_gape;
    P.seed_len = p.seed_len;
    P.seed_diff = p.seed_diff;
    P.ies = p.indel_end_skip;
    P.s_mm = p.s_mm;
    P.s_gapo = p.s_gapo;
    P.s_gape = p.s_gape;
    P.mode = p.mode;
    P.max_best = p.max_best;
    P.max_hits = p.max_hits;
    P.minc = std::min(p.s_mm, std::min(p.s_gapo, p.s_gape));
    (void)p.form;
    P.s1 = std::max(p.indel_end_skip, 1);
    return P;
}

// The workspace of a stream on this index, created on first use.
bwfm::Workspace &stream_ws(bwfm_index *ix, hipStream_t st) {
    std::lock_guard<std::mutex> g(ix->ws_mu);
    auto &w = ix->ws[(void *)st];
    if (!w) w.reset(new bwfm::Workspace());
    return *w;
}

// Grow a workspace buffer to at least `bytes` (grow-only).  The stream's
// earlier work may still read the old buffer, so it is drained first.
int ws_grow(void *&ptr, size_t &have, size_t bytes, hipStream_t st) {
    if (have >= bytes && ptr) return BWFM_OK;
    if (ptr) {
        HIPCHK(hipStreamSynchronize(st));
        (void)hipFree(ptr);
    }
    ptr = nullptr;
    have = 0;
    const size_t want = std::max<size_t>(bytes + bytes / 8, 4096);
    if (hipMalloc(&ptr, want) != hipSuccess) {
        ptr = nullptr;
        (void)hipGetLastError();
        return fail(BWFM_E_NOMEM, "workspace allocation of " + std::to_string(want) + " bytes failed");
    }
    have = want;
    return BWFM_OK;
}

int ws_reserve(bwfm::Workspace &w, size_t bytes, hipStream_t st, void **out) {
    if (int rc = ws_grow(w.ptr, w.bytes, bytes, st)) return rc;
    *out = w.ptr;
    return BWFM_OK;
}

struct Carver {
    char *p;
    size_t used = 0;
    template <typename T>
    T *take(size_t n) {
        used = (used + 255) & ~size_t(255);
        T *r = reinterpret_cast<T *>(p + used);
        used += n * sizeof(T);
        return r;
    }
};

// Exclusive scan of n u32 counts into n + 1 u64 offsets (out[n] = total).
// With n_dev the count is read on the device (at most n; the grid covers n).
int scan_counts(const uint32_t *cnt, uint64_t n, uint64_t *out, uint64_t *part, hipStream_t st,
                const uint64_t *n_dev = nullptr) {
    uint64_t nb = (n + SCAN_BLOCK - 1) / SCAN_BLOCK;
    if (n == 0) {
        k_fill_u32<<<1, 64, 0, st>>>(reinterpret_cast<uint32_t *>(out), 2, 0u);
        HIPCHK(hipGetLastError());
        return BWFM_OK;
    }
    k_scan_reduce<<<(uint32_t)nb, SCAN_BLOCK, 0, st>>>(cnt, n, part, n_dev);
    k_scan_parts<<<1, SCAN_BLOCK, 0, st>>>(part, nb);
    k_scan_apply<<<(uint32_t)nb, SCAN_BLOCK, 0, st>>>(cnt, n, part, out, n_dev);
    HIPCHK(hipGetLastError());
    return BWFM_OK;
}

size_t scan_part_elems(uint64_t n) { return (n + SCAN_BLOCK - 1) / SCAN_BLOCK + 1; }

// Lanes of a persistent grid that fit on the device at once, for a block
// size and its dynamic LDS, at most waves_per_simd waves per SIMD (0 = no
// cap; a CU has 4 SIMDs).
template <int LW>
uint32_t persistent_lanes(uint32_t bs, size_t lds, int waves_per_simd, bool dp = false) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persistent_kernel<LW>(waves_per_simd, dp), (int)bs, lds) !=
            hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    if (waves_per_simd > 0) {
        const int cap = std::max(1, waves_per_simd * 4 * 64 / (int)bs);
        per_cu = std::min(per_cu, cap);
    }
    return (uint32_t)cus * (uint32_t)per_cu * bs;
}

// LDS bytes per lane for reads up to mlen bases (an odd number of dwords,
// which spreads the lanes' rows over the banks) and the largest block that
// keeps a block's LDS (rows plus the per-wave sharing blocks) within 64 KB.
inline uint32_t lds_stride_for(uint32_t mlen) {
    uint32_t dw = (mlen + 3) / 4;
    if ((dw & 1) == 0) dw++;
    return dw * 4;
}
inline uint32_t block_for(uint32_t stride) {
    uint32_t bs = BLOCK;
    while (bs > 64 && (size_t)bs * stride + (bs / 64) * sizeof(WaveShare) > 65536) bs /= 2;
    return bs;
}

constexpr uint32_t SLOW_LANES = BWFM_SLOW_LANES;  // most lanes of the second pass
constexpr uint32_t SPLIT_DEFAULT = 16384;         // split budget unless the caller sets one

// Expansions between splits for a parameter block; 0: no splitting (the
// plain form never splits).
inline uint32_t split_budget_of(const bwfm_aln_params &p) {
    if (p.form == BWFM_FORM_PLAIN || p.split_budget < 0) return 0;
    return p.split_budget == 0 ? SPLIT_DEFAULT : (uint32_t)p.split_budget;
}

// Room of the split searches for a batch of n reads of at most mlen bases:
// a slot for one read in eight (at least 64, at most 2^26) and sixteen task entries a
// read (at least 4096, at most 2^26) per generation.  A split hands out a
// few hundred entries on long reads.  Running out is not an error: a read
// or task that finds no room goes on alone.
struct SplitShape {
    uint32_t slot_cap, task_cap, dstride;
};
inline SplitShape split_shape(uint32_t n, uint32_t mlen) {
    SplitShape z;
    z.slot_cap = std::min<uint32_t>(std::min<uint32_t>(std::max<uint32_t>(n, 1), std::max<uint32_t>(64, n / 8)), 1u << 26);
    z.task_cap = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(16ull * n, 4096), 1ull << 26);
    z.dstride = ((mlen + 15) / 16) * 16;
    return z;
}
inline size_t split_bytes(const SplitShape &z) {
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    return 9 * al((size_t)z.slot_cap * 4) + al((size_t)z.slot_cap * 2 * z.dstride) +
           al((size_t)z.slot_cap * SLOT_HITS * 16) + 2 * al((size_t)z.task_cap * 16) + 2 * al((size_t)z.task_cap * 4) +
           al(SPLIT_CTL * 4) + al(sizeof(TaskArgs)) + 256;
}
inline SplitBufs carve_split(Carver &cv, const SplitShape &z, uint32_t budget, TaskArgs **targs) {
    SplitBufs X{};
    X.slot_read = cv.take<uint32_t>(z.slot_cap);
    X.slot_meta = cv.take<uint32_t>(z.slot_cap);
    X.slot_best = cv.take<int>(z.slot_cap);
    X.slot_nhit = cv.take<uint32_t>(z.slot_cap);
    X.slot_fail = cv.take<uint32_t>(z.slot_cap);
    X.slot_exp = cv.take<uint32_t>(z.slot_cap);
    X.slot_owner = cv.take<uint32_t>(z.slot_cap);
    X.slot_own = cv.take<uint32_t>(z.slot_cap);
    X.slot_obest = cv.take<int>(z.slot_cap);
    X.slot_rows = cv.take<uint8_t>((size_t)z.slot_cap * 2 * z.dstride);
    X.slot_hits = cv.take<uint4>((size_t)z.slot_cap * SLOT_HITS);
    for (int k = 0; k < 2; k++) {
        X.tasks[k] = cv.take<uint4>(z.task_cap);
        X.task_ref[k] = cv.take<uint32_t>(z.task_cap);
    }
    X.ctl = cv.take<uint32_t>(SPLIT_CTL);
    *targs = cv.take<TaskArgs>(1);
    X.slot_cap = z.slot_cap;
    X.task_cap = z.task_cap;
    X.dstride = z.dstride;
    X.budget = budget;
    return X;
}

// Lanes of the task rounds' grid (blocks of BLOCK lanes, no LDS): as many
// as fit on the device at once, but at most sixteen per read of the batch
// (n_up lanes) or the first pass's lanes, whichever is more, since they
// all need lane buffers.
template <int LW>
uint32_t task_lanes(uint32_t n_up, uint32_t lanes) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_align_tasks<LW>, (int)BLOCK, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const uint64_t fit = (uint64_t)cus * (uint64_t)per_cu * BLOCK;
    const uint64_t want = std::max<uint64_t>(lanes, ((16ull * n_up + BLOCK - 1) / BLOCK) * BLOCK);
    return (uint32_t)std::max<uint64_t>(std::min(fit, want), BLOCK);
}

// After the first pass (split searches on): the collection of the split
// reads' first-pass hits, the task rounds on their own grid of tlanes
// lanes, on the first pass's lane buffers (allocated for both grids), the
// last round without a drain, then the publication of the split reads.  Every launch reads its counts on the device, so the
// sequence can be captured.
template <int LW>
void enqueue_split(const DevIndex &D, const Params &P, const SplitBufs &X, TaskArgs *targs, const LaneBufs &lb,
                   const ReadOut &O, uint32_t tlanes, hipStream_t st) {
    SplitBufs Xc = X;
    Xc.lane_cand = lb.cand;
    k_split_collect<<<blocks(X.slot_cap, 256), 256, 0, st>>>(Xc);
    k_set_task_args<<<1, 64, 0, st>>>(targs, TaskArgs{lb, X});
    for (uint32_t g = 0; g < (uint32_t)SPLIT_ROUNDS; g++)
        k_align_tasks<LW><<<tlanes / BLOCK, BLOCK, 0, st>>>(D, P, targs, g, g + 1 < (uint32_t)SPLIT_ROUNDS ? 1u : 0u);
    k_split_publish<<<blocks(X.slot_cap, 256), 256, 0, st>>>(P, X, O);
}

template <int LW>
int align_impl(bwfm_index *ix, bwfm::Workspace &ws, const bwfm_reads *rd, const bwfm_aln_params *p,
               bwfm_aln_result *res, hipStream_t st, uint32_t *expand, uint64_t *work = nullptr) {
    const uint32_t n = rd->n_reads;
    const DevIndex D = dev_index(ix);
    const Params P = make_params(*p);
    ReadsView rv{rd->bases, rd->offsets, rd->lengths, rd->max_diff, rd->n_reads, rd->max_len, nullptr};
    const uint32_t mlen = std::max<uint32_t>(rd->max_len, 1);
    const uint32_t worst_stack = 8 * (mlen + BWFM_MAX_DIFF) + 1;  // never overflows
    const uint32_t lstride = lds_stride_for(mlen);
    const bool plain = p->form == BWFM_FORM_PLAIN;
    const uint32_t sbud = plain ? 0u : split_budget_of(*p);  // split searches (batched form)
    // the D-array pre-pass (batched form, long reads or when that gene is on)
    const bool dpre = !plain && (BWFM_GENE_DPREPASS == 1 || mlen >= DPRE_MIN_LEN);
    const uint32_t bs = block_for(lstride);
    const size_t lds = (size_t)bs * lstride + (plain ? 0 : (bs / 64) * sizeof(WaveShare));
    const uint32_t nr_up = ((std::max<uint32_t>(n, 1) + bs - 1) / bs) * bs;
    const uint32_t lanes =
        plain ? nr_up : std::min<uint32_t>(persistent_lanes<LW>(bs, lds, p->waves_per_simd, dpre), nr_up);
    const uint32_t stack_cap = plain ? std::min<uint32_t>(worst_stack, PLAIN_STACK) : worst_stack;
    // the task rounds' grid shares the lane buffers: room for the larger one
    const uint32_t tlanes = sbud ? task_lanes<LW>(nr_up, lanes) : 0u;
    const uint32_t blanes = std::max(lanes, tlanes);
    // the staging arena holds the reported hits of every read: as many as
    // the output can take
    const uint64_t stage_cap = res->hit_capacity;
    const uint32_t slow_lanes = std::min<uint32_t>(nr_up, SLOW_LANES);
    const uint32_t scap = P.max_hits + 1;
    size_t need = (size_t)blanes * stack_cap * 16 + (size_t)blanes * FAST_CAND * 16;
    need += (size_t)slow_lanes * worst_stack * 16 + (size_t)slow_lanes * scap * 16;
    need += (size_t)n * 4 * 2 + (size_t)n * 8 + stage_cap * 16 + scan_part_elems(n) * 8 + 16 * 256;
    need += sizeof(PersistentArgs) + 256;
    // the D-array pre-pass's rows
    const uint32_t dstride = ((mlen + 15) / 16) * 16;
    if (dpre) need += (size_t)n * 2 * dstride + n + 2 * 256;
    const SplitShape zs = split_shape(n, mlen);
    if (sbud) need += split_bytes(zs) + (size_t)lanes * 4 + 256;
    void *w;
    int rc = ws_reserve(ws, need, st, &w);
    if (rc) return rc;
    Carver cv{(char *)w};
    uint4 *lstack = cv.take<uint4>((size_t)blanes * stack_cap);
    uint4 *lcand = cv.take<uint4>((size_t)blanes * FAST_CAND);
    uint4 *sstack = cv.take<uint4>((size_t)slow_lanes * worst_stack);
    uint4 *scand = cv.take<uint4>((size_t)slow_lanes * scap);
    uint32_t *n_rep = cv.take<uint32_t>(n);
    uint32_t *slow_list = cv.take<uint32_t>(n);
    uint64_t *stage_off = cv.take<uint64_t>(n);
    uint4 *stage = cv.take<uint4>(stage_cap);
    uint64_t *part = cv.take<uint64_t>(scan_part_elems(n));
    PersistentArgs *pargs = cv.take<PersistentArgs>(1);
    uint8_t *drows = dpre ? cv.take<uint8_t>((size_t)n * 2 * dstride) : nullptr;
    uint8_t *dflag = dpre ? cv.take<uint8_t>(n) : nullptr;
    TaskArgs *targs = nullptr;
    SplitBufs X = sbud ? carve_split(cv, zs, sbud, &targs) : SplitBufs{};
    X.count = expand != nullptr;
    uint32_t *lane_read = sbud ? cv.take<uint32_t>(lanes) : nullptr;
    uint32_t *ctl = cv.take<uint32_t>(16);  // n_slow, next_read, stage_used (64-bit), slow_next
    uint32_t *n_slow = ctl, *next_read = ctl + 1, *slow_next = ctl + 4;
    unsigned long long *stage_used = reinterpret_cast<unsigned long long *>(ctl + 2);
    k_fill_u32<<<1, 64, 0, st>>>(ctl, 16, 0u);
    // plain lanes start together and stay roughly in step: interleave their
    // buffers; persistent lanes drift apart: give each a contiguous run
    LaneBufs lb = plain ? LaneBufs{lstack, lcand, 1, lanes, stack_cap, 1, lanes, FAST_CAND, lstride}
                        : LaneBufs{lstack, lcand, stack_cap, 1, stack_cap, FAST_CAND, 1, FAST_CAND, lstride};
    ReadOut O{n_rep,     res->c1,   res->c2,   res->status, slow_list,
              n_slow,    stage,     stage_used, stage_cap,  stage_off,
              expand,    reinterpret_cast<unsigned long long *>(work)};
    if (work) k_fill_u32<<<1, 64, 0, st>>>(reinterpret_cast<uint32_t *>(work), 2 * (6 + SPLIT_ROUNDS), 0u);
    if (sbud) k_fill_u32<<<1, 64, 0, st>>>(X.ctl, SPLIT_CTL, 0u);
    CallTimer tm(st);
    if (n) {
        if (plain) {
            int t = tm.begin("align_plain");
            k_align_plain<LW><<<nr_up / bs, bs, lds, st>>>(D, rv, P, lb, O);
            tm.end(t);
        } else {
            if (dpre) {
                int td = tm.begin("dscan");
                k_dscan<LW><<<nr_up / bs, bs, (size_t)bs * lstride, st>>>(D, rv, P, drows, dflag, dstride, lstride);
                tm.end(td);
            }
            k_set_args<<<1, 64, 0, st>>>(pargs, PersistentArgs{rv, lb, O, next_read, drows, dflag, dstride, X, lane_read});
            int ts = tm.begin("align_search");
            int t = tm.begin("align_persistent");
            hipLaunchKernelGGL(persistent_kernel<LW>(p->waves_per_simd, dpre), dim3(lanes / bs), dim3(bs), lds, st, D, P,
                               (const PersistentArgs *)pargs);
            tm.end(t);
            if (sbud) {
                int tt = tm.begin("align_tasks");
                enqueue_split<LW>(D, P, X, targs, lb, O, tlanes, st);
                tm.end(tt);
            }
            tm.end(ts);
        }
        // the second pass reads its count on the device: no host round trip
        const size_t slds = (size_t)bs * lstride;
        LaneBufs sb{sstack, scand, worst_stack, 1, worst_stack, scap, 1, scap, lstride};
        int t = tm.begin("align_slow");
        k_align_slow<LW><<<slow_lanes / bs, bs, slds, st>>>(D, rv, P, sb, O, slow_next);
        tm.end(t);
        if (work && sbud)
            k_split_stats<<<blocks(X.slot_cap, 256), 256, 0, st>>>(X, reinterpret_cast<unsigned long long *>(work));
        HIPCHK(hipGetLastError());
    }
    rc = scan_counts(n_rep, n, res->hit_offsets, part, st);
    if (rc) return rc;
    uint64_t total = 0;
    HIPCHK(hipMemcpyAsync(&total, res->hit_offsets + n, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (total > res->hit_capacity)
        return fail(BWFM_E_CAPACITY, "hit capacity " + std::to_string(res->hit_capacity) + " < " + std::to_string(total));
    if (n && total) {
        int t = tm.begin("compact");
        k_compact<<<blocks(n, 256), 256, 0, st>>>(n, res->hit_offsets, stage, stage_off,
                                                  reinterpret_cast<uint4 *>(res->hits), nullptr, nullptr);
        tm.end(t);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipStreamSynchronize(st));
    return BWFM_OK;
}

// positions of all hits of one result; pos_off has n_hits + 1 entries
template <int LW>
int locate_impl(bwfm_index *ix, uint64_t n_hits, const uint4 *hits, uint32_t max_occ, uint64_t *pos_off,
                uint32_t *pos, uint64_t cap, uint32_t *cnt, uint64_t *part, uint32_t *big, uint32_t *n_big,
                hipStream_t st, uint64_t *total_out, bool timed = true) {
    const DevIndex D = dev_index(ix);
    if (n_hits) {
        k_loc_count<<<blocks(n_hits, 256), 256, 0, st>>>(n_hits, hits, max_occ, cnt, nullptr);
        HIPCHK(hipGetLastError());
    }
    int rc = scan_counts(cnt, n_hits, pos_off, part, st);
    if (rc) return rc;
    uint64_t total = 0;
    HIPCHK(hipMemcpyAsync(&total, pos_off + n_hits, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *total_out = total;
    if (total > cap) return fail(BWFM_E_CAPACITY, "position capacity too small");
    if (total) {
        CallTimer tm(st, timed);
        int t = tm.begin("locate_rows");
        k_loc_rows<LW><<<(uint32_t)std::min<uint64_t>(blocks(total, 256), 65536), 256, 0, st>>>(D, n_hits, hits, pos_off, total,
                                                                                            pos, nullptr, nullptr);
        tm.end(t);
        HIPCHK(hipGetLastError());
        k_fill_u32<<<1, 64, 0, st>>>(n_big, 1, 0u);
        t = tm.begin("sort");
        k_sort_small<<<blocks(n_hits, 256), 256, 0, st>>>(n_hits, pos_off, pos, big, n_big, nullptr);
        k_sort_big<<<1024, 256, 0, st>>>(pos_off, pos, big, n_big);
        tm.end(t);
        HIPCHK(hipGetLastError());
    }
    return BWFM_OK;
}

bool check_index(const bwfm_index *ix) { return ix && ix->device >= 0; }

// result buffers: per-read arrays may be NULL only for an empty batch
int check_result(const bwfm_aln_result *r, uint32_t n) {
    return r && r->hit_offsets && (n == 0 || (r->c1 && r->c2 && r->status)) && (r->hits || r->hit_capacity == 0);
}

}  // namespace

// Call f with the index's rank-line format as a compile-time tag.
template <class F> auto by_layout(const bwfm_index *ix, F &&f) {
    if (ix->rank_format == BWFM_RANK_SUBCOUNTS) return f(std::integral_constant<int, LW_SUB>());
    if (ix->rank_format == BWFM_RANK_SUB128) return f(std::integral_constant<int, LW_SUB128>());
    if (ix->line_bytes == 128) return f(std::integral_constant<int, 32>());
    if (ix->line_bytes == 32) return f(std::integral_constant<int, 8>());
    return f(std::integral_constant<int, 16>());
}

// ===================================================================== C ABI

extern "C" int bwfm_index_upload(bwfm_index *ix, void *stream) {
    if (!ix) return fail(BWFM_E_INVAL, "upload: NULL index");
    std::unique_lock<std::shared_mutex> g(ix->mu);
    if (ix->device >= 0) return BWFM_OK;
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    uint64_t bytes = 0;
    for (int d = 0; d < 2; d++) {
        size_t lb = ix->dir[d].lines.size() * 4, sb = ix->dir[d].sa.size() * 4;
        if (hipMalloc(&ix->d_lines[d], lb) != hipSuccess || hipMalloc(&ix->d_sa[d], sb) != hipSuccess)
            return fail(BWFM_E_NOMEM, "index upload: device allocation failed");
        HIPCHK(hipMemcpyAsync(ix->d_lines[d], ix->dir[d].lines.data(), lb, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(ix->d_sa[d], ix->dir[d].sa.data(), sb, hipMemcpyHostToDevice, st));
        bytes += lb + sb;
    }
    const size_t pb = std::max<size_t>(ix->pac.size(), 1) * 4;
    if (hipMalloc(&ix->d_pac, pb) != hipSuccess) return fail(BWFM_E_NOMEM, "index upload: device allocation failed");
    if (!ix->pac.empty())
        HIPCHK(hipMemcpyAsync(ix->d_pac, ix->pac.data(), ix->pac.size() * 4, hipMemcpyHostToDevice, st));
    bytes += pb;
    HIPCHK(hipStreamSynchronize(st));
    ix->device_bytes = bytes;
    ix->device = dev;
    return BWFM_OK;
}

// table bytes per direction, padded to a multiple of 256 so that a lane's
// line-sized, line-aligned read around its 32 entry bytes stays inside
static uint64_t kt_bytes(uint32_t levels) {
    return levels ? (kt_level_start((int)levels + 1) * 8 + 255) / 256 * 256 : 0;
}

extern "C" int bwfm_index_kmer_table(bwfm_index *ix, int levels, void *stream) {
    if (!ix) return fail(BWFM_E_INVAL, "kmer_table: NULL index");
    std::unique_lock<std::shared_mutex> g(ix->mu);
    if (ix->device < 0) return fail(BWFM_E_INVAL, "kmer_table: the index is not uploaded");
    if (levels < -1 || levels > 15) return fail(BWFM_E_INVAL, "kmer_table: levels must be -1, 0 or 1..15");
    if (levels == -1) {
        levels = 1;
        while (levels < 14 && ((uint64_t)1 << (2 * levels)) < ix->n) levels++;
    }
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipStreamSynchronize(st));
    ix->device_bytes -= 2 * kt_bytes(ix->kt_levels);
    ix->kt_levels = 0;
    ix->kt_gen++;
    for (int d = 0; d < 2; d++) {
        if (ix->d_kt[d]) (void)hipFree(ix->d_kt[d]);
        ix->d_kt[d] = nullptr;
    }
    if (levels == 0) return BWFM_OK;
    const uint64_t bytes = kt_bytes((uint32_t)levels);
    for (int d = 0; d < 2; d++)
        if (hipMalloc(&ix->d_kt[d], bytes) != hipSuccess) {
            for (int e = 0; e < 2; e++) {
                if (ix->d_kt[e]) (void)hipFree(ix->d_kt[e]);
                ix->d_kt[e] = nullptr;
            }
            (void)hipGetLastError();
            return fail(BWFM_E_NOMEM, "kmer_table: device allocation failed");
        }
    const DevIndex D = dev_index(ix);  // kt_levels 0: the builder reads rank lines only
    for (int d = 0; d < 2; d++) {
        k_kt_root<<<1, 64, 0, st>>>((uint32_t *)ix->d_kt[d], (uint32_t)ix->n);
        for (int lv = 1; lv <= levels; lv++) {
            const uint64_t np = (uint64_t)1 << (2 * (lv - 1));
            by_layout(ix, [&](auto t) {
                k_kt_level<decltype(t)::value><<<blocks(np, 256), 256, 0, st>>>(D, d, lv);
                return 0;
            });
        }
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    ix->kt_levels = (uint32_t)levels;
    ix->device_bytes += 2 * bytes;
    return BWFM_OK;
}

extern "C" int bwfm_index_kmer_get(const bwfm_index *ix, int which, int level, uint64_t first, uint64_t count,
                                   uint32_t *out) {
    if (!ix || !out || (which != 0 && which != 1)) return fail(BWFM_E_INVAL, "kmer_get: bad argument");
    if (level < 0 || (uint32_t)level > ix->kt_levels || !ix->d_kt[which])
        return fail(BWFM_E_INVAL, "kmer_get: no such table level");
    const uint64_t codes = (uint64_t)1 << (2 * level);
    if (first > codes || count > codes - first) return fail(BWFM_E_INVAL, "kmer_get: codes out of range");
    if (!count) return BWFM_OK;
    const char *src = (const char *)ix->d_kt[which] + (kt_level_start(level) + first) * 8;
    HIPCHK(hipMemcpy(out, src, count * 8, hipMemcpyDeviceToHost));
    return BWFM_OK;
}

extern "C" void bwfm_index_free(bwfm_index *ix) {
    if (!ix) return;
    for (int d = 0; d < 2; d++) {
        if (ix->d_lines[d]) (void)hipFree(ix->d_lines[d]);
        if (ix->d_sa[d]) (void)hipFree(ix->d_sa[d]);
        if (ix->d_kt[d]) (void)hipFree(ix->d_kt[d]);
    }
    if (ix->d_pac) (void)hipFree(ix->d_pac);
    for (auto &kv : ix->ws) {
        if (kv.second->ptr) (void)hipFree(kv.second->ptr);
        if (kv.second->pos) (void)hipFree(kv.second->pos);
    }
    delete ix;
}

// Search parameters in range; 0 or a bwfm_err.
static int check_aln_params(const bwfm_aln_params *p) {
    if (p->max_diff < 0 || p->max_diff > BWFM_MAX_DIFF || p->max_gapo < 0 || p->seed_len < 0 || p->seed_diff < 0 ||
        p->indel_end_skip < 0 || p->s_mm < 0 || p->s_gapo < 0 || p->s_gape < 0 ||
        (p->mode != BWFM_MODE_ALL && p->mode != BWFM_MODE_BEST) || p->max_best < 0 || p->max_hits < 1 ||
        (p->form != BWFM_FORM_BATCHED && p->form != BWFM_FORM_PLAIN) || p->waves_per_simd < 0 ||
        p->waves_per_simd > 8 || p->max_hits > 65536 || p->s_mm > 63 || p->s_gapo > 63 || p->s_gape > 63)
        return fail(BWFM_E_INVAL, "align_batch: parameter out of range");
    const int32_t b = p->split_budget;
    if (b != 0 && b != -1 && (b < 16 || b > (1 << 24)))
        return fail(BWFM_E_INVAL, "align_batch: split_budget must be 0, -1 or in [16, 2^24]");
    return BWFM_OK;
}

// Argument checks shared by the align entry points; 0 or a bwfm_err.
static int check_align_args(bwfm_index *ix, const bwfm_reads *rd, const bwfm_aln_params *p, const bwfm_aln_result *res) {
    if (!ix || !rd || !p || !check_result(res, rd->n_reads)) return fail(BWFM_E_INVAL, "align_batch: NULL argument");
    if (!check_index(ix)) return fail(BWFM_E_STATE, "align_batch: index not uploaded");
    if (rd->n_reads && (!rd->bases || !rd->offsets)) return fail(BWFM_E_INVAL, "align_batch: NULL reads");
    if (rd->max_len > BWFM_MAX_READ) return fail(BWFM_E_TOOLONG, "align_batch: max_len above 512");
    return check_aln_params(p);
}

extern "C" int bwfm_align_batch(const bwfm_index *cix, const bwfm_reads *rd, const bwfm_aln_params *p,
                                bwfm_aln_result *res, void *stream) {
    bwfm_index *ix = const_cast<bwfm_index *>(cix);
    if (int rc = check_align_args(ix, rd, p, res)) return rc;
    std::shared_lock<std::shared_mutex> g(ix->mu);
    hipStream_t st = (hipStream_t)stream;
    bwfm::Workspace &ws = stream_ws(ix, st);
    std::lock_guard<std::mutex> wg(ws.mu);
    return by_layout(ix, [&](auto lw) { return align_impl<decltype(lw)::value>(ix, ws, rd, p, res, st, nullptr); });
}

// Same as bwfm_align_batch, also writing per-read search work (states
// expanded, summed over both passes) to expand (device, n_reads).
extern "C" int bwfm_align_batch_counted(const bwfm_index *cix, const bwfm_reads *rd, const bwfm_aln_params *p,
                                        bwfm_aln_result *res, uint32_t *expand, uint64_t *work, void *stream) {
    bwfm_index *ix = const_cast<bwfm_index *>(cix);
    if (!expand) return fail(BWFM_E_INVAL, "align_batch_counted: NULL counter array");
    if (int rc = check_align_args(ix, rd, p, res)) return rc;
    std::shared_lock<std::shared_mutex> g(ix->mu);
    hipStream_t st = (hipStream_t)stream;
    bwfm::Workspace &ws = stream_ws(ix, st);
    std::lock_guard<std::mutex> wg(ws.mu);
    return by_layout(ix, [&](auto lw) {
        return align_impl<decltype(lw)::value>(ix, ws, rd, p, res, st, expand, work);
    });
}

extern "C" int bwfm_locate(const bwfm_index *cix, uint32_t n_reads, const bwfm_aln_result *res, uint32_t max_occ,
                           uint64_t *pos_off, uint32_t *pos, uint64_t cap, void *stream) {
    bwfm_index *ix = const_cast<bwfm_index *>(cix);
    if (!ix || !check_result(res, n_reads) || !pos_off || (!pos && cap)) return fail(BWFM_E_INVAL, "locate: NULL argument");
    if (!check_index(ix)) return fail(BWFM_E_STATE, "locate: index not uploaded");
    std::shared_lock<std::shared_mutex> g(ix->mu);
    hipStream_t st = (hipStream_t)stream;
    bwfm::Workspace &ws = stream_ws(ix, st);
    std::lock_guard<std::mutex> wg(ws.mu);
    uint64_t h0 = 0, h1 = 0;
    HIPCHK(hipMemcpyAsync(&h0, res->hit_offsets, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&h1, res->hit_offsets + n_reads, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (h1 < h0) return fail(BWFM_E_INVAL, "locate: hit offsets decrease");
    const uint64_t n_hits = h1 - h0;
    size_t need = n_hits * 4 + scan_part_elems(n_hits) * 8 + n_hits * 4 + 4096;
    void *w;
    int rc = ws_reserve(ws, need, st, &w);
    if (rc) return rc;
    Carver cv{(char *)w};
    uint32_t *cnt = cv.take<uint32_t>(n_hits);
    uint64_t *part = cv.take<uint64_t>(scan_part_elems(n_hits));
    uint32_t *big = cv.take<uint32_t>(n_hits);
    uint32_t *n_big = cv.take<uint32_t>(1);
    uint64_t total = 0;
    const uint4 *hits = (const uint4 *)res->hits + h0;
    rc = by_layout(ix, [&](auto lw) {
        return locate_impl<decltype(lw)::value>(ix, n_hits, hits, max_occ, pos_off, pos, cap, cnt, part, big, n_big,
                                                st, &total);
    });
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(st));
    return BWFM_OK;
}

namespace {

// Buffers of one pair_reads call: `ctl` returns the control area (counts,
// scan partials, per-hit position offsets of both ends), `pos` the located
// positions of both ends; either may fail with an error code.
struct PairMem {
    std::function<int(size_t, void **)> ctl, pos;
};

// Locate every hit of both ends, then pair: the body shared by the
// allocating and the non-allocating entry points.  The stream must be held
// by the caller (workspace mutex or the scratch contract).
int pair_impl(bwfm_index *ix, uint32_t n_pairs, const bwfm_aln_result *r1, const bwfm_aln_result *r2,
              const bwfm_pair_params *pp, bwfm_pair *out, hipStream_t st, const PairMem &mem, bool timed) {
    const bwfm_aln_result *rr[2] = {r1, r2};
    uint64_t hb[2] = {0, 0}, he[2] = {0, 0}, nh[2] = {0, 0};
    for (int e = 0; e < 2; e++)
        if (rr[e]) {
            HIPCHK(hipMemcpyAsync(&hb[e], rr[e]->hit_offsets, 8, hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(&he[e], rr[e]->hit_offsets + n_pairs, 8, hipMemcpyDeviceToHost, st));
        }
    HIPCHK(hipStreamSynchronize(st));
    for (int e = 0; e < 2; e++) {
        if (he[e] < hb[e]) return fail(BWFM_E_INVAL, "pair_reads: hit offsets decrease");
        nh[e] = he[e] - hb[e];
    }
    // control buffers and each end's position offsets first; the positions
    // of both ends in the second buffer, sized by a counting pass
    const uint64_t nmax = std::max(nh[0], nh[1]);
    const size_t ctl = nmax * 4 * 2 + scan_part_elems(nmax) * 8 + 4096 + (nh[0] + nh[1] + 2) * 8 + 6 * 256;
    void *wmem;
    if (int rc = mem.ctl(ctl, &wmem)) return rc;
    Carver cv{(char *)wmem};
    uint32_t *cnt = cv.take<uint32_t>(nmax);
    uint32_t *big = cv.take<uint32_t>(nmax);
    uint64_t *part = cv.take<uint64_t>(scan_part_elems(nmax));
    uint32_t *n_big = cv.take<uint32_t>(1);
    uint64_t *poff[2] = {cv.take<uint64_t>(nh[0] + 1), cv.take<uint64_t>(nh[1] + 1)};
    uint64_t total[2] = {0, 0};
    for (int e = 0; e < 2; e++) {
        if (!rr[e]) continue;
        const uint4 *hits = (const uint4 *)rr[e]->hits + hb[e];
        // counting pass: capacity 0 reports the total
        int rc = by_layout(ix, [&](auto lw) {
            return locate_impl<decltype(lw)::value>(ix, nh[e], hits, pp->max_occ, poff[e], nullptr, 0, cnt, part, big,
                                                    n_big, st, &total[e], timed);
        });
        if (rc != BWFM_OK && rc != BWFM_E_CAPACITY) return rc;
    }
    void *pmem;
    if (int rc = mem.pos((total[0] + total[1] + 1) * 4, &pmem)) return rc;
    uint32_t *pos[2] = {(uint32_t *)pmem, (uint32_t *)pmem + total[0]};
    for (int e = 0; e < 2; e++) {
        if (!rr[e] || !total[e]) continue;
        const uint4 *hits = (const uint4 *)rr[e]->hits + hb[e];
        uint64_t t2 = 0;
        int rc = by_layout(ix, [&](auto lw) {
            return locate_impl<decltype(lw)::value>(ix, nh[e], hits, pp->max_occ, poff[e], pos[e], total[e], cnt,
                                                    part, big, n_big, st, &t2, timed);
        });
        if (rc) return rc;
    }
    if (n_pairs) {
        EndView e1{r1->hit_offsets, (const uint4 *)r1->hits, poff[0], pos[0], hb[0]};
        EndView e2 = e1;
        if (r2) e2 = EndView{r2->hit_offsets, (const uint4 *)r2->hits, poff[1], pos[1], hb[1]};
        CallTimer tm(st, timed);
        int t = tm.begin("pair");
        k_pair<<<blocks(n_pairs, 256), 256, 0, st>>>(n_pairs, e1, e2, r2 ? 1 : 0, pp->lo, pp->hi, pp->mu, out, nullptr,
                                                     nullptr);
        tm.end(t);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipStreamSynchronize(st));
    return BWFM_OK;
}

int check_pair_args(const bwfm_index *ix, uint32_t n_pairs, const bwfm_aln_result *r1, const bwfm_aln_result *r2,
                    const bwfm_pair_params *pp, const bwfm_pair *out) {
    if (!ix || !check_result(r1, n_pairs) || (r2 && !check_result(r2, n_pairs)) || !pp || (!out && n_pairs))
        return fail(BWFM_E_INVAL, "pair_reads: NULL argument");
    if (!check_index(ix)) return fail(BWFM_E_STATE, "pair_reads: index not uploaded");
    if (pp->lo > pp->hi) return fail(BWFM_E_INVAL, "pair_reads: lo > hi");
    return BWFM_OK;
}

}  // namespace

extern "C" int bwfm_pair_reads(const bwfm_index *cix, uint32_t n_pairs, const bwfm_aln_result *r1,
                               const bwfm_aln_result *r2, const bwfm_pair_params *pp, bwfm_pair *out, void *stream) {
    bwfm_index *ix = const_cast<bwfm_index *>(cix);
    if (int rc = check_pair_args(ix, n_pairs, r1, r2, pp, out)) return rc;
    std::shared_lock<std::shared_mutex> g(ix->mu);
    hipStream_t st = (hipStream_t)stream;
    bwfm::Workspace &ws = stream_ws(ix, st);
    std::lock_guard<std::mutex> wg(ws.mu);
    PairMem mem{[&](size_t b, void **p) { return ws_reserve(ws, b, st, p); },
                [&](size_t b, void **p) {
                    if (int rc = ws_grow(ws.pos, ws.pos_bytes, b, st)) return rc;
                    *p = ws.pos;
                    return (int)BWFM_OK;
                }};
    return pair_impl(ix, n_pairs, r1, r2, pp, out, st, mem, true);
}

// ------------------------------------------------------------------ fixed scratch

// Device scratch of bwfm_pair_reads_noalloc: the control area at its start,
// the located positions after it.  Each device holds its own copy; in host
// code `scratch` names a host-side stand-in, so only the address returned
// by hipGetSymbolAddress (kept per device below) reaches kernels.
static __device__ __align__(256) uint8_t scratch[BWFM_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// the device address of `scratch` on device dev, looked up on the first
// call made with that device current
int scratch_of(int dev, uint8_t **out) {
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return fail(BWFM_E_DEVICE, "noalloc: device ordinal out of range");
    std::lock_guard<std::mutex> g(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(BWFM_E_DEVICE, std::string("noalloc: scratch address lookup failed: ") + hipGetErrorString(e));
        scratch_ptr[dev] = p;
    }
    *out = (uint8_t *)scratch_ptr[dev];
    return BWFM_OK;
}
}  // namespace

extern "C" int bwfm_pair_reads_noalloc(const bwfm_index *cix, uint32_t n_pairs, const bwfm_aln_result *r1,
                                       const bwfm_aln_result *r2, const bwfm_pair_params *pp, bwfm_pair *out,
                                       void *stream) {
    bwfm_index *ix = const_cast<bwfm_index *>(cix);
    if (int rc = check_pair_args(ix, n_pairs, r1, r2, pp, out)) return rc;
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev != ix->device) return fail(BWFM_E_INVAL, "pair_reads_noalloc: the index's device must be current");
    uint8_t *base;
    if (int rc = scratch_of(dev, &base)) return rc;
    std::shared_lock<std::shared_mutex> g(ix->mu);
    hipStream_t st = (hipStream_t)stream;
    size_t ctl_end = 0;
    PairMem mem{[&](size_t b, void **p) {
                    if (b > BWFM_NOALLOC_SCRATCH_BYTES)
                        return fail(BWFM_E_CAPACITY, "pair_reads_noalloc: the hits need " + std::to_string(b) +
                                                         " bytes of control buffers, more than the " +
                                                         std::to_string((size_t)BWFM_NOALLOC_SCRATCH_BYTES) +
                                                         "-byte scratch");
                    ctl_end = (b + 255) & ~(size_t)255;
                    *p = base;
                    return (int)BWFM_OK;
                },
                [&](size_t b, void **p) {
                    if (ctl_end + b > BWFM_NOALLOC_SCRATCH_BYTES)
                        return fail(BWFM_E_CAPACITY, "pair_reads_noalloc: control buffers and positions need " +
                                                         std::to_string(ctl_end + b) + " bytes, more than the " +
                                                         std::to_string((size_t)BWFM_NOALLOC_SCRATCH_BYTES) +
                                                         "-byte scratch");
                    *p = base + ctl_end;
                    return (int)BWFM_OK;
                }};
    return pair_impl(ix, n_pairs, r1, r2, pp, out, st, mem, false);
}

extern "C" int bwfm_max_diff_rule(uint32_t len, double err, double thres) {
    // accumulate the Poisson(err * len) distribution until its tail drops
    // below thres
    double lambda = err * (double)len;
    double pk = std::exp(-lambda);
    double cdf = pk;
    for (int k = 0; k < 1000; k++) {
        if (1.0 - cdf < thres) return k;
        pk = pk * lambda / (double)(k + 1);
        cdf += pk;
    }
    return 1000;
}

extern "C" int bwfm_estimate_insert(const int32_t *ins, uint64_t n, bwfm_pair_params *out) {
    if (!out || (!ins && n)) return fail(BWFM_E_INVAL, "estimate_insert: NULL argument");
    if (n < 100) {
        out->lo = 0;
        out->hi = 500;
        out->mu = 250;
        return BWFM_OK;
    }
    std::vector<int32_t> v(ins, ins + n);
    std::sort(v.begin(), v.end());
    const double q1 = v[(size_t)std::floor(0.25 * (double)(n - 1))];
    const double q3 = v[(size_t)std::floor(0.75 * (double)(n - 1))];
    const double lo_k = q1 - 2 * (q3 - q1), hi_k = q3 + 2 * (q3 - q1);
    double sum = 0;
    uint64_t cnt = 0;
    for (int32_t x : v)
        if (x >= lo_k && x <= hi_k) {
            sum += x;
            cnt++;
        }
    const double mu = sum / (double)cnt;
    double ss = 0;
    for (int32_t x : v)
        if (x >= lo_k && x <= hi_k) ss += ((double)x - mu) * ((double)x - mu);
    const double sd = std::sqrt(ss / (double)cnt);
    const double lo = std::floor(mu - 4 * sd);
    out->lo = (int32_t)(lo < 0 ? 0 : lo);
    out->hi = (int32_t)std::ceil(mu + 4 * sd);
    out->mu = (int32_t)std::nearbyint(mu);
    return BWFM_OK;
}

extern "C" int bwfm_timing_enable(int on) {
    std::lock_guard<std::mutex> g(timing().mu);
    timing().on = on != 0;
    return BWFM_OK;
}

extern "C" int bwfm_timing_reset(void) {
    std::lock_guard<std::mutex> g(timing().mu);
    timing().acc.clear();
    return BWFM_OK;
}

extern "C" int bwfm_timing_get(const char *kernel, double *total_ms, uint64_t *launches) {
    if (!kernel || !total_ms || !launches) return fail(BWFM_E_INVAL, "timing_get: NULL argument");
    std::lock_guard<std::mutex> g(timing().mu);
    auto it = timing().acc.find(kernel);
    *total_ms = it == timing().acc.end() ? 0.0 : it->second.first;
    *launches = it == timing().acc.end() ? 0 : it->second.second;
    return BWFM_OK;
}

extern "C" int bwfm_probe_gather(const void *buf, uint64_t bytes, uint32_t line_bytes, uint32_t lanes, uint32_t iters,
                                 uint32_t *sink, double *ms_out, void *stream) {
    if (!buf || !sink || !ms_out || (line_bytes != 32 && line_bytes != 64 && line_bytes != 128) || lanes == 0 ||
        lanes % 256 ||
        bytes < line_bytes)
        return fail(BWFM_E_INVAL, "probe_gather: bad argument");
    hipStream_t st = (hipStream_t)stream;
    const uint64_t n_lines = bytes / line_bytes;
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    HIPCHK(hipEventRecord(a, st));
    if (line_bytes == 128)
        k_probe_gather<32><<<lanes / 256, 256, 0, st>>>((const uint4 *)buf, n_lines, iters, sink);
    else if (line_bytes == 32)
        k_probe_gather<8><<<lanes / 256, 256, 0, st>>>((const uint4 *)buf, n_lines, iters, sink);
    else
        k_probe_gather<16><<<lanes / 256, 256, 0, st>>>((const uint4 *)buf, n_lines, iters, sink);
    hipError_t e = hipGetLastError();
    HIPCHK(hipEventRecord(b, st));
    HIPCHK(hipEventSynchronize(b));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) return fail(BWFM_E_DEVICE, std::string("k_probe_gather: ") + hipGetErrorString(e));
    *ms_out = ms;
    return BWFM_OK;
}

// ------------------------------------------------------------------ captured pipeline

namespace {

// control words of a pipeline (uint64 indices)
enum {
    PC_PAIRS = 0,     // pairs in this run
    PC_READS = 1,     // reads in this run (2 * pairs)
    PC_HITS = 2,      // reported hits, 0 when they do not fit
    PC_POS = 3,       // located positions, 0 when they do not fit
    PC_NEED_HITS = 4, // reported hits
    PC_NEED_POS = 5,  // located positions
    PC_ERR = 6,       // BWFM_PIPE_E_* bits (low 32 bits)
    PC_BIG = 7,       // hits sorted by a workgroup (low 32 bits)
    PC_ALIGN = 8,     // 16 uint32 of the align kernels' counters
    PC_WORDS = 16
};

__global__ void k_pipe_begin(uint64_t *ctl, uint32_t n_pairs, uint32_t ends) {
    const uint32_t i = threadIdx.x;
    if (i < PC_WORDS) ctl[i] = i == PC_PAIRS ? n_pairs : (i == PC_READS ? (uint64_t)ends * n_pairs : 0ull);
}

// dst = offs[*n_dev], the total of a scan, or 0 with an error bit when it
// exceeds cap or an earlier stage already failed; need keeps the total
__global__ void k_take_total(const uint64_t *offs, const uint64_t *n_dev, uint64_t cap, uint64_t *dst, uint64_t *need,
                             uint32_t *err, uint32_t bit) {
    if (threadIdx.x != 0) return;
    const uint64_t t = (*err) ? 0 : offs[*n_dev];
    *need = t;
    if (t > cap) *err |= bit;
    *dst = (*err) ? 0 : t;
}

}  // namespace

struct bwfm_pipeline {
    bwfm_index *ix = nullptr;
    bwfm_aln_params ap{};
    bwfm_pair_params pp{};
    bwfm_pipeline_params q{};
    void *mem = nullptr;
    // inputs
    uint8_t *bases = nullptr;
    uint64_t *offsets = nullptr;
    uint8_t *maxd = nullptr;
    // search buffers
    uint4 *lstack = nullptr, *lcand = nullptr, *sstack = nullptr, *scand = nullptr, *stage = nullptr;
    uint32_t *n_rep = nullptr, *slow_list = nullptr;
    uint64_t *stage_off = nullptr, *part = nullptr;
    // outputs
    uint64_t *hoff = nullptr, *poff = nullptr;
    uint4 *hits = nullptr;
    uint32_t *c1 = nullptr, *c2 = nullptr, *cnt = nullptr, *big = nullptr, *pos = nullptr;
    uint8_t *status = nullptr;
    bwfm_pair *pairs = nullptr;
    uint64_t *ctl = nullptr;
    PersistentArgs *pargs = nullptr;
    uint8_t *drows = nullptr, *dflag = nullptr;  // D-array pre-pass output (gene DPREPASS)
    uint32_t dstride = 0;
    SplitBufs X{};               // split searches (X.budget 0: off)
    TaskArgs *targs = nullptr;
    uint32_t *lane_read = nullptr;
    // launch shape
    uint32_t lanes = 0, slow_lanes = 0, bs = 0, lstride = 0, stack_cap = 0, worst_stack = 0, scap = 0;
    uint32_t tlanes = 0;  // the split searches' round grid (shares the lane buffers)
    size_t lds = 0;
    uint32_t n_pairs = 0;  // of the batch last set
    uint32_t ends = 2;     // reads per pair record
    bool bound = false;    // input from caller-owned buffers
    bwfm_reads in{};       // the bound input
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};  // first pass start, end; the search's end
    hipStream_t cap = nullptr;  // capture only: nothing runs on it
    bool timed_graph = false, timed_last = false;
    bool timing_uncapturable = false;  // a capture with event nodes failed once
    uint64_t kt_gen = 0;               // the index's table generation the graph was captured with
};

namespace {

// Enqueue the step.  Every count comes from the control words.
template <int LW>
int pipe_enqueue(bwfm_pipeline *pl, hipStream_t st, bool timed, bool capture) {
    const DevIndex D = dev_index(pl->ix);
    const Params P = make_params(pl->ap);
    const uint32_t nmax = pl->ends * pl->q.max_pairs;
    uint64_t *ctl = pl->ctl;
    uint32_t *actl = reinterpret_cast<uint32_t *>(ctl + PC_ALIGN);
    uint32_t *err = reinterpret_cast<uint32_t *>(ctl + PC_ERR);
    ReadsView rv = pl->bound ? ReadsView{pl->in.bases, pl->in.offsets, pl->in.lengths, pl->in.max_diff, nmax,
                                         pl->in.max_len, ctl + PC_READS}
                             : ReadsView{pl->bases, pl->offsets, nullptr, pl->maxd, nmax, pl->q.max_len, ctl + PC_READS};
    const bool plain = pl->ap.form == BWFM_FORM_PLAIN;
    LaneBufs lb = plain ? LaneBufs{pl->lstack, pl->lcand, 1, pl->lanes, pl->stack_cap, 1, pl->lanes, FAST_CAND, pl->lstride}
                        : LaneBufs{pl->lstack, pl->lcand, pl->stack_cap, 1, pl->stack_cap, FAST_CAND, 1, FAST_CAND,
                                   pl->lstride};
    ReadOut O{pl->n_rep, pl->c1, pl->c2, pl->status, pl->slow_list, actl, pl->stage,
              reinterpret_cast<unsigned long long *>(actl + 2), pl->q.hit_capacity, pl->stage_off, nullptr, nullptr};
    // under capture the events become event-record nodes of the graph
    auto mark = [&](hipEvent_t e) {
        return capture ? hipEventRecordWithFlags(e, st, hipEventRecordExternal) : hipEventRecord(e, st);
    };
    if (!plain && pl->drows) {
        const uint32_t nr_up = ((nmax + pl->bs - 1) / pl->bs) * pl->bs;
        k_dscan<LW><<<nr_up / pl->bs, pl->bs, (size_t)pl->bs * pl->lstride, st>>>(D, rv, P, pl->drows, pl->dflag,
                                                                               pl->dstride, pl->lstride);
    }
    if (pl->X.budget) k_fill_u32<<<1, 64, 0, st>>>(pl->X.ctl, SPLIT_CTL, 0u);
    if (!plain)
        k_set_args<<<1, 64, 0, st>>>(pl->pargs,
                                     PersistentArgs{rv, lb, O, actl + 1, pl->drows, pl->dflag, pl->dstride, pl->X,
                                                    pl->lane_read});
    if (timed) HIPCHK(mark(pl->ev[0]));
    if (plain)
        k_align_plain<LW><<<pl->lanes / pl->bs, pl->bs, pl->lds, st>>>(D, rv, P, lb, O);
    else
        hipLaunchKernelGGL(persistent_kernel<LW>(pl->ap.waves_per_simd, pl->drows != nullptr), dim3(pl->lanes / pl->bs),
                           dim3(pl->bs),
                           pl->lds, st, D, P, (const PersistentArgs *)pl->pargs);
    if (timed) HIPCHK(mark(pl->ev[1]));
    if (pl->X.budget) enqueue_split<LW>(D, P, pl->X, pl->targs, lb, O, pl->tlanes, st);
    if (timed) HIPCHK(mark(pl->ev[2]));
    LaneBufs sb{pl->sstack, pl->scand, pl->worst_stack, 1, pl->worst_stack, pl->scap, 1, pl->scap, pl->lstride};
    k_align_slow<LW><<<pl->slow_lanes / pl->bs, pl->bs, (size_t)pl->bs * pl->lstride, st>>>(D, rv, P, sb, O, actl + 4);
    HIPCHK(hipGetLastError());
    int rc = scan_counts(pl->n_rep, nmax, pl->hoff, pl->part, st, ctl + PC_READS);
    if (rc) return rc;
    k_take_total<<<1, 64, 0, st>>>(pl->hoff, ctl + PC_READS, pl->q.hit_capacity, ctl + PC_HITS, ctl + PC_NEED_HITS, err,
                                   BWFM_PIPE_E_HITS);
    k_compact<<<blocks(nmax, 256), 256, 0, st>>>(nmax, pl->hoff, pl->stage, pl->stage_off, pl->hits, ctl + PC_READS,
                                                 err);
    // every hit of both ends is located in one pass
    const uint64_t hcap = std::max<uint64_t>(pl->q.hit_capacity, 1);
    k_loc_count<<<blocks(hcap, 256), 256, 0, st>>>(hcap, pl->hits, pl->pp.max_occ, pl->cnt, ctl + PC_HITS);
    rc = scan_counts(pl->cnt, hcap, pl->poff, pl->part, st, ctl + PC_HITS);
    if (rc) return rc;
    k_take_total<<<1, 64, 0, st>>>(pl->poff, ctl + PC_HITS, pl->q.pos_capacity, ctl + PC_POS, ctl + PC_NEED_POS, err,
                                   BWFM_PIPE_E_POSITIONS);
    k_loc_rows<LW><<<2048, 256, 0, st>>>(D, hcap, pl->hits, pl->poff, pl->q.pos_capacity, pl->pos, ctl + PC_HITS,
                                         ctl + PC_POS);
    uint32_t *n_big = reinterpret_cast<uint32_t *>(ctl + PC_BIG);
    k_sort_small<<<blocks(hcap, 256), 256, 0, st>>>(hcap, pl->poff, pl->pos, pl->big, n_big, ctl + PC_HITS);
    k_sort_big<<<1024, 256, 0, st>>>(pl->poff, pl->pos, pl->big, n_big);
    EndView e1{pl->hoff, pl->hits, pl->poff, pl->pos, 0};
    EndView e2{pl->hoff, pl->hits, pl->poff, pl->pos, 0};  // offsets moved by n on the device
    k_pair<<<blocks(pl->q.max_pairs, 256), 256, 0, st>>>(pl->q.max_pairs, e1, e2, pl->ends == 2 ? 1 : 0, pl->pp.lo,
                                                         pl->pp.hi, pl->pp.mu, pl->pairs, ctl + PC_PAIRS, err);
    HIPCHK(hipGetLastError());
    return BWFM_OK;
}

int pipe_enqueue_any(bwfm_pipeline *pl, hipStream_t st, bool timed, bool capture) {
    return by_layout(pl->ix, [&](auto lw) { return pipe_enqueue<decltype(lw)::value>(pl, st, timed, capture); });
}

}  // namespace

namespace {

void drop_graph(bwfm_pipeline *pl) {
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    pl->exec = nullptr;
    pl->graph = nullptr;
}

}  // namespace

extern "C" int bwfm_pipeline_create(const bwfm_index *cix, const bwfm_aln_params *ap, const bwfm_pair_params *pp,
                                    const bwfm_pipeline_params *q, bwfm_pipeline **out) {
    bwfm_index *ix = const_cast<bwfm_index *>(cix);
    if (!out) return fail(BWFM_E_INVAL, "pipeline_create: NULL argument");
    *out = nullptr;
    if (!ix || !ap || !pp || !q) return fail(BWFM_E_INVAL, "pipeline_create: NULL argument");
    if (!check_index(ix)) return fail(BWFM_E_STATE, "pipeline_create: index not uploaded");
    if (q->max_pairs == 0 || q->max_len == 0 || q->max_bases == 0 || q->max_pairs > (1u << 30))
        return fail(BWFM_E_INVAL, "pipeline_create: empty or oversized capacity");
    if (q->max_len > BWFM_MAX_READ) return fail(BWFM_E_TOOLONG, "pipeline_create: max_len above 512");
    if (pp->lo > pp->hi) return fail(BWFM_E_INVAL, "pipeline_create: lo > hi");
    if (int rc = check_aln_params(ap)) return rc;
    std::unique_ptr<bwfm_pipeline> pl(new (std::nothrow) bwfm_pipeline);
    if (!pl) return fail(BWFM_E_NOMEM, "out of host memory");
    pl->ix = ix;
    pl->ap = *ap;
    pl->pp = *pp;
    pl->q = *q;
    pl->ends = q->paired ? 2 : 1;
    const uint32_t nmax = pl->ends * q->max_pairs;
    const uint32_t mlen = q->max_len;
    pl->worst_stack = 8 * (mlen + BWFM_MAX_DIFF) + 1;
    pl->lstride = lds_stride_for(mlen);
    const bool plain = ap->form == BWFM_FORM_PLAIN;
    const uint32_t sbud = plain ? 0u : split_budget_of(*ap);
    const bool dpre = !plain && (BWFM_GENE_DPREPASS == 1 || mlen >= DPRE_MIN_LEN);
    pl->bs = block_for(pl->lstride);
    pl->lds = (size_t)pl->bs * pl->lstride + (plain ? 0 : (pl->bs / 64) * sizeof(WaveShare));
    const uint32_t nr_up = ((nmax + pl->bs - 1) / pl->bs) * pl->bs;
    pl->lanes = plain ? nr_up
                      : std::min<uint32_t>(by_layout(ix,
                                                     [&](auto lw) {
                                                         return persistent_lanes<decltype(lw)::value>(
                                                             pl->bs, pl->lds, ap->waves_per_simd, dpre);
                                                     }),
                                           nr_up);
    pl->stack_cap = plain ? std::min<uint32_t>(pl->worst_stack, PLAIN_STACK) : pl->worst_stack;
    pl->tlanes = sbud ? by_layout(ix, [&](auto lw) { return task_lanes<decltype(lw)::value>(nr_up, pl->lanes); }) : 0u;
    const uint32_t blanes = std::max(pl->lanes, pl->tlanes);
    pl->slow_lanes = std::min<uint32_t>(nr_up, SLOW_LANES);
    pl->scap = ap->max_hits + 1;
    const uint64_t hcap = std::max<uint64_t>(q->hit_capacity, 1);
    const uint64_t pcap = std::max<uint64_t>(q->pos_capacity, 1);
    size_t need = 0;
    auto add = [&](size_t b) { need += (b + 255) & ~size_t(255); };
    add(q->max_bases); add((size_t)(nmax + 1) * 8); add(nmax);
    add((size_t)blanes * pl->stack_cap * 16); add((size_t)blanes * FAST_CAND * 16);
    add((size_t)pl->slow_lanes * pl->worst_stack * 16); add((size_t)pl->slow_lanes * pl->scap * 16);
    add((size_t)nmax * 4); add((size_t)nmax * 4); add((size_t)nmax * 8); add(hcap * 16);
    add(scan_part_elems(std::max<uint64_t>(nmax, hcap)) * 8);
    add((size_t)(nmax + 1) * 8); add(hcap * 16); add((size_t)nmax * 4); add((size_t)nmax * 4); add(nmax);
    add(hcap * 4); add(hcap * 4); add((hcap + 1) * 8); add(pcap * 4); add((size_t)q->max_pairs * sizeof(bwfm_pair));
    add(PC_WORDS * 8);
    add(sizeof(PersistentArgs));
    pl->dstride = ((mlen + 15) / 16) * 16;
    if (dpre) {
        add((size_t)nmax * 2 * pl->dstride);
        add(nmax);
    }
    const SplitShape zs = split_shape(nmax, mlen);
    if (sbud) need += split_bytes(zs) + (size_t)pl->lanes * 4 + 256;
    need += 4096;
    if (hipMalloc(&pl->mem, need) != hipSuccess) return fail(BWFM_E_NOMEM, "pipeline: device allocation failed");
    Carver cv{(char *)pl->mem};
    pl->bases = cv.take<uint8_t>(q->max_bases);
    pl->offsets = cv.take<uint64_t>(nmax + 1);
    pl->maxd = cv.take<uint8_t>(nmax);
    pl->lstack = cv.take<uint4>((size_t)blanes * pl->stack_cap);
    pl->lcand = cv.take<uint4>((size_t)blanes * FAST_CAND);
    pl->sstack = cv.take<uint4>((size_t)pl->slow_lanes * pl->worst_stack);
    pl->scand = cv.take<uint4>((size_t)pl->slow_lanes * pl->scap);
    pl->n_rep = cv.take<uint32_t>(nmax);
    pl->slow_list = cv.take<uint32_t>(nmax);
    pl->stage_off = cv.take<uint64_t>(nmax);
    pl->stage = cv.take<uint4>(hcap);
    pl->part = cv.take<uint64_t>(scan_part_elems(std::max<uint64_t>(nmax, hcap)));
    pl->hoff = cv.take<uint64_t>(nmax + 1);
    pl->hits = cv.take<uint4>(hcap);
    pl->c1 = cv.take<uint32_t>(nmax);
    pl->c2 = cv.take<uint32_t>(nmax);
    pl->status = cv.take<uint8_t>(nmax);
    pl->cnt = cv.take<uint32_t>(hcap);
    pl->big = cv.take<uint32_t>(hcap);
    pl->poff = cv.take<uint64_t>(hcap + 1);
    pl->pos = cv.take<uint32_t>(pcap);
    pl->pairs = cv.take<bwfm_pair>(q->max_pairs);
    pl->ctl = cv.take<uint64_t>(PC_WORDS);
    pl->pargs = cv.take<PersistentArgs>(1);
    if (dpre) {
        pl->drows = cv.take<uint8_t>((size_t)nmax * 2 * pl->dstride);
        pl->dflag = cv.take<uint8_t>(nmax);
    }
    if (sbud) {
        pl->X = carve_split(cv, zs, sbud, &pl->targs);
        pl->lane_read = cv.take<uint32_t>(pl->lanes);
    }
    if (hipEventCreate(&pl->ev[0]) != hipSuccess || hipEventCreate(&pl->ev[1]) != hipSuccess ||
        hipEventCreate(&pl->ev[2]) != hipSuccess ||
        hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking) != hipSuccess) {
        bwfm_pipeline_destroy(pl.release());
        return fail(BWFM_E_DEVICE, "pipeline: event or stream creation failed");
    }
    *out = pl.release();
    return BWFM_OK;
}

extern "C" int bwfm_pipeline_set_reads(bwfm_pipeline *pl, const bwfm_reads *rd, uint32_t n_pairs, void *stream) {
    if (!pl || !rd) return fail(BWFM_E_INVAL, "pipeline_set_reads: NULL argument");
    if (rd->lengths) return fail(BWFM_E_INVAL, "pipeline_set_reads: lengths must be NULL");
    if (rd->n_reads != pl->ends * n_pairs)
        return fail(BWFM_E_INVAL, "pipeline_set_reads: n_reads must be n_pairs times the reads per pair");
    if (n_pairs > pl->q.max_pairs) return fail(BWFM_E_CAPACITY, "pipeline_set_reads: more pairs than max_pairs");
    if (rd->max_len > pl->q.max_len) return fail(BWFM_E_CAPACITY, "pipeline_set_reads: max_len above the pipeline's");
    if (n_pairs && (!rd->bases || !rd->offsets)) return fail(BWFM_E_INVAL, "pipeline_set_reads: NULL reads");
    hipStream_t st = (hipStream_t)stream;
    const uint32_t n = pl->ends * n_pairs;
    if (pl->bound) drop_graph(pl);
    pl->bound = false;
    if (n) {
        uint64_t o[2] = {0, 0};
        HIPCHK(hipMemcpyAsync(&o[0], rd->offsets, 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(&o[1], rd->offsets + n, 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (o[0] != 0) return fail(BWFM_E_INVAL, "pipeline_set_reads: offsets must start at 0");
        if (o[1] > pl->q.max_bases) return fail(BWFM_E_CAPACITY, "pipeline_set_reads: more bases than max_bases");
        if (o[1]) HIPCHK(hipMemcpyAsync(pl->bases, rd->bases, o[1], hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(pl->offsets, rd->offsets, (size_t)(n + 1) * 8, hipMemcpyDeviceToDevice, st));
        if (rd->max_diff)
            HIPCHK(hipMemcpyAsync(pl->maxd, rd->max_diff, n, hipMemcpyDeviceToDevice, st));
        else
            HIPCHK(hipMemsetAsync(pl->maxd, pl->ap.max_diff, n, st));
    }
    pl->n_pairs = n_pairs;
    return BWFM_OK;
}

extern "C" int bwfm_pipeline_bind_reads(bwfm_pipeline *pl, const bwfm_reads *rd) {
    if (!pl || !rd || !rd->bases || !rd->offsets) return fail(BWFM_E_INVAL, "pipeline_bind_reads: NULL argument");
    if (rd->n_reads < pl->ends * pl->q.max_pairs)
        return fail(BWFM_E_CAPACITY, "pipeline_bind_reads: fewer read slots than the pipeline's maximum");
    if (rd->max_len > pl->q.max_len) return fail(BWFM_E_CAPACITY, "pipeline_bind_reads: max_len above the pipeline's");
    drop_graph(pl);
    pl->in = *rd;
    pl->in.max_len = pl->q.max_len;  // reads longer than the LDS rows allow are flagged invalid
    pl->bound = true;
    pl->n_pairs = 0;
    return BWFM_OK;
}

extern "C" int bwfm_pipeline_set_count(bwfm_pipeline *pl, uint32_t n_pairs) {
    if (!pl || !pl->bound) return fail(BWFM_E_INVAL, "pipeline_set_count: no bound reads");
    if (n_pairs > pl->q.max_pairs) return fail(BWFM_E_CAPACITY, "pipeline_set_count: more pairs than max_pairs");
    pl->n_pairs = n_pairs;
    return BWFM_OK;
}

extern "C" int bwfm_pipeline_run(bwfm_pipeline *pl, int graph, void *stream) {
    if (!pl) return fail(BWFM_E_INVAL, "pipeline_run: NULL pipeline");
    hipStream_t st = (hipStream_t)stream;
    bool timed;
    {
        std::lock_guard<std::mutex> g(timing().mu);
        timed = timing().on;
    }
    // the batch size goes in by a launch of its own: the graph's kernels
    // read it from the control words
    k_pipe_begin<<<1, 64, 0, st>>>(pl->ctl, pl->n_pairs, pl->ends);
    HIPCHK(hipGetLastError());
    if (!graph) {
        pl->timed_last = timed;
        return pipe_enqueue_any(pl, st, timed, false);
    }
    if (pl->timing_uncapturable) timed = false;
    if (pl->exec && (pl->timed_graph != timed || pl->kt_gen != pl->ix->kt_gen)) drop_graph(pl);
    if (!pl->exec) {
        // recorded on the pipeline's own stream (the caller's may be the
        // null stream, which cannot be captured); launched on the caller's
        hipGraph_t gph = nullptr;
        for (;;) {
            HIPCHK(hipStreamBeginCapture(pl->cap, hipStreamCaptureModeThreadLocal));
            int rc = pipe_enqueue_any(pl, pl->cap, timed, true);
            hipError_t e = hipStreamEndCapture(pl->cap, &gph);
            (void)hipGetLastError();
            if (!rc && e == hipSuccess) break;
            if (gph) (void)hipGraphDestroy(gph);
            gph = nullptr;
            if (!timed) {
                if (rc) return rc;
                return fail(BWFM_E_DEVICE, std::string("pipeline capture: ") + hipGetErrorString(e));
            }
            // without event nodes: the step still runs, its kernel time is not taken
            pl->timing_uncapturable = true;
            timed = false;
        }
        hipGraphExec_t ex = nullptr;
        hipError_t e;
        e = hipGraphInstantiate(&ex, gph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(gph);
            return fail(BWFM_E_DEVICE, std::string("pipeline graph instantiation: ") + hipGetErrorString(e));
        }
        pl->graph = gph;
        pl->exec = ex;
        pl->timed_graph = timed;
        pl->kt_gen = pl->ix->kt_gen;
    }
    pl->timed_last = pl->timed_graph;
    HIPCHK(hipGraphLaunch(pl->exec, st));
    return BWFM_OK;
}

extern "C" int bwfm_pipeline_finish(bwfm_pipeline *pl, void *stream, bwfm_pipeline_status *out) {
    if (!pl || !out) return fail(BWFM_E_INVAL, "pipeline_finish: NULL argument");
    hipStream_t st = (hipStream_t)stream;
    uint64_t c[PC_WORDS];
    HIPCHK(hipMemcpyAsync(c, pl->ctl, sizeof c, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    out->n_pairs = (uint32_t)c[PC_PAIRS];
    out->error = (uint32_t)c[PC_ERR];
    out->n_hits = c[PC_NEED_HITS];
    out->n_positions = c[PC_NEED_POS];
    out->kernel_ms = 0;
    if (pl->timed_last) {
        float ms = 0;
        float ms_all = 0;
        if (hipEventElapsedTime(&ms, pl->ev[0], pl->ev[1]) == hipSuccess &&
            hipEventElapsedTime(&ms_all, pl->ev[0], pl->ev[2]) == hipSuccess) {
            out->kernel_ms = ms_all;
            std::lock_guard<std::mutex> g(timing().mu);
            auto &e = timing().acc[pl->ap.form == BWFM_FORM_PLAIN ? "align_plain" : "align_persistent"];
            e.first += ms;
            e.second += 1;
            if (pl->ap.form != BWFM_FORM_PLAIN) {
                auto &f = timing().acc["align_search"];
                f.first += ms_all;
                f.second += 1;
            }
        }
    }
    return BWFM_OK;
}

extern "C" int bwfm_pipeline_outputs(bwfm_pipeline *pl, int end, bwfm_aln_result *res, uint64_t **pos_offsets,
                                     uint32_t **positions, bwfm_pair **pairs) {
    if (!pl || (end != 0 && end != 1)) return fail(BWFM_E_INVAL, "pipeline_outputs: bad argument");
    if (end == 1 && pl->ends == 1) return fail(BWFM_E_INVAL, "pipeline_outputs: single-end pipeline has no end 2");
    const uint64_t base = end ? pl->n_pairs : 0;
    if (res) {
        res->hit_offsets = pl->hoff + base;
        res->hits = reinterpret_cast<bwfm_hit *>(pl->hits);
        res->hit_capacity = pl->q.hit_capacity;
        res->c1 = pl->c1 + base;
        res->c2 = pl->c2 + base;
        res->status = pl->status + base;
    }
    if (pos_offsets) *pos_offsets = pl->poff;
    if (positions) *positions = pl->pos;
    if (pairs) *pairs = pl->pairs;
    return BWFM_OK;
}

extern "C" void bwfm_pipeline_destroy(bwfm_pipeline *pl) {
    if (!pl) return;
    drop_graph(pl);
    for (auto &e : pl->ev)
        if (e) (void)hipEventDestroy(e);
    if (pl->cap) (void)hipStreamDestroy(pl->cap);
    if (pl->mem) (void)hipFree(pl->mem);
    delete pl;
}

extern "C" const char *bwfm_last_error(void) { return last_error().c_str(); }
