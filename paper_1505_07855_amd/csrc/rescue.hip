// Mate rescue on the device: the end of a pair left without a partner is
// aligned locally (affine gaps) inside the reference window that the insert
// bounds allow around its mate's primary (section 3.7 closes the pipeline
// with BWA's pairing step, of which this is the rescue part).
//
// One wave per rescued pair (a wave takes a few pair records and works
// through those that need a rescue, one after another).  The mate's m bases
// are the rows of the dynamic-programming matrices, R consecutive rows per
// lane; the window's reference bases are its columns.  The wave sweeps the
// columns in skewed order -- lane l works on column t - l at step t -- so
// each lane receives the row above its first row (the previous lane's last
// row) one step after it was made, through a one-lane DPP shift.  Every cell
// is computed once; a step costs R cells per lane.  A cell is one int32 key
// holding its score, the move it prefers on ties and the window column its
// alignment starts at, so the recurrence's maxima carry the tie order and
// the start along at no extra cost.  The window is decoded from the packed
// reference into LDS first.  Work per pair is m x window cells, a few
// hundred steps: the kernel is bound by integer ALU work, not memory.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>

#include "bwfm_internal.h"

using namespace bwfm;

namespace {

constexpr int RB = 64;   // threads per block: one wave, so the hardware hands out work one wave at a time
constexpr int PPW = 4;   // pair records a wave takes (lanes 0 .. PPW - 1): few, so waves end evenly
// cell keys: score * KS + preference * KP + start column
constexpr int KS = 1 << 15, KP = 1 << 13;
constexpr int NEGK = -(1 << 30);  // no alignment can end here (score -32768)

struct EndView {
    const uint8_t *bases;
    const uint64_t *off;
    const uint32_t *len;  // or NULL: read r ends where read r + 1 starts
};

struct Scores {
    int a, b, o, e, min_score;
};

__device__ __forceinline__ void end_span(const EndView &v, uint32_t r, uint64_t &o0, int &m) {
    o0 = v.off[r];
    if (v.len) {
        m = (int)min(v.len[r], 1u << 20);
    } else {
        const uint64_t o1 = v.off[r + 1];
        m = o1 < o0 ? -1 : (int)min(o1 - o0, (uint64_t)1 << 20);
    }
}

// order this wave's LDS writes before its later reads by other lanes
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// v from the previous lane of the wave (a DPP shift right by one lane);
// lane 0, which has no previous lane, gets 0
__device__ __forceinline__ int row_above(int v) {
    return __builtin_amdgcn_mov_dpp(v, 0x138 /* wave_shr:1 */, 0xF, 0xF, true);
}

// Rescue one pair with the whole wave (all arguments wave-uniform).
template <int R>
__device__ void rescue_one(const uint32_t *pac, uint64_t n, const EndView &ev, uint32_t pair, uint64_t o0, int m,
                           int mate, uint32_t pa, int la, int sa, int lo, int hi, int max_len, const Scores &S,
                           uint8_t *win,
                           bwfm_rescue *out) {
    const int lane = threadIdx.x & 63;
    int64_t w0, w1;
    if (sa == 0) {
        w0 = pa;
        w1 = std::min<int64_t>((int64_t)pa + hi, (int64_t)n);
    } else {
        w1 = std::min<int64_t>((int64_t)pa + la, (int64_t)n);
        w0 = std::max<int64_t>(w1 - hi, 0);
    }
    const int w = (int)std::max<int64_t>(w1 - w0, 0);
    bwfm_rescue res;
    std::memset(&res, 0, sizeof res);
    if (m <= 0 || m > max_len || m > 64 * R || w <= 0) {
        if (lane == 0) out[pair] = res;
        return;
    }
    // the window, in the orientation the query reads it: forward after a +
    // anchor, reversed (from pr + lr - 1 down) after a - anchor
    // (each base stored times 8: the bit offset of its score in a row's profile)
    for (int j = lane; j < w; j += 64) {
        const uint64_t p = sa == 0 ? (uint64_t)(w0 + j) : (uint64_t)(w1 - 1 - j);
        win[j] = (uint8_t)(8 * ((pac[p >> 4] >> (2 * (p & 15))) & 3));
    }
    // this lane's rows: query base i is mate base m - 1 - i, complemented
    // after a + anchor (the mate then lies on -).  Each row keeps its
    // substitution scores against A, C, G, T as four signed bytes.
    int prof[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int i = lane * R + r;
        int c = 5;  // rows past the mate: match nothing, never reported
        if (i < m) {
            c = ev.bases[o0 + (uint64_t)(m - 1 - i)];
            if (sa == 0 && c < 4) c = 3 - c;
        }
        uint32_t pk = 0;
        for (int b = 0; b < 4; b++) pk |= (uint32_t)(uint8_t)(int8_t)(c == b ? S.a : -S.b) << (8 * b);
        prof[r] = (int)pk;
    }
    wave_sync();
    const int used = (m + R - 1) / R;        // lanes holding rows
    const int e_min = lo > 0 ? lo - 1 : -1;  // the alignment must end at column >= lo - 1
    // Cells are int32 keys: score * 2^15 + preference * 2^13 + the window
    // column the cell's alignment starts at (< 2^13).  One max over keys then
    // takes the highest score and, on equal scores, the preferred move
    // (diagonal 3 > gap along the reference 2 > gap along the read 1 > no
    // alignment 0), carrying the start column along.  H keys are kept with
    // preference 3, so a gap opened from H arrives with preference 3 and
    // beats the extension of a gap (E kept at 2, F at 1) on equal scores;
    // clearing one bit then brings E back to 2 and F back to 1.  The edge
    // row and column are key 0; cells of score 0 or below never pass their
    // start column on to a cell of positive score, so their keys' low bits
    // do not matter.
    const int oek = (S.o + S.e) * KS, ek = S.e * KS;
    int Hp[R], Ep[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        Hp[r] = 3 * KP;
        Ep[r] = NEGK;
    }
    int outH = 0, outF = 0;  // last row of this lane, current column
    int prevH = 0;           // row above, previous column
    int bestK = 0, bj = -1, bi = 0;
    int bestT = KS;  // a cell reports when its key reaches this: a score above the best
    const int steps = w + used - 1;
    const bool holds = lane < used;
    int j = -lane;
    for (int t = 0; t < steps; t++, j++) {
        // the row above this lane's first row, from the previous lane
        const int upH = row_above(outH), upF = row_above(outF);
        if (holds && (unsigned)j < (unsigned)w) {
            const int sh = win[j];
            const bool elig = j >= e_min;
            int Hd = prevH, Hu = upH, F = upF;
            const int j3 = j + 3 * KP;
#pragma unroll
            for (int r = 0; r < R; r++) {
                const int E = max(Hp[r] - oek, Ep[r] - ek) & ~KP;
                F = max(Hu - oek, F - ek) & ~(2 * KP);
                const int base = Hd >= KS ? Hd : j3;  // extend a positive cell, or start here
                const int dg = base + __builtin_amdgcn_sbfe(prof[r], sh, 8) * KS;
                const int H = max(max(dg, E), max(F, 0)) | (3 * KP);
                Hd = Hp[r];
                Hp[r] = H;
                Ep[r] = E;
                Hu = H;
                if (elig && H >= bestT && lane * R + r < m) {
                    bestK = H;
                    bestT = (H & ~(KS - 1)) + KS;
                    bj = j;
                    bi = lane * R + r + 1;
                }
            }
            outH = Hu;
            outF = F;
        }
        prevH = upH;
    }
    // the first best cell in column order: highest score, then smallest
    // column, then smallest row (each cell lives in exactly one lane)
    const int best = bestK >> 15;
    uint64_t key = best > 0 ? ((uint64_t)(uint32_t)best << 32) | ((uint64_t)(0xFFFFu - (uint32_t)bj) << 16) |
                                  (uint64_t)(0xFFFFu - (uint32_t)bi)
                            : 0;
    uint64_t top = key;
    for (int k = 32; k > 0; k >>= 1) {
        const uint64_t o = __shfl_xor(top, k);
        top = o > top ? o : top;
    }
    const unsigned long long who = __ballot(key == top && top != 0);
    if (who) {
        const int src = __ffsll((long long)who) - 1;
        const int sbest = __shfl(best, src);
        const int sbj = __shfl(bj, src);
        const int sbO = __shfl(bestK & (KP - 1), src);
        if (sbest >= S.min_score) {
            res.end = (uint8_t)mate;
            res.score = (int16_t)sbest;
            res.len = (uint16_t)(sbj - sbO + 1);
            res.insert = sbj + 1;
            if (sa == 0) {
                res.strand = 1;
                res.pos = (uint32_t)(w0 + sbO);
            } else {
                res.strand = 0;
                res.pos = (uint32_t)(w1 - 1 - sbj);
            }
        }
    }
    if (lane == 0) out[pair] = res;
}

// RMAX: rows per lane that hold the batch's longest mate; each mate is
// rescued by the build of the fewest rows per lane that hold it, so short
// mates of a mixed batch keep more lanes busy and the sweep shorter.
template <int RMAX>
__global__ __launch_bounds__(RB) void k_rescue(const uint32_t *pac, uint64_t n, EndView e1, EndView e2,
                                               const bwfm_pair *pairs, uint32_t n_pairs, int lo, int hi, int max_len,
                                               Scores S, int win_stride, bwfm_rescue *out) {
    extern __shared__ uint8_t lds[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint8_t *win = lds + (size_t)wv * win_stride;
    // the wave's first pair (uniform across the wave; said so, so that the
    // per-pair values derived from it live in scalar registers)
    const uint32_t base = __builtin_amdgcn_readfirstlane(((uint32_t)blockIdx.x * (RB / 64) + (uint32_t)wv) * PPW);
    const uint32_t p = base + (uint32_t)lane;
    bool cand = false;
    int mate = 0, la = 0, sa = 0;
    uint32_t pa = 0;
    if (lane < PPW && p < n_pairs) {
        const bwfm_pair pr = pairs[p];
        const bool m1 = (pr.flags & BWFM_PF_MAPPED1) != 0, m2 = (pr.flags & BWFM_PF_MAPPED2) != 0;
        cand = !(pr.flags & BWFM_PF_PAIRED) && (m1 || m2);
        // the anchor: the mapped end, or of two the lower search score (end 1 on ties)
        const int anchor = (m1 && m2) ? (pr.score1 <= pr.score2 ? 1 : 2) : (m1 ? 1 : 2);
        mate = 3 - anchor;
        pa = anchor == 1 ? pr.pos1 : pr.pos2;
        la = anchor == 1 ? pr.len1 : pr.len2;
        sa = anchor == 1 ? pr.strand1 : pr.strand2;
        if (!cand) {
            bwfm_rescue z;
            std::memset(&z, 0, sizeof z);
            out[p] = z;
        }
    }
    unsigned long long todo = __ballot(cand);
    while (todo) {
        const int src = __ffsll((long long)todo) - 1;
        todo &= todo - 1;
        const int c_mate = __builtin_amdgcn_readlane(mate, src), c_la = __builtin_amdgcn_readlane(la, src),
                  c_sa = __builtin_amdgcn_readlane(sa, src);
        const uint32_t c_pa = (uint32_t)__builtin_amdgcn_readlane((int)pa, src);
        const EndView &ev = c_mate == 1 ? e1 : e2;
        const uint32_t pair = base + (uint32_t)src;
        uint64_t o0;
        int m;
        end_span(ev, pair, o0, m);
        const int need = m <= 64 ? 1 : m <= 128 ? 2 : m <= 256 ? 4 : 8;
        if (RMAX >= 8 && need == 8)
            rescue_one<(RMAX >= 8 ? 8 : 1)>(pac, n, ev, pair, o0, m, c_mate, c_pa, c_la, c_sa, lo, hi, max_len, S, win,
                                           out);
        else if (RMAX >= 4 && need == 4)
            rescue_one<(RMAX >= 4 ? 4 : 1)>(pac, n, ev, pair, o0, m, c_mate, c_pa, c_la, c_sa, lo, hi, max_len, S, win,
                                           out);
        else if (RMAX >= 2 && need == 2)
            rescue_one<(RMAX >= 2 ? 2 : 1)>(pac, n, ev, pair, o0, m, c_mate, c_pa, c_la, c_sa, lo, hi, max_len, S, win,
                                           out);
        else  // one row per lane; a mate longer than the batch's bound is reported unrescued there
            rescue_one<1>(pac, n, ev, pair, o0, m, c_mate, c_pa, c_la, c_sa, lo, hi, max_len, S, win, out);
        wave_sync();  // the window is rewritten for the next pair
    }
}

}  // namespace

extern "C" int bwfm_rescue_mates(const bwfm_index *ix, const bwfm_reads *end1, const bwfm_reads *end2,
                                 uint32_t n_pairs, const bwfm_pair *pairs, const bwfm_pair_params *pp,
                                 const bwfm_rescue_params *rp, bwfm_rescue *out, void *stream) {
    if (!ix || !end1 || !end2 || !pp || (n_pairs && (!pairs || !out)))
        return fail(BWFM_E_INVAL, "rescue_mates: NULL argument");
    if (ix->device < 0 || !ix->d_pac) return fail(BWFM_E_STATE, "rescue_mates: index not uploaded");
    if (n_pairs && (!end1->bases || !end1->offsets || !end2->bases || !end2->offsets))
        return fail(BWFM_E_INVAL, "rescue_mates: NULL reads");
    if (end1->n_reads < n_pairs || end2->n_reads < n_pairs)
        return fail(BWFM_E_INVAL, "rescue_mates: fewer reads than pairs");
    if (pp->lo > pp->hi) return fail(BWFM_E_INVAL, "rescue_mates: lo > hi");
    if (pp->hi > BWFM_RESCUE_MAX_WINDOW) return fail(BWFM_E_INVAL, "rescue_mates: hi above the largest window");
    const bwfm_rescue_params q = rp ? *rp : bwfm_rescue_params BWFM_RESCUE_DEFAULTS;
    if (q.match < 1 || q.match > 32 || q.mismatch < 0 || q.mismatch > 64 || q.gap_open < 0 || q.gap_open > 64 ||
        q.gap_extend < 0 || q.gap_extend > 64 || q.min_score < 1)
        return fail(BWFM_E_INVAL, "rescue_mates: scores out of range");
    const uint32_t max_len = std::max(end1->max_len, end2->max_len);
    if (max_len > BWFM_MAX_READ) return fail(BWFM_E_TOOLONG, "rescue_mates: max_len above 512");
    if (n_pairs == 0) return BWFM_OK;
    hipStream_t st = (hipStream_t)stream;
    const EndView e1{end1->bases, end1->offsets, end1->lengths}, e2{end2->bases, end2->offsets, end2->lengths};
    const Scores S{q.match, q.mismatch, q.gap_open, q.gap_extend, q.min_score};
    const int hi = std::max(pp->hi, 0);
    const int win_stride = std::max((hi + 15) & ~15, 16);
    const uint64_t per_block = (uint64_t)(RB / 64) * PPW;
    const uint32_t grid = (uint32_t)(((uint64_t)n_pairs + per_block - 1) / per_block);
    const size_t lds = (size_t)(RB / 64) * win_stride;
    const uint32_t *pac = (const uint32_t *)ix->d_pac;
    const int ml = (int)max_len;
    if (max_len <= 64)
        k_rescue<1><<<grid, RB, lds, st>>>(pac, ix->n, e1, e2, pairs, n_pairs, pp->lo, hi, ml, S, win_stride, out);
    else if (max_len <= 128)
        k_rescue<2><<<grid, RB, lds, st>>>(pac, ix->n, e1, e2, pairs, n_pairs, pp->lo, hi, ml, S, win_stride, out);
    else if (max_len <= 256)
        k_rescue<4><<<grid, RB, lds, st>>>(pac, ix->n, e1, e2, pairs, n_pairs, pp->lo, hi, ml, S, win_stride, out);
    else
        k_rescue<8><<<grid, RB, lds, st>>>(pac, ix->n, e1, e2, pairs, n_pairs, pp->lo, hi, ml, S, win_stride, out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(BWFM_E_DEVICE, std::string("rescue_mates: launch: ") + hipGetErrorString(e));
    return BWFM_OK;
}
