// Mapping quality of each end of each pair, from the search's tiers, the
// difference budget and the pair's outcome (the pairing step that closes
// the pipeline, section 3.7, reports one; the paper gives no formula, so it
// is a reading, stated at bwfm_mapq).  One thread per pair: it reads the
// pair record, each end's c1, c2 and status, and the end's leading hits
// (those of the best score, reported first), and writes two bytes.  Work is
// a few dozen bytes per pair: the kernel streams.

#include <hip/hip_runtime.h>

#include <string>

#include "bwfm_internal.h"

using namespace bwfm;

namespace {

struct EndRes {
    const uint64_t *hoff;
    const bwfm_hit *hits;
    const uint32_t *c1, *c2;
    const uint8_t *st;
    const uint8_t *budget;  // per read, or NULL: max_diff for every read
};

struct Caps {
    double r;  // weight of a tier-2 placement, 10^(-q_tier / 10), computed on the host
    int q_unique, q_budget, q_pair, max_diff;
};

// single-end quality of end e (1 or 2) of pair p
__device__ int quality_se(const bwfm_pair &pr, int e, const EndRes &R, uint32_t p, const Caps &K) {
    const uint32_t pos = e == 1 ? pr.pos1 : pr.pos2;
    const int score = e == 1 ? pr.score1 : pr.score2;
    const uint64_t h0 = R.hoff[p], h1 = R.hoff[p + 1];
    if (pos == 0xFFFFFFFFu || (R.st[p] & BWFM_ST_OVERFLOW) || R.c1[p] == 0 || h1 <= h0) return 0;
    const int best = R.hits[h0].score;
    int dmin = 1 << 30;
    for (uint64_t i = h0; i < h1; i++) {
        const bwfm_hit h = R.hits[i];
        if (h.score != best) break;
        dmin = min(dmin, (int)h.n_mm + (int)h.n_gapo + (int)h.n_gape);
    }
    const double w = score == best ? 1.0 : K.r;
    const double den = (double)R.c1[p] + (double)R.c2[p] * K.r;
    int q;
    if (den - w <= 0.0) {
        q = K.q_unique;
    } else {
        q = (int)floor(-10.0 * log10((den - w) / den) + 0.5);
        q = max(0, min(q, K.q_unique));
    }
    const int budget = R.budget ? (int)R.budget[p] : K.max_diff;
    if (dmin >= budget) q = min(q, K.q_budget);
    return q;
}

__global__ __launch_bounds__(256) void k_mapq(uint32_t n, EndRes R1, EndRes R2, bool paired, const bwfm_pair *pairs,
                                              const bwfm_rescue *rescue, Caps K, uint8_t *out) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const bwfm_pair pr = pairs[p];
    const int q1 = quality_se(pr, 1, R1, p, K);
    const int q2 = paired ? quality_se(pr, 2, R2, p, K) : 0;
    int o1 = q1, o2 = q2;
    const int rescued = rescue ? rescue[p].end : 0;
    if (pr.flags & BWFM_PF_PAIRED) {
        o1 = o2 = min(K.q_pair, q1 + q2);  // the pair is wrong only if both placements are
    } else if (rescued == 2) {
        o2 = q1;  // placed relative to its anchor
    } else if (rescued == 1) {
        o1 = q2;
    }
    out[2 * (size_t)p] = (uint8_t)o1;
    out[2 * (size_t)p + 1] = (uint8_t)o2;
}

bool result_ok(const bwfm_aln_result *r) { return r && r->hit_offsets && r->c1 && r->c2 && r->status; }

}  // namespace

extern "C" int bwfm_mapq(uint32_t n_pairs, const bwfm_aln_result *r1, const bwfm_aln_result *r2,
                         const uint8_t *budget1, const uint8_t *budget2, uint32_t max_diff, const bwfm_pair *pairs,
                         const bwfm_rescue *rescue, const bwfm_mapq_params *mp, uint8_t *out, void *stream) {
    if (n_pairs == 0) return BWFM_OK;
    if (!result_ok(r1) || (r2 && !result_ok(r2)) || !pairs || !out) return fail(BWFM_E_INVAL, "mapq: NULL argument");
    const bwfm_mapq_params q = mp ? *mp : bwfm_mapq_params BWFM_MAPQ_DEFAULTS;
    if (q.q_tier < 1 || q.q_tier > 60 || q.q_unique < 0 || q.q_unique > 60 || q.q_budget < 0 || q.q_budget > 60 ||
        q.q_pair < 0 || q.q_pair > 254)
        return fail(BWFM_E_INVAL, "mapq: qualities out of range");
    const Caps K{pow(10.0, -q.q_tier / 10.0), q.q_unique, q.q_budget, q.q_pair, (int)max_diff};
    const EndRes R1{r1->hit_offsets, r1->hits, r1->c1, r1->c2, r1->status, budget1};
    const EndRes R2 = r2 ? EndRes{r2->hit_offsets, r2->hits, r2->c1, r2->c2, r2->status, budget2} : EndRes{};
    const uint32_t grid = (uint32_t)(((uint64_t)n_pairs + 255) / 256);
    k_mapq<<<grid, 256, 0, (hipStream_t)stream>>>(n_pairs, R1, R2, r2 != nullptr, pairs, rescue, K, out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(BWFM_E_DEVICE, std::string("mapq: launch: ") + hipGetErrorString(e));
    return BWFM_OK;
}
