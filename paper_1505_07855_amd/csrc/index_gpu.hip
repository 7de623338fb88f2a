// Index construction on the device: the suffix array of T$ by prefix
// doubling over radix sorts, then the BWT as bit-plane rank lines with
// per-line counts, and the row-sampled SA -- the same bytes the host
// builder (index_host.cpp) writes, produced in device memory so that a
// human-scale reference is indexed in seconds rather than tens of minutes.
//
// Suffix order (section 2 of the paper; FM-index background): suffixes of
// T$ with $ < A < C < G < T.  Prefix doubling: after sorting by the first h
// symbols, rank[i] is 1 + the first sorted row whose h-prefix equals that of
// suffix i; sorting by (rank[i], rank[i + h]) orders by the first 2h
// symbols.  The first round sorts 21-symbol keys (3 bits per symbol, $ and
// the padding past it as 0), so a random genome needs about
// log2(longest repeat / 21) further rounds.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <rocprim/rocprim.hpp>
#include <string>
#include <vector>

#include "bwfm_internal.h"

using namespace bwfm;

namespace {

constexpr int K0 = 21;  // symbols in a first-round key

#define DCHK(expr)                                                                          \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(BWFM_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));  \
    } while (0)

inline uint32_t grid_for(uint64_t n, uint32_t block) {
    return (uint32_t)std::min<uint64_t>((n + block - 1) / block, 1u << 16);
}

__global__ void k_reverse(const uint8_t *t, uint64_t n, uint8_t *r) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        r[i] = t[n - 1 - i];
}

// the reference two bits per base, 16 bases per word (base i in bits 2 (i % 16) of word i / 16)
__global__ void k_pack_ref(const uint8_t *t, uint64_t n, uint32_t *pac) {
    const uint64_t words = (n + 15) / 16;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < words; w += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t v = 0;
        const uint64_t i0 = w * 16;
        for (int k = 0; k < 16 && i0 + k < n; k++) v |= (uint32_t)(t[i0 + k] & 3) << (2 * k);
        pac[w] = v;
    }
}

// planar 64-byte lines of 160 rows rewritten in place as sub-counted ones:
// counts of C, G, T before the line, per base a word of the counts in the
// first 32, 64, 96 and 128 rows (a byte each), then the ten row words
__global__ void k_ix_subcount(uint32_t *lines, uint64_t n_lines) {
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n_lines; x += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t *L = lines + x * 16;
        uint32_t P[16];
        for (int w = 0; w < 16; w++) P[w] = L[w];
        uint32_t cC = 0, cG = 0, cT = 0, sC = 0, sG = 0, sT = 0;
        for (int g = 0; g < 5; g++) {
            if (g > 0) {
                sC |= cC << (8 * (g - 1));
                sG |= cG << (8 * (g - 1));
                sT |= cT << (8 * (g - 1));
            }
            const uint32_t h = P[4 + 2 * g], l = P[5 + 2 * g];
            cC += __popc(~h & l);
            cG += __popc(h & ~l);
            cT += __popc(h & l);
        }
        L[0] = P[1];
        L[1] = P[2];
        L[2] = P[3];
        L[3] = sC;
        L[4] = sG;
        L[5] = sT;
        for (int w = 0; w < 10; w++) L[6 + w] = P[4 + w];
    }
}

// planar 128-byte lines of 384 rows rewritten in place as 128-byte
// sub-counted ones: counts of C, G, T before the line, the boundary words
// of rows 64, 128, 192, 256 and 320 (C | G << 9 | T << 18), then the 24 row
// words
__global__ void k_ix_sub128(uint32_t *lines, uint64_t n_lines) {
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n_lines; x += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t *L = lines + x * 32;
        uint32_t P[32];
        for (int w = 0; w < 32; w++) P[w] = L[w];
        uint32_t cC = 0, cG = 0, cT = 0;
        for (int g = 0; g < 6; g++) {
            if (g > 0) L[2 + g] = cC | (cG << 9) | (cT << 18);
            for (int w = 0; w < 2; w++) {
                const uint32_t h = P[4 + 4 * g + 2 * w], l = P[5 + 4 * g + 2 * w];
                cC += __popc(~h & l);
                cG += __popc(h & ~l);
                cT += __popc(h & l);
            }
        }
        L[0] = P[1];
        L[1] = P[2];
        L[2] = P[3];
        for (int w = 0; w < 24; w++) L[8 + w] = P[4 + w];
    }
}

// first-round keys: the 21 symbols from i, each code + 1, 0 from $ on
__global__ void k_sa_init(const uint8_t *t, uint64_t n, uint64_t N, uint64_t *key, uint32_t *val) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t k = 0;
        for (int q = 0; q < K0; q++) {
            const uint64_t p = i + q;
            k = (k << 3) | (p < n ? (uint64_t)(t[p] + 1) : 0ull);
        }
        key[i] = k;
        val[i] = (uint32_t)i;
    }
}

// g[j] = j where sorted row j starts a group of equal keys, else 0; counts groups
__global__ void k_sa_heads(const uint64_t *key, uint64_t N, uint32_t *g, unsigned long long *n_groups) {
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < N; j += (uint64_t)gridDim.x * blockDim.x) {
        const bool head = j == 0 || key[j] != key[j - 1];
        g[j] = head ? (uint32_t)j : 0u;
        const unsigned long long b = __ballot(head);
        if (b && (threadIdx.x & 63) == (unsigned)(__ffsll((long long)__ballot(1)) - 1))
            atomicAdd(n_groups, (unsigned long long)__popcll(b));
    }
}

// rank of each suffix: 1 + the first row of its group
__global__ void k_sa_rank(const uint32_t *val, const uint32_t *grp, uint64_t N, uint32_t *rank) {
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < N; j += (uint64_t)gridDim.x * blockDim.x)
        rank[val[j]] = grp[j] + 1;
}

// next-round keys in the current row order: (rank[p], rank[p + h])
__global__ void k_sa_pairs(const uint32_t *val, const uint32_t *rank, uint64_t N, uint64_t h, uint64_t *key) {
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < N; j += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t p = val[j];
        key[j] = ((uint64_t)rank[p] << 32) | (p + h < N ? (uint64_t)rank[p + h] : 0ull);
    }
}

// One lane per 32-row group: the group's two bit-plane words, its symbol
// counts ($ as A), the $ row, and the SA samples among its rows.
__global__ void k_ix_groups(const uint8_t *t, const uint32_t *sa, uint64_t N, uint32_t bpl, uint32_t lw,
                            uint32_t sa_sample, uint32_t *lines, uint32_t *gcnt, uint64_t n_groups, uint32_t *samp,
                            unsigned long long *primary) {
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_groups;
         g += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t hi = 0, lo = 0, c[4] = {0, 0, 0, 0};
        for (uint32_t r = 0; r < 32; r++) {
            const uint64_t j = g * 32 + r;
            if (j >= N) break;
            const uint32_t q = sa[j];
            const uint32_t code = q == 0 ? 0u : t[q - 1];
            if (q == 0) *primary = j;
            hi |= (code >> 1) << r;
            lo |= (code & 1u) << r;
            c[code]++;
            if ((j & (sa_sample - 1)) == 0) samp[j / sa_sample] = q;
        }
        const uint64_t row = g * 32, line = row / bpl, rr = row - line * bpl;
        uint32_t *L = lines + line * lw;
        L[4 + 2 * (rr >> 5)] = hi;
        L[5 + 2 * (rr >> 5)] = lo;
        for (int a = 0; a < 4; a++) gcnt[(size_t)a * n_groups + g] = c[a];
    }
}

// per line and base: the count of its rows (a sum over its groups)
__global__ void k_ix_linecnt(const uint32_t *gcnt, uint64_t n_groups, uint32_t gpl, uint64_t n_lines, uint32_t *lc) {
    for (uint64_t L = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; L < n_lines;
         L += (uint64_t)gridDim.x * blockDim.x)
        for (int a = 0; a < 4; a++) {
            uint32_t s = 0;
            const uint64_t g1 = (L + 1) * gpl < n_groups ? (L + 1) * gpl : n_groups;
            for (uint64_t g = L * gpl; g < g1; g++)
                s += gcnt[(size_t)a * n_groups + g];
            lc[(size_t)a * n_lines + L] = s;
        }
}

// the counts before each line into its header words
__global__ void k_ix_heads(const uint64_t *off, uint64_t n_lines, uint32_t lw, uint32_t *lines) {
    for (uint64_t L = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; L < n_lines;
         L += (uint64_t)gridDim.x * blockDim.x)
        for (int a = 0; a < 4; a++) lines[L * lw + a] = (uint32_t)off[(size_t)a * n_lines + L];
}

// Device buffers of one build, freed on every exit path.
struct DevScratch {
    std::vector<void *> ptrs;
    ~DevScratch() {
        for (void *p : ptrs) (void)hipFree(p);
    }
    template <class T> T *alloc(size_t n) {
        void *p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return static_cast<T *>(p);
    }
};

// Suffix array of t$ (N = n + 1 rows) into sa (device).
int suffix_sort(const uint8_t *t, uint64_t n, uint32_t *sa, hipStream_t st) {
    const uint64_t N = n + 1;
    DevScratch s;
    uint64_t *k0 = s.alloc<uint64_t>(N), *k1 = s.alloc<uint64_t>(N);
    uint32_t *v1 = s.alloc<uint32_t>(N), *rank = s.alloc<uint32_t>(N);
    unsigned long long *ng = s.alloc<unsigned long long>(1);
    if (!k0 || !k1 || !v1 || !rank || !ng) return fail(BWFM_E_NOMEM, "index build: device scratch for the suffix sort");
    const uint32_t B = 256, G = grid_for(N, B);
    k_sa_init<<<G, B, 0, st>>>(t, n, N, k0, sa);
    rocprim::double_buffer<uint64_t> keys(k0, k1);
    rocprim::double_buffer<uint32_t> vals(sa, v1);
    size_t tmp_sort = 0, tmp_scan = 0;
    DCHK(rocprim::radix_sort_pairs(nullptr, tmp_sort, keys, vals, N, 0, 64, st));
    uint32_t *dummy = nullptr;
    DCHK(rocprim::inclusive_scan(nullptr, tmp_scan, dummy, dummy, N, rocprim::maximum<uint32_t>(), st));
    void *tmp = s.alloc<uint8_t>(std::max(tmp_sort, tmp_scan));
    if (!tmp) return fail(BWFM_E_NOMEM, "index build: sort scratch");
    unsigned end_bit = 3 * K0;
    for (uint64_t h = K0;; h *= 2) {
        size_t ts = tmp_sort;
        DCHK(rocprim::radix_sort_pairs(tmp, ts, keys, vals, N, 0, end_bit, st));
        // groups of equal keys; the free halves of the double buffers hold
        // the head marks and their running maximum
        uint32_t *g = vals.alternate();
        uint32_t *grp = reinterpret_cast<uint32_t *>(keys.alternate());
        DCHK(hipMemsetAsync(ng, 0, 8, st));
        k_sa_heads<<<G, B, 0, st>>>(keys.current(), N, g, ng);
        size_t tc = tmp_scan;
        DCHK(rocprim::inclusive_scan(tmp, tc, g, grp, N, rocprim::maximum<uint32_t>(), st));
        unsigned long long groups = 0;
        DCHK(hipMemcpyAsync(&groups, ng, 8, hipMemcpyDeviceToHost, st));
        DCHK(hipStreamSynchronize(st));
        if (groups == N) break;
        if (h >= N) return fail(BWFM_E_DEVICE, "index build: suffix sort did not converge");
        k_sa_rank<<<G, B, 0, st>>>(vals.current(), grp, N, rank);
        k_sa_pairs<<<G, B, 0, st>>>(vals.current(), rank, N, h, keys.current());
        end_bit = 64;
        DCHK(hipGetLastError());
    }
    if (vals.current() != sa) DCHK(hipMemcpyAsync(sa, vals.current(), N * 4, hipMemcpyDeviceToDevice, st));
    DCHK(hipStreamSynchronize(st));
    return BWFM_OK;
}

// One direction: suffix sort, then rank lines and samples straight into
// the index's device buffers, and host copies of both.
int build_dir_device(const uint8_t *t, uint64_t n, uint32_t line_bytes, uint32_t bpl, uint32_t sa_sample,
                     uint32_t rank_format, HostDir &out, void *&d_lines, void *&d_sa, hipStream_t st) {
    const uint64_t N = n + 1;
    const uint32_t lw = line_bytes / 4;
    const uint64_t n_lines = N / bpl + 1, n_samples = n / sa_sample + 1, n_groups = (N + 31) / 32;
    DevScratch s;
    uint32_t *sa = s.alloc<uint32_t>(N);
    if (!sa) return fail(BWFM_E_NOMEM, "index build: device suffix array");
    if (int rc = suffix_sort(t, n, sa, st)) return rc;
    if (hipMalloc(&d_lines, n_lines * lw * 4) != hipSuccess || hipMalloc(&d_sa, n_samples * 4) != hipSuccess)
        return fail(BWFM_E_NOMEM, "index build: device index");
    uint32_t *lines = static_cast<uint32_t *>(d_lines), *samp = static_cast<uint32_t *>(d_sa);
    uint32_t *gcnt = s.alloc<uint32_t>(4 * n_groups), *lc = s.alloc<uint32_t>(4 * n_lines);
    uint64_t *off = s.alloc<uint64_t>(4 * n_lines);
    unsigned long long *prim = s.alloc<unsigned long long>(1);
    if (!gcnt || !lc || !off || !prim) return fail(BWFM_E_NOMEM, "index build: device line scratch");
    DCHK(hipMemsetAsync(lines, 0, n_lines * lw * 4, st));
    const uint32_t B = 256;
    k_ix_groups<<<grid_for(n_groups, B), B, 0, st>>>(t, sa, N, bpl, lw, sa_sample, lines, gcnt, n_groups, samp, prim);
    k_ix_linecnt<<<grid_for(n_lines, B), B, 0, st>>>(gcnt, n_groups, bpl / 32, n_lines, lc);
    size_t tmp_bytes = 0;
    DCHK(rocprim::exclusive_scan(nullptr, tmp_bytes, lc, off, (uint64_t)0, n_lines, rocprim::plus<uint64_t>(), st));
    void *tmp = s.alloc<uint8_t>(tmp_bytes);
    if (!tmp) return fail(BWFM_E_NOMEM, "index build: scan scratch");
    for (int a = 0; a < 4; a++) {
        size_t tb = tmp_bytes;
        DCHK(rocprim::exclusive_scan(tmp, tb, lc + (size_t)a * n_lines, off + (size_t)a * n_lines, (uint64_t)0, n_lines,
                                     rocprim::plus<uint64_t>(), st));
    }
    k_ix_heads<<<grid_for(n_lines, B), B, 0, st>>>(off, n_lines, lw, lines);
    if (rank_format == BWFM_RANK_SUBCOUNTS) k_ix_subcount<<<grid_for(n_lines, B), B, 0, st>>>(lines, n_lines);
    if (rank_format == BWFM_RANK_SUB128) k_ix_sub128<<<grid_for(n_lines, B), B, 0, st>>>(lines, n_lines);
    DCHK(hipGetLastError());
    // totals per base ($ counted as A) and the $ row
    uint64_t last_off[4];
    uint32_t last_cnt[4];
    unsigned long long primary = 0;
    for (int a = 0; a < 4; a++) {
        DCHK(hipMemcpyAsync(&last_off[a], off + (size_t)a * n_lines + n_lines - 1, 8, hipMemcpyDeviceToHost, st));
        DCHK(hipMemcpyAsync(&last_cnt[a], lc + (size_t)a * n_lines + n_lines - 1, 4, hipMemcpyDeviceToHost, st));
    }
    DCHK(hipMemcpyAsync(&primary, prim, 8, hipMemcpyDeviceToHost, st));
    out.lines.resize(n_lines * lw);
    out.sa.resize(n_samples);
    DCHK(hipMemcpyAsync(out.lines.data(), lines, n_lines * lw * 4, hipMemcpyDeviceToHost, st));
    DCHK(hipMemcpyAsync(out.sa.data(), samp, n_samples * 4, hipMemcpyDeviceToHost, st));
    DCHK(hipStreamSynchronize(st));
    uint64_t cnt[4];
    for (int a = 0; a < 4; a++) cnt[a] = last_off[a] + last_cnt[a];
    cnt[0] -= 1;  // the $ row was counted as A
    out.C[0] = 1;
    for (int a = 1; a < 4; a++) out.C[a] = out.C[a - 1] + cnt[a - 1];
    out.primary = primary;
    return BWFM_OK;
}

}  // namespace

extern "C" int bwfm_build_index_device(const uint8_t *ref, uint64_t n, const bwfm_index_params *p, void *stream,
                                       bwfm_index **out) {
    if (!ref || !out) return fail(BWFM_E_INVAL, "build_index_device: NULL argument");
    *out = nullptr;
    bwfm_index_params q = p ? *p : bwfm_index_params{128, 0, 32, 0, BWFM_RANK_PLANES};
    if (int rc = check_index_params(q, n)) return rc;
    for (uint64_t i = 0; i < n; i++)
        if (ref[i] > 3) return fail(BWFM_E_BASE, "reference holds a code outside 0..3 at " + std::to_string(i));
    std::unique_ptr<bwfm_index> ix(new (std::nothrow) bwfm_index);
    if (!ix) return fail(BWFM_E_NOMEM, "out of host memory");
    ix->n = n;
    ix->line_bytes = q.line_bytes;
    ix->bpl = q.bases_per_line;
    ix->sa_sample = q.sa_sample;
    ix->rank_format = q.rank_format;
    ix->n_lines = (n + 1) / q.bases_per_line + 1;
    ix->n_samples = n / q.sa_sample + 1;
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    DCHK(hipGetDevice(&dev));
    uint8_t *t = nullptr, *r = nullptr;
    if (hipMalloc(&t, n) != hipSuccess) return fail(BWFM_E_NOMEM, "index build: device text");
    int rc = BWFM_OK;
    if (hipMemcpyAsync(t, ref, n, hipMemcpyHostToDevice, st) != hipSuccess)
        rc = fail(BWFM_E_DEVICE, "index build: text upload");
    const uint64_t pac_words = (n + 15) / 16;
    if (!rc && hipMalloc(&ix->d_pac, pac_words * 4) != hipSuccess) rc = fail(BWFM_E_NOMEM, "index build: packed text");
    if (!rc) {
        k_pack_ref<<<grid_for(pac_words, 256), 256, 0, st>>>(t, n, (uint32_t *)ix->d_pac);
        try {
            ix->pac.resize(pac_words);
        } catch (const std::bad_alloc &) {
            rc = fail(BWFM_E_NOMEM, "out of host memory");
        }
        if (!rc && hipMemcpyAsync(ix->pac.data(), ix->d_pac, pac_words * 4, hipMemcpyDeviceToHost, st) != hipSuccess)
            rc = fail(BWFM_E_DEVICE, "index build: packed text copy");
    }
    if (!rc) rc = build_dir_device(t, n, q.line_bytes, q.bases_per_line, q.sa_sample, q.rank_format, ix->dir[0],
                                   ix->d_lines[0],
                                   ix->d_sa[0], st);
    if (!rc) {
        // reverse(T) in place of T
        if (hipMalloc(&r, n) != hipSuccess) {
            rc = fail(BWFM_E_NOMEM, "index build: device text");
        } else {
            k_reverse<<<grid_for(n, 256), 256, 0, st>>>(t, n, r);
            rc = build_dir_device(r, n, q.line_bytes, q.bases_per_line, q.sa_sample, q.rank_format, ix->dir[1],
                                  ix->d_lines[1],
                                  ix->d_sa[1], st);
        }
    }
    (void)hipStreamSynchronize(st);
    if (t) (void)hipFree(t);
    if (r) (void)hipFree(r);
    if (rc) {
        for (int d = 0; d < 2; d++) {
            if (ix->d_lines[d]) (void)hipFree(ix->d_lines[d]);
            if (ix->d_sa[d]) (void)hipFree(ix->d_sa[d]);
            ix->d_lines[d] = ix->d_sa[d] = nullptr;
        }
        if (ix->d_pac) (void)hipFree(ix->d_pac);
        ix->d_pac = nullptr;
        return rc;
    }
    ix->device = dev;
    ix->device_bytes = 0;
    for (int d = 0; d < 2; d++) ix->device_bytes += ix->dir[d].lines.size() * 4 + ix->dir[d].sa.size() * 4;
    ix->device_bytes += pac_words * 4;
    *out = ix.release();
    return BWFM_OK;
}
