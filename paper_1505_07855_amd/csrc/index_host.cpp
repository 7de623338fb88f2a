// Host-side construction of the packed FM-index (the offline encoding of
// the reference, Genetically Improved BarraCUDA section 2).
//
// Suffix sorting uses induced sorting (SA-IS: Nong, Zhang and Chan, "Two
// efficient algorithms for linear time suffix array construction", IEEE
// Trans. Computers 2011), written from that description.  The BWT is then
// packed into rank lines: each line starts with the counts of A, C, G and T
// in the rows before it ($ counted as A, since $ is stored as A) followed by
// its rows, so one rank query reads one line.  Rows are stored as bit
// planes: for every 32 rows one word holds the high bits of their 2-bit
// codes and the next word the low bits, so a single 32-bit popcount counts
// a symbol over 32 rows.  Every sa_sample-th row keeps its suffix array
// value.
#include <algorithm>
#include <cstdio>
#include <memory>
#include <cstring>
#include <stdexcept>
#include <thread>

#include "bwfm_internal.h"

namespace bwfm {

namespace {

constexpr uint32_t EMPTY = 0xffffffffu;

struct Bits {
    std::vector<uint64_t> w;
    explicit Bits(uint64_t n) : w((n + 63) / 64, 0) {}
    bool get(uint64_t i) const { return (w[i >> 6] >> (i & 63)) & 1; }
    void set(uint64_t i) { w[i >> 6] |= 1ULL << (i & 63); }
};

// Suffix array of s[0, n) over alphabet [0, K); s[n - 1] must be the unique
// smallest symbol.  SA receives the n sorted suffix starts.
template <typename Ch>
void sais(const Ch *s, uint32_t *SA, uint64_t n, uint64_t K) {
    if (n == 1) {
        SA[0] = 0;
        return;
    }
    // type of each suffix: S (bit set) or L
    Bits st(n);
    st.set(n - 1);
    for (uint64_t i = n - 1; i-- > 0;)
        if (s[i] < s[i + 1] || (s[i] == s[i + 1] && st.get(i + 1))) st.set(i);
    auto lms = [&](uint64_t i) { return i > 0 && st.get(i) && !st.get(i - 1); };

    std::vector<uint64_t> bkt(K + 1, 0);
    for (uint64_t i = 0; i < n; i++) bkt[s[i] + 1]++;
    for (uint64_t c = 0; c < K; c++) bkt[c + 1] += bkt[c];  // bkt[c] = start of bucket c
    std::vector<uint64_t> ptr(K);
    auto tails = [&] { for (uint64_t c = 0; c < K; c++) ptr[c] = bkt[c + 1]; };
    auto heads = [&] { for (uint64_t c = 0; c < K; c++) ptr[c] = bkt[c]; };
    auto induce = [&] {
        heads();
        for (uint64_t i = 0; i < n; i++) {
            uint32_t j = SA[i];
            if (j != EMPTY && j > 0 && !st.get(j - 1)) SA[ptr[s[j - 1]]++] = j - 1;
        }
        tails();
        for (uint64_t i = n; i-- > 0;) {
            uint32_t j = SA[i];
            if (j != EMPTY && j > 0 && st.get(j - 1)) SA[--ptr[s[j - 1]]] = j - 1;
        }
    };

    // 1. sort the LMS substrings: LMS suffixes at their bucket ends, induce
    std::fill(SA, SA + n, EMPTY);
    tails();
    for (uint64_t i = 1; i < n; i++)
        if (lms(i)) SA[--ptr[s[i]]] = (uint32_t)i;
    induce();

    // 2. gather the sorted LMS positions in SA[0, n1)
    uint64_t n1 = 0;
    for (uint64_t i = 0; i < n; i++)
        if (lms(SA[i])) SA[n1++] = SA[i];
    // 3. name them: equal LMS substrings get equal names
    std::fill(SA + n1, SA + n, EMPTY);
    uint64_t name = 0;
    uint32_t prev = EMPTY;
    for (uint64_t i = 0; i < n1; i++) {
        uint32_t p = SA[i];
        bool diff = prev == EMPTY;
        for (uint64_t d = 0; !diff; d++) {
            if (s[p + d] != s[prev + d] || st.get(p + d) != st.get(prev + d)) {
                diff = true;
            } else if (d > 0 && (lms(p + d) || lms(prev + d))) {
                diff = !(lms(p + d) && lms(prev + d));
                break;
            }
        }
        if (diff) {
            name++;
            prev = p;
        }
        SA[n1 + p / 2] = (uint32_t)(name - 1);
    }
    // the reduced string, in text order of its LMS positions, at SA's end
    {
        uint64_t j = n;
        for (uint64_t i = n; i-- > n1;)
            if (SA[i] != EMPTY) SA[--j] = SA[i];
    }
    uint32_t *s1 = SA + n - n1;
    uint32_t *SA1 = SA;
    // 4. sort the reduced string's suffixes
    if (name < n1) {
        sais<uint32_t>(s1, SA1, n1, name);
    } else {
        for (uint64_t i = 0; i < n1; i++) SA1[s1[i]] = (uint32_t)i;
    }
    // 5. map back to text positions and induce the full order
    {
        uint64_t j = 0;
        for (uint64_t i = 1; i < n; i++)
            if (lms(i)) s1[j++] = (uint32_t)i;
        for (uint64_t i = 0; i < n1; i++) SA1[i] = s1[SA1[i]];
        std::fill(SA + n1, SA + n, EMPTY);
        tails();
        for (uint64_t i = n1; i-- > 0;) {
            uint32_t p = SA[i];
            SA[i] = EMPTY;
            SA[--ptr[s[p]]] = p;
        }
    }
    induce();
}

}  // namespace

int build_dir(const uint8_t *text, uint64_t n, uint32_t line_bytes, uint32_t bpl, uint32_t sa_sample,
              uint32_t rank_format, HostDir &out) {
    const uint64_t N = n + 1;
    std::vector<uint8_t> s(N);
    for (uint64_t i = 0; i < n; i++) s[i] = (uint8_t)(text[i] + 1);
    s[n] = 0;
    std::vector<uint32_t> SA;
    try {
        SA.resize(N);
    } catch (const std::bad_alloc &) {
        return BWFM_E_NOMEM;
    }
    sais<uint8_t>(s.data(), SA.data(), N, 5);
    std::vector<uint8_t>().swap(s);

    const uint32_t lw = line_bytes / 4;
    const uint64_t n_lines = N / bpl + 1;
    out.lines.assign(n_lines * lw, 0);
    out.sa.assign(n / sa_sample + 1, 0);
    uint64_t cnt[4] = {0, 0, 0, 0};
    for (uint64_t j = 0; j < N; j++) {
        uint64_t line = j / bpl, r = j - line * bpl;
        uint32_t *L = &out.lines[line * lw];
        if (r == 0)
            for (int a = 0; a < 4; a++) L[a] = (uint32_t)cnt[a];
        uint32_t q = SA[j];
        uint32_t c = q == 0 ? 0 : text[q - 1];  // $ stored as A
        if (q == 0) out.primary = j;
        L[4 + 2 * (r >> 5)] |= (c >> 1) << (r & 31);
        L[5 + 2 * (r >> 5)] |= (c & 1) << (r & 31);
        cnt[c]++;
        if ((j & (sa_sample - 1)) == 0) out.sa[j / sa_sample] = q;
    }
    if (N % bpl == 0) {
        uint32_t *L = &out.lines[(N / bpl) * lw];
        for (int a = 0; a < 4; a++) L[a] = (uint32_t)cnt[a];
    }
    cnt[0] -= 1;  // the $ row was counted as A
    out.C[0] = 1;
    for (int a = 1; a < 4; a++) out.C[a] = out.C[a - 1] + cnt[a - 1];
    if (rank_format == BWFM_RANK_SUBCOUNTS) subcount_lines(out.lines.data(), n_lines);
    if (rank_format == BWFM_RANK_SUB128) sub128_lines(out.lines.data(), n_lines);
    return BWFM_OK;
}

// Plane lines of 128 bytes and 384 rows (counts of A, C, G, T, then 24
// plane words) rewritten in place as 128-byte sub-counted lines.
void sub128_lines(uint32_t *lines, uint64_t n_lines) {
    for (uint64_t x = 0; x < n_lines; x++) {
        uint32_t *L = lines + x * 32, P[32];
        std::memcpy(P, L, sizeof P);
        uint32_t cum[3] = {0, 0, 0};  // C, G, T in the rows before the group
        for (int g = 0; g < 6; g++) {
            if (g > 0) L[2 + g] = cum[0] | (cum[1] << 9) | (cum[2] << 18);
            for (int w = 0; w < 2; w++) {
                const uint32_t h = P[4 + 4 * g + 2 * w], l = P[5 + 4 * g + 2 * w];
                cum[0] += (uint32_t)__builtin_popcount(~h & l);
                cum[1] += (uint32_t)__builtin_popcount(h & ~l);
                cum[2] += (uint32_t)__builtin_popcount(h & l);
            }
        }
        L[0] = P[1];
        L[1] = P[2];
        L[2] = P[3];
        for (int w = 0; w < 24; w++) L[8 + w] = P[4 + w];
    }
}

void subcount_lines(uint32_t *lines, uint64_t n_lines) {
    for (uint64_t x = 0; x < n_lines; x++) {
        uint32_t *L = lines + x * 16, P[16];
        std::memcpy(P, L, sizeof P);
        uint32_t cum[3] = {0, 0, 0}, sub[3] = {0, 0, 0};
        for (int g = 0; g < 5; g++) {
            const uint32_t h = P[4 + 2 * g], l = P[5 + 2 * g];
            if (g > 0)
                for (int b = 0; b < 3; b++) sub[b] |= cum[b] << (8 * (g - 1));
            cum[0] += (uint32_t)__builtin_popcount(~h & l);  // C
            cum[1] += (uint32_t)__builtin_popcount(h & ~l);  // G
            cum[2] += (uint32_t)__builtin_popcount(h & l);   // T
        }
        L[0] = P[1];
        L[1] = P[2];
        L[2] = P[3];
        for (int b = 0; b < 3; b++) L[3 + b] = sub[b];
        for (int w = 0; w < 10; w++) L[6 + w] = P[4 + w];
    }
}

static inline uint32_t planes_at(uint32_t rank_format) {
    return rank_format == BWFM_RANK_SUBCOUNTS ? 6 : (rank_format == BWFM_RANK_SUB128 ? 8 : 4);
}

static inline uint32_t code_at(const uint32_t *L, uint32_t po, uint64_t r) {
    return (((L[po + 2 * (r >> 5)] >> (r & 31)) & 1) << 1) | ((L[po + 1 + 2 * (r >> 5)] >> (r & 31)) & 1);
}

uint8_t bwt_host(const HostDir &d, uint32_t lw, uint32_t bpl, uint32_t rank_format, uint64_t row) {
    if (row == d.primary) return 4;
    uint64_t line = row / bpl, r = row - line * bpl;
    return (uint8_t)code_at(&d.lines[line * lw], planes_at(rank_format), r);
}

void occ_host(const HostDir &d, uint32_t lw, uint32_t bpl, uint32_t rank_format, uint64_t i, uint64_t out[4]) {
    uint64_t line = i / bpl, r = i - line * bpl;
    const uint32_t *L = &d.lines[line * lw];
    if (rank_format == BWFM_RANK_SUBCOUNTS) {
        // counts before the line, then at the start of row r's 32-row group
        // (the stored bytes), then the group's rows before r; A is the rest
        const uint64_t g = r >> 5;
        for (int b = 0; b < 3; b++) out[1 + b] = L[b] + (g ? (L[3 + b] >> (8 * (g - 1))) & 255u : 0u);
        for (uint64_t x = 32 * g; x < r; x++) {
            const uint32_t c = code_at(L, planes_at(rank_format), x);
            if (c) out[c]++;
        }
        out[0] = i - out[1] - out[2] - out[3] - (i > d.primary ? 1 : 0);
        return;
    }
    if (rank_format == BWFM_RANK_SUB128) {
        // counts before the line, at the start of row r's 64-row group (the
        // boundary word), then the group's rows before r
        const uint64_t g = r >> 6;
        const uint32_t bw = g ? L[2 + g] : 0u;
        for (int b = 0; b < 3; b++) out[1 + b] = L[b] + ((bw >> (9 * b)) & 511u);
        for (uint64_t x = 64 * g; x < r; x++) {
            const uint32_t c = code_at(L, planes_at(rank_format), x);
            if (c) out[c]++;
        }
        out[0] = i - out[1] - out[2] - out[3] - (i > d.primary ? 1 : 0);
        return;
    }
    for (int a = 0; a < 4; a++) out[a] = L[a];
    for (uint64_t x = 0; x < r; x++) out[code_at(L, planes_at(rank_format), x)]++;
    if (i > d.primary) out[0]--;
}

std::string &last_error() {
    thread_local std::string e;
    return e;
}

int fail(int code, const std::string &msg) {
    last_error() = msg;
    return code;
}

}  // namespace bwfm

using namespace bwfm;

namespace bwfm {

int check_index_params(bwfm_index_params &q, uint64_t n) {
    if (q.line_bytes != 32 && q.line_bytes != 64 && q.line_bytes != 128)
        return fail(BWFM_E_INVAL, "line_bytes must be 32, 64 or 128");
    if (q.rank_format != BWFM_RANK_PLANES && q.rank_format != BWFM_RANK_SUBCOUNTS &&
        q.rank_format != BWFM_RANK_SUB128)
        return fail(BWFM_E_INVAL, "unknown rank_format");
    if (q.rank_format == BWFM_RANK_SUBCOUNTS) {
        if (q.bases_per_line == 0) q.bases_per_line = 160;
        if (q.line_bytes != 64 || q.bases_per_line != 160)
            return fail(BWFM_E_INVAL, "sub-counted rank lines are 64 bytes of 160 rows");
    }
    if (q.rank_format == BWFM_RANK_SUB128) {
        if (q.bases_per_line == 0) q.bases_per_line = 384;
        if (q.line_bytes != 128 || q.bases_per_line != 384)
            return fail(BWFM_E_INVAL, "128-byte sub-counted rank lines are 128 bytes of 384 rows");
    }
    uint32_t maxb = (q.line_bytes - 16) * 4;
    if (q.bases_per_line == 0) q.bases_per_line = maxb;
    if (q.bases_per_line % 32 || q.bases_per_line < 32 || q.bases_per_line > maxb)
        return fail(BWFM_E_INVAL, "bases_per_line must be a multiple of 32 in [32, (line_bytes-16)*4]");
    if (q.sa_sample < 1 || q.sa_sample > 1024 || (q.sa_sample & (q.sa_sample - 1)))
        return fail(BWFM_E_INVAL, "sa_sample must be a power of two in [1, 1024]");
    if (n < 1) return fail(BWFM_E_INVAL, "empty reference");
    if (n + 1 >= (1ULL << 32)) return fail(BWFM_E_TOOLONG, "reference too long for 32-bit positions");
    return BWFM_OK;
}

void pack_ref(const uint8_t *text, uint64_t n, std::vector<uint32_t> &out) {
    out.assign((n + 15) / 16, 0u);
    for (uint64_t i = 0; i < n; i++) out[i >> 4] |= (uint32_t)(text[i] & 3) << (2 * (i & 15));
}

}  // namespace bwfm

extern "C" int bwfm_build_index(const uint8_t *ref, uint64_t n, const bwfm_index_params *p, bwfm_index **out) {
    if (!ref || !out) return fail(BWFM_E_INVAL, "build_index: NULL argument");
    *out = nullptr;
    bwfm_index_params q = p ? *p : bwfm_index_params{128, 0, 32, 0, BWFM_RANK_PLANES};
    if (int rc = check_index_params(q, n)) return rc;
    for (uint64_t i = 0; i < n; i++)
        if (ref[i] > 3) return fail(BWFM_E_BASE, "reference holds a code outside 0..3 at " + std::to_string(i));
    bwfm_index *ix = new (std::nothrow) bwfm_index;
    if (!ix) return fail(BWFM_E_NOMEM, "out of host memory");
    ix->n = n;
    ix->line_bytes = q.line_bytes;
    ix->bpl = q.bases_per_line;
    ix->sa_sample = q.sa_sample;
    ix->rank_format = q.rank_format;
    ix->n_lines = (n + 1) / q.bases_per_line + 1;
    ix->n_samples = n / q.sa_sample + 1;
    std::vector<uint8_t> rev(ref, ref + n);
    std::reverse(rev.begin(), rev.end());
    int rc[2] = {BWFM_OK, BWFM_OK};
    auto job = [&](int d) {
        try {
            rc[d] = build_dir(d == 0 ? ref : rev.data(), n, q.line_bytes, q.bases_per_line, q.sa_sample,
                              q.rank_format, ix->dir[d]);
        } catch (const std::bad_alloc &) {
            rc[d] = BWFM_E_NOMEM;
        }
    };
    bool par = q.n_threads != 1;
    if (par) {
        std::thread t(job, 1);
        job(0);
        t.join();
    } else {
        job(0);
        job(1);
    }
    if (rc[0] || rc[1]) {
        delete ix;
        return fail(rc[0] ? rc[0] : rc[1], "index build failed (out of memory)");
    }
    try {
        pack_ref(ref, n, ix->pac);
    } catch (const std::bad_alloc &) {
        delete ix;
        return fail(BWFM_E_NOMEM, "index build failed (out of memory)");
    }
    *out = ix;
    return BWFM_OK;
}

extern "C" int bwfm_index_get_info(const bwfm_index *ix, bwfm_index_info *o) {
    if (!ix || !o) return fail(BWFM_E_INVAL, "get_info: NULL argument");
    std::memset(o, 0, sizeof(*o));
    o->n = ix->n;
    for (int d = 0; d < 2; d++) {
        o->primary[d] = ix->dir[d].primary;
        for (int a = 0; a < 4; a++) o->C[d][a] = ix->dir[d].C[a];
    }
    o->lines = ix->n_lines;
    o->sa_samples = ix->n_samples;
    o->device_bytes = ix->device_bytes;
    o->line_bytes = ix->line_bytes;
    o->bases_per_line = ix->bpl;
    o->sa_sample = ix->sa_sample;
    o->uploaded = ix->device >= 0;
    o->rank_format = ix->rank_format;
    o->kmer_levels = ix->kt_levels;
    o->kmer_bytes = ix->kt_levels ? 2 * ((8 * bwfm::kt_level_start((int)ix->kt_levels + 1) + 255) / 256 * 256) : 0;
    bwfm_index *mix = const_cast<bwfm_index *>(ix);
    std::lock_guard<std::mutex> g(mix->ws_mu);
    for (auto &kv : mix->ws) o->ws_bytes += kv.second->bytes + kv.second->pos_bytes;
    o->ws_streams = (uint32_t)mix->ws.size();
    return BWFM_OK;
}

extern "C" int bwfm_index_get_bwt(const bwfm_index *ix, int which, uint8_t *out) {
    if (!ix || !out || which < 0 || which > 1) return fail(BWFM_E_INVAL, "get_bwt: bad argument");
    for (uint64_t r = 0; r <= ix->n; r++)
        out[r] = bwt_host(ix->dir[which], ix->line_bytes / 4, ix->bpl, ix->rank_format, r);
    return BWFM_OK;
}

extern "C" int bwfm_index_get_sa_samples(const bwfm_index *ix, int which, uint32_t *out) {
    if (!ix || !out || which < 0 || which > 1) return fail(BWFM_E_INVAL, "get_sa_samples: bad argument");
    std::memcpy(out, ix->dir[which].sa.data(), ix->dir[which].sa.size() * 4);
    return BWFM_OK;
}

extern "C" int bwfm_index_get_ref(const bwfm_index *ix, uint64_t start, uint64_t len, uint8_t *out) {
    if (!ix || (!out && len) || start > ix->n || len > ix->n - start) return fail(BWFM_E_INVAL, "get_ref: bad argument");
    for (uint64_t i = 0; i < len; i++) {
        const uint64_t p = start + i;
        out[i] = (uint8_t)((ix->pac[p >> 4] >> (2 * (p & 15))) & 3);
    }
    return BWFM_OK;
}

extern "C" int bwfm_index_occ(const bwfm_index *ix, int which, uint64_t i, uint64_t *out) {
    if (!ix || !out || which < 0 || which > 1 || i > ix->n + 1) return fail(BWFM_E_INVAL, "occ: bad argument");
    occ_host(ix->dir[which], ix->line_bytes / 4, ix->bpl, ix->rank_format, i, out);
    return BWFM_OK;
}

// ------------------------------------------------------------------ index files

namespace {

constexpr char FILE_MAGIC[8] = {'B', 'W', 'F', 'M', 'I', 'D', 'X', 0};
constexpr uint32_t FILE_VERSION = 2;

struct Fnv {
    uint64_t h = 1469598103934665603ULL;
    void add(const void *p, size_t n) {
        const uint8_t *b = static_cast<const uint8_t *>(p);
        for (size_t i = 0; i < n; i++) {
            h ^= b[i];
            h *= 1099511628211ULL;
        }
    }
};

struct Writer {
    FILE *f;
    Fnv sum;
    bool ok = true;
    void put(const void *p, size_t n) {
        if (!ok || n == 0) return;
        sum.add(p, n);
        ok = std::fwrite(p, 1, n, f) == n;
    }
    template <class T> void val(T v) { put(&v, sizeof v); }
};

struct Reader {
    FILE *f;
    Fnv sum;
    bool ok = true;
    void get(void *p, size_t n) {
        if (!ok || n == 0) return;
        ok = std::fread(p, 1, n, f) == n;
        if (ok) sum.add(p, n);
    }
    template <class T> T val() {
        T v{};
        get(&v, sizeof v);
        return v;
    }
};

}  // namespace

extern "C" int bwfm_index_save(const bwfm_index *ix, const char *path) {
    if (!ix || !path) return fail(BWFM_E_INVAL, "index_save: NULL argument");
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(BWFM_E_IO, std::string("index_save: cannot open ") + path);
    Writer w{f};
    w.put(FILE_MAGIC, 8);
    w.val<uint32_t>(FILE_VERSION);
    w.val<uint32_t>(ix->line_bytes);
    w.val<uint32_t>(ix->bpl);
    w.val<uint32_t>(ix->sa_sample);
    w.val<uint32_t>(ix->rank_format);
    w.val<uint64_t>(ix->n);
    w.val<uint64_t>(ix->n_lines);
    w.val<uint64_t>(ix->n_samples);
    for (int d = 0; d < 2; d++) {
        const HostDir &h = ix->dir[d];
        for (int a = 0; a < 4; a++) w.val<uint64_t>(h.C[a]);
        w.val<uint64_t>(h.primary);
        w.val<uint64_t>(h.lines.size());
        w.put(h.lines.data(), h.lines.size() * 4);
        w.val<uint64_t>(h.sa.size());
        w.put(h.sa.data(), h.sa.size() * 4);
    }
    w.val<uint64_t>(ix->pac.size());
    w.put(ix->pac.data(), ix->pac.size() * 4);
    const uint64_t sum = w.sum.h;
    if (w.ok) w.ok = std::fwrite(&sum, 1, 8, f) == 8;
    const bool closed = std::fclose(f) == 0;
    if (!w.ok || !closed) return fail(BWFM_E_IO, std::string("index_save: write failed on ") + path);
    return BWFM_OK;
}

extern "C" int bwfm_index_load(const char *path, bwfm_index **out) {
    if (!path || !out) return fail(BWFM_E_INVAL, "index_load: NULL argument");
    *out = nullptr;
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(BWFM_E_IO, std::string("index_load: cannot open ") + path);
    std::unique_ptr<FILE, int (*)(FILE *)> guard(f, std::fclose);
    std::fseek(f, 0, SEEK_END);
    const long fsize = std::ftell(f);
    std::fseek(f, 0, SEEK_SET);
    Reader r{f};
    char magic[8];
    r.get(magic, 8);
    if (!r.ok || std::memcmp(magic, FILE_MAGIC, 8) != 0) return fail(BWFM_E_IO, "index_load: not an index file");
    if (r.val<uint32_t>() != FILE_VERSION) return fail(BWFM_E_IO, "index_load: unsupported file version");
    std::unique_ptr<bwfm_index> ix(new (std::nothrow) bwfm_index);
    if (!ix) return fail(BWFM_E_NOMEM, "out of host memory");
    ix->line_bytes = r.val<uint32_t>();
    ix->bpl = r.val<uint32_t>();
    ix->sa_sample = r.val<uint32_t>();
    ix->rank_format = r.val<uint32_t>();
    ix->n = r.val<uint64_t>();
    ix->n_lines = r.val<uint64_t>();
    ix->n_samples = r.val<uint64_t>();
    // the layout must be one the builder could have made, and the sizes
    // must follow from it, before anything is allocated
    const bool layout_ok = (ix->line_bytes == 32 || ix->line_bytes == 64 || ix->line_bytes == 128) && ix->bpl % 32 == 0 &&
                           ix->bpl >= 32 &&
                           ix->bpl <= (ix->line_bytes - 16) * 4 && ix->sa_sample >= 1 && ix->sa_sample <= 1024 &&
                           (ix->sa_sample & (ix->sa_sample - 1)) == 0 && ix->n >= 1 && ix->n + 1 < (1ULL << 32) &&
                           (ix->rank_format == BWFM_RANK_PLANES ||
                            (ix->rank_format == BWFM_RANK_SUBCOUNTS && ix->line_bytes == 64 && ix->bpl == 160) ||
                            (ix->rank_format == BWFM_RANK_SUB128 && ix->line_bytes == 128 && ix->bpl == 384)) &&
                           ix->n_lines == (ix->n + 1) / ix->bpl + 1 && ix->n_samples == ix->n / ix->sa_sample + 1;
    if (!r.ok || !layout_ok) return fail(BWFM_E_IO, "index_load: corrupt header");
    const uint64_t words = ix->n_lines * (ix->line_bytes / 4);
    const uint64_t pac_words = (ix->n + 15) / 16;
    const uint64_t expect =
        8 + 5 * 4 + 3 * 8 + 2 * (6 * 8 + words * 4 + 8 + ix->n_samples * 4) + 8 + pac_words * 4 + 8;
    if (fsize < 0 || (uint64_t)fsize != expect) return fail(BWFM_E_IO, "index_load: file size does not match header");
    try {
        for (int d = 0; d < 2; d++) {
            HostDir &h = ix->dir[d];
            for (int a = 0; a < 4; a++) h.C[a] = r.val<uint64_t>();
            h.primary = r.val<uint64_t>();
            if (r.val<uint64_t>() != words) return fail(BWFM_E_IO, "index_load: corrupt rank-line count");
            h.lines.resize(words);
            r.get(h.lines.data(), words * 4);
            if (r.val<uint64_t>() != ix->n_samples) return fail(BWFM_E_IO, "index_load: corrupt SA sample count");
            h.sa.resize(ix->n_samples);
            r.get(h.sa.data(), ix->n_samples * 4);
            if (h.primary > ix->n) return fail(BWFM_E_IO, "index_load: corrupt $ row");
        }
        if (r.val<uint64_t>() != pac_words) return fail(BWFM_E_IO, "index_load: corrupt reference size");
        ix->pac.resize(pac_words);
        r.get(ix->pac.data(), pac_words * 4);
    } catch (const std::bad_alloc &) {
        return fail(BWFM_E_NOMEM, "out of host memory");
    }
    const uint64_t sum = r.sum.h;
    uint64_t stored = 0;
    if (!r.ok || std::fread(&stored, 1, 8, f) != 8) return fail(BWFM_E_IO, "index_load: truncated file");
    if (stored != sum) return fail(BWFM_E_IO, "index_load: checksum mismatch");
    *out = ix.release();
    return BWFM_OK;
}
