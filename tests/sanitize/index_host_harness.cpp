// Host index builder under AddressSanitizer and UndefinedBehaviorSanitizer:
// builds, queries, saves and reloads indexes of several texts in every
// rank-line layout, and takes each argument-error path once.  Consistency
// checks here are light (Occ totals, the LF walk back to position 0, a
// reloaded copy equal to the original); exactness against the oracle is the
// job of the library's CPU tests.  Exit status 0 = every check passed and
// no sanitizer reported.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../../paper_1505_07855_amd/csrc/bwfm_internal.h"

// The library's bwfm_index_free also releases device memory; indexes built
// here never reach a device, so releasing the host object is all it does.
extern "C" void bwfm_index_free(bwfm_index *ix) { delete ix; }

static int failures = 0;
#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            failures++;                                                      \
        }                                                                    \
    } while (0)

static std::vector<std::vector<uint8_t>> texts() {
    std::mt19937_64 rng(7);
    std::vector<std::vector<uint8_t>> out;
    std::vector<uint8_t> t(20000);
    for (auto &x : t) x = (uint8_t)(rng() & 3);
    out.push_back(t);
    out.push_back(std::vector<uint8_t>(1, 2));
    out.push_back(std::vector<uint8_t>(3000, 0));
    std::vector<uint8_t> per(5001);
    for (size_t i = 0; i < per.size(); i++) per[i] = (uint8_t)"\x00\x01\x02\x03\x03"[i % 5];
    out.push_back(per);
    std::vector<uint8_t> rep(12000);
    for (auto &x : rep) x = (uint8_t)(rng() & 3);
    std::memcpy(rep.data() + 6000, rep.data() + 1000, 4000);
    out.push_back(rep);
    std::vector<uint8_t> exact(383);  // n + 1 a multiple of 384 and of 32
    for (auto &x : exact) x = (uint8_t)(rng() & 3);
    out.push_back(exact);
    return out;
}

static void check_one(const std::vector<uint8_t> &t, bwfm_index_params q, const char *tmp) {
    bwfm_index *ix = nullptr;
    int rc = bwfm_build_index(t.data(), t.size(), &q, &ix);
    CHECK(rc == BWFM_OK && ix);
    if (rc) return;
    bwfm_index_info info;
    CHECK(bwfm_index_get_info(ix, &info) == BWFM_OK);
    const uint64_t n = t.size();
    std::vector<uint8_t> bwt(n + 1), bwt2(n + 1), ref(n);
    std::vector<uint32_t> sa(info.sa_samples), sa2(info.sa_samples);
    for (int which = 0; which < 2; which++) {
        CHECK(bwfm_index_get_bwt(ix, which, bwt.data()) == BWFM_OK);
        CHECK(bwfm_index_get_sa_samples(ix, which, sa.data()) == BWFM_OK);
        uint64_t tot[4] = {0, 0, 0, 0};
        CHECK(bwfm_index_occ(ix, which, n + 1, tot) == BWFM_OK);
        uint64_t cnt[4] = {0, 0, 0, 0};
        for (uint8_t c : t) cnt[c]++;
        for (int a = 0; a < 4; a++) CHECK(tot[a] == cnt[a]);
        // LF walk from the $ row's successor back through the whole text
        uint64_t row = 0;
        for (uint64_t step = 0; step < n; step++) {
            const uint8_t a = bwt[row];
            CHECK(a < 4);
            if (a >= 4) break;
            uint64_t o[4];
            CHECK(bwfm_index_occ(ix, which, row, o) == BWFM_OK);
            const uint8_t want = which == 0 ? t[n - 1 - step] : t[step];
            CHECK(a == want);
            row = info.C[which][a] + o[a];
        }
        CHECK(row == info.primary[which]);
    }
    CHECK(bwfm_index_get_ref(ix, 0, n, ref.data()) == BWFM_OK && ref == t);
    CHECK(bwfm_index_get_ref(ix, n, 1, ref.data()) != BWFM_OK);
    // save, reload, compare
    CHECK(bwfm_index_save(ix, tmp) == BWFM_OK);
    bwfm_index *iy = nullptr;
    CHECK(bwfm_index_load(tmp, &iy) == BWFM_OK && iy);
    if (iy) {
        for (int which = 0; which < 2; which++) {
            CHECK(bwfm_index_get_bwt(ix, which, bwt.data()) == BWFM_OK);
            CHECK(bwfm_index_get_bwt(iy, which, bwt2.data()) == BWFM_OK);
            CHECK(bwt == bwt2);
            CHECK(bwfm_index_get_sa_samples(ix, which, sa.data()) == BWFM_OK);
            CHECK(bwfm_index_get_sa_samples(iy, which, sa2.data()) == BWFM_OK);
            CHECK(sa == sa2);
            for (uint64_t i = 0; i <= n + 1; i += 1 + n / 97) {
                uint64_t a[4], b[4];
                CHECK(bwfm_index_occ(ix, which, i, a) == BWFM_OK && bwfm_index_occ(iy, which, i, b) == BWFM_OK);
                CHECK(std::memcmp(a, b, sizeof a) == 0);
            }
        }
        bwfm_index_free(iy);
    }
    // a corrupted copy is refused
    if (FILE *f = std::fopen(tmp, "r+b")) {
        std::fseek(f, 40, SEEK_SET);
        int c = std::fgetc(f);
        std::fseek(f, 40, SEEK_SET);
        std::fputc(c ^ 0x5a, f);
        std::fclose(f);
        bwfm_index *iz = nullptr;
        CHECK(bwfm_index_load(tmp, &iz) != BWFM_OK && !iz);
    }
    bwfm_index_free(ix);
}

int main(int argc, char **argv) {
    const std::string tmp = std::string(argc > 1 ? argv[1] : "/tmp") + "/bwfm_sanitize_index.bin";
    const bwfm_index_params layouts[] = {
        {128, 0, 32, 0, BWFM_RANK_PLANES},      {64, 0, 32, 1, BWFM_RANK_PLANES},
        {64, 128, 1, 2, BWFM_RANK_PLANES},      {32, 0, 8, 0, BWFM_RANK_PLANES},
        {128, 448, 1024, 0, BWFM_RANK_PLANES},  {64, 0, 32, 0, BWFM_RANK_SUBCOUNTS},
        {64, 160, 4, 1, BWFM_RANK_SUBCOUNTS},   {128, 0, 32, 0, BWFM_RANK_SUB128},
        {128, 384, 2, 2, BWFM_RANK_SUB128},
    };
    for (const auto &t : texts())
        for (const auto &q : layouts) check_one(t, q, tmp.c_str());
    // argument errors
    std::vector<uint8_t> t(100, 1);
    bwfm_index *ix = nullptr;
    const bwfm_index_params bad[] = {
        {48, 0, 32, 0, BWFM_RANK_PLANES},   {64, 100, 32, 0, BWFM_RANK_PLANES}, {64, 0, 3, 0, BWFM_RANK_PLANES},
        {64, 0, 32, 0, 7},                  {128, 0, 32, 0, BWFM_RANK_SUBCOUNTS}, {64, 0, 32, 0, BWFM_RANK_SUB128},
        {128, 448, 32, 0, BWFM_RANK_SUB128},
    };
    for (const auto &q : bad) {
        CHECK(bwfm_build_index(t.data(), t.size(), &q, &ix) == BWFM_E_INVAL && !ix);
    }
    t[50] = 4;
    CHECK(bwfm_build_index(t.data(), t.size(), nullptr, &ix) == BWFM_E_BASE && !ix);
    CHECK(bwfm_build_index(t.data(), 0, nullptr, &ix) == BWFM_E_INVAL && !ix);
    CHECK(bwfm_build_index(nullptr, 10, nullptr, &ix) == BWFM_E_INVAL);
    CHECK(bwfm_index_load((tmp + ".missing").c_str(), &ix) == BWFM_E_IO && !ix);
    std::remove(tmp.c_str());
    if (failures) std::fprintf(stderr, "%d checks failed\n", failures);
    else std::printf("index host harness: all checks passed\n");
    return failures ? 1 : 0;
}
