// Library-internal definitions shared by the host index builder, the C ABI
// and the kernel launchers.  Not part of the public interface.
#pragma once

#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <shared_mutex>
#include <string>
#include <vector>

#include "../../include/bwfm.h"

namespace bwfm {

// One direction of the index (0: index of T, 1: index of reverse(T)).
struct HostDir {
    std::vector<uint32_t> lines;  // lines * line_words32: 4 counts, then packed rows
    std::vector<uint32_t> sa;     // SA[r] for r % sa_sample == 0
    uint64_t C[4] = {0, 0, 0, 0};
    uint64_t primary = 0;
};

// Device-side view of one direction, passed to kernels by value.
struct DevDir {
    const uint32_t *lines;  // line_words32 uint32 per line, 16-byte aligned
    const uint32_t *sa;
    uint32_t C[4];
    uint32_t primary;
    uint32_t pad;
    const uint32_t *kt;  // short-string interval table, (k, l) word pairs (kt_level_start), or null
};

struct DevIndex {
    DevDir dir[2];
    uint64_t magic;       // floor(2^64 / bases_per_line) + 1: row / bpl = mulhi(row, magic)
    uint32_t n;           // text length (n + 1 < 2^32)
    uint32_t bpl;         // rows per rank line
    uint32_t sa_shift;    // log2(sa_sample)
    uint32_t line_words;  // uint32 words per line
    uint32_t kt_levels;   // levels of the short-string table (0: none)
};

// First entry of level d of the short-string table: level 0 is entry 0,
// level d >= 1 starts at 4 + (4^d - 4) / 3, a multiple of 4.
constexpr uint64_t kt_level_start(int d) {
    return d == 0 ? 0 : 4 + (((uint64_t)1 << (2 * d)) - 4) / 3;
}

// Grow-only device scratch of one stream: calls on that stream carve their
// temporaries from it; its mutex is held for the whole of a call, so calls
// on one stream from several threads take turns while calls on different
// streams proceed together.
struct Workspace {
    void *ptr = nullptr;  // control buffers and per-read temporaries
    size_t bytes = 0;
    void *pos = nullptr;  // located positions (bwfm_pair_reads)
    size_t pos_bytes = 0;
    std::mutex mu;
};

std::string &last_error();
int fail(int code, const std::string &msg);

// Validate a layout (filling in bases_per_line = 0) for a reference of n
// bases; 0 or a bwfm_err with the message set.
int check_index_params(bwfm_index_params &q, uint64_t n);

// Host index builder and inspection (index_host.cpp).
int build_dir(const uint8_t *text, uint64_t n, uint32_t line_bytes, uint32_t bpl, uint32_t sa_sample,
              uint32_t rank_format, HostDir &out);
// rewrite planar 64-byte lines of 160 rows as sub-counted ones, in place
void subcount_lines(uint32_t *lines, uint64_t n_lines);
void sub128_lines(uint32_t *lines, uint64_t n_lines);
void occ_host(const HostDir &d, uint32_t line_words, uint32_t bpl, uint32_t rank_format, uint64_t i,
              uint64_t out[4]);
uint8_t bwt_host(const HostDir &d, uint32_t line_words, uint32_t bpl, uint32_t rank_format, uint64_t row);
// T packed two bits per base, 16 bases per word, base i in bits 2 (i % 16)
// of word i / 16 (unused high bits of the last word zero)
void pack_ref(const uint8_t *text, uint64_t n, std::vector<uint32_t> &out);

}  // namespace bwfm

struct bwfm_index {
    uint64_t n = 0;
    uint32_t line_bytes = 128, bpl = 448, sa_sample = 32, rank_format = BWFM_RANK_PLANES;
    uint64_t n_lines = 0, n_samples = 0;
    bwfm::HostDir dir[2];
    std::vector<uint32_t> pac;  // the reference itself (pack_ref), for mate rescue
    // device copies (valid when uploaded)
    int device = -1;
    void *d_lines[2] = {nullptr, nullptr};
    void *d_sa[2] = {nullptr, nullptr};
    void *d_pac = nullptr;
    void *d_kt[2] = {nullptr, nullptr};  // short-string interval tables
    uint32_t kt_levels = 0;
    uint64_t kt_gen = 0;  // bumped whenever the table changes (captured graphs hold its address)
    uint64_t device_bytes = 0;
    // held shared by calls that only read the index's device state (align,
    // locate, pair), exclusively by calls that change it (upload, the
    // short-string table)
    std::shared_mutex mu;
    std::mutex ws_mu;                                           // guards ws
    std::map<void *, std::unique_ptr<bwfm::Workspace>> ws;      // one per stream used
};
