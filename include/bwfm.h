/*
 * bwfm -- FM-index short-read alignment on AMD Instinct MI355X (gfx950).
 *
 * The method is the one BarraCUDA runs on the GPU (W. B. Langdon and
 * B. Y. H. Lam, "Genetically Improved BarraCUDA", 2015, section 2): the
 * reference genome is encoded offline into an index in which all suffixes
 * that share a prefix sit together; each read is looked up by keeping an
 * upper and a lower pointer into that index and narrowing them one base at
 * a time (their distance is the number of matching positions; crossed
 * pointers mean no match); inexact reads are handled by backing up the
 * search and trying alternatives; the whole index lives in GPU memory; the
 * two ends of a pair are aligned separately and then combined ("aln" then
 * "sampe", section 3.7), using the approximate fragment length to discard
 * placements that lie too far apart.  The search details follow the BWA
 * short-read backtracking method that BarraCUDA derives from.
 *
 * Conventions
 *  - Base codes: A=0, C=1, G=2, T=3; reads may also hold 4 (N), which
 *    mismatches every reference base.  Symbol order $ < A < C < G < T.
 *  - Every call returns 0 (BWFM_OK) or a negative bwfm_err.  On error
 *    nothing is written to caller buffers except where a call says so;
 *    bwfm_last_error() then describes the failure (per calling thread).
 *  - "device" pointers are HIP device memory on the current device (for
 *    example torch tensors' data_ptr()); "host" pointers are ordinary host
 *    memory.  Work is issued on the hip_stream argument (a hipStream_t
 *    passed as void *, NULL = the default stream).
 *  - The caller owns every buffer it passes in.  The library owns the
 *    index (host and device copies) and, per index, one grow-only device
 *    workspace for each stream it has been called on, all released by
 *    bwfm_index_free.
 *  - Concurrency.  The index is read-only after upload: bwfm_align_batch,
 *    bwfm_locate and bwfm_pair_reads calls on different streams may run at
 *    the same time from different host threads, and their kernels overlap
 *    on the device; each uses its own stream's workspace.  Calls on one
 *    stream from several threads take turns.  bwfm_index_upload and
 *    bwfm_index_kmer_table change the index and wait for the calls in
 *    flight; bwfm_index_free must not overlap any other call on the index.
 *  - The three calls above block the calling thread until their own stream
 *    has finished the call's work (the number of hits decides the output
 *    size, which they check); the captured step (bwfm_pipeline_*) is the
 *    fully asynchronous form, with every count and capacity checked on the
 *    device.
 */
#ifndef BWFM_H
#define BWFM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum bwfm_err {
    BWFM_OK = 0,
    BWFM_E_INVAL = -1,    /* bad argument (NULL pointer, bad size or parameter) */
    BWFM_E_NOMEM = -2,    /* host or device allocation failed */
    BWFM_E_BASE = -3,     /* reference holds a code other than 0..3 */
    BWFM_E_TOOLONG = -4,  /* reference too long (n + 1 >= 2^32) or read bound above 512 */
    BWFM_E_CAPACITY = -5, /* a caller buffer is too small; see the call for what is reported */
    BWFM_E_DEVICE = -6,   /* a HIP runtime call failed */
    BWFM_E_STATE = -7,    /* index not uploaded to the device */
    BWFM_E_IO = -8        /* a file could not be read or written, or is not an index file */
};

/* Longest read and largest per-read difference budget accepted. */
#define BWFM_MAX_READ 512
#define BWFM_MAX_DIFF 15

/* ------------------------------------------------------------------ */
/* Index (section 2: the offline encoding of the reference; section 3.4:
 * it must be resident in GPU memory for the search)                    */
/* ------------------------------------------------------------------ */

typedef struct bwfm_index bwfm_index;

typedef struct {
    uint32_t line_bytes;     /* rank line size: 32, 64 or 128 bytes */
    uint32_t bases_per_line; /* BWT rows per rank line: a multiple of 32 in
                                [32, (line_bytes - 16) * 4]; 0 = the maximum
                                (64 for 32-byte lines, 192 for 64, 448 for 128) */
    uint32_t sa_sample;      /* rows r with r % sa_sample == 0 keep SA[r];
                                a power of two in [1, 1024] */
    uint32_t n_threads;      /* host threads for the build; 0 = all cores */
    uint32_t rank_format;    /* BWFM_RANK_PLANES, BWFM_RANK_SUBCOUNTS or BWFM_RANK_SUB128 */
} bwfm_index_params;

/* Rank-line formats.  PLANES: 16 bytes of counts (A, C, G, T before the
 * line), then the rows.  SUBCOUNTS (64-byte lines of 160 rows only): 12
 * bytes of counts (C, G, T before the line; A follows from the row number),
 * then for each of C, G and T a uint32 of four bytes, byte g - 1 counting
 * that base in the line's first 32 g rows (g = 1..4), then the rows; a rank
 * query then counts bits in one 32-row group only.  SUB128 (128-byte lines
 * of 384 rows only): C, G, T before the line (12 bytes), then five uint32
 * boundary words, word g - 1 holding the counts of C, G and T in the
 * line's first 64 g rows (g = 1..5) as C | G << 9 | T << 18, then the rows;
 * a rank query reads the line's first 32 bytes at most and the 16 bytes of
 * its row's 64-row group, all inside the one 128-byte line.  Rows in every
 * format: for each 32 rows a uint32 of the 2-bit codes' high bits, then one
 * of their low bits. */
#define BWFM_RANK_PLANES 0
#define BWFM_RANK_SUBCOUNTS 1
#define BWFM_RANK_SUB128 2

/*
 * Build the FM-index of T = ref[0, n) and of reverse(T) on the host.
 *   ref: host, n codes 0..3 (borrowed for the call only).
 *   p:   layout; NULL = {128, 0, 32, 0, BWFM_RANK_PLANES}.
 *   out: receives a new index (host part only; see bwfm_index_upload).
 * Each direction holds the BWT of S$ with $ stored as A, the row of $
 * ("primary"), C[a] = 1 + #symbols < a, rank lines (4 x uint32 counts of
 * A, C, G, T before the line, $ counted as A, then the line's rows as bit
 * planes: for each 32 rows a uint32 of the 2-bit codes' high bits followed
 * by a uint32 of their low bits), and SA samples.  The index also keeps T
 * itself, two bits per base (16 bases per uint32, base i in bits 2 (i % 16)
 * of word i / 16), for mate rescue.  Errors: E_INVAL (NULL or bad layout),
 * E_BASE, E_TOOLONG (n + 1 >= 2^32), E_NOMEM.
 */
int bwfm_build_index(const uint8_t *ref, uint64_t n, const bwfm_index_params *p, bwfm_index **out);

/* The same index built on the current device: the suffix arrays of T$ and
 * reverse(T)$ by prefix doubling over device radix sorts (first keys of 21
 * symbols, then (rank, rank h further) pairs until all ranks differ), then
 * the rank lines and SA samples in device memory.  The result is uploaded
 * already and holds host copies too, byte for byte equal to
 * bwfm_build_index's.  Device scratch: about 30 bytes per reference base,
 * released before return.  ref is a host array.  Synchronises hip_stream.
 * Errors: as bwfm_build_index, plus E_DEVICE. */
int bwfm_build_index_device(const uint8_t *ref, uint64_t n, const bwfm_index_params *p, void *hip_stream,
                            bwfm_index **out);

/* Copy the index to the current device's memory (once; later calls are
 * no-ops).  Synchronises hip_stream.  Errors: E_INVAL, E_NOMEM, E_DEVICE. */
int bwfm_index_upload(bwfm_index *idx, void *hip_stream);

/* Short-string interval table (a device-side accelerator of the search in
 * section 2; it changes no result).  For each direction and each string S
 * of d <= levels bases (2 bits per base, the base prepended last in the
 * low bits: code(aS) = 4 code(S) + a), the table holds the SA interval
 * (k, l) of S on that direction's index, exactly as backward search steps
 * reach it (k > l when S does not occur).  Level d starts at entry
 * 4 + (4^d - 4) / 3 (level 0, entry 0, is the empty string's (0, n)), so
 * the four one-base extensions of a string are 32 contiguous,
 * 32-byte-aligned bytes.  The plain form's search and D-array scan, and
 * the batched form's second pass, take the children of a state whose
 * matched string is shorter than `levels` bases from there: one access in
 * place of two rank-line fetches.  The batched form's persistent first
 * pass does not: there it measured slower.  Built on the device from the
 * uploaded rank lines; replaces an existing table (no call that uses the
 * index may run meanwhile; captured pipeline steps are captured again on
 * their next run).  levels: 0 releases the table, -1 picks the smallest d
 * with 4^d >= n (at most 14: 2.9 GB per direction), 1..15 as given (15:
 * 11.5 GB per direction).  Synchronises hip_stream.  Errors: E_INVAL
 * (NULL, not uploaded, levels out of range; the index is left as it was),
 * E_NOMEM (the index is left without a table), E_DEVICE (it may be). */
int bwfm_index_kmer_table(bwfm_index *idx, int levels, void *hip_stream);

/* Host copy of count entries of level `level` of direction `which`'s
 * table, from string code `first` on, as (k, l) pairs: out (host,
 * 2 * count uint32).  For tests.  Errors: E_INVAL (no table, level above
 * its levels, range beyond 4^level codes), E_DEVICE. */
int bwfm_index_kmer_get(const bwfm_index *idx, int which, int level, uint64_t first, uint64_t count,
                        uint32_t *out);

/* Release host and device memory of the index and its workspace. */
void bwfm_index_free(bwfm_index *idx);

/* Write the host part of an index to path (created or truncated): a
 * little-endian header (magic, version 2, layout, n), then per direction C,
 * the $ row, the rank lines and the SA samples, then the packed reference,
 * then a 64-bit FNV-1a checksum of everything before it.  Errors: E_INVAL,
 * E_IO. */
int bwfm_index_save(const bwfm_index *idx, const char *path);

/* Read an index written by bwfm_index_save into a new host-only index
 * (upload it with bwfm_index_upload).  The checksum and every size are
 * verified before use.  Errors: E_INVAL (NULL), E_IO (unreadable, short,
 * corrupt or another version), E_NOMEM. */
int bwfm_index_load(const char *path, bwfm_index **out);

typedef struct {
    uint64_t n;             /* reference length */
    uint64_t primary[2];    /* row of $: [0] index of T, [1] index of reverse(T) */
    uint64_t C[2][4];       /* C[a] per direction */
    uint64_t lines;         /* rank lines per direction */
    uint64_t sa_samples;    /* SA samples per direction */
    uint64_t device_bytes;  /* device memory the uploaded index occupies */
    uint32_t line_bytes, bases_per_line, sa_sample, uploaded, rank_format;
    uint32_t kmer_levels;   /* levels of the device k-mer interval table (0: none) */
    uint64_t kmer_bytes;    /* device memory of that table, both directions (each padded to 256 bytes) */
    uint64_t ws_bytes;      /* device memory of the per-stream workspaces, summed */
    uint32_t ws_streams;    /* streams that have a workspace */
    uint32_t pad;
} bwfm_index_info;

int bwfm_index_get_info(const bwfm_index *idx, bwfm_index_info *out);

/* Host-side inspection of the packed index, for tests.  which: 0 = index
 * of T, 1 = index of reverse(T).
 *   get_bwt:  out (host, n + 1 bytes) <- BWT symbols, 4 at the $ row.
 *   get_sa_samples: out (host, info.sa_samples uint32) <- SA[r], r % sa_sample == 0.
 *   occ: out (host, 4 uint64) <- Occ(a, i) = #a in BWT[0, i), 0 <= i <= n + 1,
 *        decoded from the rank line holding row i. */
int bwfm_index_get_bwt(const bwfm_index *idx, int which, uint8_t *out);
int bwfm_index_get_sa_samples(const bwfm_index *idx, int which, uint32_t *out);
int bwfm_index_occ(const bwfm_index *idx, int which, uint64_t i, uint64_t *out);
/*   get_ref: out (host, len bytes) <- T[start, start + len), codes 0..3,
 *        decoded from the index's packed copy; start + len <= n. */
int bwfm_index_get_ref(const bwfm_index *idx, uint64_t start, uint64_t len, uint8_t *out);

/* ------------------------------------------------------------------ */
/* Alignment ("aln"; section 2: per-read search with backtracking)     */
/* ------------------------------------------------------------------ */

typedef struct {
    const uint8_t *bases;     /* device: read r starts at bases[offsets[r]] */
    const uint64_t *offsets;  /* device: n_reads + 1 non-decreasing offsets (read r
                                 ends at offsets[r+1]), or n_reads start offsets
                                 when lengths is given */
    const uint8_t *max_diff;  /* device, n_reads per-read budgets, or NULL */
    uint32_t n_reads;
    uint32_t max_len;         /* host-known bound on read length, <= 512 */
    const uint32_t *lengths;  /* device, n_reads read lengths, or NULL; with
                                 lengths, reads may sit anywhere in bases */
} bwfm_reads;

enum { BWFM_MODE_ALL = 0, BWFM_MODE_BEST = 1 };

/* Execution form; results are identical.  BATCHED: one persistent launch
 * whose lanes pull reads from a shared counter, each lane taking the next
 * read as soon as its current one is done.  PLAIN: one lane per read, one
 * launch per batch. */
enum { BWFM_FORM_BATCHED = 0, BWFM_FORM_PLAIN = 1 };

typedef struct {
    int32_t max_diff;       /* budget when reads.max_diff is NULL, 0..15 */
    int32_t max_gapo;       /* most gap opens */
    int32_t max_gape;       /* most gap extensions; -1 = limited by max_diff only */
    int32_t seed_len;       /* 5' seed length; 0 = no seed rule */
    int32_t seed_diff;      /* most differences inside the seed */
    int32_t indel_end_skip; /* no insertion within this many bases of either end */
    int32_t s_mm, s_gapo, s_gape; /* score of a mismatch, gap open, gap extension, 0..63 */
    int32_t mode;           /* BWFM_MODE_ALL or BWFM_MODE_BEST */
    int32_t max_best;       /* BEST: second tier reported only if c1 <= max_best */
    uint32_t max_hits;      /* reads with more candidate hits report none, 1..65536 */
    int32_t form;           /* BWFM_FORM_BATCHED or BWFM_FORM_PLAIN */
    int32_t waves_per_simd; /* batched form residency, 0..8.  0 or >= 4: the
                               kernel build held to 128 VGPRs, 4 waves per
                               SIMD; 3: the compiler's own register budget
                               (3 waves); 1, 2: that build capped at 1 or 2
                               waves per SIMD.  A tuning knob: results do not
                               depend on it. */
    int32_t split_budget;   /* batched form: once the batch's reads are all
                               taken, a lane whose part of a read's search
                               has expanded this many states hands the rest of
                               it to tasks that every lane of the device may
                               take (rounds of one launch each); the lanes
                               of a wave share the rest of their reads in
                               flight either way.  0 = the library's default
                               (16384), -1 = no splitting, else 16 .. 2^24.
                               A tuning knob: results do not depend on it. */
} bwfm_aln_params;

/*
 * One hit: a distinct reference string X matched by the read on one
 * strand, with the best transcript's counts.  Strand 0 (+): [k, l] is the
 * SA interval of reverse(X) in the index of reverse(T) (the read is
 * searched 5' end first); strand 1 (-): [k, l] is the interval of X in the
 * index of T, X matching revcomp(read).  len = |X|.
 */
typedef struct {
    uint32_t k, l;
    uint16_t len, score;
    uint8_t strand, n_mm, n_gapo, n_gape;
} bwfm_hit;

/* per-read status bits */
#define BWFM_ST_HIT 1      /* at least one hit reported */
#define BWFM_ST_OVERFLOW 2 /* more than max_hits candidates: none reported, c1 = c2 = 0xFFFFFFFF */
#define BWFM_ST_INVALID 4  /* read longer than reads.max_len / 512, or budget above 15 */
#define BWFM_ST_RESEARCH 8 /* informational: the read's search outgrew the first pass's
                              per-lane buffers and was redone with worst-case buffers */
#define BWFM_ST_SHARED 16  /* informational (batched form): parts of the read's search
                              tree were handed to other lanes once the batch ran dry;
                              results are unaffected, its work counter then covers a
                              different traversal than one lane's depth-first order */
#define BWFM_ST_SPLIT 32   /* informational (batched form): the read's search outgrew
                              split_budget and was finished by tasks spread over the
                              device; results are unaffected, its work counter covers
                              every part */

typedef struct {
    uint64_t *hit_offsets;  /* device, n_reads + 1: hits of read r are [hit_offsets[r], hit_offsets[r+1]) */
    bwfm_hit *hits;         /* device, hit_capacity entries */
    uint64_t hit_capacity;
    uint32_t *c1, *c2;      /* device, n_reads: summed widths of tier 1 and tier 2 */
    uint8_t *status;        /* device, n_reads */
} bwfm_aln_result;

/*
 * Align every read on both strands.  A transcript of read W against a
 * reference string X uses match/mismatch, insertion (read base only) and
 * deletion (reference base only); a gap is a maximal run of insertions or
 * of deletions; diffs = mismatches + gap opens + gap extensions; score =
 * s_mm n_mm + s_gapo n_gapo + s_gape n_gape.  Valid transcripts keep
 * diffs <= budget, gap opens <= max_gapo, extensions <= max_gape (if >= 0),
 * insertions at read indices [s, m - s), deletions at boundaries
 * [max(s,1), m - max(s,1)] (s = indel_end_skip), and at most seed_diff
 * differences inside the first seed_len bases as sequenced.  ALL mode
 * reports every (strand, X) with a valid transcript, each with its smallest
 * (score, diffs, n_gapo, n_mm).  BEST mode keeps tier 1 (minimum score S*)
 * and, when c1 <= max_best, tier 2 (S* < score <= S* + s_mm).  Hits are
 * ordered by (score, strand, k, len).  Reads longer than max_len or with a
 * budget above 15 get BWFM_ST_INVALID; empty reads get status 0.
 *
 * Synchronous: returns after the results are complete on hip_stream.
 * Errors: E_INVAL, E_STATE (index not uploaded), E_TOOLONG (max_len > 512),
 * E_NOMEM, E_DEVICE; E_CAPACITY when the hits do not fit hit_capacity --
 * then hit_offsets, c1, c2 and status are complete, hits is untouched, and
 * hit_offsets[n_reads] holds the capacity needed.
 */
int bwfm_align_batch(const bwfm_index *idx, const bwfm_reads *reads, const bwfm_aln_params *p,
                     bwfm_aln_result *res, void *hip_stream);

/* As bwfm_align_batch, also writing each read's search work -- the number
 * of search states expanded (each expansion issues the two rank queries at
 * k and l + 1), summed over both passes -- to expand (device, n_reads).
 * work (device, 14 uint64, or NULL; batched form only) receives the first
 * pass's loop iterations summed over waves, lane iterations spent on a read,
 * and lane iterations that issued a rank query, then the reads whose search
 * was split, the tasks handed out over all rounds, the split reads that went
 * on to the second pass, and for each of the eight task generations (the
 * first pass's, then each round's but the last) the task entries asked for
 * (more than the room when some split found none). */
int bwfm_align_batch_counted(const bwfm_index *idx, const bwfm_reads *reads, const bwfm_aln_params *p,
                             bwfm_aln_result *res, uint32_t *expand, uint64_t *work, void *hip_stream);

/* ------------------------------------------------------------------ */
/* Locate and pairing ("sampe"; section 2: repeats give several
 * placements, the other end and the fragment length decide)           */
/* ------------------------------------------------------------------ */

/*
 * Reference positions of every hit of res (n_reads reads) whose width
 * l - k + 1 is at most max_occ: pos_offsets (device, n_hits + 1, n_hits =
 * hit_offsets[n_reads] - hit_offsets[0]) receives CSR offsets per hit
 * (hit hit_offsets[0] + j has entry j), positions (device, pos_capacity)
 * the sorted 0-based leftmost forward coordinates of X.  res may be a
 * window of a larger result (hit_offsets need not start at 0).
 * Synchronous.  E_CAPACITY when the positions do not fit: pos_offsets is
 * complete and pos_offsets[n_hits] holds the capacity needed.
 */
int bwfm_locate(const bwfm_index *idx, uint32_t n_reads, const bwfm_aln_result *res, uint32_t max_occ,
                uint64_t *pos_offsets, uint32_t *positions, uint64_t pos_capacity, void *hip_stream);

typedef struct {
    int32_t lo, hi, mu;  /* proper insert window [lo, hi] and its centre */
    uint32_t max_occ;    /* hits wider than this are not located */
} bwfm_pair_params;

/* pair flags */
#define BWFM_PF_PAIRED 1
#define BWFM_PF_MAPPED1 2
#define BWFM_PF_MAPPED2 4
#define BWFM_PF_REP1 8   /* end 1 has a reported hit wider than max_occ */
#define BWFM_PF_REP2 16

typedef struct {
    uint32_t pos1, pos2;       /* 0xFFFFFFFF when that end is unplaced */
    int32_t insert;            /* pr + lr - pf of the chosen pair, 0 if unpaired */
    uint16_t len1, len2;       /* |X| per end */
    uint16_t score1, score2;
    uint8_t strand1, strand2, flags, pad;
} bwfm_pair;

/*
 * Pair n_pairs reads: r1 holds end 1's alignment of the pairs, r2 end 2's
 * (NULL: single-end, each record gets end 1's primary only).  Either may be
 * a window of a larger result (for example both ends aligned in one call).  A proper pair
 * puts the ends on opposite strands with pf <= pr and lo <= pr + lr - pf <=
 * hi (pf: position of the + end; pr, lr: position and length of the - end);
 * the chosen pair minimises (score1 + score2, |insert - mu|, pf, strand1,
 * pos1, len1, pos2, len2).  Without one, each end takes its primary: the
 * smallest (score, diffs, strand, pos, len) over its located hits.
 * out: device, n_pairs records.  Synchronous.  The located positions live
 * in the stream's workspace, which grows only when a call needs more than
 * any earlier one on that stream.  Errors: E_INVAL, E_STATE, E_NOMEM,
 * E_DEVICE.
 */
int bwfm_pair_reads(const bwfm_index *idx, uint32_t n_pairs, const bwfm_aln_result *r1,
                    const bwfm_aln_result *r2, const bwfm_pair_params *p, bwfm_pair *out, void *hip_stream);

/* bytes of device scratch bwfm_pair_reads_noalloc works in (per device) */
#define BWFM_NOALLOC_SCRATCH_BYTES (64u << 20)

/*
 * bwfm_pair_reads for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, hosts that forbid hipMalloc):
 * the same arguments, checks and results, but its control buffers and
 * located positions live in a fixed device array of
 * BWFM_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs
 * on until the process ends; it calls no hipMalloc or hipFree.  The index's
 * device must be current.  Limit: the control area (about 16 bytes per hit
 * of the larger end plus 8 per hit of each end) and the positions (4 bytes
 * each, both ends) must fit the scratch together; otherwise E_CAPACITY with
 * the bytes needed in bwfm_last_error() and `out` unwritten.  Every call on
 * a device shares that device's scratch: calls that overlap on one device,
 * on any streams or threads, race and must be serialised by the caller.
 * Synchronous.  Errors: E_INVAL, E_STATE, E_CAPACITY, E_DEVICE.
 */
int bwfm_pair_reads_noalloc(const bwfm_index *idx, uint32_t n_pairs, const bwfm_aln_result *r1,
                            const bwfm_aln_result *r2, const bwfm_pair_params *p, bwfm_pair *out,
                            void *hip_stream);

/* ------------------------------------------------------------------ */
/* Mate rescue (section 3.7: the pipeline ends with BWA's pairing step,  */
/* which gives an end without a partner a local alignment near its mate) */
/* ------------------------------------------------------------------ */

typedef struct {
    int32_t match;       /* score of a matching base, 1..32 */
    int32_t mismatch;    /* penalty of a mismatch (a read N mismatches everything), 0..64 */
    int32_t gap_open;    /* a gap of g bases costs gap_open + g * gap_extend; 0..64 each */
    int32_t gap_extend;
    int32_t min_score;   /* an alignment is reported when its score reaches this (>= 1) */
} bwfm_rescue_params;

/* the defaults: BWA-MEM's documented local-alignment scores, 20 to report */
#define BWFM_RESCUE_DEFAULTS {1, 4, 6, 1, 20}
/* largest fragment window (hi) rescue accepts */
#define BWFM_RESCUE_MAX_WINDOW 8192

typedef struct {
    uint32_t pos;      /* leftmost reference base of the rescued alignment */
    uint16_t len;      /* reference bases it spans */
    int16_t score;     /* its local alignment score */
    int32_t insert;    /* pr + lr - pf of the pair it forms (lo <= insert <= hi) */
    uint8_t end;       /* 0: nothing rescued; else the end rescued (1 or 2) */
    uint8_t strand;    /* strand of the rescued end (1: its reverse complement aligned) */
    uint8_t pad[2];
} bwfm_rescue;

/*
 * For every pair without a proper pair (BWFM_PF_PAIRED clear) and with a
 * primary for at least one end, align the other end (the mate) locally
 * inside the reference window the insert bounds allow around the primary
 * (the anchor; with primaries for both ends the one of lower score, end 1 on
 * ties):
 *   anchor on + at pf:            window [pf, pf + hi), mate on -;
 *   anchor on - at pr, length lr: window [pr + lr - hi, pr + lr), mate on +;
 * both clipped to the reference, and the alignment must give an insert of at
 * least lo.  Affine-gap local alignment (bwfm_rescue_params); among the best
 * cells the one of smallest insert, then smallest mate base, is reported; a
 * cell prefers the diagonal, then the gap along the reference, then the gap
 * along the read, and a gap prefers opening over extending, which fixes the
 * reported start.  Pairs that are proper, have no primary, or whose best score
 * is below min_score get end = 0.
 *   idx:   uploaded index (its packed reference is read).
 *   end1, end2: device, the pairs' reads (n_reads >= n_pairs each; the
 *          budgets are ignored); max_len bounds both ends' lengths.
 *   pairs: device, n_pairs records from bwfm_pair_reads.
 *   pp:    lo, hi as given to bwfm_pair_reads (hi <= BWFM_RESCUE_MAX_WINDOW).
 *   rp:    scores; NULL = BWFM_RESCUE_DEFAULTS.
 *   out:   device, n_pairs records (every one written).
 * Allocates nothing and does not wait: the work is enqueued on hip_stream.
 * Errors: E_INVAL (NULL, lo > hi, hi above the maximum, scores out of
 * range), E_TOOLONG (max_len above 512), E_STATE (index not uploaded),
 * E_DEVICE.
 */
int bwfm_rescue_mates(const bwfm_index *idx, const bwfm_reads *end1, const bwfm_reads *end2, uint32_t n_pairs,
                      const bwfm_pair *pairs, const bwfm_pair_params *pp, const bwfm_rescue_params *rp,
                      bwfm_rescue *out, void *hip_stream);

/* ------------------------------------------------------------------ */
/* Mapping quality (the pairing step of section 3.7 reports one per end; */
/* the paper gives no formula, so this is a stated reading)             */
/* ------------------------------------------------------------------ */

typedef struct {
    int32_t q_tier;    /* phred weight of a tier-2 placement against a tier-1 one, 1..60 */
    int32_t q_unique;  /* single-end cap (a unique placement), 0..60 */
    int32_t q_budget;  /* cap when every tier-1 hit spends the whole budget, 0..60 */
    int32_t q_pair;    /* cap for the ends of a proper pair, 0..254 */
} bwfm_mapq_params;

#define BWFM_MAPQ_DEFAULTS {22, 37, 25, 60}

/*
 * MAPQ of both ends of n_pairs pairs.  Each placement the search reported
 * weighs 1 in tier 1 and r = 10^(-q_tier / 10) in tier 2; an end placed by a
 * hit of its read's best score has P = 1 / (c1 + c2 r) of being right (r /
 * (c1 + c2 r) when placed by a tier-2 hit), and Q = round(-10 log10(1 - P))
 * (half up, double precision), at most q_unique, and at most q_budget when
 * every hit of the best score has diffs (mismatches + gap opens + gap
 * extensions) >= the read's budget.  0 for an end not placed in its pair
 * record or whose candidate set overflowed.  Both ends of a proper pair get
 * min(q_pair, Q1 + Q2); an end rescued by bwfm_rescue_mates takes its
 * anchor's Q.
 *   r1, r2:  the alignments the pairs were made from (r2 NULL: single-end,
 *            end 2 gets 0); windows of a larger result are fine.
 *   budget1, budget2: device, per-read difference budgets, or NULL: max_diff.
 *   pairs:   device, n_pairs records from bwfm_pair_reads.
 *   rescue:  device, n_pairs records from bwfm_rescue_mates, or NULL.
 *   mp:      NULL = BWFM_MAPQ_DEFAULTS.
 *   out:     device, 2 n_pairs bytes: end 1's then end 2's MAPQ per pair.
 * Allocates nothing and does not wait.  Errors: E_INVAL, E_DEVICE.
 */
int bwfm_mapq(uint32_t n_pairs, const bwfm_aln_result *r1, const bwfm_aln_result *r2, const uint8_t *budget1,
              const uint8_t *budget2, uint32_t max_diff, const bwfm_pair *pairs, const bwfm_rescue *rescue,
              const bwfm_mapq_params *mp, uint8_t *out, void *hip_stream);

/* ------------------------------------------------------------------ */
/* Captured step: one batch of pairs through align, locate and pairing  */
/* as a single hipGraph replay                                          */
/* ------------------------------------------------------------------ */

/*
 * A pipeline owns fixed-capacity device buffers for one step of the path
 * over up to max_pairs read pairs -- both ends aligned by one launch of the
 * batched form, every reported hit located, pairs chosen -- and enqueues the
 * step with every count read on the device and every capacity checked on
 * the device, so that no call in it waits for the host.  The step is
 * captured into a hipGraph at its first run and replayed by later runs; the
 * eager form enqueues the same kernels one by one.  Results equal those of
 * bwfm_align_batch (on end 1's reads followed by end 2's) and
 * bwfm_pair_reads.  Calls on one pipeline must not overlap; runs on one
 * stream may be queued back to back only if each one's results are read
 * before the next run is enqueued.
 */
typedef struct bwfm_pipeline bwfm_pipeline;

typedef struct {
    uint32_t max_pairs;    /* most pairs per run */
    uint32_t max_len;      /* longest read, 1..512 */
    uint64_t max_bases;    /* most read bases per run, both ends */
    uint64_t hit_capacity; /* most reported hits per run, both ends */
    uint64_t pos_capacity; /* most located positions per run, both ends */
    int32_t paired;        /* 1: each pair has two reads (end 1's, then end 2's);
                              0: single-end, one read per "pair" record */
} bwfm_pipeline_params;

/* Allocate the pipeline on the current device (the index must be
 * uploaded).  ap, pp: search and pairing parameters, fixed for the
 * pipeline's life.  Errors: E_INVAL, E_STATE, E_TOOLONG, E_NOMEM, E_DEVICE. */
int bwfm_pipeline_create(const bwfm_index *idx, const bwfm_aln_params *ap, const bwfm_pair_params *pp,
                         const bwfm_pipeline_params *q, bwfm_pipeline **out);

/* Enqueue on hip_stream a device-to-device copy of the next batch into the
 * pipeline's own input buffers (and unbind any bound reads):
 * reads.bases/offsets/max_diff hold 2 * n_pairs reads, end 1's then end
 * 2's (n_pairs reads single-end), in the bwfm_reads format (CSR offsets
 * starting at 0; lengths must be NULL; max_diff may be NULL: then every read
 * takes ap->max_diff).  The source buffers must
 * stay valid until the copy has run.  Errors: E_INVAL, E_CAPACITY (n_pairs
 * or the base count above the pipeline's maxima), E_DEVICE. */
int bwfm_pipeline_set_reads(bwfm_pipeline *pl, const bwfm_reads *reads, uint32_t n_pairs, void *hip_stream);

/* Bind caller-owned device buffers as the pipeline's input instead of its
 * own: reads->bases, offsets (start offsets when lengths is given, else
 * CSR offsets), lengths and max_diff (NULL: ap->max_diff for every read)
 * are read by every later run; reads->n_reads (at least 2 * max_pairs, or
 * max_pairs single-end) and max_len (at most the pipeline's) bound them.
 * The caller rewrites their contents between runs (on the run's stream,
 * before it) and sets the batch size with bwfm_pipeline_set_count.  A
 * captured graph is dropped and captured again at the next graph run.
 * Errors: E_INVAL, E_CAPACITY. */
int bwfm_pipeline_bind_reads(bwfm_pipeline *pl, const bwfm_reads *reads);

/* Batch size of the next run with bound reads.  Errors: E_INVAL, E_CAPACITY. */
int bwfm_pipeline_set_count(bwfm_pipeline *pl, uint32_t n_pairs);

/* Enqueue one step over the batch last set.  graph: 1 = replay the captured
 * graph (captured now if this is the first graph run), 0 = enqueue eagerly.
 * Errors: E_INVAL, E_DEVICE. */
int bwfm_pipeline_run(bwfm_pipeline *pl, int graph, void *hip_stream);

typedef struct {
    uint32_t n_pairs;
    uint32_t error;         /* 0, or BWFM_PIPE_E_* bits: a capacity was too small */
    uint64_t n_hits;        /* reported hits, both ends (needed size when too small) */
    uint64_t n_positions;   /* located positions, both ends */
    double kernel_ms;       /* the search's duration in this run (the first
                               pass, then for the batched form the split
                               searches' rounds and publication), from HIP
                               events captured around it; 0 when timing is
                               off */
} bwfm_pipeline_status;
#define BWFM_PIPE_E_HITS 1
#define BWFM_PIPE_E_POSITIONS 2

/* Wait for the last run on hip_stream and report it.  With timing enabled
 * (bwfm_timing_enable) the search kernel's duration is also added to the
 * timing store under "align_persistent" ("align_plain" for the plain form).
 * Errors: E_INVAL, E_DEVICE. */
int bwfm_pipeline_finish(bwfm_pipeline *pl, void *hip_stream, bwfm_pipeline_status *out);

/* Views of the last run's outputs (device memory owned by the pipeline,
 * valid until the next run): end 0 or 1 as an alignment result whose
 * hit_offsets index the shared hit array (see bwfm_locate on windows), the
 * per-hit position offsets (n_hits + 1, over both ends' hits in order) and
 * positions, and the n_pairs pair records. */
int bwfm_pipeline_outputs(bwfm_pipeline *pl, int end, bwfm_aln_result *res, uint64_t **pos_offsets,
                          uint32_t **positions, bwfm_pair **pairs);

void bwfm_pipeline_destroy(bwfm_pipeline *pl);

/* ------------------------------------------------------------------ */
/* Serving (continuous batching over the path above)                    */
/* ------------------------------------------------------------------ */

/*
 * A request server for the paired-end path.  Requests (host buffers) are
 * copied at submit and queued; a worker thread admits them in arrival order
 * while their reads fit in a device arena of arena_bytes, then runs
 * scheduling steps of at most step_pairs pairs taken from every admitted
 * request, oldest first -- so requests that arrive while others are on the
 * GPU join the next step and share its launch.  Two steps are in flight at
 * once, on two streams of the worker's own, so staging, the tail of one
 * step and the collection of its records overlap the next step.  Each step
 * aligns both ends in one call (form and search parameters from ap), pairs
 * them (pp) and copies the pair records back.  A request's results are the
 * same whatever it was mixed with.  The index must stay alive and uploaded
 * while the server exists.
 */
typedef struct bwfm_server bwfm_server;

typedef struct {
    uint64_t arena_bytes;  /* device bytes for admitted requests' bases */
    uint32_t step_pairs;   /* most pairs per scheduling step */
    uint32_t max_len;      /* longest read accepted, <= 512 */
    int32_t paired;        /* 1: requests carry both ends, 0: single-end */
    int32_t budget_rule;   /* 1: each read's difference budget is
                              bwfm_max_diff_rule(length, 0.02, 0.04);
                              0: ap->max_diff for every read */
    int32_t rescue_mapq;   /* 1: after pairing, rescue mates (paired servers;
                              bwfm_rescue_mates with default scores, pp->hi
                              <= BWFM_RESCUE_MAX_WINDOW) and assign MAPQ
                              (bwfm_mapq, default qualities) */
} bwfm_server_params;

typedef struct {
    double queued_ms;   /* submit -> admitted */
    double service_ms;  /* admitted -> results ready */
    double latency_ms;  /* submit -> results ready */
} bwfm_request_times;

typedef struct {
    uint64_t steps, pairs, requests_done;
    double busy_ms;     /* summed step durations, launch to collection
                           (two steps overlap, so it can exceed wall time) */
} bwfm_server_stats;

/* Errors: E_INVAL, E_STATE (index not uploaded), E_NOMEM, E_DEVICE. */
int bwfm_server_create(const bwfm_index *idx, const bwfm_aln_params *ap, const bwfm_pair_params *pp,
                       const bwfm_server_params *sp, bwfm_server **out);

/* Queue a request of n_pairs pairs: end e's pair j is bases_e[offsets_e[j],
 * offsets_e[j+1]) (host; offsets need not start at 0).  bases2/offsets2 are
 * ignored for a single-end server.  *ticket identifies it for
 * bwfm_server_wait.  Errors: E_INVAL, E_CAPACITY (larger than the arena),
 * E_STATE (server stopping). */
int bwfm_server_submit(bwfm_server *srv, const uint8_t *bases1, const uint64_t *offsets1, const uint8_t *bases2,
                       const uint64_t *offsets2, uint32_t n_pairs, uint64_t *ticket);

/* Block until the request is done; copy its n_pairs pair records to out,
 * with rescue_mapq its n_pairs rescue records to rescue and its 2 n_pairs
 * MAPQ bytes (end 1, end 2 per pair) to mapq, and its times to *times (host
 * buffers; each may be NULL; rescue and mapq are left untouched without
 * rescue_mapq).  Each ticket can be waited for once. */
int bwfm_server_wait(bwfm_server *srv, uint64_t ticket, bwfm_pair *out, bwfm_rescue *rescue, uint8_t *mapq,
                     bwfm_request_times *times);

int bwfm_server_get_stats(bwfm_server *srv, bwfm_server_stats *out);

/* Finish every queued request, stop the worker, free device memory. */
void bwfm_server_destroy(bwfm_server *srv);

/* ------------------------------------------------------------------ */
/* Host helpers                                                         */
/* ------------------------------------------------------------------ */

/*
 * Insert window from n inserts (host) of uniquely placed proper pairs
 * (section 2: the fragment length is known or estimated from the data): quartiles at index
 * floor(q (n - 1)) of the sorted inserts; inserts outside [p25 - 2 IQR,
 * p75 + 2 IQR] dropped; mu = mean, sigma = population sd of the rest;
 * lo = max(0, floor(mu - 4 sigma)), hi = ceil(mu + 4 sigma), mu rounded
 * half to even.  n < 100 gives {0, 500, 250}.  out->max_occ is untouched.
 */
int bwfm_estimate_insert(const int32_t *inserts, uint64_t n, bwfm_pair_params *out);

/* Difference budget for a read of length len: the smallest k >= 0 with
 * P[Poisson(err * len) > k] < thres (BWA's rule for a fractional budget;
 * err = 0.02 and thres = 0.04 give 2/3/4/5/6 at 36/51/76/100/150 bases). */
int bwfm_max_diff_rule(uint32_t len, double err, double thres);

/*
 * Kernel timing (off by default).  When on, the library brackets its
 * kernel launches with HIP events on the caller's stream and, when the
 * call completes, adds each launch's elapsed time under the kernel's name
 * ("align_fast", "align_slow", "compact", "locate_rows", "sort", "pair").
 * Process-wide; for measurement, not for concurrent production use.
 *   timing_get: *total_ms and *launches for one name (0 if never run).
 */
int bwfm_timing_enable(int on);
int bwfm_timing_reset(void);
int bwfm_timing_get(const char *kernel, double *total_ms, uint64_t *launches);

/*
 * Random-line probe: the achievable rate of dependent random line fetches,
 * the access pattern of the search (each rank query is one line at an index
 * the previous query decided).  lanes (a multiple of 256) each perform iters
 * dependent fetches of whole line_bytes (32, 64 or 128) lines at pseudo-random
 * line indices within buf (device, bytes long; contents arbitrary).  sink:
 * device, lanes uint32 (defeats dead-code removal).  *ms_out receives the
 * kernel time from HIP events on hip_stream.  Synchronous.  Lines/s =
 * lanes * iters / (ms / 1000).
 */
int bwfm_probe_gather(const void *buf, uint64_t bytes, uint32_t line_bytes, uint32_t lanes, uint32_t iters,
                      uint32_t *sink, double *ms_out, void *hip_stream);

/* Description of the last error on the calling thread ("" if none). */
const char *bwfm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BWFM_H */
