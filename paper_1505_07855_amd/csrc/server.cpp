// Continuous-batching request server over the alignment path.
//
// Requests (read pairs in host memory) are queued by bwfm_server_submit.  A
// worker thread owns a device arena of fixed size and two step slots, each
// with its own HIP stream, captured step (bwfm_pipeline), step buffers and
// pinned host staging.  It admits queued requests in arrival order while
// their reads fit in the arena, copies them there, and runs scheduling
// steps.  Each step takes up to step_pairs pairs from the admitted requests,
// oldest first, so the tail of one request and the head of the next share a
// launch; it aligns both ends of every selected pair in one batched launch
// (reads addressed by start offset and length inside the arena), pairs them,
// and copies the pair records back.  While one slot's step runs on the
// device the worker stages and launches the next step in the other slot and
// then collects the first one's records, so host staging, result scatter
// and the tail of one step's search overlap the next step's work.  A request
// completes when its last pair has been processed; its arena range is then
// freed, which admits the next waiting request.  Results do not depend on
// how requests are mixed or which slot ran them: every read is aligned and
// every pair decided on its own.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <thread>
#include <tuple>
#include <unordered_map>

#include "bwfm_internal.h"

using namespace bwfm;

namespace {

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t id = 0;
    uint32_t n_pairs = 0;
    std::vector<uint8_t> bases[2];
    std::vector<uint64_t> offs[2];  // n_pairs + 1 each
    uint64_t bytes = 0;             // arena bytes (both ends, 256-byte aligned)
    uint64_t arena_off = 0;
    uint64_t end_off[2] = {0, 0};   // arena offset of each end's bases
    uint32_t next_pair = 0;         // first pair not yet scheduled
    uint32_t done_pairs = 0;
    std::vector<bwfm_pair> out;
    std::vector<bwfm_rescue> resc;  // with rescue_mapq
    std::vector<uint8_t> mapq;      // with rescue_mapq: 2 per pair
    double t_submit = 0, t_admit = 0, t_done = 0;
    int state = 0;  // 0 queued, 1 admitted, 2 done, 3 failed
    int err = 0;
};

// first-fit allocator over [0, size)
struct Arena {
    std::map<uint64_t, uint64_t> free_;  // offset -> size
    explicit Arena(uint64_t size) { free_[0] = size; }
    bool alloc(uint64_t n, uint64_t &off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                off = it->first;
                uint64_t rest = it->second - n;
                free_.erase(it);
                if (rest) free_[off + n] = rest;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t n) {
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

inline uint64_t round256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

using Chunks = std::vector<std::tuple<std::shared_ptr<Request>, uint32_t, uint32_t>>;

// One step in flight: its buffers, stream and captured step.
struct StepSlot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;  // recorded after the step's results reach the host staging
    uint64_t *d_off = nullptr;  // 2 * step_pairs start offsets
    uint32_t *d_len = nullptr;  // 2 * step_pairs lengths
    uint8_t *d_md = nullptr;    // 2 * step_pairs budgets (length rule)
    // the step as a captured graph over the buffers above
    bwfm_pipeline *pipe = nullptr;
    uint64_t pipe_hits = 0, pipe_pos = 0;
    // outputs of a step redone by eager calls (a pipeline capacity was short)
    uint64_t *d_hoff = nullptr;  // 2 * step_pairs + 1
    uint4 *d_hits = nullptr;
    uint64_t hit_cap = 0;
    uint32_t *d_c1 = nullptr, *d_c2 = nullptr;
    uint8_t *d_status = nullptr;
    bwfm_pair *d_pairs = nullptr;
    bwfm_rescue *d_resc = nullptr;  // with rescue_mapq
    uint8_t *d_mapq = nullptr;
    // pinned host staging
    uint64_t *h_off = nullptr;
    uint32_t *h_len = nullptr;
    uint8_t *h_md = nullptr;
    bwfm_pair *h_pairs = nullptr;
    bwfm_rescue *h_resc = nullptr;
    uint8_t *h_mapq = nullptr;
    // the step in flight
    Chunks chunks;
    uint32_t P = 0;
    bool busy = false;
    double t_start = 0;
};

}  // namespace

struct bwfm_server {
    const bwfm_index *ix = nullptr;
    bwfm_aln_params ap{};
    bwfm_pair_params pp{};
    bwfm_server_params sp{};
    int device = 0;
    uint8_t *arena_mem = nullptr;  // admitted requests' bases
    StepSlot slot[2];
    uint8_t rule[BWFM_MAX_READ + 1];
    // state
    Arena arena{0};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> queued;
    std::vector<std::shared_ptr<Request>> active;  // admission order
    std::unordered_map<uint64_t, std::shared_ptr<Request>> all;
    uint64_t next_id = 1;
    bool stop = false;
    int worker_error = 0;
    std::string worker_msg;
    bwfm_server_stats stats{};
    std::thread worker;
};

namespace {

// (Re)create a slot's step pipeline with the given capacities, reading the
// arena and the slot's start offsets, lengths and budgets.
int make_pipeline(bwfm_server *s, StepSlot &k, uint64_t hits, uint64_t pos) {
    if (k.pipe) bwfm_pipeline_destroy(k.pipe);
    k.pipe = nullptr;
    const bool paired = s->sp.paired != 0;
    bwfm_pipeline_params q{s->sp.step_pairs, s->sp.max_len, 256, hits, pos, paired ? 1 : 0};
    int rc = bwfm_pipeline_create(s->ix, &s->ap, &s->pp, &q, &k.pipe);
    if (rc) return rc;
    const uint32_t R = (paired ? 2u : 1u) * s->sp.step_pairs;
    bwfm_reads rd{s->arena_mem, k.d_off, s->sp.budget_rule ? k.d_md : nullptr, R, s->sp.max_len, k.d_len};
    rc = bwfm_pipeline_bind_reads(k.pipe, &rd);
    if (rc) {
        bwfm_pipeline_destroy(k.pipe);
        k.pipe = nullptr;
        return rc;
    }
    k.pipe_hits = hits;
    k.pipe_pos = pos;
    return BWFM_OK;
}

void release_slot(StepSlot &k) {
    if (k.pipe) bwfm_pipeline_destroy(k.pipe);
    k.pipe = nullptr;
    void *ptrs[] = {k.d_off, k.d_len, k.d_md, k.d_hoff, k.d_hits, k.d_c1, k.d_c2, k.d_status, k.d_pairs, k.d_resc,
                    k.d_mapq};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    void *hptrs[] = {k.h_off, k.h_len, k.h_md, k.h_pairs, k.h_resc, k.h_mapq};
    for (void *p : hptrs)
        if (p) (void)hipHostFree(p);
    if (k.done) (void)hipEventDestroy(k.done);
    if (k.stream) (void)hipStreamDestroy(k.stream);
    k = StepSlot{};
}

void release_device(bwfm_server *s) {
    for (auto &k : s->slot) release_slot(k);
    if (s->arena_mem) (void)hipFree(s->arena_mem);
    s->arena_mem = nullptr;
}

// Device buffers, pinned staging, stream, event and captured step of a slot.
int make_slot(bwfm_server *s, StepSlot &k) {
    const uint64_t R = 2ull * s->sp.step_pairs;
    const uint64_t SP = s->sp.step_pairs;
    k.hit_cap = 4 * R + 1024;
    if (hipStreamCreateWithFlags(&k.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&k.done, hipEventDisableTiming) != hipSuccess)
        return fail(BWFM_E_DEVICE, "server_create: stream or event creation failed");
    if (hipMalloc(&k.d_off, 8 * R) != hipSuccess || hipMalloc(&k.d_len, 4 * R) != hipSuccess ||
        hipMalloc(&k.d_md, R) != hipSuccess || hipMalloc(&k.d_hoff, 8 * (R + 1)) != hipSuccess ||
        hipMalloc(&k.d_hits, 16 * k.hit_cap) != hipSuccess || hipMalloc(&k.d_c1, 4 * R) != hipSuccess ||
        hipMalloc(&k.d_c2, 4 * R) != hipSuccess || hipMalloc(&k.d_status, R) != hipSuccess ||
        hipMalloc(&k.d_pairs, sizeof(bwfm_pair) * SP) != hipSuccess ||
        (s->sp.rescue_mapq && (hipMalloc(&k.d_resc, sizeof(bwfm_rescue) * SP) != hipSuccess ||
                               hipMalloc(&k.d_mapq, 2 * SP) != hipSuccess)))
        return fail(BWFM_E_NOMEM, "server_create: device allocation failed");
    if (hipHostMalloc(&k.h_off, 8 * R) != hipSuccess || hipHostMalloc(&k.h_len, 4 * R) != hipSuccess ||
        hipHostMalloc(&k.h_md, R) != hipSuccess || hipHostMalloc(&k.h_pairs, sizeof(bwfm_pair) * SP) != hipSuccess ||
        (s->sp.rescue_mapq && (hipHostMalloc(&k.h_resc, sizeof(bwfm_rescue) * SP) != hipSuccess ||
                               hipHostMalloc(&k.h_mapq, 2 * SP) != hipSuccess)))
        return fail(BWFM_E_NOMEM, "server_create: pinned host allocation failed");
    return make_pipeline(s, k, k.hit_cap, 64 * R + 4096);
}

// hand a step's records (in chunk order) to their requests
void scatter_pairs(bwfm_server *s, const StepSlot &k) {
    uint32_t o = 0;
    for (auto &c : k.chunks) {
        Request &q = *std::get<0>(c);
        const uint32_t j = std::get<1>(c), n = std::get<2>(c);
        std::memcpy(q.out.data() + j, k.h_pairs + o, sizeof(bwfm_pair) * n);
        if (s->sp.rescue_mapq) {
            std::memcpy(q.resc.data() + j, k.h_resc + o, sizeof(bwfm_rescue) * n);
            std::memcpy(q.mapq.data() + 2 * (size_t)j, k.h_mapq + 2 * (size_t)o, 2 * (size_t)n);
        }
        o += n;
    }
}

// After pairing (records at dp, device): with rescue_mapq, the mates' rescue
// and the MAPQ of both ends from the step's alignments (r2 NULL:
// single-end); then the step's results to the slot's pinned staging and its
// event.  Nothing here waits.
int enqueue_results(bwfm_server *s, StepSlot &k, const bwfm_pair *dp, const bwfm_aln_result &r1,
                    const bwfm_aln_result *r2) {
    const uint32_t P = k.P;
    if (s->sp.rescue_mapq) {
        const bool rule = s->sp.budget_rule != 0;
        if (r2) {
            bwfm_reads e1{s->arena_mem, k.d_off, nullptr, P, s->sp.max_len, k.d_len};
            bwfm_reads e2{s->arena_mem, k.d_off + P, nullptr, P, s->sp.max_len, k.d_len + P};
            if (int rc = bwfm_rescue_mates(s->ix, &e1, &e2, P, dp, &s->pp, nullptr, k.d_resc, k.stream)) return rc;
        } else if (P && hipMemsetAsync(k.d_resc, 0, sizeof(bwfm_rescue) * P, k.stream) != hipSuccess) {
            return fail(BWFM_E_DEVICE, "server: clearing rescue records failed");
        }
        if (int rc = bwfm_mapq(P, &r1, r2, rule ? k.d_md : nullptr, rule && r2 ? k.d_md + P : nullptr,
                               (uint32_t)s->ap.max_diff, dp, r2 ? k.d_resc : nullptr, nullptr, k.d_mapq, k.stream))
            return rc;
        if (hipMemcpyAsync(k.h_resc, k.d_resc, sizeof(bwfm_rescue) * P, hipMemcpyDeviceToHost, k.stream) !=
                hipSuccess ||
            hipMemcpyAsync(k.h_mapq, k.d_mapq, 2ull * P, hipMemcpyDeviceToHost, k.stream) != hipSuccess)
            return fail(BWFM_E_DEVICE, "server: result download failed");
    }
    if (hipMemcpyAsync(k.h_pairs, dp, sizeof(bwfm_pair) * P, hipMemcpyDeviceToHost, k.stream) != hipSuccess ||
        hipEventRecord(k.done, k.stream) != hipSuccess)
        return fail(BWFM_E_DEVICE, "server: result download failed");
    return BWFM_OK;
}

// The step by eager calls over the slot's own output buffers (a captured
// step outgrew its capacities; the pipeline has been grown for the next
// steps).  Synchronous.
int run_step_eager(bwfm_server *s, StepSlot &k) {
    const bool paired = s->sp.paired != 0;
    const uint32_t P = k.P, n = (paired ? 2 : 1) * P;
    const bool rule = s->sp.budget_rule != 0;
    bwfm_reads rd{s->arena_mem, k.d_off, rule ? k.d_md : nullptr, n, s->sp.max_len, k.d_len};
    bwfm_aln_result res{k.d_hoff, reinterpret_cast<bwfm_hit *>(k.d_hits), k.hit_cap, k.d_c1, k.d_c2, k.d_status};
    int rc = bwfm_align_batch(s->ix, &rd, &s->ap, &res, k.stream);
    if (rc == BWFM_E_CAPACITY) {
        uint64_t need = 0;
        if (hipMemcpy(&need, k.d_hoff + n, 8, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(BWFM_E_DEVICE, "server: reading hit need failed");
        (void)hipFree(k.d_hits);
        k.d_hits = nullptr;
        k.hit_cap = need + need / 4 + 1024;
        if (hipMalloc(&k.d_hits, k.hit_cap * 16) != hipSuccess) return fail(BWFM_E_NOMEM, "server: hit buffer");
        res.hits = reinterpret_cast<bwfm_hit *>(k.d_hits);
        res.hit_capacity = k.hit_cap;
        rc = bwfm_align_batch(s->ix, &rd, &s->ap, &res, k.stream);
    }
    if (rc) return rc;
    bwfm_aln_result r1 = res, r2 = res;
    r2.hit_offsets = k.d_hoff + P;
    r2.c1 = k.d_c1 + P;
    r2.c2 = k.d_c2 + P;
    r2.status = k.d_status + P;
    rc = bwfm_pair_reads(s->ix, P, &r1, paired ? &r2 : nullptr, &s->pp, k.d_pairs, k.stream);
    if (rc) return rc;
    rc = enqueue_results(s, k, k.d_pairs, r1, paired ? &r2 : nullptr);
    if (rc) return rc;
    return hipStreamSynchronize(k.stream) == hipSuccess ? BWFM_OK : fail(BWFM_E_DEVICE, "server: step failed");
}

// Stage and launch the slot's step (its chunks are set): start offsets,
// lengths and budgets of all end-1 reads of the step, then all end-2 reads,
// to the device; the captured step; the results to the pinned staging.
int launch_step(bwfm_server *s, StepSlot &k) {
    const bool paired = s->sp.paired != 0;
    const uint32_t ends = paired ? 2 : 1;
    uint32_t P = 0;
    for (auto &c : k.chunks) P += std::get<2>(c);
    k.P = P;
    uint32_t n = 0;
    for (uint32_t e = 0; e < ends; e++)
        for (auto &c : k.chunks) {
            Request &q = *std::get<0>(c);
            for (uint32_t j = std::get<1>(c); j < std::get<1>(c) + std::get<2>(c); j++) {
                k.h_off[n] = q.end_off[e] + q.offs[e][j];
                k.h_len[n] = (uint32_t)(q.offs[e][j + 1] - q.offs[e][j]);
                k.h_md[n] = s->rule[std::min<uint32_t>(k.h_len[n], BWFM_MAX_READ)];
                n++;
            }
        }
    const bool rule = s->sp.budget_rule != 0;
    if (hipMemcpyAsync(k.d_off, k.h_off, 8ull * n, hipMemcpyHostToDevice, k.stream) != hipSuccess ||
        hipMemcpyAsync(k.d_len, k.h_len, 4ull * n, hipMemcpyHostToDevice, k.stream) != hipSuccess ||
        (rule && hipMemcpyAsync(k.d_md, k.h_md, n, hipMemcpyHostToDevice, k.stream) != hipSuccess))
        return fail(BWFM_E_DEVICE, "server: step upload failed");
    int rc = bwfm_pipeline_set_count(k.pipe, P);
    if (!rc) rc = bwfm_pipeline_run(k.pipe, 1, k.stream);
    if (rc) return rc;
    bwfm_pair *dp = nullptr;
    bwfm_aln_result pr1{}, pr2{};
    rc = bwfm_pipeline_outputs(k.pipe, 0, &pr1, nullptr, nullptr, &dp);
    if (!rc && paired) rc = bwfm_pipeline_outputs(k.pipe, 1, &pr2, nullptr, nullptr, nullptr);
    if (rc) return rc;
    return enqueue_results(s, k, dp, pr1, paired ? &pr2 : nullptr);
}

// Wait for the slot's step; when its captured step ran out of room, grow
// the pipeline and redo the step eagerly; then hand the records out.
int collect_step(bwfm_server *s, StepSlot &k) {
    if (hipEventSynchronize(k.done) != hipSuccess) return fail(BWFM_E_DEVICE, "server: step failed");
    bwfm_pipeline_status ps{};
    int rc = bwfm_pipeline_finish(k.pipe, k.stream, &ps);
    if (rc) return rc;
    if (ps.error) {
        rc = make_pipeline(s, k, std::max(k.pipe_hits, ps.n_hits + ps.n_hits / 4 + 1024),
                           std::max(k.pipe_pos, ps.n_positions + ps.n_positions / 4 + 4096));
        if (!rc) rc = run_step_eager(s, k);
        if (rc) return rc;
    }
    scatter_pairs(s, k);
    return BWFM_OK;
}

// Under the lock: admit queued requests in arrival order while the arena
// has room; return them (their bases still to be uploaded).
std::vector<std::shared_ptr<Request>> admit(bwfm_server *s) {
    std::vector<std::shared_ptr<Request>> admitted;
    while (!s->queued.empty()) {
        auto q = s->queued.front();
        uint64_t off;
        if (!s->arena.alloc(q->bytes, off)) break;
        s->queued.pop_front();
        q->arena_off = off;
        q->end_off[0] = off;
        q->end_off[1] = off + round256(q->bases[0].size());
        q->state = 1;
        q->t_admit = now_ms();
        s->active.push_back(q);
        admitted.push_back(q);
    }
    return admitted;
}

// Under the lock: the next step's chunks (request, first pair, count),
// oldest request first.
Chunks choose(bwfm_server *s) {
    Chunks chunks;
    uint32_t room = s->sp.step_pairs;
    for (auto &q : s->active) {
        if (!room) break;
        const uint32_t left = q->n_pairs - q->next_pair;
        if (!left || q->state == 3) continue;
        const uint32_t take = std::min(left, room);
        chunks.emplace_back(q, q->next_pair, take);
        q->next_pair += take;
        room -= take;
    }
    return chunks;
}

// Under the lock: account a collected (or failed) step and retire the
// requests it completed.
void retire(bwfm_server *s, StepSlot &k, int rc, const std::string &msg, double t1) {
    s->stats.steps++;
    s->stats.busy_ms += t1 - k.t_start;
    for (auto &c : k.chunks) {
        auto &q = std::get<0>(c);
        if (rc) {
            q->state = 3;
            q->err = rc;
        }
        q->done_pairs += std::get<2>(c);
        s->stats.pairs += std::get<2>(c);
    }
    if (rc) {
        s->worker_error = rc;
        s->worker_msg = msg;
    }
    std::vector<std::shared_ptr<Request>> keep;
    for (auto &q : s->active) {
        // a failed request waits for its steps still in flight
        const bool finished = q->done_pairs == q->n_pairs || (q->state == 3 && q->done_pairs == q->next_pair);
        if (finished) {
            if (q->state != 3) q->state = 2;
            q->t_done = now_ms();
            s->arena.release(q->arena_off, q->bytes);
            for (int e = 0; e < 2; e++) std::vector<uint8_t>().swap(q->bases[e]);
            s->stats.requests_done++;
        } else {
            keep.push_back(q);
        }
    }
    s->active.swap(keep);
    k.chunks.clear();
    k.busy = false;
    s->cv_done.notify_all();
}

void worker_main(bwfm_server *s) {
    (void)hipSetDevice(s->device);
    int inflight[2] = {-1, -1};  // slots with a step on the device, oldest first
    int n_inflight = 0;
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // launch a step into a free slot while there is work for one
        int free_slot = !s->slot[0].busy ? 0 : (!s->slot[1].busy ? 1 : -1);
        std::vector<std::shared_ptr<Request>> admitted;
        Chunks chunks;
        if (free_slot >= 0) {
            admitted = admit(s);
            chunks = choose(s);
        }
        if (!chunks.empty()) {
            StepSlot &k = s->slot[free_slot];
            k.chunks = std::move(chunks);
            k.busy = true;
            lk.unlock();
            int rc = BWFM_OK;
            k.t_start = now_ms();
            // new requests' bases, on this slot's (idle) stream, before the
            // step: the other slot's later steps may read them, so wait here
            for (auto &q : admitted)
                for (int e = 0; e < 2 && rc == BWFM_OK; e++)
                    if (!q->bases[e].empty() &&
                        hipMemcpyAsync(s->arena_mem + q->end_off[e], q->bases[e].data(), q->bases[e].size(),
                                       hipMemcpyHostToDevice, k.stream) != hipSuccess)
                        rc = fail(BWFM_E_DEVICE, "server: request upload failed");
            if (rc == BWFM_OK && !admitted.empty() && hipStreamSynchronize(k.stream) != hipSuccess)
                rc = fail(BWFM_E_DEVICE, "server: request upload failed");
            if (rc == BWFM_OK) rc = launch_step(s, k);
            if (rc) {
                (void)hipStreamSynchronize(k.stream);
                const std::string msg = last_error();
                lk.lock();
                retire(s, k, rc, msg, now_ms());
                continue;
            }
            inflight[n_inflight++] = free_slot;
            lk.lock();
            // keep the device fed: a second step goes in before the first
            // is collected, when there is work for it
            if (n_inflight < 2) continue;
        }
        if (n_inflight > 0) {
            StepSlot &k = s->slot[inflight[0]];
            if (n_inflight == 1 && hipEventQuery(k.done) == hipErrorNotReady) {
                // one step on the device and no work for the other slot:
                // look again shortly, so that requests arriving meanwhile
                // are launched before this step is collected
                s->cv_work.wait_for(lk, std::chrono::microseconds(200));
                continue;
            }
            lk.unlock();
            int rc = collect_step(s, k);
            const double t1 = now_ms();
            const std::string msg = rc ? last_error() : std::string();
            lk.lock();
            retire(s, k, rc, msg, t1);
            inflight[0] = inflight[1];
            inflight[1] = -1;
            n_inflight--;
            continue;
        }
        if (s->stop && s->queued.empty()) break;
        s->cv_work.wait(lk);
    }
}

}  // namespace

extern "C" int bwfm_server_create(const bwfm_index *ix, const bwfm_aln_params *ap, const bwfm_pair_params *pp,
                                  const bwfm_server_params *sp, bwfm_server **out) {
    if (!ix || !ap || !pp || !sp || !out) return fail(BWFM_E_INVAL, "server_create: NULL argument");
    *out = nullptr;
    if (ix->device < 0) return fail(BWFM_E_STATE, "server_create: index not uploaded");
    if (sp->step_pairs < 1 || sp->arena_bytes < 4096 || sp->max_len < 1 || sp->max_len > BWFM_MAX_READ)
        return fail(BWFM_E_INVAL, "server_create: bad server parameters");
    if (ap->form != BWFM_FORM_BATCHED && ap->form != BWFM_FORM_PLAIN)
        return fail(BWFM_E_INVAL, "server_create: bad form");
    if (sp->rescue_mapq && sp->paired && (pp->hi > BWFM_RESCUE_MAX_WINDOW || pp->lo > pp->hi))
        return fail(BWFM_E_INVAL, "server_create: insert window unfit for mate rescue");
    auto s = std::make_unique<bwfm_server>();
    s->ix = ix;
    s->ap = *ap;
    s->pp = *pp;
    s->sp = *sp;
    s->device = ix->device;
    s->arena = Arena(sp->arena_bytes);
    for (uint32_t L = 0; L <= BWFM_MAX_READ; L++)
        s->rule[L] = (uint8_t)std::min(bwfm_max_diff_rule(L, 0.02, 0.04), BWFM_MAX_DIFF);
    if (hipSetDevice(s->device) != hipSuccess) return fail(BWFM_E_DEVICE, "server_create: device not available");
    if (hipMalloc(&s->arena_mem, sp->arena_bytes) != hipSuccess) {
        s->arena_mem = nullptr;
        return fail(BWFM_E_NOMEM, "server_create: arena allocation failed");
    }
    for (auto &k : s->slot) {
        if (int rc = make_slot(s.get(), k)) {
            release_device(s.get());
            return rc;
        }
    }
    bwfm_server *raw = s.release();
    raw->worker = std::thread(worker_main, raw);
    *out = raw;
    return BWFM_OK;
}

extern "C" int bwfm_server_submit(bwfm_server *s, const uint8_t *b1, const uint64_t *o1, const uint8_t *b2,
                                  const uint64_t *o2, uint32_t n_pairs, uint64_t *ticket) {
    if (!s || !o1 || !ticket || (s->sp.paired && !o2)) return fail(BWFM_E_INVAL, "server_submit: NULL argument");
    if (n_pairs == 0) return fail(BWFM_E_INVAL, "server_submit: empty request");
    auto q = std::make_shared<Request>();
    q->n_pairs = n_pairs;
    const int ends = s->sp.paired ? 2 : 1;
    const uint8_t *bb[2] = {b1, b2};
    const uint64_t *oo[2] = {o1, o2};
    for (int e = 0; e < ends; e++) {
        const uint64_t base = oo[e][0], total = oo[e][n_pairs] - base;
        if (oo[e][n_pairs] < base || (total && !bb[e])) return fail(BWFM_E_INVAL, "server_submit: bad offsets");
        for (uint32_t j = 0; j < n_pairs; j++)
            if (oo[e][j + 1] < oo[e][j]) return fail(BWFM_E_INVAL, "server_submit: offsets decrease");
        q->bases[e].assign(bb[e] + base, bb[e] + base + total);
        q->offs[e].resize(n_pairs + 1);
        for (uint32_t j = 0; j <= n_pairs; j++) q->offs[e][j] = oo[e][j] - base;
        q->bytes += round256(total);
    }
    q->bytes = std::max<uint64_t>(q->bytes, 256);
    if (q->bytes > s->sp.arena_bytes)
        return fail(BWFM_E_CAPACITY, "server_submit: request larger than the arena");
    q->out.resize(n_pairs);
    if (s->sp.rescue_mapq) {
        q->resc.resize(n_pairs);
        q->mapq.resize(2 * (size_t)n_pairs);
    }
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return fail(BWFM_E_STATE, "server_submit: server is stopping");
    q->id = s->next_id++;
    q->t_submit = now_ms();
    s->all[q->id] = q;
    s->queued.push_back(q);
    *ticket = q->id;
    s->cv_work.notify_one();
    return BWFM_OK;
}

extern "C" int bwfm_server_wait(bwfm_server *s, uint64_t ticket, bwfm_pair *out, bwfm_rescue *rescue, uint8_t *mapq,
                                bwfm_request_times *times) {
    if (!s) return fail(BWFM_E_INVAL, "server_wait: NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(BWFM_E_INVAL, "server_wait: unknown ticket");
    auto q = it->second;
    s->cv_done.wait(lk, [&] { return q->state >= 2; });
    s->all.erase(it);
    if (q->state == 3) return fail(q->err, "server: request failed: " + s->worker_msg);
    if (out) std::memcpy(out, q->out.data(), sizeof(bwfm_pair) * q->n_pairs);
    if (rescue && s->sp.rescue_mapq) std::memcpy(rescue, q->resc.data(), sizeof(bwfm_rescue) * q->n_pairs);
    if (mapq && s->sp.rescue_mapq) std::memcpy(mapq, q->mapq.data(), 2 * (size_t)q->n_pairs);
    if (times) {
        times->queued_ms = q->t_admit - q->t_submit;
        times->latency_ms = q->t_done - q->t_submit;
        times->service_ms = q->t_done - q->t_admit;
    }
    return BWFM_OK;
}

extern "C" int bwfm_server_get_stats(bwfm_server *s, bwfm_server_stats *out) {
    if (!s || !out) return fail(BWFM_E_INVAL, "server_get_stats: NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->stats;
    return BWFM_OK;
}

extern "C" void bwfm_server_destroy(bwfm_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    release_device(s);
    delete s;
}
