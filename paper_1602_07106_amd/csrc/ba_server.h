// ba_server.h -- continuous batching of generation requests on one GPU.
//
// Requests (a whole edge list, or the first-k degrees and checksum of a
// graph) queue on the host.  Each pump admits queued requests in arrival
// order while their outputs fit the caller's device arena (admission by
// HBM bytes), launches all admitted edge-list requests as ONE batched
// persistent launch (the instance table goes to the arena from pinned
// staging) and every admitted degree request as a streaming launch, and
// records one event for the step.  Steps queue on the server's stream, so
// the host admits the next batch while earlier ones run; results stay in
// the arena (device-resident) until the client releases them.
//
// The paper hands batches of edge IDs to processors as they become free
// (Section 2, last paragraph); here whole requests are the units and the
// GPU is the processor.  Included at the end of ba.hip.
#pragma once

#include <chrono>
#include <deque>
#include <map>
#include <vector>

namespace ba {

// First-fit allocator over [0, bytes) of the arena, 256-byte granules.
class ArenaAlloc {
  public:
    explicit ArenaAlloc(uint64_t bytes) : total_(bytes & ~(uint64_t)255)
    {
        if (total_) free_[0] = total_;
    }
    bool alloc(uint64_t bytes, uint64_t *off)
    {
        if (bytes > total_) return false;  // also keeps the rounding below from wrapping
        bytes = align256(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const uint64_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes)
    {
        bytes = align256(bytes ? bytes : 1);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
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
    uint64_t used() const { return used_; }

  private:
    uint64_t total_;
    std::map<uint64_t, uint64_t> free_;
    uint64_t used_ = 0;
};

struct ServerJob {
    ba_request req;
    uint64_t m = 0;
    uint64_t out_off = 0, out_bytes = 0;
    int state = BA_JOB_QUEUED;
    double done_ms = 0.0;
};

struct ServerStep {
    hipEvent_t ev = nullptr;
    uint64_t table_off = 0, table_bytes = 0;
    int slot = -1;  // pinned staging slot holding the table, returned when the step retires
    std::vector<uint64_t> jobs;
};

constexpr uint32_t kServerSlots = 8;         // steps in flight at most
constexpr uint32_t kServerMaxBatch = 4096;   // edge requests per step at most

}  // namespace ba

struct ba_server {
    unsigned char *arena = nullptr;
    uint64_t arena_bytes = 0;
    hipStream_t stream = nullptr;
    hipEvent_t start = nullptr;
    ba::ArenaAlloc alloc{0};
    // jobs of tickets job_base .. job_base + jobs.size() - 1; released jobs
    // leave from the front, so memory follows the jobs still held
    std::deque<ba::ServerJob> jobs;
    uint64_t job_base = 0;
    std::deque<uint64_t> queue;
    std::deque<ba::ServerStep> steps;  // in flight, oldest first (they finish in order on one stream)
    std::vector<uint64_t> completed;   // tickets finished since the client last asked
    uint32_t inflight = 0;
    unsigned char *staging = nullptr;  // kServerSlots pinned table slots
    uint64_t slot_bytes = 0;
    std::vector<int> free_slots;
};

namespace ba {

static ServerJob *server_job(ba_server *s, uint64_t ticket)
{
    if (ticket < s->job_base || ticket - s->job_base >= s->jobs.size()) return nullptr;
    return &s->jobs[ticket - s->job_base];
}

static void server_trim(ba_server *s)
{
    while (!s->jobs.empty() && s->jobs.front().state == BA_JOB_RELEASED) {
        s->jobs.pop_front();
        s->job_base++;
    }
}

static uint64_t job_output_bytes(const ba_request &r, uint64_t m)
{
    return r.kind == BA_REQ_EDGES ? 8 * m : 8 * (r.first_k + 1);  // degrees: first_k counts + checksum
}

// Retire finished steps (non-blocking): mark their jobs ready with the GPU
// completion time and free their tables.  Steps finish in launch order.
static int server_retire(ba_server *s)
{
    while (!s->steps.empty()) {
        ServerStep &st = s->steps.front();
        const hipError_t q = hipEventQuery(st.ev);
        if (q == hipErrorNotReady) break;
        int rc = hip_check(q);
        if (rc) return rc;
        float ms = 0.0f;
        if ((rc = hip_check(hipEventElapsedTime(&ms, s->start, st.ev)))) return rc;
        for (uint64_t j : st.jobs) {
            ServerJob *J = server_job(s, j);
            J->state = BA_JOB_READY;
            J->done_ms = ms;
            s->completed.push_back(j);
        }
        if (st.table_bytes) s->alloc.release(st.table_off, st.table_bytes);
        if (st.slot >= 0) s->free_slots.push_back(st.slot);
        st.slot = -1;
        (void)hipEventDestroy(st.ev);
        s->steps.pop_front();
        s->inflight--;
    }
    return BA_OK;
}

// One step: admit queued jobs in order while they fit, launch them.
static int server_launch_step(ba_server *s, uint32_t *launched)
{
    std::vector<uint64_t> edge_jobs, deg_jobs;
    *launched = 0;
    if (s->free_slots.empty()) return BA_OK;  // every staging slot is in flight
    while (!s->queue.empty()) {
        ServerJob &J = *server_job(s, s->queue.front());
        if (J.req.kind == BA_REQ_EDGES && edge_jobs.size() == kServerMaxBatch) break;
        uint64_t off;
        if (!s->alloc.alloc(J.out_bytes, &off)) break;
        J.out_off = off;
        (J.req.kind == BA_REQ_EDGES ? edge_jobs : deg_jobs).push_back(s->queue.front());
        s->queue.pop_front();
    }
    if (edge_jobs.empty() && deg_jobs.empty()) {
        *launched = 0;
        // a head job that can never fit an empty arena fails instead of blocking the queue
        if (!s->queue.empty() && s->inflight == 0 && s->alloc.used() == 0) {
            server_job(s, s->queue.front())->state = BA_JOB_FAILED;
            s->completed.push_back(s->queue.front());
            s->queue.pop_front();
        }
        return BA_OK;
    }
    ServerStep st;
    int rc = BA_OK;
    // A launch of the step failed: part of it may already be queued, so wait
    // for the stream, then fail the step's requests and free what they held.
    auto fail_step = [&](int err) {
        (void)hipStreamSynchronize(s->stream);
        for (const auto *list : {&edge_jobs, &deg_jobs}) {
            for (uint64_t j : *list) {
                ServerJob &J = *server_job(s, j);
                s->alloc.release(J.out_off, J.out_bytes);
                J.state = BA_JOB_FAILED;
                s->completed.push_back(j);
            }
        }
        if (st.table_bytes) s->alloc.release(st.table_off, st.table_bytes);
        if (st.slot >= 0) s->free_slots.push_back(st.slot);
        if (st.ev) (void)hipEventDestroy(st.ev);
        *launched = 0;
        return err;
    };
    const uint32_t ne = (uint32_t)edge_jobs.size();
    if (ne) {
        const BatchLayout L = batch_layout(ne);
        if (!s->alloc.alloc(L.bytes, &st.table_off)) {
            // no room for the table: give the outputs back and retry next pump
            for (auto it = deg_jobs.rbegin(); it != deg_jobs.rend(); ++it) {
                s->alloc.release(server_job(s, *it)->out_off, server_job(s, *it)->out_bytes);
                s->queue.push_front(*it);
            }
            for (auto it = edge_jobs.rbegin(); it != edge_jobs.rend(); ++it) {
                s->alloc.release(server_job(s, *it)->out_off, server_job(s, *it)->out_bytes);
                s->queue.push_front(*it);
            }
            *launched = 0;
            return BA_OK;
        }
        st.table_bytes = L.bytes;
        st.slot = s->free_slots.back();
        s->free_slots.pop_back();
        unsigned char *stage = s->staging + (uint64_t)st.slot * s->slot_bytes;
        memset(stage, 0, L.bytes);
        BatchInst *I = (BatchInst *)(stage + L.o_inst);
        uint64_t *T[3];
        for (int t = 0; t < 3; t++) T[t] = (uint64_t *)(stage + L.o_tile0[t]);
        uint64_t tiles[3] = {0, 0, 0};
        for (uint32_t q = 0; q < ne; q++) {
            const ServerJob &J = *server_job(s, edge_jobs[q]);
            I[q].key = make_hash_key(J.req.seed);
            I[q].narrow = 2 * J.m <= ((uint64_t)1 << 32) ? 1u : 0u;
            I[q].div = make_divider(J.req.d ? J.req.d : 1u);
            I[q].m = J.m;
            I[q].out = J.out_off / 4;  // uint32 elements from the arena base
            for (int t = 0; t < 3; t++) {
                T[t][q] = tiles[t];
                tiles[t] += (J.m + kBatchTiles[t] - 1) / kBatchTiles[t];
            }
        }
        for (int t = 0; t < 3; t++) T[t][ne] = tiles[t];
        if ((rc = hip_check(hipMemcpyAsync(s->arena + st.table_off, stage, L.bytes, hipMemcpyHostToDevice,
                                           s->stream))))
            return fail_step(rc);
        ba_batch_info info{};
        info.count = ne;
        for (int t = 0; t < 3; t++) info.tiles[t] = tiles[t];
        info.edges_len = s->arena_bytes / 4;
        if ((rc = ba_batch_launch(&info, s->arena + st.table_off, (uint32_t *)s->arena, s->arena_bytes / 4,
                                  s->stream)))
            return fail_step(rc);
    }
    for (uint64_t j : deg_jobs) {
        const ServerJob &J = *server_job(s, j);
        uint64_t *deg = (uint64_t *)(s->arena + J.out_off);
        if ((rc = ba_degrees(J.req.n, J.req.d, J.req.seed, J.req.first_k, deg, deg + J.req.first_k, s->stream)))
            return fail_step(rc);
    }
    if ((rc = hip_check(hipEventCreate(&st.ev)))) return fail_step(rc);
    if ((rc = hip_check(hipEventRecord(st.ev, s->stream)))) return fail_step(rc);
    for (uint64_t j : edge_jobs) st.jobs.push_back(j);
    for (uint64_t j : deg_jobs) st.jobs.push_back(j);
    for (uint64_t j : st.jobs) server_job(s, j)->state = BA_JOB_RUNNING;
    s->steps.push_back(std::move(st));
    s->inflight++;
    *launched = (uint32_t)(edge_jobs.size() + deg_jobs.size());
    return BA_OK;
}

}  // namespace ba
