// ba_server.h -- continuous batching of generation requests on one GPU.
//
// Requests (a whole edge list, or the first-k degrees and checksum of a
// graph) queue on the host.  Each pump admits queued requests in arrival
// order whose outputs fit the caller's device arena (admission by HBM
// bytes); a request that does not fit is passed over, not waited for, until
// it has been passed over kServerMaxBypass steps in a row, after which
// nothing behind it is admitted until it fits.  All admitted edge-list
// requests run as ONE batched persistent launch on the caller's stream, all
// admitted degree requests as one batched streaming launch per LDS tier on
// the server's own stream, which follows the step's table copy (the tables
// go to the arena from pinned staging), so the two kinds overlap.  Steps
// queue on the two streams, so the host admits the next batch while earlier
// ones run; a step retires once both streams have passed it, and results
// stay in the arena (device-resident) until the client releases them.
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
    hipEvent_t ev = nullptr;     // the caller's stream: table copy and edge batch done
    hipEvent_t tab = nullptr;    // the caller's stream: table copy done (the degree stream waits for it)
    hipEvent_t ev2 = nullptr;    // the degree stream: degree requests done (none without them)
    uint64_t table_off = 0, table_bytes = 0;  // the step's tables in the arena (edge batch, then degree requests)
    int slot = -1;  // pinned staging slot holding the tables, returned when the step retires
    ba_batch_info info{};         // the edge batch
    uint64_t units[2] = {0, 0};   // units of the batched streaming launches (16K, 64K tier)
    std::vector<uint64_t> jobs;
};

constexpr uint32_t kServerSlots = 8;         // steps in flight at most
constexpr uint32_t kServerMaxBatch = 4096;   // edge requests per step at most
constexpr uint32_t kServerMaxDeg = kStreamBatchJobs;  // degree requests per step at most
constexpr uint32_t kServerLookahead = 1024;  // queued requests one pump examines
constexpr uint32_t kServerMaxBypass = 8;     // steps a head request may be passed over
// degree requests with more edges than this run as single streaming launches
constexpr uint64_t kServerBatchedEdges = 1ull << 40;

// The degree requests' table of a step: StreamJob entries (16K-tier
// requests, then 64K-tier ones) and the two tiers' unit counters.
static inline uint64_t stream_table_bytes(uint32_t njobs)
{
    return align256(sizeof(StreamJob) * (uint64_t)njobs + 2 * sizeof(uint32_t));
}

}  // namespace ba

struct ba_server {
    unsigned char *arena = nullptr;
    uint64_t arena_bytes = 0;
    hipStream_t stream = nullptr;  // the caller's: tables and edge batches
    hipStream_t side = nullptr;    // the server's own (default priority): degree requests
    hipEvent_t start = nullptr;
    ba::ArenaAlloc alloc{0};
    // jobs of tickets job_base .. job_base + jobs.size() - 1; released jobs
    // leave from the front, so memory follows the jobs still held
    std::deque<ba::ServerJob> jobs;
    uint64_t job_base = 0;
    std::deque<uint64_t> queue;
    std::deque<ba::ServerStep> steps;  // in flight, oldest first (retired in that order)
    std::vector<uint64_t> completed;   // tickets finished since the client last asked
    uint32_t inflight = 0;
    unsigned char *staging = nullptr;  // kServerSlots pinned table slots
    uint64_t slot_bytes = 0;
    std::vector<int> free_slots;
    uint32_t head_passed = 0;  // steps in a row that admitted requests behind a head that did not fit
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

static void server_step_events_free(ServerStep &st)
{
    for (hipEvent_t *e : {&st.ev, &st.tab, &st.ev2}) {
        if (*e) (void)hipEventDestroy(*e);
        *e = nullptr;
    }
}

// Retire finished steps (non-blocking): mark their jobs ready with the GPU
// completion time and free their tables, oldest first; a step is finished
// when both streams have passed its events.
static int server_retire(ba_server *s)
{
    while (!s->steps.empty()) {
        ServerStep &st = s->steps.front();
        const hipError_t q = hipEventQuery(st.ev);
        if (q == hipErrorNotReady) break;
        int rc = hip_check(q);
        if (rc) return rc;
        if (st.ev2) {
            const hipError_t q2 = hipEventQuery(st.ev2);
            if (q2 == hipErrorNotReady) break;
            if ((rc = hip_check(q2))) return rc;
        }
        float ms = 0.0f, ms2 = 0.0f;
        if ((rc = hip_check(hipEventElapsedTime(&ms, s->start, st.ev)))) return rc;
        if (st.ev2 && (rc = hip_check(hipEventElapsedTime(&ms2, s->start, st.ev2)))) return rc;
        ms = std::max(ms, ms2);  // the step ends with the later of its two streams
        for (uint64_t j : st.jobs) {
            ServerJob *J = server_job(s, j);
            J->state = BA_JOB_READY;
            J->done_ms = ms;
            s->completed.push_back(j);
        }
        if (st.table_bytes) s->alloc.release(st.table_off, st.table_bytes);
        if (st.slot >= 0) s->free_slots.push_back(st.slot);
        st.slot = -1;
        server_step_events_free(st);
        s->steps.pop_front();
        s->inflight--;
    }
    return BA_OK;
}

// Fills the StreamJob of a degree request for a batched streaming launch of
// `grid` blocks on the given tier; returns its units.
static uint64_t stream_job(const ServerJob &J, bool packed, uint32_t grid, StreamJob *out)
{
    StreamJob &S = *out;
    S = StreamJob{};
    S.key = make_hash_key(J.req.seed);
    S.narrow = 2 * J.m <= ((uint64_t)1 << 32) ? 1u : 0u;
    S.div = make_divider(J.req.d ? J.req.d : 1u);
    S.m = J.m;
    S.k = J.req.first_k;
    S.out = J.out_off / 8;  // uint64 elements from the arena base
    // runs sized so the request's units spread over the grid once
    uint64_t pw = (J.m + (uint64_t)kStreamWaves * grid - 1) / ((uint64_t)kStreamWaves * grid);
    if (packed) {
        pw = (pw + kStreamRoundClaims - 1) / kStreamRoundClaims * kStreamRoundClaims;
        pw = std::min<uint64_t>(std::max<uint64_t>(pw, kStreamRoundClaims), (uint64_t)kStreamRoundClaims << 16);
        S.rounds = pw / kStreamRoundClaims;  // no wave takes more barriers in its run
    } else {
        pw = (pw + kWave - 1) / kWave * kWave;
        // a block's 32-bit LDS counts of one unit stay below 16 * 2^26 = 2^30
        pw = std::min<uint64_t>(std::max<uint64_t>(pw, 4 * kWave), (uint64_t)1 << 26);
    }
    S.per_wave = pw;
    return J.m ? (J.m + (uint64_t)kStreamWaves * pw - 1) / ((uint64_t)kStreamWaves * pw) : 0;
}

// One step: admit queued jobs that fit (in arrival order, passing over
// those that do not), launch them.
static int server_launch_step(ba_server *s, uint32_t *launched)
{
    std::vector<uint64_t> edge_jobs, deg_jobs;
    *launched = 0;
    if (s->free_slots.empty() || s->queue.empty()) return BA_OK;  // every staging slot is in flight
    // room for the step's tables first, sized for what the examined requests
    // could need, so admitted outputs never leave the tables without room
    const size_t look = std::min<size_t>(s->queue.size(), kServerLookahead);
    uint32_t ce = 0, cd = 0;
    for (size_t q = 0; q < look; q++) (server_job(s, s->queue[q])->req.kind == BA_REQ_EDGES ? ce : cd)++;
    ce = std::min(ce, kServerMaxBatch);
    cd = std::min(cd, kServerMaxDeg);
    const uint64_t table_max = (ce ? batch_layout(ce).bytes : 0) + (cd ? stream_table_bytes(cd) : 0);
    ServerStep st;
    // a head job that can never fit the arena beside its step's table fails
    // instead of blocking the queue
    auto fail_head_if_stuck = [&]() {
        if (s->inflight == 0 && s->alloc.used() == align256(st.table_bytes)) {
            server_job(s, s->queue.front())->state = BA_JOB_FAILED;
            s->completed.push_back(s->queue.front());
            s->queue.pop_front();
            s->head_passed = 0;
        }
    };
    if (!s->alloc.alloc(table_max, &st.table_off)) {
        fail_head_if_stuck();
        return BA_OK;
    }
    st.table_bytes = table_max;
    bool head_fits = true;
    std::vector<size_t> taken;  // queue positions admitted
    for (size_t q = 0; q < look; q++) {
        if (!head_fits && s->head_passed >= kServerMaxBypass) break;  // the head waits for room first
        ServerJob &J = *server_job(s, s->queue[q]);
        auto &list = J.req.kind == BA_REQ_EDGES ? edge_jobs : deg_jobs;
        if (list.size() == (J.req.kind == BA_REQ_EDGES ? kServerMaxBatch : kServerMaxDeg)) continue;
        uint64_t off;
        if (!s->alloc.alloc(J.out_bytes, &off)) {
            if (q == 0) head_fits = false;
            continue;
        }
        J.out_off = off;
        list.push_back(s->queue[q]);
        taken.push_back(q);
    }
    if (edge_jobs.empty() && deg_jobs.empty()) {
        fail_head_if_stuck();
        s->alloc.release(st.table_off, st.table_bytes);
        return BA_OK;
    }
    // the admitted requests leave the queue
    {
        std::deque<uint64_t> rest;
        size_t t = 0;
        for (size_t q = 0; q < s->queue.size(); q++) {
            if (t < taken.size() && taken[t] == q) t++;
            else rest.push_back(s->queue[q]);
        }
        s->queue.swap(rest);
    }
    s->head_passed = head_fits ? 0 : s->head_passed + 1;
    // the degree requests: batched per LDS tier, the largest ones alone
    std::vector<uint64_t> deg16, deg64, deg_single;
    for (uint64_t j : deg_jobs) {
        const ServerJob &J = *server_job(s, j);
        if (J.m > kServerBatchedEdges) {
            deg_single.push_back(j);
            continue;
        }
        const bool narrow = 2 * J.m <= ((uint64_t)1 << 32);
        (stream_tier(J.req.n, J.req.first_k, narrow, BA_TIER_AUTO) == BA_TIER_64K ? deg64 : deg16).push_back(j);
    }
    const uint32_t ne = (uint32_t)edge_jobs.size(), nd = (uint32_t)(deg16.size() + deg64.size());
    uint32_t g16 = 0, g64 = 0;
    int rc = BA_OK;
    if (!deg16.empty() && (rc = persistent_grid(k_stream_batch<false>, kStreamBlock, &g16))) return rc;
    if (!deg64.empty() && (rc = persistent_grid(k_stream_batch<true>, kStreamBlock, &g64))) return rc;
    const BatchLayout L = batch_layout(ne);
    const uint64_t eb_bytes = ne ? L.bytes : 0, sb_bytes = nd ? stream_table_bytes(nd) : 0;
    // A launch of the step failed: part of it may already be queued, so wait
    // for both streams, then fail the step's requests and free what they held.
    auto fail_step = [&](int err) {
        (void)hipStreamSynchronize(s->stream);
        (void)hipStreamSynchronize(s->side);
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
        server_step_events_free(st);
        *launched = 0;
        return err;
    };
    if (eb_bytes + sb_bytes) {
        st.slot = s->free_slots.back();
        s->free_slots.pop_back();
        unsigned char *stage = s->staging + (uint64_t)st.slot * s->slot_bytes;
        memset(stage, 0, eb_bytes + sb_bytes);
        if (ne) {
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
            st.info.count = ne;
            for (int t = 0; t < 3; t++) st.info.tiles[t] = tiles[t];
            st.info.edges_len = s->arena_bytes / 4;
        }
        if (nd) {
            // per tier: requests with the longest runs first (their units are taken first)
            StreamJob *SJ = (StreamJob *)(stage + eb_bytes);
            uint32_t at = 0;
            for (int tier = 0; tier < 2; tier++) {
                const auto &list = tier ? deg64 : deg16;
                const uint32_t first = at;
                for (uint64_t j : list) (void)stream_job(*server_job(s, j), tier == 1, tier ? g64 : g16, &SJ[at++]);
                std::stable_sort(SJ + first, SJ + at,
                                 [](const StreamJob &x, const StreamJob &y) { return x.per_wave > y.per_wave; });
                uint64_t units = 0;
                for (uint32_t q = first; q < at; q++) {
                    SJ[q].unit0 = units;
                    units += (SJ[q].m + (uint64_t)kStreamWaves * SJ[q].per_wave - 1) /
                             ((uint64_t)kStreamWaves * SJ[q].per_wave);
                }
                st.units[tier] = units;
            }
        }
        int rc2 = hip_check(hipMemcpyAsync(s->arena + st.table_off, stage, eb_bytes + sb_bytes, hipMemcpyHostToDevice,
                                           s->stream));
        if (rc2) return fail_step(rc2);
    }
    // The degree requests run on the server's own stream, after the table
    // copy, beside the edge batch: each launch's tail then overlaps the other.
    const bool degs = nd || !deg_single.empty();
    if (degs) {
        if ((rc = hip_check(hipEventCreateWithFlags(&st.tab, hipEventDisableTiming)))) return fail_step(rc);
        if ((rc = hip_check(hipEventRecord(st.tab, s->stream)))) return fail_step(rc);
        if ((rc = hip_check(hipStreamWaitEvent(s->side, st.tab, 0)))) return fail_step(rc);
    }
    if (ne) {
        if ((rc = ba_batch_launch(&st.info, s->arena + st.table_off, (uint32_t *)s->arena, s->arena_bytes / 4,
                                  s->stream)))
            return fail_step(rc);
    }
    if (nd) {
        StreamBatchArgs a{};
        const StreamJob *SJ = (const StreamJob *)(s->arena + st.table_off + eb_bytes);
        uint32_t *next = (uint32_t *)(s->arena + st.table_off + eb_bytes + sizeof(StreamJob) * (uint64_t)nd);
        a.base = (uint64_t *)s->arena;
        a.jobs = SJ;
        a.njobs = nd;
        if ((rc = launch_timed(BA_KT_OTHER, s->side, [&] {
                 hipLaunchKernelGGL(k_stream_batch_init, dim3(std::min<uint32_t>(nd, 1024)), dim3(256), 0, s->side,
                                    a);
             })))
            return fail_step(rc);
        const uint32_t n16 = (uint32_t)deg16.size();
        for (int tier = 0; tier < 2; tier++) {
            if (!st.units[tier]) continue;
            a.jobs = SJ + (tier ? n16 : 0);
            a.njobs = tier ? nd - n16 : n16;
            a.units = (uint32_t)st.units[tier];
            a.next = next + tier;
            const uint32_t grid = (uint32_t)std::min<uint64_t>(tier ? g64 : g16, st.units[tier]);
            if ((rc = launch_timed(BA_KT_STREAM, s->side, [&] {
                     if (tier)
                         hipLaunchKernelGGL(k_stream_batch<true>, dim3(grid), dim3(kStreamBlock), 0, s->side, a);
                     else
                         hipLaunchKernelGGL(k_stream_batch<false>, dim3(grid), dim3(kStreamBlock), 0, s->side, a);
                 })))
                return fail_step(rc);
        }
    }
    for (uint64_t j : deg_single) {
        const ServerJob &J = *server_job(s, j);
        uint64_t *deg = (uint64_t *)(s->arena + J.out_off);
        if ((rc = ba_degrees(J.req.n, J.req.d, J.req.seed, J.req.first_k, deg, deg + J.req.first_k, s->side)))
            return fail_step(rc);
    }
    if ((rc = hip_check(hipEventCreate(&st.ev)))) return fail_step(rc);
    if ((rc = hip_check(hipEventRecord(st.ev, s->stream)))) return fail_step(rc);
    if (degs) {
        if ((rc = hip_check(hipEventCreate(&st.ev2)))) return fail_step(rc);
        if ((rc = hip_check(hipEventRecord(st.ev2, s->side)))) return fail_step(rc);
    }
    for (uint64_t j : edge_jobs) st.jobs.push_back(j);
    for (uint64_t j : deg_jobs) st.jobs.push_back(j);
    for (uint64_t j : st.jobs) server_job(s, j)->state = BA_JOB_RUNNING;
    s->steps.push_back(std::move(st));
    s->inflight++;
    *launched = (uint32_t)(edge_jobs.size() + deg_jobs.size());
    return BA_OK;
}

}  // namespace ba
