// ba_stream.h -- the streaming consumer of paper Section 3 on gfx950:
// degrees of the first k nodes and an edge checksum, with no edge stored.
//
// Each wave owns a contiguous run of edge IDs and runs the per-edge chain
// (paper Section 2, figure generateEdge) with lane refill.  A finished edge
// (u, v) adds one to the degree of v when v < k (first endpoints are counted
// in closed form by the caller) and XORs (u * 2^32 + v) * (2i + 1) into a
// per-lane checksum.  Counts of the lowest node IDs, which take most of the
// targets, go to LDS-privatised tables; the rest are 64-bit global atomics.
// Two tiers: k_stream (16384 nodes, 32-bit counters) and k_stream_packed
// (65536 nodes, 16-bit counters kept from wrapping by block-wide rounds).
//
// Included by ba.hip after its host helpers (persistent_grid, launch_timed).
#pragma once

#include <algorithm>
#include <atomic>
#include <cmath>
#include <type_traits>

namespace ba {

constexpr int kStreamBlock = 1024;  // 16 waves share one LDS degree table
constexpr int kStreamWaves = kStreamBlock / kWave;
constexpr uint32_t kLdsNodes = 16384;  // LDS-privatised degree counters per block

struct StreamArgs {
    HashKey key;
    Divider div;
    uint64_t begin, count;
    uint64_t per_wave;  // edges per wave (multiple of 64)
    uint64_t rounds;    // packed tier: barriers every wave takes
    uint64_t k;         // first_k
    uint32_t klds;      // min(k, kLdsNodes)
    uint64_t *deg;      // first_k uint64 (second endpoints added here)
    uint64_t *cs;       // nullable
};

// floor(x / d) with the divider's kind fixed at compile time (the streaming
// kernels divide on every finished edge; d is a power of two when POW2),
// otherwise the same multiply-high steps as div32 (x < 2^31) / div64.
template <bool POW2>
__device__ __forceinline__ uint32_t sdiv32(uint32_t x, const Divider &v)
{
    if constexpr (POW2) return x >> v.shift;
    return mulhi32(x, v.m32) >> v.shift;
}

template <bool POW2>
__device__ __forceinline__ uint64_t sdiv64(uint64_t x, const Divider &v)
{
    if constexpr (POW2) return x >> v.shift;
    return mulhi64(x, v.m64) >> v.shift;  // x < 2^63
}

// floor(x / 2d): a power-of-two d takes one 64-bit shift (shift + 1 <= 32)
template <bool POW2>
__device__ __forceinline__ uint64_t shalf64(uint64_t x, const Divider &v)
{
    if constexpr (POW2) return x >> (v.shift + 1);
    return sdiv64<false>(x >> 1, v);
}

// The checksum word of the edge with start position r0 = 2i + 1 and
// endpoints (u, v): ((u << 32) + v) * r0 mod 2^64, from 32-bit halves.  The
// word's low half is v's and its high half is u + (v >> 32) mod 2^32, or u's
// alone when every node ID is below 2^32 (ID32: n <= 2^32); only the low
// halves of the cross products reach the result.
template <bool ID32>
__device__ __forceinline__ uint64_t edge_word(uint64_t u, uint64_t v, uint64_t r0)
{
    const uint32_t xl = (uint32_t)v, xh = ID32 ? (uint32_t)u : (uint32_t)u + (uint32_t)(v >> 32);
    const uint32_t r0l = (uint32_t)r0, r0h = (uint32_t)(r0 >> 32);
    return mad64(xl, r0l, 0) + ((uint64_t)(xl * r0h + xh * r0l) << 32);
}

// One wave's run of tn edges starting at edge ibase: the chain of every
// edge, its second endpoint counted (cnt: LDS counters of nodes below klds;
// deg: global counts of nodes below k) and its checksum word XORed into xs.
// ID32: every node ID is below 2^32 (always so for 32-bit positions).
template <bool NARROW, bool POW2, bool ID32 = NARROW>
__device__ __forceinline__ void stream_run16(const HashKey &key, const Divider &div, uint64_t ibase, uint32_t tn,
                                             uint32_t klds, uint64_t k, uint32_t *cnt, uint64_t *deg, uint64_t &xs)
{
    using R = typename std::conditional<NARROW, uint32_t, uint64_t>::type;
    chain_run_visit(
        tn, __lane_id(), (R)(2 * ibase + 1),
        [&](R r) -> R {
            if constexpr (NARROW) return hash_narrow(r, key);
            else return hash_wide(r, key);
        },
        [](R r) { return !((uint32_t)r & 1u); },
        [&](R r0, R r) {  // r0 = 2i + 1, the edge's start position
            uint64_t u, v;
            if constexpr (NARROW) {
                v = sdiv32<POW2>((uint32_t)r >> 1, div);
                u = sdiv32<POW2>((uint32_t)r0 >> 1, div);
            } else {
                v = shalf64<POW2>(r, div);
                u = shalf64<POW2>(r0, div);
            }
            if (v < klds)
                atomicAdd(&cnt[v], 1u);
            else if (v < k)
                __hip_atomic_fetch_add(deg + v, (uint64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            xs ^= edge_word<ID32>(u, v, r0);
        });
}

// The wave's checksum XORed into *cs (one atomic per wave).
__device__ __forceinline__ void stream_xor_out(uint64_t xs, uint64_t *cs)
{
    if (cs) {
        for (int o = 32; o > 0; o >>= 1) xs ^= __shfl_xor(xs, o);
        if (__lane_id() == 0 && xs) __hip_atomic_fetch_xor(cs, xs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <bool NARROW, bool POW2, bool ID32>
__global__ __launch_bounds__(kStreamBlock) void k_stream(StreamArgs a)
{
    __shared__ uint32_t cnt[kLdsNodes];
    for (uint32_t v = threadIdx.x; v < a.klds; v += kStreamBlock) cnt[v] = 0;
    __syncthreads();

    // wave-uniform (readfirstlane): keeps the loop control scalar
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint64_t gw = (uint64_t)blockIdx.x * kStreamWaves + wv;
    const uint64_t w0 = gw * a.per_wave;
    uint64_t xs = 0;
    if (w0 < a.count) {
        // per_wave < 2^32: the host splits larger launches
        const uint32_t tn = (uint32_t)min(a.per_wave, a.count - w0);
        stream_run16<NARROW, POW2, ID32>(a.key, a.div, a.begin + w0, tn, a.klds, a.k, cnt, a.deg, xs);
    }
    stream_xor_out(xs, a.cs);
    __syncthreads();
    for (uint32_t v = threadIdx.x; v < a.klds; v += kStreamBlock) {
        const uint32_t c = cnt[v];
        if (c) __hip_atomic_fetch_add(a.deg + v, (uint64_t)c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// k_stream with a wider LDS tier for first_k > 16384: nodes 0..65535 count in
// 16-bit counters, two to an LDS word (node v: word v >> 1, half v & 1;
// 128 KiB, one block per compute unit), so only targets in [65536, first_k)
// need global atomics.
//
// A 16-bit counter could wrap, so the block synchronises in rounds.  Chains
// in flight carry across a round boundary; a wave takes its next barrier as
// soon as it has handed out kStreamRoundClaims more edges, so it finishes at
// most kStreamRoundClaims + 127 edges between two barriers (two chains per
// lane), and the block at most 16 * 2047 = 32752.  A counter below 0x8000 at
// a barrier therefore stays at or below 0xFFFF until the next one; the lane
// whose increment takes it from 0x7FFF to 0x8000 moves those 32768 counts to
// the global degree before its wave's next barrier.  Every counter is below
// 0x8000 again at each barrier, and the counts are exact.  Waves that run
// out of edges early take their remaining barriers at the end, so all take
// a.rounds of them.
constexpr uint32_t kPackedNodes = 65536;
constexpr uint32_t kStreamRoundClaims = 1920;
static_assert(kStreamWaves * (kStreamRoundClaims + 2 * kWave - 1) <= 0x8000, "a round must not wrap a 16-bit counter");

// The packed counters of nodes below ktier added to deg (and cleared, for
// the next unit of a batched launch).
__device__ __forceinline__ void packed_flush(uint32_t *cnt, uint32_t ktier, uint64_t *deg)
{
    for (uint32_t w = threadIdx.x; w < kPackedNodes / 2; w += kStreamBlock) {
        const uint32_t c = cnt[w];
        cnt[w] = 0;
        const uint32_t lo = c & 0xFFFFu, hi = c >> 16;
        if (lo && 2 * w < ktier)
            __hip_atomic_fetch_add(deg + 2 * w, (uint64_t)lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (hi && 2 * w + 1 < ktier)
            __hip_atomic_fetch_add(deg + 2 * w + 1, (uint64_t)hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// One wave's run of tot edges starting at edge ibase on the 64K tier (see
// above): two chains per lane, counts of nodes below ktier in the packed
// LDS counters cnt, of nodes below k in deg, checksum words into xs.  The
// wave takes exactly `rounds` block barriers (at least its own claims /
// kStreamRoundClaims), so every wave of the block must pass the same rounds.
template <bool NARROW, bool POW2, bool ID32 = NARROW>
__device__ __forceinline__ void stream_run_packed(const HashKey &key, const Divider &div, uint64_t ibase, uint32_t tot,
                                                  uint32_t ktier, uint64_t k, uint32_t *cnt, uint64_t *deg,
                                                  uint64_t rounds, uint64_t &xs)
{
    using R = typename std::conditional<NARROW, uint32_t, uint64_t>::type;
    const uint32_t lane = __lane_id();
    const R rbase = (R)(2 * ibase + 1);

    // The value a lane's last LDS increment returned is examined at its next
    // finished edge of the same chain (or before its wave's next barrier),
    // so the wave does not wait for the atomic's result right after issuing
    // it.
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    auto settle = [&](uint32_t &pend_old, uint32_t &pend_v) {
        if (pend_v != kNone) {
            const uint32_t sh = (pend_v & 1u) << 4;
            if (((pend_old >> sh) & 0xFFFFu) == 0x7FFFu) {
                atomicSub(&cnt[pend_v >> 1], 0x8000u << sh);
                __hip_atomic_fetch_add(deg + pend_v, (uint64_t)0x8000, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            pend_v = kNone;
        }
    };
    auto hash = [&](R r) -> R {
        if constexpr (NARROW) return hash_narrow(r, key);
        else return hash_wide(r, key);
    };
    // r0 = 2i + 1: the edge's start position (i = r0 >> 1, and the checksum
    // multiplier itself)
    auto finish = [&](R r0, R r, uint32_t &pend_old, uint32_t &pend_v) {
        uint64_t u, v;
        if constexpr (NARROW) {
            v = sdiv32<POW2>((uint32_t)r >> 1, div);
            u = sdiv32<POW2>((uint32_t)r0 >> 1, div);
        } else {
            v = shalf64<POW2>(r, div);
            u = shalf64<POW2>(r0, div);
        }
        settle(pend_old, pend_v);
        if (v < ktier) {
            pend_old = atomicAdd(&cnt[(uint32_t)v >> 1], 1u << (((uint32_t)v & 1u) << 4));
            pend_v = (uint32_t)v;
        } else if (v < k) {
            __hip_atomic_fetch_add(deg + v, (uint64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        xs ^= edge_word<ID32>(u, v, r0);
    };

    // Every lane runs two chains (A and B): their hash evaluations are
    // independent, which hides latency at the one block per compute unit
    // this tier allows.  claimed (wave-uniform): edges handed out so far,
    // the first 128 at the start and one more per finished edge (those past
    // tot stay idle).  Up to 128 edges finish per step, so a wave finishes
    // at most kStreamRoundClaims + 127 edges between two barriers.
    uint32_t pa_old = 0, pa_v = kNone, pb_old = 0, pb_v = kNone;
    uint32_t claimed = 2 * kWave, next_bar = 2 * kWave + kStreamRoundClaims;
    uint64_t bars = 0;
    auto round_edge = [&]() {
        if (claimed >= next_bar) {
            settle(pa_old, pa_v);
            settle(pb_old, pb_v);
            lds_barrier();
            bars++;
            next_bar += kStreamRoundClaims;
        }
    };
    // start positions of the lane's two edges (edge index li = (r0 - rbase) / 2);
    // a refill is one multiply-add of the rank onto a wave-uniform base
    R ra0 = rbase + 2 * (R)lane, rb0 = rbase + 2 * (R)(lane + kWave);
    R ra = ra0, rb = rb0;
    if (tot >= 2 * kWave) {
        while (claimed + 2 * kWave <= tot) {  // every lane holds two live edges
            ra = hash(ra);
            rb = hash(rb);
            const bool fa = !((uint32_t)ra & 1u), fb = !((uint32_t)rb & 1u);
            const uint64_t ma = __ballot(fa), mb = __ballot(fb);
            if (fa) {
                finish(ra0, ra, pa_old, pa_v);
                ra0 = wave_uniform((R)(rbase + 2 * (R)claimed)) + 2 * (R)lane_rank(ma);
                ra = ra0;
            }
            claimed += (uint32_t)__popcll(ma);
            if (fb) {
                finish(rb0, rb, pb_old, pb_v);
                rb0 = wave_uniform((R)(rbase + 2 * (R)claimed)) + 2 * (R)lane_rank(mb);
                rb = rb0;
            }
            claimed += (uint32_t)__popcll(mb);
            round_edge();
        }
    }
    uint32_t la = (uint32_t)((ra0 - rbase) >> 1), lb = (uint32_t)((rb0 - rbase) >> 1);
    bool aa = la < tot, ab = lb < tot;
    uint64_t live = __ballot(aa || ab);
    while (live) {
        ra = hash(ra);
        rb = hash(rb);
        const bool fa = aa && !((uint32_t)ra & 1u), fb = ab && !((uint32_t)rb & 1u);
        const uint64_t ma = __ballot(fa), mb = __ballot(fb);
        if (fa) {
            finish(ra0, ra, pa_old, pa_v);
            la = claimed + lane_rank(ma);
            aa = la < tot;
            ra0 = rbase + 2 * (R)la;
            ra = ra0;
        }
        claimed += (uint32_t)__popcll(ma);
        if (fb) {
            finish(rb0, rb, pb_old, pb_v);
            lb = claimed + lane_rank(mb);
            ab = lb < tot;
            rb0 = rbase + 2 * (R)lb;
            rb = rb0;
        }
        claimed += (uint32_t)__popcll(mb);
        round_edge();
        live = __ballot(aa || ab);
    }
    settle(pa_old, pa_v);
    settle(pb_old, pb_v);
    for (; bars < rounds; bars++) lds_barrier();
}

template <bool NARROW, bool POW2, bool ID32>
__global__ __launch_bounds__(kStreamBlock) void k_stream_packed(StreamArgs a)
{
    __shared__ uint32_t cnt[kPackedNodes / 2];  // node v: word v >> 1, half v & 1
    for (uint32_t w = threadIdx.x; w < kPackedNodes / 2; w += kStreamBlock) cnt[w] = 0;
    __syncthreads();
    // wave-uniform (readfirstlane): keeps the loop control scalar
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint64_t gw = (uint64_t)blockIdx.x * kStreamWaves + wv;
    const uint64_t w0 = gw * a.per_wave;
    // edges of this wave (per_wave < 2^32: the host splits larger launches)
    const uint32_t tot = w0 < a.count ? (uint32_t)min(a.per_wave, a.count - w0) : 0u;
    const uint32_t ktier = a.klds;  // min(first_k, 65536)
    uint64_t xs = 0;
    stream_run_packed<NARROW, POW2, ID32>(a.key, a.div, a.begin + w0, tot, ktier, a.k, cnt, a.deg, a.rounds, xs);
    stream_xor_out(xs, a.cs);
    __syncthreads();
    packed_flush(cnt, ktier, a.deg);
}

// ---------------------------------------------------------------------------
// Batched streaming: many degree requests (graphs) in one persistent launch,
// for the served path.  Each request j is cut into units of kStreamWaves
// wave runs of jobs[j].per_wave edges; blocks take units from a device
// counter in table order (the host lists the requests with the longest runs
// first), so one block works on one request at a time: its waves run the
// unit's edges into the block's LDS table, which is then added to that
// request's degrees and cleared.  Results do not depend on which block takes
// which unit (counts are added, checksum words XORed).

struct StreamJob {
    HashKey key;
    uint32_t narrow;    // every position of the graph below 2^32
    Divider div;
    uint64_t m;         // edges of the graph
    uint64_t k;         // first_k
    uint64_t out;       // uint64 elements from the launch's base: k degrees, then the checksum
    uint64_t per_wave;  // edges per wave run (a multiple of 64; 64K tier: of kStreamRoundClaims too)
    uint64_t unit0;     // the request's first unit
    uint64_t rounds;    // 64K tier: block barriers per unit
};

struct StreamBatchArgs {
    const StreamJob *jobs;
    uint32_t njobs;
    uint32_t units;     // units of all requests
    uint32_t *next;     // next unit to take (zero at launch)
    uint64_t *base;     // outputs
};

// deg = d for each request's nodes below first_k (their first endpoints, in
// closed form) and checksum = 0, before the batched streaming launch.
__global__ __launch_bounds__(256) void k_stream_batch_init(StreamBatchArgs a)
{
    for (uint32_t j = blockIdx.x; j < a.njobs; j += gridDim.x) {
        const StreamJob J = a.jobs[j];
        uint64_t *deg = a.base + J.out;
        const uint64_t d = J.div.d;
        for (uint64_t v = threadIdx.x; v < J.k; v += 256) deg[v] = J.m ? d : 0;
        if (threadIdx.x == 0) deg[J.k] = 0;
    }
}

// Requests of one batched streaming launch at most: their first units are
// cached in LDS (16 KB beside the 64 KB table keeps two 16K-tier blocks per
// compute unit).
constexpr uint32_t kStreamBatchJobs = 4000;

template <bool PACKED>
__global__ __launch_bounds__(kStreamBlock) void k_stream_batch(StreamBatchArgs a)
{
    constexpr uint32_t kWords = PACKED ? kPackedNodes / 2 : kLdsNodes;
    __shared__ uint32_t cnt[kWords];
    __shared__ uint32_t unit0[kStreamBatchJobs];  // first unit of each request (the search runs in LDS)
    __shared__ uint32_t unit_sh;
    for (uint32_t w = threadIdx.x; w < kWords; w += kStreamBlock) cnt[w] = 0;
    for (uint32_t j = threadIdx.x; j < a.njobs; j += kStreamBlock) unit0[j] = (uint32_t)a.jobs[j].unit0;
    if (threadIdx.x == 0) unit_sh = atomicAdd(a.next, 1u);
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    for (;;) {
        __syncthreads();
        const uint32_t u = __builtin_amdgcn_readfirstlane(unit_sh);
        if (u >= a.units) break;  // every wave sees the same u: the whole block leaves
        // the next unit is taken now; its index is needed only after this one
        uint32_t u_next = 0;
        if (threadIdx.x == 0) u_next = atomicAdd(a.next, 1u);
        uint32_t lo = 0, hi = a.njobs;  // the request j with unit0[j] <= u < unit0[j+1]
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) / 2;
            if (unit0[mid] <= u) lo = mid; else hi = mid;
        }
        const uint32_t j = __builtin_amdgcn_readfirstlane(lo);
        // a copy: the hot loop stores to global memory, so fields read through
        // a reference would be reloaded after every degree update
        const StreamJob J = a.jobs[j];
        const uint64_t w0 = ((u - J.unit0) * (uint64_t)kStreamWaves + wv) * J.per_wave;
        const uint32_t tn = w0 < J.m ? (uint32_t)min(J.per_wave, J.m - w0) : 0u;
        const uint32_t klds = (uint32_t)min(J.k, (uint64_t)(PACKED ? kPackedNodes : kLdsNodes));
        uint64_t *deg = a.base + J.out;
        uint64_t xs = 0;
        auto run = [&](auto n_t, auto p_t) {
            constexpr bool N = decltype(n_t)::value, P = decltype(p_t)::value;
            if constexpr (PACKED)
                stream_run_packed<N, P>(J.key, J.div, w0, tn, klds, J.k, cnt, deg, J.rounds, xs);
            else if (tn)
                stream_run16<N, P>(J.key, J.div, w0, tn, klds, J.k, cnt, deg, xs);
        };
        using T = std::true_type;
        using F = std::false_type;
        if (J.narrow) {
            if (J.div.pow2) run(T{}, T{}); else run(T{}, F{});
        } else {
            if (J.div.pow2) run(F{}, T{}); else run(F{}, F{});
        }
        stream_xor_out(xs, deg + J.k);
        __syncthreads();  // every wave has read unit_sh and counted its run
        if (threadIdx.x == 0) unit_sh = u_next;
        if constexpr (PACKED) {
            packed_flush(cnt, klds, deg);
        } else {
            for (uint32_t v = threadIdx.x; v < klds; v += kStreamBlock) {
                const uint32_t c = cnt[v];
                cnt[v] = 0;
                if (c) __hip_atomic_fetch_add(deg + v, (uint64_t)c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

// ------------------------------------------------------------ host side

// One streaming launch per slice of at most max_waves << wave_log2 edges, so
// no wave takes more than 2^wave_log2 of them (launches accumulate).
template <class L>
static int launch_stream_slices(const StreamArgs &a0, uint64_t max_waves, unsigned wave_log2, L launch)
{
    const uint64_t slice = max_waves << wave_log2;
    for (uint64_t off = 0; off < a0.count; off += slice) {
        StreamArgs a = a0;
        a.begin = a0.begin + off;
        a.count = std::min(slice, a0.count - off);
        const int rc = launch(a);
        if (rc) return rc;
    }
    return BA_OK;
}

// 16K tier: a block's LDS counts stay below 16 * 2^27 = 2^31.
template <bool N, bool P, bool I>
static int launch_stream_one(const StreamArgs &a0, hipStream_t st)
{
    uint32_t grid0 = 0;
    int rc = persistent_grid(k_stream<N, P, I>, kStreamBlock, &grid0);
    if (rc) return rc;
    const uint64_t max_waves = (uint64_t)grid0 * kStreamWaves;
    return launch_stream_slices(a0, max_waves, 27, [&](StreamArgs a) {
        uint64_t per_wave = (a.count + max_waves - 1) / max_waves;
        per_wave = (per_wave + kWave - 1) / kWave * kWave;
        if (per_wave < 4 * kWave) per_wave = 4 * kWave;
        a.per_wave = per_wave;
        const uint64_t waves = (a.count + per_wave - 1) / per_wave;
        const uint32_t grid = (uint32_t)((waves + kStreamWaves - 1) / kStreamWaves);
        return launch_timed(BA_KT_STREAM, st,
                            [&] { hipLaunchKernelGGL((k_stream<N, P, I>), dim3(grid), dim3(kStreamBlock), 0, st, a); });
    });
}

// 64K tier: a wave's share stays below 2^30 edges (32-bit claim counters).
template <bool N, bool P, bool I>
static int launch_stream_packed(const StreamArgs &a0, hipStream_t st)
{
    uint32_t grid0 = 0;
    int rc = persistent_grid(k_stream_packed<N, P, I>, kStreamBlock, &grid0);
    if (rc) return rc;
    const uint64_t max_waves = (uint64_t)grid0 * kStreamWaves;
    return launch_stream_slices(a0, max_waves, 30, [&](StreamArgs a) {
        uint64_t per_wave = (a.count + max_waves - 1) / max_waves;
        per_wave = (per_wave + kWave - 1) / kWave * kWave;
        if (per_wave < kStreamRoundClaims) per_wave = kStreamRoundClaims;
        a.per_wave = per_wave;
        a.rounds = per_wave / kStreamRoundClaims;  // no wave takes more barriers in its loop
        const uint64_t waves = (a.count + per_wave - 1) / per_wave;
        const uint32_t grid = (uint32_t)((waves + kStreamWaves - 1) / kStreamWaves);
        a.klds = (uint32_t)(a.k < kPackedNodes ? a.k : kPackedNodes);
        return launch_timed(BA_KT_STREAM, st,
                            [&] { hipLaunchKernelGGL((k_stream_packed<N, P, I>), dim3(grid), dim3(kStreamBlock), 0, st, a); });
    });
}

// BA_TIER_AUTO.  A target lands on node v with probability close to
// 1 / (2 sqrt(v n)), so about (sqrt(min(k, 65536)) - 128) / sqrt(n) of all
// targets fall in [16384, min(k, 65536)): the global atomics the 64K tier
// saves.  Their cost per atomic grows with their share (~140 ps apiece
// around n = 2^26, ~35 ps near n = 2^28, measured).  The 64K tier's one
// block per compute unit and round barriers cost ~45% more compute per edge
// with 32-bit positions and more with 64-bit ones.  Measured on MI355X
// (first_k = 10^5, 32-bit positions) the tiers break even near n = 7e7, a
// share of ~1.5%.  With 64-bit positions the 64K tier costs more compute
// (~35% at n = 2^30) but the served mix still favours it above ~1.8%.
static int stream_tier(uint64_t n, uint64_t k, bool narrow, int tier)
{
    if (tier != BA_TIER_AUTO) return tier;
    if (k <= kLdsNodes) return BA_TIER_16K;
    const double share = (std::sqrt((double)std::min<uint64_t>(k, kPackedNodes)) - 128.0) / std::sqrt((double)n);
    return share > (narrow ? 0.015 : 0.018) ? BA_TIER_64K : BA_TIER_16K;
}

static int launch_stream(uint64_t n, uint64_t begin, uint64_t count, uint32_t d, uint64_t seed, uint64_t k,
                         uint64_t *deg, uint64_t *cs, int tier, hipStream_t st)
{
    if (count == 0) return BA_OK;
    StreamArgs a{};
    a.key = make_hash_key(seed);
    a.div = make_divider(d);
    a.begin = begin;
    a.count = count;
    a.k = k;
    a.klds = (uint32_t)(k < kLdsNodes ? k : kLdsNodes);
    a.deg = deg;
    a.cs = cs;
    const bool narrow = 2 * (begin + count) <= ((uint64_t)1 << 32);
    const bool id32 = n <= ((uint64_t)1 << 32);  // every node ID below 2^32 (implied by narrow)
    const bool pow2 = a.div.pow2 != 0;
    const bool packed = stream_tier(n, k, narrow, tier) == BA_TIER_64K;
    auto go = [&](auto n_, auto p_, auto i_) {
        constexpr bool N = decltype(n_)::value, P = decltype(p_)::value, I = decltype(i_)::value;
        return packed ? launch_stream_packed<N, P, I>(a, st) : launch_stream_one<N, P, I>(a, st);
    };
    using T = std::true_type;
    using F = std::false_type;
    if (narrow) return pow2 ? go(T{}, T{}, T{}) : go(T{}, F{}, T{});
    if (id32) return pow2 ? go(F{}, T{}, T{}) : go(F{}, F{}, T{});
    return pow2 ? go(F{}, T{}, F{}) : go(F{}, F{}, F{});
}

}  // namespace ba
