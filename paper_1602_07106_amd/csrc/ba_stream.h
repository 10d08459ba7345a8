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

template <bool NARROW, bool POW2>
__global__ __launch_bounds__(kStreamBlock) void k_stream(StreamArgs a)
{
    __shared__ uint32_t cnt[kLdsNodes];
    for (uint32_t v = threadIdx.x; v < a.klds; v += kStreamBlock) cnt[v] = 0;
    __syncthreads();

    using R = typename std::conditional<NARROW, uint32_t, uint64_t>::type;
    const uint32_t lane = __lane_id();
    // wave-uniform (readfirstlane): keeps the loop control scalar
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint64_t gw = (uint64_t)blockIdx.x * kStreamWaves + wv;
    const uint64_t w0 = gw * a.per_wave;
    uint64_t xs = 0;
    if (w0 < a.count) {
        // per_wave < 2^32: the host splits larger launches
        const uint32_t tn = (uint32_t)min(a.per_wave, a.count - w0);
        const uint64_t ibase = a.begin + w0;
        chain_run_visit(
            tn, lane, (R)(2 * ibase + 1),
            [&](R r) -> R {
                if constexpr (NARROW) return hash_narrow(r, a.key);
                else return hash_wide(r, a.key);
            },
            [](R r) { return !((uint32_t)r & 1u); },
            [&](R r0, R r) {  // r0 = 2i + 1, the edge's start position
                uint64_t u, v;
                if constexpr (NARROW) {
                    v = sdiv32<POW2>((uint32_t)r >> 1, a.div);
                    u = sdiv32<POW2>((uint32_t)r0 >> 1, a.div);
                } else {
                    v = shalf64<POW2>(r, a.div);
                    u = shalf64<POW2>(r0, a.div);
                }
                if (v < a.klds)
                    atomicAdd(&cnt[v], 1u);
                else if (v < a.k)
                    __hip_atomic_fetch_add(a.deg + v, (uint64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                xs ^= ((u << 32) + v) * (uint64_t)r0;
            });
    }
    if (a.cs) {
        for (int o = 32; o > 0; o >>= 1) xs ^= __shfl_xor(xs, o);
        if (lane == 0 && xs) __hip_atomic_fetch_xor(a.cs, xs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
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

template <bool NARROW, bool POW2>
__global__ __launch_bounds__(kStreamBlock) void k_stream_packed(StreamArgs a)
{
    __shared__ uint32_t cnt[kPackedNodes / 2];  // node v: word v >> 1, half v & 1
    for (uint32_t w = threadIdx.x; w < kPackedNodes / 2; w += kStreamBlock) cnt[w] = 0;
    __syncthreads();
    using R = typename std::conditional<NARROW, uint32_t, uint64_t>::type;
    const uint32_t lane = __lane_id();
    // wave-uniform (readfirstlane): keeps the loop control scalar
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint64_t gw = (uint64_t)blockIdx.x * kStreamWaves + wv;
    const uint64_t w0 = gw * a.per_wave;
    // edges of this wave (per_wave < 2^32: the host splits larger launches)
    const uint32_t tot = w0 < a.count ? (uint32_t)min(a.per_wave, a.count - w0) : 0u;
    const uint64_t ibase = a.begin + w0;
    const R rbase = (R)(2 * ibase + 1);
    const uint32_t ktier = a.klds;  // min(first_k, 65536)
    uint64_t xs = 0;

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
                __hip_atomic_fetch_add(a.deg + pend_v, (uint64_t)0x8000, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            pend_v = kNone;
        }
    };
    auto hash = [&](R r) -> R {
        if constexpr (NARROW) return hash_narrow(r, a.key);
        else return hash_wide(r, a.key);
    };
    // r0 = 2i + 1: the edge's start position (i = r0 >> 1, and the checksum
    // multiplier itself)
    auto finish = [&](R r0, R r, uint32_t &pend_old, uint32_t &pend_v) {
        uint64_t u, v;
        if constexpr (NARROW) {
            v = sdiv32<POW2>((uint32_t)r >> 1, a.div);
            u = sdiv32<POW2>((uint32_t)r0 >> 1, a.div);
        } else {
            v = shalf64<POW2>(r, a.div);
            u = shalf64<POW2>(r0, a.div);
        }
        settle(pend_old, pend_v);
        if (v < ktier) {
            pend_old = atomicAdd(&cnt[(uint32_t)v >> 1], 1u << (((uint32_t)v & 1u) << 4));
            pend_v = (uint32_t)v;
        } else if (v < a.k) {
            __hip_atomic_fetch_add(a.deg + v, (uint64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        xs ^= ((u << 32) + v) * (uint64_t)r0;
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
    for (; bars < a.rounds; bars++) lds_barrier();

    if (a.cs) {
        for (int o = 32; o > 0; o >>= 1) xs ^= __shfl_xor(xs, o);
        if (lane == 0 && xs) __hip_atomic_fetch_xor(a.cs, xs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    for (uint32_t w = threadIdx.x; w < kPackedNodes / 2; w += kStreamBlock) {
        const uint32_t c = cnt[w];
        const uint32_t lo = c & 0xFFFFu, hi = c >> 16;
        if (lo && 2 * w < ktier)
            __hip_atomic_fetch_add(a.deg + 2 * w, (uint64_t)lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (hi && 2 * w + 1 < ktier)
            __hip_atomic_fetch_add(a.deg + 2 * w + 1, (uint64_t)hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
template <bool N, bool P>
static int launch_stream_one(const StreamArgs &a0, hipStream_t st)
{
    uint32_t grid0 = 0;
    int rc = persistent_grid(k_stream<N, P>, kStreamBlock, &grid0);
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
                            [&] { hipLaunchKernelGGL((k_stream<N, P>), dim3(grid), dim3(kStreamBlock), 0, st, a); });
    });
}

// 64K tier: a wave's share stays below 2^30 edges (32-bit claim counters).
template <bool N, bool P>
static int launch_stream_packed(const StreamArgs &a0, hipStream_t st)
{
    uint32_t grid0 = 0;
    int rc = persistent_grid(k_stream_packed<N, P>, kStreamBlock, &grid0);
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
                            [&] { hipLaunchKernelGGL((k_stream_packed<N, P>), dim3(grid), dim3(kStreamBlock), 0, st, a); });
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
    const bool pow2 = a.div.pow2 != 0;
    if (stream_tier(n, k, narrow, tier) == BA_TIER_64K) {
        if (narrow) return pow2 ? launch_stream_packed<true, true>(a, st) : launch_stream_packed<true, false>(a, st);
        return pow2 ? launch_stream_packed<false, true>(a, st) : launch_stream_packed<false, false>(a, st);
    }
    if (narrow) return pow2 ? launch_stream_one<true, true>(a, st) : launch_stream_one<true, false>(a, st);
    return pow2 ? launch_stream_one<false, true>(a, st) : launch_stream_one<false, false>(a, st);
}

}  // namespace ba
