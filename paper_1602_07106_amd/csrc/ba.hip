// ba.hip -- gfx950 kernels and the C ABI of libba (declared in include/ba.h).
//
// The method (paper Section 2, figure generateEdge): edge i of a
// Barabasi-Albert graph with an empty seed graph is computed on its own, with
// no access to the edge array: r = 2i+1, then r = h(r) (at least once) until r
// is even, and the edge is (floor(i/d), floor(r/(2d))).  Edges are
// independent units, so a launch is a set of waves that each own a
// contiguous run of edge IDs (the batches of edge IDs of paper Section 2).
//
// Wavefront-level refill.  The number of hash steps of an edge is geometric
// with mean about 2 (paper Section 2: P(more than k steps) <= 2^-k).  One
// edge per lane would keep a wave64 busy for the longest of 64 chains
// (about 7 steps) for 2 steps of useful work per lane.  Instead each lane runs
// one chain step per iteration; a lane whose chain ends hands its result to
// LDS and takes the next unclaimed edge of its wave's tile (ballot + mbcnt
// give every finishing lane a distinct next edge).  All lanes stay busy
// until the tile runs dry.
//
// Output.  The stored kernel writes edge pairs (u, v) as uint32.  Finished
// chains leave their final position r (narrow path) or v (wide path) in a
// per-wave LDS tile; when the tile is complete the wave writes it out as
// 16-byte (two-edge) coalesced stores, computing u = floor(i/d) and v on the
// way.  The degree array (ba_degree.h) is computed from the target list by a
// radix partition and LDS histograms; first endpoints contribute exactly d
// per node, in closed form.
//
// The streaming kernels (paper Section 3, ba_stream.h) store nothing: each
// finished edge updates the degree counts of the first k nodes (an
// LDS-privatised table for the hottest low IDs, 64-bit global atomics above)
// and a per-lane XOR checksum, reduced per wave at the end.

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <mutex>
#include <new>
#include <type_traits>
#include <utility>
#include <vector>

#include "ba_degree.h"
#include "ba_device.h"
#include "../../include/ba.h"

namespace ba {

constexpr int kWave = 64;
constexpr int kGenBlock = 256;  // 4 waves
constexpr int kGenWaves = kGenBlock / kWave;
constexpr uint32_t kTile = 1024;  // edges per wave tile (4 KiB of LDS per wave)
constexpr uint32_t kGenCarry = 192;  // next-tile edges a wave's chain tail may claim (8 waves/SIMD still fit)

struct GenArgs {
    HashKey key;
    Divider div;
    uint64_t begin;   // first edge ID of the launch
    uint64_t count;   // number of edges
    uint64_t ntiles;  // ceil(count / kTile)
    uint32_t d;
    uint32_t *edges;  // 2*count uint32
    uint32_t *vlist;  // count uint32 second endpoints (degree pipeline), or null
    uint32_t *deg;    // degree counts the second endpoints are added to (kDegAtomic)
};

// What the generator does with second endpoints besides storing the edges.
enum DegMode { kDegNone = 0, kDegList = 1, kDegAtomic = 2 };

__device__ __forceinline__ uint32_t lane_rank(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Edges of a tile: min(cap, rest) in 64 bits, then narrowed (at most cap).
__device__ __forceinline__ uint32_t tile_len(uint32_t cap, uint64_t rest)
{
    return rest < cap ? (uint32_t)rest : cap;
}


// floor(x / d) with the divider's kind (a power of two or not) fixed at
// compile time, so the flush loops carry no per-step branch on it.  x < 2^31
// (the 31-bit multiplier); values of a pair past the end of a tile may break
// that, and they are never stored.
template <bool POW2>
__device__ __forceinline__ uint32_t fdiv32(uint32_t x, const Divider &v)
{
    if constexpr (POW2) return x >> v.shift;
    return mulhi32(x, v.m32) >> v.shift;
}

template <bool POW2>
__device__ __forceinline__ uint64_t fdiv64(uint64_t x, const Divider &v)
{
    if constexpr (POW2) return x >> v.shift;
    return mulhi64(x, v.m64) >> v.shift;  // x < 2^63
}

// Edge pair j, j+1 of a tile from the stage: u = floor(i/d) and v (the
// stage holds the final position r on the narrow path, v itself on the wide
// path).
template <bool NARROW, bool POW2>
__device__ __forceinline__ void flush_pair(const GenArgs &a, const uint32_t *stage, uint64_t ibase, uint32_t j,
                                           uint32_t &u0, uint32_t &u1, uint32_t &v0, uint32_t &v1)
{
    const uint2 s = *reinterpret_cast<const uint2 *>(stage + j);
    if constexpr (NARROW) {
        const uint32_t i0 = (uint32_t)ibase + j;
        u0 = fdiv32<POW2>(i0, a.div);
        u1 = fdiv32<POW2>(i0 + 1, a.div);
        v0 = fdiv32<POW2>(s.x >> 1, a.div);
        v1 = fdiv32<POW2>(s.y >> 1, a.div);
    } else {
        const uint64_t i0 = ibase + j;
        u0 = (uint32_t)fdiv64<POW2>(i0, a.div);
        u1 = (uint32_t)fdiv64<POW2>(i0 + 1, a.div);
        v0 = s.x;
        v1 = s.y;
    }
}

// Edge-pair output is written once and never read back by the kernel that
// writes it, so its stores are non-temporal (NT): they stream through L2
// instead of taking its lines from data that is still being assembled there
// (the fused generator's partially written partition regions; with plain
// pair stores those cost the fused kernel about 0.4 ms more, for the same
// HBM bytes).  The batched generator keeps plain stores: NT measured slower
// there.
template <bool NT>
__device__ __forceinline__ void store_u32(uint32_t *p, uint32_t x)
{
    if constexpr (NT)
        __builtin_nontemporal_store(x, p);
    else
        *p = x;
}

// (u0, v0, u1, v1) to a 16-byte aligned p.
template <bool NT = true>
__device__ __forceinline__ void store_edges16(uint32_t *p, uint32_t u0, uint32_t v0, uint32_t u1, uint32_t v1)
{
    if constexpr (NT) {
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
        const u32x4 x = {u0, v0, u1, v1};
        __builtin_nontemporal_store(x, reinterpret_cast<u32x4 *>(p));
    } else {
        *reinterpret_cast<uint4 *>(p) = make_uint4(u0, v0, u1, v1);
    }
}

// Edges j and j+1 (when j+1 < tn) to the output, one 16-byte store when aligned.
template <bool VEC16, bool NT = true>
__device__ __forceinline__ void store_pair(uint32_t *out, uint32_t j, uint32_t tn, uint32_t u0, uint32_t v0,
                                           uint32_t u1, uint32_t v1)
{
    const bool two = j + 1 < tn;
    if (VEC16 && two) {
        store_edges16<NT>(out + 2 * j, u0, v0, u1, v1);
    } else {
        store_u32<NT>(out + 2 * j, u0);
        store_u32<NT>(out + 2 * j + 1, v0);
        if (two) {
            store_u32<NT>(out + 2 * j + 2, u1);
            store_u32<NT>(out + 2 * j + 3, v1);
        }
    }
}

// The chain loop of one tile of tn edges (paper Section 2, figure
// generateEdge): lane-refill over the tile.  rbase = 2*(first edge)+1, so
// edge li of the tile starts at position rbase + 2*li.  A lane whose chain
// reaches a final position (stop(r): an even position, or a seed-graph
// position in the generalized model) stores out(r) at stage[li] and takes
// the next unclaimed edge.  While a whole wave's worth of edges is
// unclaimed every lane is busy and no per-lane bounds test is needed; the
// tail then runs the last chains with finished lanes idle.
template <class R, class H, class S, class V>
__device__ __forceinline__ void chain_tile_visit(uint32_t tn, uint32_t lane, R rbase, H hash, S stop, V visit)
{
    tn = __builtin_amdgcn_readfirstlane(tn);  // wave-uniform: keeps loop control scalar
    uint32_t li = lane;
    uint32_t next = kWave;  // next unclaimed edge (wave-uniform)
    R r = rbase + 2 * (R)li;
    if (tn >= kWave) {
        while (next + kWave <= tn) {
            r = hash(r);
            const bool fin = stop(r);
            const uint64_t dm = __ballot(fin);
            if (fin) {
                visit(li, r);
                li = next + lane_rank(dm);
                r = rbase + 2 * (R)li;
            }
            next += (uint32_t)__popcll(dm);
        }
    }
    // tail: at most 64 chains in flight, no more than tn - next left to claim.
    // A lane is live iff li < tn; the masks come from ballots of plain
    // compares (a ballot of a combined condition costs two more instructions).
    uint64_t live = __ballot(li < tn);
    while (live) {
        r = hash(r);
        const bool fin = stop(r);
        const uint64_t dm = __ballot(fin) & live;
        if (fin && li < tn) {
            visit(li, r);
            li = next + lane_rank(dm);
            r = rbase + 2 * (R)li;
        }
        next += (uint32_t)__popcll(dm);
        live = __ballot(li < tn);
    }
}

// A wave-uniform value kept opaque to the compiler, so that an expression
// built on it is not reassociated into one that needs per-lane work first.
// (readfirstlane returns int: each half goes through uint32_t, so the low
// half is not sign-extended into the high one)
__device__ __forceinline__ uint32_t wave_uniform(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t wave_uniform(uint64_t x)
{
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)x);
    return ((uint64_t)hi << 32) | lo;
}

// The same refill as chain_tile_visit for consumers that need the edge's
// start position 2i+1 rather than its index in the run: visit(r0, r) gets the
// lane's start position r0 and its final position r.  A finishing lane's
// next start position is one multiply-add of its rank onto a wave-uniform
// base, and the consumer gets i = r0 >> 1 and the checksum multiplier 2i+1 =
// r0 without recomputing them from li.
template <class R, class H, class S, class V>
__device__ __forceinline__ void chain_run_visit(uint32_t tn, uint32_t lane, R rbase, H hash, S stop, V visit)
{
    tn = __builtin_amdgcn_readfirstlane(tn);  // wave-uniform: keeps loop control scalar
    uint32_t next = kWave;                    // next unclaimed edge (wave-uniform)
    R r0 = rbase + 2 * (R)lane;
    R r = r0;
    if (tn >= kWave) {
        while (next + kWave <= tn) {
            r = hash(r);
            const bool fin = stop(r);
            const uint64_t dm = __ballot(fin);
            if (fin) {
                visit(r0, r);
                r0 = wave_uniform((R)(rbase + 2 * (R)next)) + 2 * (R)lane_rank(dm);
                r = r0;
            }
            next += (uint32_t)__popcll(dm);
        }
    }
    // tail: live iff li < tn
    uint32_t li = (uint32_t)((r0 - rbase) >> 1);
    uint64_t live = __ballot(li < tn);
    while (live) {
        r = hash(r);
        const bool fin = stop(r);
        const uint64_t dm = __ballot(fin) & live;
        if (fin && li < tn) {
            visit(r0, r);
            li = next + lane_rank(dm);
            r0 = rbase + 2 * (R)li;
            r = r0;
        }
        next += (uint32_t)__popcll(dm);
        live = __ballot(li < tn);
    }
}

typedef __attribute__((address_space(3))) uint32_t lds_u32;

// Chain-loop state a wave carries from one of its tiles into its next
// (chain_tile_carry): the next tile's first ncl edges are claimed; a lane
// still running one of them keeps its position and its index there, and
// the results of those that already finished wait in the wave's side buffer.
constexpr uint32_t kIdle = 0xFFFFFFFFu;
template <class R>
struct ChainCarry {
    R r = 0;             // per lane: the chain's current position (valid iff li < ncl)
    uint32_t li = kIdle; // per lane: index of its edge in the next tile, or kIdle
    uint32_t ncl = 0;    // wave-uniform: edges of the next tile claimed (a prefix)
};

// The chain loop of one tile of tn edges of the plain model (chains end at
// the first even position), writing out(r) of edge li to stage[li], with
// the tail filled from the wave's next tile (tn2 edges from position
// rbase2; none if tn2 = 0).  The refill is chain_tile_visit's, but a lane
// keeps the LDS byte address of its stage slot instead of li: a finishing
// lane's next slot and restart position are each one multiply-add of its
// rank onto a wave-uniform base (the slot and position of edge `next`).
// Once every edge of this tile is claimed, a finishing lane takes the next
// unclaimed edge of the next tile, at most CAP of them, instead of idling
// while the tile's last chains run; a finished next-tile edge stores its
// result at side[index].  The call for the next tile, with the same carry,
// copies those into its stage and resumes the chains still running.  Every
// edge's result lands at the same stage slot whatever order its chain runs
// in, so nothing downstream changes.
template <uint32_t CAP, class R, class H, class O>
__device__ __forceinline__ void chain_tile_carry(uint32_t *stage, uint32_t *side, uint32_t tn, uint32_t lane,
                                                 R rbase, uint32_t tn2, R rbase2, H hash, O out, ChainCarry<R> &c)
{
    tn = wave_uniform(tn);
    const uint32_t ncl = wave_uniform(c.ncl);  // <= tn: at most min(tn, CAP) were claimed
    for (uint32_t j = lane; j < ncl; j += kWave) stage[j] = side[j];  // slots of running chains: rewritten later
    // Edges in one index space: li < tn this tile, tn <= li < lim the next one.
    const uint32_t lim = tn + min(wave_uniform(tn2), CAP);
    const R rb2 = wave_uniform((R)(rbase2 - 2 * (R)tn));  // start position of index li >= tn: rb2 + 2 li
    const uint32_t sbase = wave_uniform((uint32_t)(uintptr_t)(lds_u32 *)stage);    // LDS byte address of slot 0
    const uint32_t xbase = wave_uniform((uint32_t)(uintptr_t)(lds_u32 *)side) - 4 * tn;  // of index li >= tn: xbase + 4 li
    // lanes without a running chain claim ncl, ncl+1, ...
    const bool held = c.li < ncl;
    const uint64_t fm = __ballot(!held);
    uint32_t li = c.li;
    R r = c.r;
    if (!held) {
        li = ncl + lane_rank(fm);
        r = (li < tn ? rbase : rb2) + 2 * (R)li;
    }
    uint32_t next = ncl + (uint32_t)__popcll(fm);  // next unclaimed index (wave-uniform)
    if (next + kWave <= tn) {
        // every lane's edge is in this tile (li < next): the steady loop
        uint32_t sa = sbase + 4 * li;
        do {
            r = hash(r);
            const bool fin = !((uint32_t)r & 1u);
            const uint64_t dm = __ballot(fin);
            if (fin) {
                *(lds_u32 *)(uintptr_t)sa = out(r);
                const uint32_t k = lane_rank(dm);
                sa = wave_uniform(sbase + 4 * next) + 4 * k;
                r = wave_uniform((R)(rbase + 2 * (R)next)) + 2 * (R)k;
            }
            next += (uint32_t)__popcll(dm);
        } while (next + kWave <= tn);
        li = (sa - sbase) >> 2;
    }
    // tail: runs until no lane holds an edge of this tile; a lane is live iff li < lim
    uint64_t cur = __ballot(li < tn);
    uint64_t live = __ballot(li < lim);
    while (cur) {
        r = hash(r);
        const bool fin = !((uint32_t)r & 1u);
        const uint64_t dm = __ballot(fin) & live;
        if (fin && li < lim) {
            *(lds_u32 *)(uintptr_t)((li < tn ? sbase : xbase) + 4 * li) = out(r);
            li = next + lane_rank(dm);  // >= lim: idle until the next call
            r = (li < tn ? rbase : rb2) + 2 * (R)li;
        }
        next += (uint32_t)__popcll(dm);
        cur = __ballot(li < tn);
        live = __ballot(li < lim);
    }
    // every index below tn was claimed (a finishing lane takes the lowest unclaimed one)
    c.ncl = min(next, lim) - tn;
    c.li = li < lim ? li - tn : kIdle;
    c.r = r;
}

// chain_tile_carry for a wave whose next tile (tn2 edges, none if 0) starts
// right after this one in edge IDs, with room for CAP more slots after the
// tile's in its stage (stage[tn .. tn+CAP)).  Index li is then edge li of
// this tile or, from tn on, of the next one, with one slot address and one
// start position formula for both: the tail claims next-tile edges with the
// steady loop's own refill, and costs one compare per step more than it
// (the test whether a lane still holds an edge of this tile).  The next call
// moves the early results (from coff on) to the front of its stage.  A chain
// ends where stop(r) holds: an even position, or a seed-graph position in
// the generalized model.
template <uint32_t CAP, class R, class H, class S, class O>
__device__ __forceinline__ void chain_tile_next_until(uint32_t *stage, uint32_t tn, uint32_t tn2, uint32_t lane,
                                                      R rbase, H hash, S stop, O out, ChainCarry<R> &c,
                                                      uint32_t &coff)
{
    tn = wave_uniform(tn);
    const uint32_t ncl = wave_uniform(c.ncl);  // <= min(tn, CAP)
    const uint32_t src = wave_uniform(coff);
    for (uint32_t j = lane; j < ncl; j += kWave) stage[j] = stage[src + j];  // slots of running chains: rewritten later
    const uint32_t lim = tn + min(wave_uniform(tn2), CAP);
    const uint32_t sbase = wave_uniform((uint32_t)(uintptr_t)(lds_u32 *)stage);  // LDS byte address of slot 0
    const uint32_t send = sbase + 4 * tn;                                        // of the tile's end
    // lanes without a running chain claim ncl, ncl+1, ...
    const bool held = c.li < ncl;
    const uint64_t fm = __ballot(!held);
    uint32_t li = held ? c.li : ncl + lane_rank(fm);
    R r = held ? c.r : rbase + 2 * (R)li;
    uint32_t sa = sbase + 4 * li;
    uint32_t next = ncl + (uint32_t)__popcll(fm);  // next unclaimed index (wave-uniform)
    auto step = [&] {  // one step of every lane; refill from `next` (no lane may claim past lim)
        r = hash(r);
        const bool fin = stop(r);
        const uint64_t dm = __ballot(fin);
        if (fin) {
            *(lds_u32 *)(uintptr_t)sa = out(r);
            const uint32_t k = lane_rank(dm);
            sa = wave_uniform(sbase + 4 * next) + 4 * k;
            r = wave_uniform((R)(rbase + 2 * (R)next)) + 2 * (R)k;
        }
        next += (uint32_t)__popcll(dm);
    };
    // steady loop: every lane's edge is in this tile (li < next <= tn)
    while (next + kWave <= tn) step();
    // tail while no claim can reach lim: every lane holds an edge below lim;
    // it ends once no lane holds one of this tile
    while (next + kWave <= lim && __ballot(sa < send)) step();
    // general tail (the claims reached lim): a lane is live iff li < lim
    li = (sa - sbase) >> 2;
    uint64_t cur = __ballot(li < tn);
    uint64_t live = __ballot(li < lim);
    while (cur) {
        r = hash(r);
        const bool fin = stop(r);
        const uint64_t dm = __ballot(fin) & live;
        if (fin && li < lim) {
            stage[li] = out(r);
            li = next + lane_rank(dm);  // >= lim: idle until the next call
            r = rbase + 2 * (R)li;
        }
        next += (uint32_t)__popcll(dm);
        cur = __ballot(li < tn);
        live = __ballot(li < lim);
    }
    c.ncl = min(next, lim) - tn;
    c.li = li < lim ? li - tn : kIdle;
    c.r = r;
    coff = tn;
}

// chain_tile_next of the plain model: chains end at the first even position.
template <uint32_t CAP, class R, class H, class O>
__device__ __forceinline__ void chain_tile_next(uint32_t *stage, uint32_t tn, uint32_t tn2, uint32_t lane, R rbase,
                                                H hash, O out, ChainCarry<R> &c, uint32_t &coff)
{
    chain_tile_next_until<CAP>(stage, tn, tn2, lane, rbase, hash, [](R r) { return !((uint32_t)r & 1u); }, out, c,
                               coff);
}

// One chain step for every lane, then refill of the lanes that finished.
// NARROW: all positions of the launch are below 2^32.  DM: the second
// endpoints also go to the degree pipeline's target list (kDegList), or are
// added to deg by global atomics (kDegAtomic, the path that needs no
// workspace: exact, but an order of magnitude slower).
template <bool NARROW, bool VEC16, int DM>
__global__ __launch_bounds__(kGenBlock) void k_gen_u32(GenArgs a)
{
    __shared__ uint32_t stage_all[kGenWaves][kTile + kGenCarry];  // a tile, then next-tile results of its tail
    const uint32_t lane = __lane_id();
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform: scalar tile bases
    uint32_t *stage = stage_all[wv];
    // wave w takes tiles t0 .. t1-1, consecutive in edge IDs, so the chain
    // tail of one tile runs straight into the next
    const uint64_t nw = (uint64_t)gridDim.x * kGenWaves, w = (uint64_t)blockIdx.x * kGenWaves + wv;
    const uint64_t per = a.ntiles / nw, extra = a.ntiles % nw;
    const uint64_t t0 = w * per + min(w, extra), t1 = t0 + per + (w < extra ? 1u : 0u);
    using R = std::conditional_t<NARROW, uint32_t, uint64_t>;
    ChainCarry<R> cc;
    uint32_t coff = 0;

    for (uint64_t tile = t0; tile < t1; tile++) {
        const uint64_t off = tile * kTile;
        const uint32_t tn = tile_len(kTile, a.count - off);
        const uint64_t ibase = a.begin + off;
        const uint32_t tn2 = tile + 1 < t1 ? tile_len(kTile, a.count - off - kTile) : 0u;

        if constexpr (NARROW)
            chain_tile_next<kGenCarry>(stage, tn, tn2, lane, (R)(2 * ibase + 1),
                                       [&](uint32_t r) { return hash_narrow(r, a.key); },
                                       [](uint32_t r) { return r; }, cc, coff);
        else
            chain_tile_next<kGenCarry>(stage, tn, tn2, lane, (R)(2 * ibase + 1),
                                       [&](uint64_t r) { return hash_wide(r, a.key); },
                                       [&](uint64_t r) { return (uint32_t)div64(r >> 1, a.div); }, cc, coff);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        // Flush: two edges per lane per step, 16-byte stores.  The divider's
        // kind and whether the tile is full are uniform, so they select a
        // loop instead of being tested in it; a full tile (all but a
        // launch's last) needs no partial-pair checks.
        uint32_t *out = a.edges + 2 * off;
        auto flush = [&](auto pow2, auto full) {
            constexpr bool P = decltype(pow2)::value, F = decltype(full)::value;
            if constexpr (F) {
                // full tile: kTile / 128 pairs per lane (a uniform trip count)
#pragma unroll 2
                for (uint32_t t = 0; t < kTile / (2 * kWave); t++) {
                    const uint32_t j = 2 * lane + t * (2 * kWave);
                    uint32_t u0, u1, v0, v1;
                    flush_pair<NARROW, P>(a, stage, ibase, j, u0, u1, v0, v1);
                    if constexpr (VEC16)
                        store_edges16(out + 2 * j, u0, v0, u1, v1);
                    else
                        store_pair<false>(out, j, kTile, u0, v0, u1, v1);
                    if constexpr (DM == kDegList) *reinterpret_cast<uint2 *>(a.vlist + off + j) = make_uint2(v0, v1);
                    if constexpr (DM == kDegAtomic) {
                        deg_atomic_add(a.deg, v0, 1u);
                        deg_atomic_add(a.deg, v1, 1u);
                    }
                }
            } else {
                for (uint32_t j = 2 * lane; j < tn; j += 2 * kWave) {
                    uint32_t u0, u1, v0, v1;
                    flush_pair<NARROW, P>(a, stage, ibase, j, u0, u1, v0, v1);
                    store_pair<VEC16>(out, j, tn, u0, v0, u1, v1);
                    if constexpr (DM == kDegList) {
                        // second endpoints alone, for the degree pipeline (8-byte aligned: j, off even)
                        if (j + 1 < tn)
                            *reinterpret_cast<uint2 *>(a.vlist + off + j) = make_uint2(v0, v1);
                        else
                            a.vlist[off + j] = v0;
                    }
                    if constexpr (DM == kDegAtomic) {
                        deg_atomic_add(a.deg, v0, 1u);
                        if (j + 1 < tn) deg_atomic_add(a.deg, v1, 1u);
                    }
                }
            }
        };
        using T = std::true_type;
        using Fa = std::false_type;
        if (a.div.pow2) {
            if (tn == kTile) flush(T{}, T{});
            else flush(T{}, Fa{});
        } else {
            if (tn == kTile) flush(Fa{}, T{});
            else flush(Fa{}, Fa{});
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

}  // namespace ba

#include "ba_genpart.h"
#include "ba_batch.h"
#include "ba_model.h"

namespace ba {

// 64-bit node IDs, any positions: each finished chain stores its edge pair
// directly (used for ranges of very large graphs; not the bandwidth path).
struct Gen64Args {
    HashKey key;
    Divider div;
    uint64_t begin, count;
    uint64_t nchunks;  // ceil(count / kTile)
    uint64_t *edges;   // 2*count uint64
};

__global__ __launch_bounds__(kGenBlock) void k_gen_u64(Gen64Args a)
{
    const uint32_t lane = __lane_id();
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform: scalar loops
    const uint64_t wstride = (uint64_t)gridDim.x * kGenWaves;
    for (uint64_t c = (uint64_t)blockIdx.x * kGenWaves + wv; c < a.nchunks; c += wstride) {
        const uint64_t off = c * kTile;
        const uint32_t tn = tile_len(kTile, a.count - off);
        const uint64_t ibase = a.begin + off;
        uint64_t *out = a.edges + 2 * off;
        chain_tile_visit(
            tn, lane, 2 * ibase + 1, [&](uint64_t r) { return hash_wide(r, a.key); },
            [](uint64_t r) { return !((uint32_t)r & 1u); },
            [&](uint32_t li, uint64_t r) {
                uint64_t *o = out + 2 * li;
                o[0] = div64(ibase + li, a.div);
                o[1] = div64(r >> 1, a.div);
            });
    }
}

// deg[v] = d for v < n (first endpoints of a whole graph, in closed form).
__global__ void k_fill_u32(uint32_t *p, uint64_t count, uint32_t value)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < count; j += stride)
        p[j] = value;
}

__global__ void k_fill_u64(uint64_t *p, uint64_t count, uint64_t value)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < count; j += stride)
        p[j] = value;
}

// First-endpoint counts of the edges b .. b+c-1 for nodes v0 .. v1-1: node v
// is the first endpoint of edges v*d .. v*d+d-1.
template <class T>
__global__ void k_first_endpoints(T *deg, uint64_t v0, uint64_t v1, uint64_t b, uint64_t c,
                                  uint64_t d)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = v0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < v1; v += stride) {
        const uint64_t lo = max(b, v * d), hi = min(b + c, v * d + d);
        if (hi > lo) atomicAdd(deg + v, (T)(hi - lo));
    }
}

// ------------------------------------------------------------ host side

static thread_local int g_last_hip = 0;

static int hip_check(hipError_t e)
{
    if (e != hipSuccess) {
        g_last_hip = (int)e;
        return BA_EDEVICE;
    }
    return BA_OK;
}

// Resident blocks per CU of a kernel, times the CU count: the persistent
// grid.  Waves take units round-robin, so a grid larger than what is resident
// would leave late blocks running alone at the end.
template <class K>
static int persistent_grid(K kernel, int block, uint32_t *grid)
{
    int dev = 0, cus = 0, per_cu = 0;
    int rc = hip_check(hipGetDevice(&dev));
    if (rc) return rc;
    rc = hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (rc) return rc;
    rc = hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0));
    if (rc) return rc;
    if (per_cu < 1) per_cu = 1;
    *grid = (uint32_t)(cus * per_cu);
    return BA_OK;
}

// 2*n*d must fit 64 bits (positions are 64-bit).
static bool graph_fits(uint64_t n, uint32_t d, uint64_t *m)
{
    unsigned __int128 mm = (unsigned __int128)n * d;
    if (mm >> 63) return false;
    *m = (uint64_t)mm;
    return true;
}

static uint32_t grid_for(uint64_t units, uint64_t per_block, uint64_t cap)
{
    uint64_t b = (units + per_block - 1) / per_block;
    if (b > cap) b = cap;
    if (b == 0) b = 1;
    return (uint32_t)b;
}

// Opt-in measurement of kernel durations (per host thread): an event pair
// recorded on the launch stream around every launch, tagged with the kind of
// kernel (BA_KT_*).
struct KernelTiming {
    struct Rec {
        int kind;
        hipEvent_t e0, e1;
    };
    bool on = false;
    std::vector<Rec> ev;
};
static thread_local KernelTiming g_timing;

// Runs `launch` (which enqueues one kernel on st), bracketed by events when
// timing is on; returns the launch status.
template <class F>
static int launch_timed(int kind, hipStream_t st, F &&launch)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc;
    if (g_timing.on) {
        if ((rc = hip_check(hipEventCreate(&e0)))) return rc;
        if ((rc = hip_check(hipEventCreate(&e1)))) {
            (void)hipEventDestroy(e0);
            return rc;
        }
        if ((rc = hip_check(hipEventRecord(e0, st)))) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return rc;
        }
    }
    launch();
    rc = hip_check(hipGetLastError());
    if (g_timing.on) {
        const int rc2 = hip_check(hipEventRecord(e1, st));
        g_timing.ev.push_back({kind, e0, e1});
        if (!rc) rc = rc2;
    }
    return rc;
}

template <bool N, bool V, int L>
static int launch_gen_one(const GenArgs &a, hipStream_t st)
{
    uint32_t grid = 0;
    int rc = persistent_grid(k_gen_u32<N, V, L>, kGenBlock, &grid);
    if (rc) return rc;
    grid = grid_for(a.ntiles, kGenWaves, grid);
    return launch_timed(BA_KT_GEN, st,
                        [&] { hipLaunchKernelGGL((k_gen_u32<N, V, L>), dim3(grid), dim3(kGenBlock), 0, st, a); });
}

// Generator over edges begin .. begin+count-1 writing edge pairs to `edges`
// and, when vlist is set (8-byte aligned), the second endpoints alone, or,
// when deg is set, adding the second endpoints to deg by atomics.
static int launch_gen_u32(uint64_t begin, uint64_t count, uint32_t d, uint64_t seed, uint32_t *edges,
                          hipStream_t st, uint32_t *vlist = nullptr, uint32_t *deg = nullptr)
{
    if (count == 0) return BA_OK;
    GenArgs a{};
    a.key = make_hash_key(seed);
    a.div = make_divider(d);
    a.begin = begin;
    a.count = count;
    a.ntiles = (count + kTile - 1) / kTile;
    a.d = d;
    a.edges = edges;
    a.vlist = vlist;
    a.deg = deg;
    const bool narrow = 2 * (begin + count) <= ((uint64_t)1 << 32);
    const bool vec16 = ((uintptr_t)edges & 15) == 0;
    const int dm = vlist ? kDegList : deg ? kDegAtomic : kDegNone;
    auto pick = [&](auto n_t, auto v_t) {
        constexpr bool N = decltype(n_t)::value, V = decltype(v_t)::value;
        if (dm == kDegList) return launch_gen_one<N, V, kDegList>(a, st);
        if (dm == kDegAtomic) return launch_gen_one<N, V, kDegAtomic>(a, st);
        return launch_gen_one<N, V, kDegNone>(a, st);
    };
    using T = std::true_type;
    using Fa = std::false_type;
    if (narrow) return vec16 ? pick(T{}, T{}) : pick(T{}, Fa{});
    return vec16 ? pick(Fa{}, T{}) : pick(Fa{}, Fa{});
}

// Largest pass (edges) of the degree pipeline whose layout for up to
// pmax partition blocks fits ws_bytes (a multiple of the partition chunk
// when several passes are needed); 0 if not even the smallest pass fits.
static uint64_t deg_piece(uint64_t n, uint64_t count, uint64_t ws_bytes, uint32_t pmax)
{
    uint64_t hi = count < kPieceMax ? count : kPieceMax;
    if (make_deg_plan(n, hi, pmax).bytes <= ws_bytes) return hi;
    uint64_t lo = hi < kPieceMin ? hi : kPieceMin;
    if (lo == hi || make_deg_plan(n, lo, pmax).bytes > ws_bytes) return 0;
    while (hi - lo > 1) {  // the layout grows with the pass
        const uint64_t mid = lo + (hi - lo) / 2;
        if (make_deg_plan(n, mid, pmax).bytes <= ws_bytes) lo = mid; else hi = mid;
    }
    return lo / kPChunk * kPChunk;
}

// Totals, part scan and histograms of a pass whose partition has run, then
// (unfused pipeline only) the targets after the partition's last whole chunk.
static int deg_count(const DegArgs &a, uint64_t count, hipStream_t st)
{
    int rc;
    if ((rc = launch_timed(BA_KT_OTHER, st,
                           [&] { hipLaunchKernelGGL(k_deg_tot, dim3(a.p.NBsub), dim3(256), 0, st, a); })))
        return rc;
    if ((rc = launch_timed(BA_KT_OTHER, st, [&] { hipLaunchKernelGGL(k_deg_scan, dim3(1), dim3(1024), 0, st, a); })))
        return rc;
    const uint32_t parts_max = (uint32_t)((uint64_t)a.p.NBsub + (count + a.p.H - 1) / a.p.H + 1);
    if ((rc = launch_timed(BA_KT_HIST, st, [&] {
             if (a.p.S == kS16)
                 hipLaunchKernelGGL(k_deg_hist16, dim3(parts_max), dim3(kHBlock), 0, st, a);
             else
                 hipLaunchKernelGGL(k_deg_hist, dim3(parts_max), dim3(kHBlock), 0, st, a);
         })))
        return rc;
    // the tail's atomics after the histogram, which may store single-part counts directly
    if (!a.p.fused && count % kPChunk) {
        const uint32_t tb = (uint32_t)((count % kPChunk + 255) / 256);
        if ((rc = launch_timed(BA_KT_OTHER, st, [&] { hipLaunchKernelGGL(k_deg_tail, dim3(tb), dim3(256), 0, st, a); })))
            return rc;
    }
    return BA_OK;
}

// Second endpoints of edges begin .. begin+count-1 (the target list the
// generator left in the workspace) added to deg: partition, totals, part
// scan, histograms.  First endpoints are the caller's (a fill of d or the
// closed-form range counts).
static int degrees_of_targets(uint64_t n, uint32_t d, uint64_t begin, uint64_t count, uint32_t *deg, void *ws,
                              bool fresh, double cap_scale, uint32_t pmax, hipStream_t st)
{
    uint32_t P = 0;
    int rc = persistent_grid(k_deg_part, kPBlock, &P);
    if (rc) return rc;
    if (P > pmax) P = pmax;
    DegArgs a{};
    a.p = make_deg_plan(n, count, P);
    a.B = begin;
    a.d = d;
    a.deg = deg;
    a.ws = (unsigned char *)ws;
    a.scale = cap_scale;
    a.fresh = fresh ? 1u : 0u;
    if ((rc = launch_timed(BA_KT_OTHER, st, [&] { hipLaunchKernelGGL(k_deg_plan, dim3(1), dim3(1024), 0, st, a); })))
        return rc;
    for (uint32_t w = 0; w < a.p.NW; w++) {
        a.g0 = w * kWin;
        if ((rc = launch_timed(BA_KT_PART, st,
                               [&] { hipLaunchKernelGGL(k_deg_part, dim3(P), dim3(kPBlock), 0, st, a); })))
            return rc;
    }
    return deg_count(a, count, st);
}

// One pass of the fused pipeline (graphs with one window of sub-buckets):
// k_gen_part writes edges begin .. begin+count-1 and partitions their second
// endpoints, then the histograms add them to deg.
static int gen_part_pass(uint64_t n, uint32_t d, uint64_t seed, uint64_t begin, uint64_t count, uint32_t *edges,
                         uint32_t *deg, void *ws, bool fresh, double cap_scale, uint32_t pmax, hipStream_t st)
{
    GenPartArgs ga{};
    ga.g.key = make_hash_key(seed);
    ga.g.div = make_divider(d);
    ga.g.begin = begin;
    ga.g.count = count;
    ga.g.ntiles = (count + kFChunk - 1) / kFChunk;
    ga.g.d = d;
    ga.g.edges = edges;
    ga.nchunks = ga.g.ntiles;
    auto run = [&](auto kern) -> int {
        uint32_t P = 0;
        int rc = persistent_grid(kern, kFBlock, &P);
        if (rc) return rc;
        if (P > pmax) P = pmax;
        DegArgs &q = ga.p;
        q.p = make_deg_plan(n, count, P);
        q.B = begin;
        q.d = d;
        q.deg = deg;
        q.ws = (unsigned char *)ws;
        q.scale = cap_scale;
        q.fresh = fresh ? 1u : 0u;
        q.g0 = 0;
        if ((rc = launch_timed(BA_KT_OTHER, st,
                               [&] { hipLaunchKernelGGL(k_deg_plan, dim3(1), dim3(1024), 0, st, q); })))
            return rc;
        if ((rc = launch_timed(BA_KT_GEN, st, [&] { hipLaunchKernelGGL(kern, dim3(P), dim3(kFBlock), 0, st, ga); })))
            return rc;
        return deg_count(q, count, st);
    };
    const bool narrow = 2 * (begin + count) <= ((uint64_t)1 << 32);
    const bool vec16 = ((uintptr_t)edges & 15) == 0;
    const bool pow2 = ga.g.div.pow2 != 0;
    if (narrow) {
        if (pow2) return vec16 ? run(k_gen_part<true, true, true>) : run(k_gen_part<true, true, false>);
        return vec16 ? run(k_gen_part<true, false, true>) : run(k_gen_part<true, false, false>);
    }
    if (pow2) return vec16 ? run(k_gen_part<false, true, true>) : run(k_gen_part<false, true, false>);
    return vec16 ? run(k_gen_part<false, false, true>) : run(k_gen_part<false, false, false>);
}

// Edges [begin, begin+count) written to `edges`, their second endpoints
// added to deg, pass by pass, with at most pmax partition blocks.  fresh:
// deg[v] = d for every node (a whole graph's first endpoints, just filled),
// so the first pass may store counts without reading deg.
static int gen_with_degrees(uint64_t n, uint32_t d, uint64_t seed, uint64_t begin, uint64_t count,
                            uint32_t *edges, uint32_t *deg, void *ws, uint64_t ws_bytes, bool fresh, hipStream_t st,
                            double cap_scale = 1.0, uint32_t pmax = kPBlocksMax)
{
    if (count == 0) return BA_OK;
    const uint64_t piece = deg_piece(n, count, ws_bytes, pmax);
    if (piece == 0 || !ws || ((uintptr_t)ws & 255)) return BA_EINVAL;
    for (uint64_t done = 0; done < count; done += piece) {
        const uint64_t C = count - done < piece ? count - done : piece;
        const DegPlan p = make_deg_plan(n, C, pmax);
        int rc;
        if (p.fused) {
            rc = gen_part_pass(n, d, seed, begin + done, C, edges + 2 * done, deg, ws, fresh && done == 0, cap_scale,
                               pmax, st);
        } else {
            rc = launch_gen_u32(begin + done, C, d, seed, edges + 2 * done, st,
                                (uint32_t *)((unsigned char *)ws + p.o_V));
            if (!rc) rc = degrees_of_targets(n, d, begin + done, C, deg, ws, fresh && done == 0, cap_scale, pmax, st);
        }
        if (rc) return rc;
    }
    return BA_OK;
}

template <class T>
static int launch_first_endpoints(T *deg, uint64_t n, uint64_t begin, uint64_t count, uint32_t d,
                                  uint64_t node_limit, hipStream_t st)
{
    if (count == 0 || d == 0) return BA_OK;
    uint64_t v0 = begin / d, v1 = (begin + count - 1) / d + 1;
    if (v1 > n) v1 = n;
    if (v1 > node_limit) v1 = node_limit;
    if (v0 >= v1) return BA_OK;
    const uint32_t grid = grid_for(v1 - v0, 256, 4096);
    hipLaunchKernelGGL((k_first_endpoints<T>), dim3(grid), dim3(256), 0, st, deg, v0, v1, begin, count,
                       (uint64_t)d);
    return hip_check(hipGetLastError());
}

}  // namespace ba

#include "ba_stream.h"

namespace ba {

// ---------------------------------------------------------------------------
// Batched generation: device table layout, upload, launch, tile-shape tuning.

struct BatchLayout {
    uint64_t o_inst, o_tile0[3], bytes;
};

static BatchLayout batch_layout(uint32_t count)
{
    BatchLayout L{};
    uint64_t o = 0;
    L.o_inst = o;
    o = align256(o + sizeof(BatchInst) * (uint64_t)count);
    for (int s = 0; s < 3; s++) {
        L.o_tile0[s] = o;
        o = align256(o + 8ull * ((uint64_t)count + 1));
    }
    L.bytes = o;
    return L;
}

// Kernel shapes the tuner chooses from: (tile edges, waves per block).
struct BatchShape {
    int tile_idx;  // index into kBatchTiles
    uint32_t waves;
};
constexpr BatchShape kBatchShapes[] = {{0, 4}, {1, 4}, {2, 4}, {0, 8}, {1, 8}};
constexpr int kBatchShapeCount = sizeof(kBatchShapes) / sizeof(kBatchShapes[0]);
constexpr int kMaxDevices = 64;
// Tuned shape per device, -1 = default (shape 0): the library's one piece of
// process-wide state, a cache that ba_batch_autotune writes and the launches
// read (atomics, so calls from several host threads do not race).
static std::atomic<int> g_batch_shape[kMaxDevices];
static int batch_shape_of(int slot)
{
    const int s = g_batch_shape[slot].load(std::memory_order_relaxed);
    return s <= 0 || s >= kBatchShapeCount ? 0 : s;
}

template <uint32_t TILE, uint32_t WAVES>
static int launch_batch_shape(BatchArgs a, hipStream_t st)
{
    uint32_t grid = 0;
    int rc = persistent_grid(k_gen_batch<TILE, WAVES>, WAVES * 64, &grid);
    if (rc) return rc;
    return launch_timed(BA_KT_GEN, st,
                        [&] { hipLaunchKernelGGL((k_gen_batch<TILE, WAVES>), dim3(grid), dim3(WAVES * 64), 0, st, a); });
}

static int launch_batch(int shape, const ba_batch_info *info, const void *ws, uint32_t *edges, hipStream_t st)
{
    const BatchShape S = kBatchShapes[shape];
    const BatchLayout L = batch_layout(info->count);
    BatchArgs a{};
    a.inst = (const BatchInst *)((const unsigned char *)ws + L.o_inst);
    a.tile0 = (const uint64_t *)((const unsigned char *)ws + L.o_tile0[S.tile_idx]);
    a.count = info->count;
    a.tiles = info->tiles[S.tile_idx];
    a.edges = edges;
    if (a.tiles == 0) return BA_OK;
    switch (shape) {
    case 0: return launch_batch_shape<1024, 4>(a, st);
    case 1: return launch_batch_shape<2048, 4>(a, st);
    case 2: return launch_batch_shape<4096, 4>(a, st);
    case 3: return launch_batch_shape<1024, 8>(a, st);
    default: return launch_batch_shape<2048, 8>(a, st);
    }
}

static int current_device_slot(int *slot)
{
    int dev = 0;
    int rc = hip_check(hipGetDevice(&dev));
    if (rc) return rc;
    if (dev < 0 || dev >= kMaxDevices) return BA_EINVAL;
    *slot = dev;
    return BA_OK;
}


// ---------------------------------------------------------------------------
// Generalized model (seed graph, self-loop-free draws, CRC hash).

static constexpr CrcTables kHostCrcTables = make_crc_tables();

template <bool C, bool L, bool N>
static int launch_model_one(const ModelArgs &a, hipStream_t st)
{
    uint32_t grid = 0;
    int rc = persistent_grid(k_gen_model<C, L, N>, kModelBlock<C>, &grid);
    if (rc) return rc;
    grid = grid_for(a.ntiles, kModelWaves<C>, grid);
    return launch_timed(BA_KT_GEN, st, [&] {
        hipLaunchKernelGGL((k_gen_model<C, L, N>), dim3(grid), dim3(kModelBlock<C>), 0, st, a);
    });
}

template <bool C, bool L>
static int launch_model_width(const ModelArgs &a, bool narrow, hipStream_t st)
{
    return narrow ? launch_model_one<C, L, true>(a, st) : launch_model_one<C, L, false>(a, st);
}

}  // namespace ba

#include "ba_server.h"

// Device scratch of ba_generate_static: the degree pipeline's workspace for
// callers that cannot allocate.  Each device holds its own copy from the
// moment the library's code is loaded on it until the process ends.  In host
// code `scratch` names a host-side stand-in, not the device copy: kernels get
// the per-device address that static_scratch() takes from the runtime.
static __device__ __align__(256) unsigned char scratch[BA_STATIC_SCRATCH_BYTES];

namespace ba {

// Partition blocks of a pass through the static scratch.  Fixed, so the
// host decides before any device call whether a graph fits (BA_ENOMEM), and
// small, since every (block, sub-bucket) region costs its slack in the
// layout; MI355X has 256 compute units, one partition block each.
constexpr uint32_t kStaticPBlocks = 256;

static std::mutex g_scratch_mu;
static std::atomic<void *> g_scratch_addr[kMaxDevices];

// Device address of the current device's copy of `scratch`, looked up once
// per device (with that device current) and kept.
static int static_scratch(void **out)
{
    int slot = 0;
    int rc = current_device_slot(&slot);
    if (rc) return rc;
    void *p = g_scratch_addr[slot].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        p = g_scratch_addr[slot].load(std::memory_order_relaxed);
        if (!p) {
            if ((rc = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))))) return rc;
            if (!p || ((uintptr_t)p & 255)) return BA_EDEVICE;
            g_scratch_addr[slot].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return BA_OK;
}

}  // namespace ba

using namespace ba;

extern "C" {

static int check_generate(uint64_t n, uint32_t d, uint64_t begin, uint64_t count, const uint32_t *edges,
                          const uint32_t *deg)
{
    uint64_t m;
    if (!graph_fits(n, d, &m) || n > ((uint64_t)1 << 32)) return BA_ERANGE;
    // uint32 degrees: node v holds its d first endpoints and at most the
    // second endpoints of edges d*v .. m-1, so every count is at most m + d
    if (deg && m + d > (uint64_t)UINT32_MAX) return BA_ERANGE;
    if (begin > m || count > m - begin) return BA_EINVAL;
    if ((count && !edges) || ((uintptr_t)edges & 3) || ((uintptr_t)deg & 3)) return BA_EINVAL;
    return BA_OK;
}

static int fill_first_endpoints_whole(uint64_t n, uint32_t d, uint32_t *deg, hipStream_t st)
{
    if (!deg || !n) return BA_OK;
    return launch_timed(BA_KT_OTHER, st, [&] {
        hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256 * 8, 8192)), dim3(256), 0, st, deg, n, d);
    });
}

int ba_generate(uint64_t n, uint32_t d, uint64_t seed, uint32_t *edges, uint32_t *deg, void *stream)
{
    uint64_t m = 0;
    int rc = check_generate(n, d, 0, 0, edges, deg);
    if (rc) return rc;
    graph_fits(n, d, &m);
    if (m && !edges) return BA_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = fill_first_endpoints_whole(n, d, deg, st))) return rc;
    // no workspace: second endpoints by global atomics (no allocation)
    return launch_gen_u32(0, m, d, seed, edges, st, nullptr, deg);
}

int ba_generate_ws(uint64_t n, uint32_t d, uint64_t seed, uint32_t *edges, uint32_t *deg, void *workspace,
                   uint64_t workspace_bytes, void *stream)
{
    uint64_t m = 0;
    int rc = check_generate(n, d, 0, 0, edges, deg);
    if (rc) return rc;
    graph_fits(n, d, &m);
    if (m && !edges) return BA_EINVAL;
    if (deg && m && (!workspace || ((uintptr_t)workspace & 255))) return BA_EINVAL;
    if (deg && m && deg_piece(n, m, workspace_bytes, kPBlocksMax) == 0) return BA_ENOMEM;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = fill_first_endpoints_whole(n, d, deg, st))) return rc;
    if (deg) return gen_with_degrees(n, d, seed, 0, m, edges, deg, workspace, workspace_bytes, true, st);
    return launch_gen_u32(0, m, d, seed, edges, st);
}

int ba_generate_static(uint64_t n, uint32_t d, uint64_t seed, uint32_t *edges, uint32_t *deg, void *stream)
{
    uint64_t m = 0;
    int rc = check_generate(n, d, 0, 0, edges, deg);
    if (rc) return rc;
    graph_fits(n, d, &m);
    if (m && !edges) return BA_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (!deg || !m) {
        if ((rc = fill_first_endpoints_whole(n, d, deg, st))) return rc;
        return launch_gen_u32(0, m, d, seed, edges, st);
    }
    if (deg_piece(n, m, BA_STATIC_SCRATCH_BYTES, kStaticPBlocks) == 0) return BA_ENOMEM;
    void *ws = nullptr;
    if ((rc = static_scratch(&ws))) return rc;
    if ((rc = fill_first_endpoints_whole(n, d, deg, st))) return rc;
    return gen_with_degrees(n, d, seed, 0, m, edges, deg, ws, BA_STATIC_SCRATCH_BYTES, true, st, 1.0,
                            kStaticPBlocks);
}

int ba_generate_range(uint64_t n, uint32_t d, uint64_t seed, uint64_t edge_begin, uint64_t edge_count,
                      uint32_t *edges, uint32_t *deg, void *stream)
{
    int rc = check_generate(n, d, edge_begin, edge_count, edges, deg);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (deg) {
        if ((rc = launch_first_endpoints<uint32_t>(deg, n, edge_begin, edge_count, d, n, st))) return rc;
        return launch_gen_u32(edge_begin, edge_count, d, seed, edges, st, nullptr, deg);
    }
    return launch_gen_u32(edge_begin, edge_count, d, seed, edges, st);
}

int ba_generate_range_ws(uint64_t n, uint32_t d, uint64_t seed, uint64_t edge_begin, uint64_t edge_count,
                         uint32_t *edges, uint32_t *deg, void *workspace, uint64_t workspace_bytes,
                         void *stream)
{
    int rc = check_generate(n, d, edge_begin, edge_count, edges, deg);
    if (rc) return rc;
    if (deg && edge_count && (!workspace || ((uintptr_t)workspace & 255))) return BA_EINVAL;
    if (deg && edge_count && deg_piece(n, edge_count, workspace_bytes, kPBlocksMax) == 0) return BA_ENOMEM;
    hipStream_t st = (hipStream_t)stream;
    if (deg) {
        if ((rc = launch_first_endpoints<uint32_t>(deg, n, edge_begin, edge_count, d, n, st))) return rc;
        return gen_with_degrees(n, d, seed, edge_begin, edge_count, edges, deg, workspace, workspace_bytes, false,
                                st);
    }
    return launch_gen_u32(edge_begin, edge_count, d, seed, edges, st);
}

int ba_test_generate_ws_scaled(uint64_t n, uint32_t d, uint64_t seed, uint32_t *edges, uint32_t *deg,
                               void *workspace, uint64_t workspace_bytes, double cap_scale, void *stream)
{
    if (!(cap_scale > 0.0 && cap_scale <= 1.0) || !deg) return BA_EINVAL;
    uint64_t m = 0;
    int rc = check_generate(n, d, 0, 0, edges, deg);
    if (rc) return rc;
    graph_fits(n, d, &m);
    if (m && (!edges || !workspace || ((uintptr_t)workspace & 255))) return BA_EINVAL;
    if (m && deg_piece(n, m, workspace_bytes, kPBlocksMax) == 0) return BA_ENOMEM;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = fill_first_endpoints_whole(n, d, deg, st))) return rc;
    return gen_with_degrees(n, d, seed, 0, m, edges, deg, workspace, workspace_bytes, true, st, cap_scale);
}

uint64_t ba_generate_workspace_bytes(uint64_t n, uint32_t d, uint64_t edge_count)
{
    uint64_t m;
    if (!graph_fits(n, d, &m) || edge_count == 0) return 0;
    const uint64_t piece = edge_count < kPieceMax ? edge_count : kPieceMax;
    return make_deg_plan(n, piece, kPBlocksMax).bytes;
}

int ba_generate_range_u64(uint64_t n, uint32_t d, uint64_t seed, uint64_t edge_begin, uint64_t edge_count,
                          uint64_t *edges, void *stream)
{
    uint64_t m;
    if (!graph_fits(n, d, &m)) return BA_ERANGE;
    if (edge_begin > m || edge_count > m - edge_begin) return BA_EINVAL;
    if ((edge_count && !edges) || ((uintptr_t)edges & 7)) return BA_EINVAL;
    if (edge_count == 0) return BA_OK;
    Gen64Args a{};
    a.key = make_hash_key(seed);
    a.div = make_divider(d);
    a.begin = edge_begin;
    a.count = edge_count;
    a.nchunks = (edge_count + kTile - 1) / kTile;
    a.edges = edges;
    uint32_t grid = 0;
    int rc = persistent_grid(k_gen_u64, kGenBlock, &grid);
    if (rc) return rc;
    grid = grid_for(a.nchunks, kGenWaves, grid);
    hipLaunchKernelGGL(k_gen_u64, dim3(grid), dim3(kGenBlock), 0, (hipStream_t)stream, a);
    return hip_check(hipGetLastError());
}

int ba_degrees_range_tier(uint64_t n, uint32_t d, uint64_t seed, uint64_t edge_begin, uint64_t edge_count,
                          uint64_t first_k, uint64_t *deg, uint64_t *xor_checksum, int tier, void *stream)
{
    uint64_t m;
    if (tier != BA_TIER_AUTO && tier != BA_TIER_16K && tier != BA_TIER_64K) return BA_EINVAL;
    if (!graph_fits(n, d, &m)) return BA_ERANGE;
    if (first_k > n || edge_begin > m || edge_count > m - edge_begin) return BA_EINVAL;
    if ((first_k && !deg) || ((uintptr_t)deg & 7) || ((uintptr_t)xor_checksum & 7)) return BA_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (first_k) {
        int rc = launch_first_endpoints<uint64_t>(deg, n, edge_begin, edge_count, d, first_k, st);
        if (rc) return rc;
    }
    return launch_stream(n, edge_begin, edge_count, d, seed, first_k, deg, xor_checksum, tier, st);
}

int ba_degrees_range(uint64_t n, uint32_t d, uint64_t seed, uint64_t edge_begin, uint64_t edge_count,
                     uint64_t first_k, uint64_t *deg, uint64_t *xor_checksum, void *stream)
{
    return ba_degrees_range_tier(n, d, seed, edge_begin, edge_count, first_k, deg, xor_checksum, BA_TIER_AUTO,
                                 stream);
}

int ba_degrees(uint64_t n, uint32_t d, uint64_t seed, uint64_t first_k, uint64_t *deg,
               uint64_t *xor_checksum, void *stream)
{
    uint64_t m;
    if (!graph_fits(n, d, &m)) return BA_ERANGE;
    if (first_k > n) return BA_EINVAL;
    if ((first_k && !deg) || ((uintptr_t)deg & 7) || ((uintptr_t)xor_checksum & 7)) return BA_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (first_k) {
        hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(first_k, 256 * 8, 4096)), dim3(256), 0, st, deg,
                           first_k, (uint64_t)0);
        int rc = hip_check(hipGetLastError());
        if (rc) return rc;
    }
    if (xor_checksum) {
        hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, xor_checksum, (uint64_t)1, (uint64_t)0);
        int rc = hip_check(hipGetLastError());
        if (rc) return rc;
    }
    return ba_degrees_range(n, d, seed, 0, m, first_k, deg, xor_checksum, stream);
}

uint64_t ba_batch_workspace_bytes(uint32_t count) { return batch_layout(count).bytes; }

int ba_batch_upload(uint32_t count, const uint64_t *n, const uint32_t *d, const uint64_t *seed,
                    const uint64_t *out_offset, void *workspace, uint64_t workspace_bytes, ba_batch_info *info,
                    void *stream)
{
    if (!info || (count && (!n || !d || !seed || !out_offset))) return BA_EINVAL;
    const BatchLayout L = batch_layout(count);
    if (count && (!workspace || ((uintptr_t)workspace & 255) || workspace_bytes < L.bytes)) return BA_EINVAL;
    std::vector<unsigned char> host(L.bytes, 0);
    BatchInst *I = (BatchInst *)(host.data() + L.o_inst);
    uint64_t *T[3];
    for (int s = 0; s < 3; s++) T[s] = (uint64_t *)(host.data() + L.o_tile0[s]);
    uint64_t tiles[3] = {0, 0, 0}, need = 0;
    for (uint32_t j = 0; j < count; j++) {
        uint64_t m;
        if (!graph_fits(n[j], d[j], &m) || n[j] > ((uint64_t)1 << 32)) return BA_ERANGE;
        const uint64_t end = out_offset[j] + 2 * m;
        if (end < out_offset[j]) return BA_ERANGE;
        if (m && end > need) need = end;
        I[j].key = make_hash_key(seed[j]);
        I[j].narrow = 2 * m <= ((uint64_t)1 << 32) ? 1u : 0u;
        I[j].div = make_divider(d[j] ? d[j] : 1u);
        I[j].m = m;
        I[j].out = out_offset[j];
        for (int s = 0; s < 3; s++) {
            T[s][j] = tiles[s];
            tiles[s] += (m + kBatchTiles[s] - 1) / kBatchTiles[s];
        }
    }
    // tiles * waves must fit 64 bits in the kernel's split of the tiles
    if (tiles[0] >= ((uint64_t)1 << 40)) return BA_ERANGE;
    for (int s = 0; s < 3; s++) T[s][count] = tiles[s];
    if (count) {
        hipStream_t st = (hipStream_t)stream;
        int rc = hip_check(hipMemcpyAsync(workspace, host.data(), L.bytes, hipMemcpyHostToDevice, st));
        if (rc) return rc;
        if ((rc = hip_check(hipStreamSynchronize(st)))) return rc;
    }
    info->count = count;
    info->reserved = 0;
    for (int s = 0; s < 3; s++) info->tiles[s] = tiles[s];
    info->edges_len = need;
    return BA_OK;
}

int ba_batch_launch(const ba_batch_info *info, const void *workspace, uint32_t *edges, uint64_t edges_len,
                    void *stream)
{
    if (!info) return BA_EINVAL;
    if (info->count == 0 || info->tiles[0] == 0) return BA_OK;
    if (!workspace || !edges || ((uintptr_t)edges & 3) || edges_len < info->edges_len) return BA_EINVAL;
    int slot = 0;
    int rc = current_device_slot(&slot);
    if (rc) return rc;
    return launch_batch(batch_shape_of(slot), info, workspace, edges, (hipStream_t)stream);
}

int ba_batch_autotune(const ba_batch_info *info, const void *workspace, uint32_t *edges, uint64_t edges_len,
                      int *shape_out, void *stream)
{
    if (!info) return BA_EINVAL;
    if (info->count == 0 || info->tiles[0] == 0) return BA_EINVAL;
    if (!workspace || !edges || ((uintptr_t)edges & 3) || edges_len < info->edges_len) return BA_EINVAL;
    int slot = 0;
    int rc = current_device_slot(&slot);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if ((rc = hip_check(hipEventCreate(&e0)))) return rc;
    if ((rc = hip_check(hipEventCreate(&e1)))) {
        (void)hipEventDestroy(e0);
        return rc;
    }
    int best = 0;
    float best_ms = 0.0f;
    const bool timing = g_timing.on;
    g_timing.on = false;  // the tuner's own launches stay out of the kernel timing
    for (int s = 0; s < kBatchShapeCount && !rc; s++) {
        rc = launch_batch(s, info, workspace, edges, st);  // warm-up
        if (!rc) rc = hip_check(hipEventRecord(e0, st));
        for (int k = 0; k < 2 && !rc; k++) rc = launch_batch(s, info, workspace, edges, st);
        if (!rc) rc = hip_check(hipEventRecord(e1, st));
        if (!rc) rc = hip_check(hipEventSynchronize(e1));
        float ms = 0.0f;
        if (!rc) rc = hip_check(hipEventElapsedTime(&ms, e0, e1));
        if (!rc && (s == 0 || ms < best_ms)) {
            best = s;
            best_ms = ms;
        }
    }
    g_timing.on = timing;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    g_batch_shape[slot].store(best, std::memory_order_relaxed);
    if (shape_out) *shape_out = best;
    return BA_OK;
}

int ba_batch_launch_shape(const ba_batch_info *info, const void *workspace, uint32_t *edges, uint64_t edges_len,
                          int shape, void *stream)
{
    if (!info || shape < 0 || shape >= kBatchShapeCount) return BA_EINVAL;
    if (info->count == 0 || info->tiles[0] == 0) return BA_OK;
    if (!workspace || !edges || ((uintptr_t)edges & 3) || edges_len < info->edges_len) return BA_EINVAL;
    return launch_batch(shape, info, workspace, edges, (hipStream_t)stream);
}

int ba_batch_current_shape(int *shape)
{
    if (!shape) return BA_EINVAL;
    int slot = 0;
    int rc = current_device_slot(&slot);
    if (rc) return rc;
    *shape = batch_shape_of(slot);
    return BA_OK;
}

int ba_batch_shape_dims(int shape, int *tile_edges, int *waves_per_block)
{
    if (shape < 0 || shape >= kBatchShapeCount || !tile_edges || !waves_per_block) return BA_EINVAL;
    *tile_edges = (int)kBatchTiles[kBatchShapes[shape].tile_idx];
    *waves_per_block = (int)kBatchShapes[shape].waves;
    return BA_OK;
}

int ba_batch_plan_rounds(uint32_t count, const uint64_t *n, const uint32_t *d, uint64_t round_elems,
                         uint32_t *round_of, uint64_t *offset_of, uint32_t *rounds)
{
    if (!rounds || (count && (!n || !d || !round_of || !offset_of))) return BA_EINVAL;
    uint32_t r = 0;
    uint64_t off = 0;
    for (uint32_t j = 0; j < count; j++) {
        uint64_t m;
        if (!graph_fits(n[j], d[j], &m) || n[j] > ((uint64_t)1 << 32) || m > (UINT64_MAX - 3) / 2) return BA_ERANGE;
        const uint64_t need = (2 * m + 3) & ~(uint64_t)3;  // each instance starts 16-byte aligned
        if (need > round_elems) return BA_EINVAL;
        if (off + need > round_elems) {
            r++;
            off = 0;
        }
        round_of[j] = r;
        offset_of[j] = off;
        off += need;
    }
    *rounds = count ? r + 1 : 0;
    return BA_OK;
}

int ba_server_create(void *arena, uint64_t arena_bytes, void *stream, ba_server **out)
{
    if (!out || !arena || ((uintptr_t)arena & 255) || arena_bytes < 4096) return BA_EINVAL;
    *out = nullptr;
    ba_server *s = new (std::nothrow) ba_server();
    if (!s) return BA_EINVAL;
    s->arena = (unsigned char *)arena;
    s->arena_bytes = arena_bytes & ~(uint64_t)255;
    s->stream = (hipStream_t)stream;
    s->alloc = ArenaAlloc(s->arena_bytes);
    s->slot_bytes = batch_layout(kServerMaxBatch).bytes + stream_table_bytes(kServerMaxDeg);
    int rc = hip_check(hipHostMalloc((void **)&s->staging, s->slot_bytes * kServerSlots, hipHostMallocDefault));
    if (!rc) rc = hip_check(hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking));  // default priority
    if (!rc) rc = hip_check(hipEventCreate(&s->start));
    if (!rc) rc = hip_check(hipEventRecord(s->start, s->stream));
    if (rc) {
        if (s->staging) (void)hipHostFree(s->staging);
        if (s->start) (void)hipEventDestroy(s->start);
        if (s->side) (void)hipStreamDestroy(s->side);
        delete s;
        return rc;
    }
    for (int k = kServerSlots - 1; k >= 0; k--) s->free_slots.push_back(k);
    *out = s;
    return BA_OK;
}

int ba_server_destroy(ba_server *s)
{
    if (!s) return BA_EINVAL;
    int rc = hip_check(hipStreamSynchronize(s->stream));
    const int rc2 = hip_check(hipStreamSynchronize(s->side));
    if (!rc) rc = rc2;
    for (auto &st : s->steps) server_step_events_free(st);
    if (s->start) (void)hipEventDestroy(s->start);
    if (s->staging) (void)hipHostFree(s->staging);
    (void)hipStreamDestroy(s->side);
    delete s;
    return rc;
}

int ba_server_submit(ba_server *s, const ba_request *r, uint64_t *ticket)
{
    if (!s || !r || !ticket) return BA_EINVAL;
    uint64_t m;
    if (!graph_fits(r->n, r->d, &m)) return BA_ERANGE;
    // result sizes (8*m, 8*(first_k+1) bytes) must fit 64 bits
    if (r->kind == BA_REQ_EDGES) {
        if (r->n > ((uint64_t)1 << 32) || m > UINT64_MAX / 8) return BA_ERANGE;
    } else if (r->kind == BA_REQ_DEGREES) {
        if (r->first_k > r->n) return BA_EINVAL;
        if (r->first_k >= UINT64_MAX / 8) return BA_ERANGE;
    } else {
        return BA_EINVAL;
    }
    ServerJob J;
    J.req = *r;
    J.m = m;
    J.out_bytes = job_output_bytes(*r, m);
    *ticket = s->job_base + s->jobs.size();
    s->jobs.push_back(J);
    s->queue.push_back(*ticket);
    return BA_OK;
}

int ba_server_pump(ba_server *s, uint32_t max_inflight, uint32_t *launched)
{
    if (!s || !launched) return BA_EINVAL;
    *launched = 0;
    int rc = server_retire(s);
    if (rc) return rc;
    if (s->queue.empty() || s->inflight >= max_inflight) return BA_OK;
    return server_launch_step(s, launched);
}

int ba_server_poll(ba_server *s, uint64_t ticket, int *state, double *done_ms, uint64_t *offset, uint64_t *bytes)
{
    if (!s || !state) return BA_EINVAL;
    int rc = server_retire(s);
    if (rc) return rc;
    const ServerJob *Jp = server_job(s, ticket);
    if (!Jp) return BA_EINVAL;
    const ServerJob &J = *Jp;
    *state = J.state;
    if (done_ms) *done_ms = J.done_ms;
    if (offset) *offset = J.out_off;
    if (bytes) *bytes = J.out_bytes;
    return BA_OK;
}

int ba_server_completed(ba_server *s, uint64_t *tickets, uint32_t capacity, uint32_t *count)
{
    if (!s || !count || (capacity && !tickets)) return BA_EINVAL;
    int rc = server_retire(s);
    if (rc) return rc;
    const uint32_t k = (uint32_t)std::min<size_t>(capacity, s->completed.size());
    for (uint32_t j = 0; j < k; j++) tickets[j] = s->completed[j];
    s->completed.erase(s->completed.begin(), s->completed.begin() + k);
    *count = k;
    return BA_OK;
}

int ba_server_release(ba_server *s, uint64_t ticket)
{
    if (!s) return BA_EINVAL;
    ServerJob *J = server_job(s, ticket);
    if (!J || (J->state != BA_JOB_READY && J->state != BA_JOB_FAILED)) return BA_EINVAL;
    if (J->state == BA_JOB_READY) s->alloc.release(J->out_off, J->out_bytes);
    J->state = BA_JOB_RELEASED;
    server_trim(s);
    return BA_OK;
}

int ba_server_stats(ba_server *s, uint64_t *queued, uint32_t *inflight, uint64_t *arena_used)
{
    if (!s) return BA_EINVAL;
    if (queued) *queued = s->queue.size();
    if (inflight) *inflight = s->inflight;
    if (arena_used) *arena_used = s->alloc.used();
    return BA_OK;
}

int ba_generate_model(uint64_t n, uint32_t d, uint64_t seed, uint64_t n0, uint64_t m0, const uint32_t *seed_edges,
                      uint32_t flags, uint64_t edge_begin, uint64_t edge_count, uint32_t *edges, void *stream)
{
    if (flags & ~(uint32_t)(BA_NO_SELF_LOOPS | BA_HASH_CRC)) return BA_EINVAL;
    if (n0 > n) return BA_EINVAL;
    if (n > ((uint64_t)1 << 32)) return BA_ERANGE;
    uint64_t m;
    if (!graph_fits(n - n0, d, &m)) return BA_ERANGE;
    const unsigned __int128 pos = (unsigned __int128)2 * m0 + (unsigned __int128)2 * m;
    if (pos >> 63) return BA_ERANGE;
    if ((m0 && !seed_edges) || ((uintptr_t)seed_edges & 3)) return BA_EINVAL;
    if ((flags & BA_NO_SELF_LOOPS) && m0 == 0 && m > 0) return BA_EINVAL;
    if (edge_begin > m || edge_count > m - edge_begin) return BA_EINVAL;
    if ((edge_count && !edges) || ((uintptr_t)edges & 3)) return BA_EINVAL;
    if (edge_count == 0) return BA_OK;
    ModelArgs a{};
    a.key = make_hash_key(seed);
    a.key64 = seed * kPhi64;
    a.k1 = crc32c_u64(kHostCrcTables.t, 1u, 0);
    a.khi = crc32c_u64(kHostCrcTables.t, 0u, a.key64 & ~(uint64_t)0xFFFFFFFFu);
    a.div = make_divider(d);
    a.P0 = 2 * m0;
    a.n0 = n0;
    a.S = seed_edges;
    a.begin = edge_begin;
    a.count = edge_count;
    a.ntiles = (edge_count + kTile - 1) / kTile;
    a.edges = edges;
    hipStream_t st = (hipStream_t)stream;
    const bool crc = flags & BA_HASH_CRC, noloops = flags & BA_NO_SELF_LOOPS;
    // every position of the graph (not only of the range) below 2^32: 32-bit arithmetic
    const bool narrow = 2 * m0 + 2 * m <= ((uint64_t)1 << 32);
    if (crc) return noloops ? launch_model_width<true, true>(a, narrow, st) : launch_model_width<true, false>(a, narrow, st);
    return noloops ? launch_model_width<false, true>(a, narrow, st) : launch_model_width<false, false>(a, narrow, st);
}

const char *ba_strerror(int status)
{
    switch (status) {
    case BA_OK: return "success";
    case BA_EINVAL: return "invalid argument (null or misaligned buffer, range past n*d, or first_k > n)";
    case BA_ERANGE:
        return "graph too large (2*n*d must fit 64 bits; uint32 output needs n <= 2^32; uint32 degrees need "
               "n*d + d < 2^32)";
    case BA_ENOMEM: return "workspace or static scratch too small for the smallest pass";
    case BA_EDEVICE: return "HIP call failed (see ba_last_hip_error)";
    default: return "unknown status";
    }
}

int ba_last_hip_error(void) { return g_last_hip; }

static void timing_release()
{
    for (auto &r : g_timing.ev) {
        (void)hipEventDestroy(r.e0);
        (void)hipEventDestroy(r.e1);
    }
    g_timing.ev.clear();
}

int ba_kernel_timing(int enable)
{
    timing_release();
    g_timing.on = enable != 0;
    return BA_OK;
}

int ba_kernel_timing_read(double *ms, uint64_t *launches)
{
    if (!ms || !launches) return BA_EINVAL;
    for (int k = 0; k < BA_KT_COUNT; k++) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    int rc = BA_OK;
    for (auto &r : g_timing.ev) {
        float t = 0.0f;
        if (!rc) rc = hip_check(hipEventSynchronize(r.e1));
        if (!rc) rc = hip_check(hipEventElapsedTime(&t, r.e0, r.e1));
        ms[r.kind] += t;
        launches[r.kind]++;
    }
    timing_release();
    return rc;
}

int ba_host_divide(uint32_t d, const uint64_t *x, uint64_t *q, uint64_t count)
{
    if (d == 0 || (count && (!x || !q))) return BA_EINVAL;
    const Divider v = make_divider(d);
    for (uint64_t j = 0; j < count; j++)
        q[j] = (x[j] >> 63) ? x[j] / d : (x[j] >> 31) ? div64(x[j], v) : (uint64_t)div32((uint32_t)x[j], v);
    return BA_OK;
}

}  // extern "C"
