// ba_genpart.h -- the stored generator with the degree pipeline's partition
// fused in, for graphs of at most 2^26 nodes (1024 sub-buckets of 65536
// nodes; their histograms are k_deg_hist16).
//
// One block of 16 waves per compute unit takes chunks of kFChunk consecutive
// edge IDs.  Each wave runs the chain loop (paper Section 2, figure
// generateEdge) over its kFTile edges into its part of the block's LDS stage,
// writes the edge pairs as the plain generator does, and keeps the second
// endpoints of its edges in registers (20 a lane).  The block then
// counting-sorts the chunk's second endpoints by sub-bucket in the same LDS
// (the stage is free again) and appends each sub-bucket's run of 16-bit local
// indices to the block's own region for it, exactly the layout k_deg_part
// builds from the target list; the totals, scan and histogram kernels of
// ba_degree.h then finish the degrees.  No target list is written or read.
// Each wave writes out the sorted entries that sit in its own stage part and
// goes on to its next chunk without waiting for the block, and its chain
// tail runs into the wave's tile of that chunk (chain_tile_carry).
//
// Chunks go to blocks round-robin (block b takes chunks b, b+P, ...), so
// every block sees second endpoints from the whole edge range, as the region
// capacities (sized for the mean) assume.  A block owning one contiguous
// range would not: the targets of early edges all fall in the lowest
// sub-buckets, whose regions then overflow into global atomics.
//
// Run length is what matters for the sort: a chunk's 20480 second endpoints
// over 1024 sub-buckets leave runs of about 20 entries (40 bytes) per region
// and chunk; shorter runs (smaller chunks, or 32768-node sub-buckets) cost
// more in scattered stores than the overlap of two smaller blocks per
// compute unit gains.
#pragma once

namespace ba {

constexpr uint32_t kFWaves = 16;
constexpr uint32_t kFBlock = kFWaves * kWave;   // 1024 threads, one block per compute unit (121 KiB of LDS)
constexpr uint32_t kFTile = 1280;               // edges per wave per chunk (a multiple of 128)
constexpr uint32_t kFChunk = kFWaves * kFTile;  // 20480 edges per block chunk
constexpr uint32_t kFPer = kFTile / kWave;      // second endpoints per thread
constexpr uint32_t kFBins = kWin16 / kFBlock;   // sub-buckets per thread in the scan
constexpr uint32_t kFCarry = 256;               // next-tile edges a wave's chain tail may claim
static_assert(kFTile % (2 * kWave) == 0 && kFPer % 2 == 0, "pair flush");
static_assert(kFChunk < 65536, "16-bit ranks");
static_assert(kWin16 % kFBlock == 0, "scan");

struct GenPartArgs {
    GenArgs g;         // chain loop and edge output: edges g.begin .. g.begin+g.count-1
    DegArgs p;         // partition layout: one window (g0 = 0), P = the grid
    uint64_t nchunks;  // ceil(g.count / kFChunk)
};

template <bool NARROW, bool POW2, bool VEC16>
__global__ __launch_bounds__(kFBlock) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_gen_part(GenPartArgs a)
{
    constexpr uint32_t kOut = kWin16 << kS16;  // no entry (past the launch's edges): lane-private dummy bins
    __shared__ uint32_t stage[kFChunk];     // chain results, then the chunk's second endpoints in sorted order
    __shared__ uint32_t cnt[kWin16 + 64];     // per chunk: counts, then run starts
    __shared__ uint32_t wpos[kWin16];         // next slot of this block's region per sub-bucket (<= wend)
    __shared__ uint32_t wend[kWin16];         // end of this block's region per sub-bucket
    __shared__ uint32_t dlx[kWin16];          // per chunk: region slot of sorted entry x is dlx[b] + x
    __shared__ uint32_t scan_sh[16];
    __shared__ uint32_t any_over;           // per chunk: some region of this block is full
    __shared__ uint32_t side_all[kFWaves][kFCarry];  // per wave: next-tile results of the chain tail
    const DegArgs &q = a.p;
    const uint32_t nb = q.p.NBsub;  // <= kWin16
    const uint32_t blk = blockIdx.x, P = gridDim.x;
    for (uint32_t b = threadIdx.x; b < kWin16; b += kFBlock) {
        const uint32_t cp = b < nb ? ws_rcap(q)[b] : 0u;
        const uint32_t base = b < nb ? (uint32_t)(ws_off(q)[b] + (uint64_t)blk * cp) : 0u;
        wpos[b] = base;
        wend[b] = base + cp;
    }
    uint16_t *L = ws_L(q);
    const uint32_t lane = __lane_id();
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform: scalar tile bases
    uint32_t *st_w = stage + wv * kFTile;
    uint32_t *side_w = side_all[wv];
    using R = std::conditional_t<NARROW, uint32_t, uint64_t>;
    ChainCarry<R> cc;
    // this wave's tile of chunk ch: first edge offset and size
    auto tile_of = [&](uint64_t ch, uint64_t &woff) -> uint32_t {
        woff = ch * kFChunk + (uint64_t)wv * kFTile;
        return ch < a.nchunks && woff < a.g.count ? tile_len(kFTile, a.g.count - woff) : 0u;
    };

    for (uint64_t ch = blk; ch < a.nchunks; ch += P) {
        // ---- this wave's edges of the chunk: chain loop, edge pairs out
        uint64_t woff, woff2;
        const uint32_t tn = tile_of(ch, woff);
        const uint32_t tn2 = tile_of(ch + P, woff2);  // the wave's tile of its next chunk (its tail runs into it)
        const uint64_t ibase = a.g.begin + woff;
        const R rbase = (R)(2 * ibase + 1), rbase2 = (R)(2 * (a.g.begin + woff2) + 1);
        uint32_t v[kFPer];
#pragma unroll
        for (uint32_t t = 0; t < kFPer; t++) v[t] = kOut;
        if (tn) {
            if constexpr (NARROW)
                chain_tile_carry<kFCarry>(st_w, side_w, tn, lane, rbase, tn2, rbase2,
                                          [&](uint32_t r) { return hash_narrow(r, a.g.key); },
                                          [](uint32_t r) { return r; }, cc);
            else
                chain_tile_carry<kFCarry>(st_w, side_w, tn, lane, rbase, tn2, rbase2,
                                          [&](uint64_t r) { return hash_wide(r, a.g.key); },
                                          [&](uint64_t r) { return (uint32_t)fdiv64<POW2>(r >> 1, a.g.div); }, cc);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            uint32_t *out = a.g.edges + 2 * woff;
            if (tn == kFTile) {
#pragma unroll
                for (uint32_t t = 0; t < kFPer / 2; t++) {
                    const uint32_t j = 2 * lane + t * (2 * kWave);
                    uint32_t u0, u1, v0, v1;
                    flush_pair<NARROW, POW2>(a.g, st_w, ibase, j, u0, u1, v0, v1);
                    if constexpr (VEC16)
                        store_edges16(out + 2 * j, u0, v0, u1, v1);
                    else
                        store_pair<false>(out, j, kFTile, u0, v0, u1, v1);
                    v[2 * t] = v0;
                    v[2 * t + 1] = v1;
                }
            } else {
#pragma unroll
                for (uint32_t t = 0; t < kFPer / 2; t++) {
                    const uint32_t j = 2 * lane + t * (2 * kWave);
                    if (j < tn) {
                        uint32_t u0, u1, v0, v1;
                        flush_pair<NARROW, POW2>(a.g, st_w, ibase, j, u0, u1, v0, v1);
                        store_pair<VEC16>(out, j, tn, u0, v0, u1, v1);
                        v[2 * t] = v0;
                        if (j + 1 < tn) v[2 * t + 1] = v1;
                    }
                }
            }
        }

        // ---- the chunk's second endpoints: counting sort by sub-bucket
        for (uint32_t b = threadIdx.x; b < kWin16 + 64; b += kFBlock) cnt[b] = 0;
        lds_barrier();  // also: every wave has read its stage part
        // counts; each entry keeps its rank in its bin, two 16-bit ranks a register
        uint32_t rk[kFPer / 2];
#pragma unroll
        for (uint32_t t = 0; t < kFPer; t += 2) {
            const uint32_t b0 = (v[t] >> kS16) + (v[t] == kOut ? lane : 0u);
            const uint32_t b1 = (v[t + 1] >> kS16) + (v[t + 1] == kOut ? lane : 0u);
            const uint32_t r0 = atomicAdd(&cnt[b0], 1u);
            const uint32_t r1 = atomicAdd(&cnt[b1], 1u);
            rk[t / 2] = (r0 & 0xFFFFu) | (r1 << 16);
        }
        if (threadIdx.x == 0) any_over = 0;
        lds_barrier();
        // run starts (exclusive scan, kFBins sub-buckets a thread) and region slots
        uint32_t c[kFBins], sum = 0;
#pragma unroll
        for (uint32_t k = 0; k < kFBins; k++) {
            c[k] = cnt[kFBins * threadIdx.x + k];
            sum += c[k];
        }
        uint32_t total;
        uint32_t s = block_exclusive_scan<uint32_t>(sum, scan_sh, &total);
#pragma unroll
        for (uint32_t k = 0; k < kFBins; k++) {
            const uint32_t b = kFBins * threadIdx.x + k;
            if (c[k]) {
                const uint32_t w = wpos[b], e = wend[b];
                const uint32_t room = e - w;
                dlx[b] = w - s;  // mod 2^32: dlx + x is the slot for x in [s, s + c)
                wpos[b] = c[k] < room ? w + c[k] : e;
                if (c[k] > room) any_over = 1;
            }
            cnt[b] = s;
            s += c[k];
        }
        lds_barrier();
        // scatter into sorted order: run start + rank (cnt[kWin16] for no entry, never stored)
#pragma unroll
        for (uint32_t t0 = 0; t0 < kFPer; t0 += kFPer / 2) {
            uint32_t sb[kFPer / 2];
#pragma unroll
            for (uint32_t j = 0; j < kFPer / 2; j++) sb[j] = cnt[v[t0 + j] >> kS16];
#pragma unroll
            for (uint32_t j = 0; j < kFPer / 2; j++) {
                const uint32_t t = t0 + j;
                if (v[t] != kOut) stage[sb[j] + ((rk[t / 2] >> (16 * (t & 1))) & 0xFFFFu)] = v[t];
            }
        }
        lds_barrier();
        // Sorted runs out.  Wave w takes the sorted entries of its own stage
        // part, consecutive lanes consecutive entries, so a store covers a
        // few runs of contiguous region slots.  It then goes straight on to
        // its next chain loop, which rewrites only that part: no block
        // barrier ends the chunk (the next chunk's sort rewrites dlx, wpos
        // and any_over only behind its first barrier, when every wave is done
        // here).
        const bool over = any_over != 0;
        const uint32_t x0 = wv * kFTile;
        if (!over && x0 + kFTile <= total) {  // no region full, a whole part (the normal case)
            constexpr uint32_t G = 2;  // entries a lane loads before it stores (more gains nothing)
            static_assert(kFPer % G == 0, "whole groups");
#pragma unroll 1
            for (uint32_t t0 = 0; t0 < kFPer; t0 += G) {
                uint32_t w[G], o[G];
#pragma unroll
                for (uint32_t u = 0; u < G; u++) w[u] = st_w[(t0 + u) * kWave + lane];
#pragma unroll
                for (uint32_t u = 0; u < G; u++) o[u] = dlx[w[u] >> kS16];
#pragma unroll
                for (uint32_t u = 0; u < G; u++)
                    L[o[u] + x0 + (t0 + u) * kWave + lane] = (uint16_t)(w[u] & (kSub16 - 1));
            }
        } else if (x0 < total) {
            if (over && wv == 0 && lane == 0) *ws_flag(q) = 1;  // deg takes atomics before the histogram
            for (uint32_t t = 0; t < kFPer; t++) {
                const uint32_t x = x0 + t * kWave + lane;
                if (x < total) {
                    const uint32_t w = stage[x];
                    const uint32_t slot = dlx[w >> kS16] + x;
                    if (!over || slot < wend[w >> kS16])
                        L[slot] = (uint16_t)(w & (kSub16 - 1));
                    else
                        deg_atomic_add(q.deg, w, 1u);
                }
            }
        }
    }
    // this block's fill per sub-bucket (k_deg_tot caps it at the region size)
    uint32_t *gfill = ws_fill(q) + (uint64_t)blk * nb;
    for (uint32_t b = threadIdx.x; b < nb; b += kFBlock)
        gfill[b] = wpos[b] - (uint32_t)(ws_off(q)[b] + (uint64_t)blk * ws_rcap(q)[b]);
}

}  // namespace ba
