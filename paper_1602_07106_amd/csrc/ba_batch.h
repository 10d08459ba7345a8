// ba_batch.h -- many independent graphs in one persistent launch (gfx950).
//
// A batch is a ragged table of instances (n_j, d_j, seed_j), each with its
// own edge array at its own offset of one output buffer.  The paper hands
// edge-ID batches to processors for load balancing (Section 2, last
// paragraph); here the unit handed out is a tile of consecutive edges of one
// instance, and the tiles of all instances are numbered one after the other
// so that one launch covers the whole table.  Every tile runs the same
// lane-refill chain loop as the single-graph generator, with the instance's
// own key and divider.
//
// Included by ba.hip after the chain loop and the pair stores.
#pragma once

namespace ba {

// One instance of a batch in device memory (64 bytes).
struct BatchInst {
    HashKey key;
    uint32_t narrow;  // 1 when every position 2m-1 of the instance is below 2^32
    Divider div;
    uint64_t m;       // edges
    uint64_t out;     // offset (uint32 elements) of its edge array in the output
    uint64_t pad;
};
static_assert(sizeof(BatchInst) == 64, "BatchInst layout");

struct BatchArgs {
    const BatchInst *inst;  // count entries
    const uint64_t *tile0;  // count + 1 entries: first tile of each instance, tile0[count] = tiles
    uint32_t count;
    uint64_t tiles;
    uint32_t *edges;
};

// Tile sizes a batch layout is prepared for (the launch picks one).
constexpr uint32_t kBatchTiles[3] = {1024, 2048, 4096};

// Wave w of W takes the contiguous tiles [T w / W, T (w+1) / W), so its
// instance index only moves forward; one binary search per wave finds the
// first.  Empty instances (m = 0) own no tile and are skipped.
template <uint32_t TILE, uint32_t WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_gen_batch(BatchArgs a)
{
    __shared__ uint32_t stage_all[WAVES][TILE + kGenCarry];  // a tile, then next-tile results of its tail
    const uint32_t lane = __lane_id();
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    uint32_t *stage = stage_all[wv];
    const uint64_t W = (uint64_t)gridDim.x * WAVES, w = (uint64_t)blockIdx.x * WAVES + wv;
    const uint64_t t0 = a.tiles * w / W, t1 = a.tiles * (w + 1) / W;
    if (t0 >= t1) return;
    uint32_t lo = 0, hi = a.count;  // tile0[lo] <= t0 < tile0[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (a.tile0[mid] <= t0) lo = mid; else hi = mid;
    }
    uint32_t j = lo;
    uint64_t tcur = a.tile0[j], tnext = a.tile0[j + 1];
    BatchInst I = a.inst[j];
    // chains carried from a tile into the next tile of the same instance
    // (none across instances: an instance's last tile claims nothing)
    ChainCarry<uint32_t> c32;
    ChainCarry<uint64_t> c64;
    uint32_t coff = 0;
    for (uint64_t t = t0; t < t1; t++) {
        while (t >= tnext) {
            j++;
            tcur = tnext;
            tnext = a.tile0[j + 1];
            I = a.inst[j];
        }
        const uint64_t off = (t - tcur) * TILE;
        const uint32_t tn = tile_len(TILE, I.m - off);
        const uint32_t tn2 = t + 1 < t1 && t + 1 < tnext ? tile_len(TILE, I.m - off - TILE) : 0u;
        if (I.narrow)
            chain_tile_next<kGenCarry>(stage, tn, tn2, lane, (uint32_t)(2 * off + 1),
                                       [&](uint32_t r) { return hash_narrow(r, I.key); },
                                       [](uint32_t r) { return r; }, c32, coff);  // the final position; the flush divides
        else
            chain_tile_next<kGenCarry>(stage, tn, tn2, lane, 2 * off + 1,
                                       [&](uint64_t r) { return hash_wide(r, I.key); },
                                       [&](uint64_t r) { return (uint32_t)div64(r >> 1, I.div); }, c64, coff);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        uint32_t *out = a.edges + I.out + 2 * off;
        const bool vec16 = (((uintptr_t)(a.edges + I.out)) & 15) == 0;  // off is a multiple of 2 edges
        // The instance's width and divider kind, and whether the tile is full
        // and 16-byte aligned, are uniform per tile: they select a loop
        // instead of being tested in it.
        auto flush = [&](auto narrow_t, auto pow2_t, auto full_t) {
            constexpr bool NW = decltype(narrow_t)::value, P = decltype(pow2_t)::value,
                           F = decltype(full_t)::value;
            auto pair = [&](uint32_t jj, uint32_t &u0, uint32_t &u1, uint32_t &v0, uint32_t &v1) {
                const uint2 s = *reinterpret_cast<const uint2 *>(stage + jj);
                if constexpr (NW) {
                    const uint32_t i0 = (uint32_t)off + jj;
                    u0 = fdiv32<P>(i0, I.div);
                    u1 = fdiv32<P>(i0 + 1, I.div);
                    v0 = fdiv32<P>(s.x >> 1, I.div);
                    v1 = fdiv32<P>(s.y >> 1, I.div);
                } else {
                    const uint64_t i0 = off + jj;
                    u0 = (uint32_t)fdiv64<P>(i0, I.div);
                    u1 = (uint32_t)fdiv64<P>(i0 + 1, I.div);
                    v0 = s.x;
                    v1 = s.y;
                }
            };
            if constexpr (F) {
                // full, aligned tile: TILE / 128 pairs per lane (a uniform trip count)
#pragma unroll 1
                for (uint32_t t = 0; t < TILE / (2 * kWave); t++) {
                    const uint32_t jj = 2 * lane + t * (2 * kWave);
                    uint32_t u0, u1, v0, v1;
                    pair(jj, u0, u1, v0, v1);
                    store_edges16<false>(out + 2 * jj, u0, v0, u1, v1);
                }
            } else {
                for (uint32_t jj = 2 * lane; jj < tn; jj += 2 * kWave) {
                    uint32_t u0, u1, v0, v1;
                    pair(jj, u0, u1, v0, v1);
                    if (vec16)
                        store_pair<true, false>(out, jj, tn, u0, v0, u1, v1);
                    else
                        store_pair<false, false>(out, jj, tn, u0, v0, u1, v1);
                }
            }
        };
        using T = std::true_type;
        using Fa = std::false_type;
        const bool full = tn == TILE && vec16;
        if (I.narrow) {
            if (I.div.pow2) {
                if (full) flush(T{}, T{}, T{}); else flush(T{}, T{}, Fa{});
            } else {
                if (full) flush(T{}, Fa{}, T{}); else flush(T{}, Fa{}, Fa{});
            }
        } else {
            // 64-bit positions (large instances only): the general loop
            if (I.div.pow2) flush(Fa{}, T{}, Fa{}); else flush(Fa{}, Fa{}, Fa{});
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

}  // namespace ba
