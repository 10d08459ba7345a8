// ba_model.h -- the generalized model on gfx950: a seed graph in front of
// the edge array, self-loop-free draws, and the paper's CRC-based hash.
//
// Paper Section "Generalizations": a seed graph of n0 nodes and m0 edges
// takes positions 0..2*m0-1 of E; new edge i sits at 2*m0 + 2i, its first
// endpoint is n0 + floor(i/d), and its chain stops at the first position
// that is either a seed position (its node is read from the seed graph) or
// even (node n0 + floor((r - 2*m0) / (2d))).  Self-loops are avoided by
// drawing below the first position of the edge's own node instead of below
// r itself; the hashed word stays the edge's own position, so the d edges
// of a node draw independently.
//
// Hashes of position r into 0..b-1 (key = seed * phi64):
//   fmix:  umul64hi(fmix64(r XOR key), b)
//   crc:   ((crc32c(0, z) << 32) + crc32c(1, z)) mod b,  z = r XOR key
// crc32c(c, z) is the CRC-32C register update over the 8 bytes of z (the
// SSE4.2 crc32 instruction of the paper's hash_crc).  CRC is affine in the
// register, so crc32c(1, z) = crc32c(0, z) XOR crc32c(1, 0): one table
// evaluation serves both halves.  The update runs slicing-by-8 from tables
// held in LDS (8 KiB per block).  With positions below 2^32 the high half of
// z is the key's, whose share of crc32c(0, z) is computed once on the host,
// so only the four tables of the low bytes are read (4 KiB).
//
// Included by ba.hip after the chain loop.
#pragma once

#include <type_traits>

namespace ba {

constexpr uint32_t kCrcPoly = 0x82F63B78u;  // CRC-32C, reflected

struct CrcTables {
    uint32_t t[8][256];  // t[k][b]: register after byte b followed by k zero bytes
};

constexpr CrcTables make_crc_tables()
{
    CrcTables T{};
    for (uint32_t b = 0; b < 256; b++) {
        uint32_t c = b;
        for (int k = 0; k < 8; k++) c = (c & 1u) ? (c >> 1) ^ kCrcPoly : (c >> 1);
        T.t[0][b] = c;
    }
    for (int k = 1; k < 8; k++)
        for (uint32_t b = 0; b < 256; b++) T.t[k][b] = (T.t[k - 1][b] >> 8) ^ T.t[0][T.t[k - 1][b] & 0xFFu];
    return T;
}

__constant__ CrcTables kCrcTables = make_crc_tables();

// Register update over the 8 bytes of x (least significant first) from c.
template <class Tab>
__host__ __device__ __forceinline__ uint32_t crc32c_u64(const Tab &t, uint32_t c, uint64_t x)
{
    const uint64_t v = x ^ (uint64_t)c;
    return t[7][v & 0xFF] ^ t[6][(v >> 8) & 0xFF] ^ t[5][(v >> 16) & 0xFF] ^ t[4][(v >> 24) & 0xFF] ^
           t[3][(v >> 32) & 0xFF] ^ t[2][(v >> 40) & 0xFF] ^ t[1][(v >> 48) & 0xFF] ^ t[0][v >> 56];
}

// crc32c(0, x) for x whose high word is fixed: the update from register 0
// is linear over GF(2) in x, so it is the update of the low word alone
// (the tables of its four bytes, t[7]..t[4], passed as lo4[3]..lo4[0])
// XOR hi_part, the update of the high word alone (high << 32).
template <class Tab>
__host__ __device__ __forceinline__ uint32_t crc32c0_low_word(const Tab &lo4, uint32_t lo, uint32_t hi_part)
{
    return lo4[3][lo & 0xFF] ^ lo4[2][(lo >> 8) & 0xFF] ^ lo4[1][(lo >> 16) & 0xFF] ^ lo4[0][lo >> 24] ^ hi_part;
}

// x mod b for 1 <= b < 2^32, exact; there is no 64-by-32-bit division
// instruction.  Two steps, each with a quotient estimate in double precision:
// r1 = hi mod b, then (r1 * 2^32 + lo) mod b, whose quotient is below 2^32.
// The reciprocal seed (float(b) rounded, then a 1-ulp reciprocal) is within
// 1.5 * 2^-23 of 1/b; one Newton step squares that to below 2^-44, so num * y
// is within 2^-12 of num / b < 2^32.  The second step forms num * y as
// r1 * (2^32 y) + lo * y (one rounded product, one rounded fma: 2^-20 more).
// The truncated (and clamped) estimate is therefore q - 1, q or q + 1, so
// num - q_est * b lies in [-b, 2b) and one signed correction, taken by
// selects, gives the remainder.  The host build perturbs its (correctly
// rounded) seed by 2^-22, a larger error than the device's, so a host
// self-test covers the device's error bound.
__host__ __device__ __forceinline__ uint32_t mod_u64_u32(uint64_t x, uint32_t b)
{
    const double bd = (double)b;
#if defined(__HIP_DEVICE_COMPILE__)
    double y = (double)__builtin_amdgcn_rcpf((float)b);
#else
    double y = (double)(1.0f / (float)b) * ((b & 1u) ? 1.0 + 0x1p-22 : 1.0 - 0x1p-22);
#endif
    y = fma(fma(-bd, y, 1.0), y, y);
    auto fix = [&](uint64_t num, double qd) -> uint32_t {  // num < b * 2^32, qd >= 0
        const uint32_t q = (uint32_t)fmin(qd, 4294967295.0);
        const int64_t r = (int64_t)(num - (uint64_t)q * b);  // in [-b, 2b)
        const uint32_t rl = (uint32_t)r;
        return r < 0 ? rl + b : (r >= (int64_t)b ? rl - b : rl);
    };
    const uint32_t hi = (uint32_t)(x >> 32), lo = (uint32_t)x;
    const uint32_t r1 = fix(hi, (double)hi * y);
    return fix(((uint64_t)r1 << 32) | lo, fma((double)r1, y * 4294967296.0, (double)lo * y));
}

enum : uint32_t { kModelNoLoops = 1, kModelCrc = 2 };

struct ModelArgs {
    HashKey key;
    uint32_t k1;       // crc32c(1, 0): the register-1 offset of the crc hash
    uint32_t khi;      // crc32c(0, (key64 >> 32) << 32): with positions below 2^32 the
                       // hashed word's high half is key64's, a constant share
    Divider div;
    uint64_t key64;    // seed * phi64 (the crc hash XORs it into r)
    uint64_t P0;       // 2*m0: first position of the new edges
    uint64_t n0;
    const uint32_t *S; // the seed graph's 2*m0 node IDs
    uint64_t begin, count, ntiles;
    uint32_t *edges;
};

// NARROW: every position of the launch (2*m0 + 2*(n-n0)*d) is below 2^32,
// so positions, bounds and the fmix high product stay 32-bit.
// Block size: the CRC variants hold their tables in LDS per block (4 KiB
// on 32-bit positions, 8 KiB on 64-bit), so they run 8 waves a block to
// share them: 40 KiB blocks (stages with their tail room, and the tables)
// still fill a CU's 160 KiB at 8 waves per SIMD on 32-bit positions, where
// 4-wave blocks stop at 6.  The others run the generator's 4 waves.
template <bool CRC>
constexpr int kModelBlock = CRC ? 512 : kGenBlock;
template <bool CRC>
constexpr int kModelWaves = kModelBlock<CRC> / kWave;
constexpr uint32_t kModelCarry = 128;  // next-tile edges a wave's chain tail may claim

template <bool CRC, bool NOLOOPS, bool NARROW>
__global__ __launch_bounds__(kModelBlock<CRC>) void k_gen_model(ModelArgs a)
{
    constexpr int kBlock = kModelBlock<CRC>, kWaves = kModelWaves<CRC>;
    using R = typename std::conditional<NARROW, uint32_t, uint64_t>::type;
    __shared__ uint32_t stage_all[kWaves][kTile + kModelCarry];  // a tile, then next-tile results of its tail
    // CRC tables in LDS: all eight for 64-bit positions; with 32-bit
    // positions only the four of the low word's bytes (t[4..7])
    constexpr int kCrcRows = CRC ? (NARROW ? 4 : 8) : 1;
    __shared__ uint32_t crc_t[kCrcRows][256];
    if constexpr (CRC) {
        for (uint32_t j = threadIdx.x; j < kCrcRows * 256; j += kBlock)
            crc_t[j / 256][j % 256] = kCrcTables.t[8 - kCrcRows + j / 256][j % 256];
        __syncthreads();
    }
    const uint32_t lane = __lane_id();
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform: scalar loops
    uint32_t *stage = stage_all[wv];
    // wave w takes tiles t0 .. t1-1, consecutive in edge IDs, so the chain
    // tail of one tile runs straight into the next
    const uint64_t nw = (uint64_t)gridDim.x * kWaves, w = (uint64_t)blockIdx.x * kWaves + wv;
    const uint64_t per = a.ntiles / nw, extra = a.ntiles % nw;
    const uint64_t t0 = w * per + min(w, extra), t1 = t0 + per + (w < extra ? 1u : 0u);
    ChainCarry<R> cc;
    uint32_t coff = 0;
    const R P0 = (R)a.P0;
    const uint32_t stop_min = 0x80000000u - (uint32_t)(a.P0 >> 1);  // 32-bit positions only
    // 16-byte stores when the output is 16-byte aligned (tiles start at even edges)
    const bool vec16 = (((uintptr_t)a.edges) & 15) == 0;

    // One tile with the divider's kind fixed at compile time: the kind is
    // uniform, so it selects a copy of the whole tile loop body instead of
    // being tested at every division.
    auto run_tile = [&](auto pow2, uint64_t tile) {
        constexpr bool P = decltype(pow2)::value;
        // floor(x / d) in the width of the launch
        auto divd = [&](R x) -> R {
            if constexpr (NARROW) return fdiv32<P>(x, a.div);
            else return fdiv64<P>(x, a.div);
        };
        // draw bound of the edge whose second endpoint sits at odd r >= P0
        auto bound = [&](R r) -> R {
            if constexpr (NOLOOPS) return P0 + 2 * (R)a.div.d * divd((r - P0) >> 1);  // (r-P0-1)/2 = edge index
            else return r;
        };
        auto hash = [&](R r) -> R {
            const R b = bound(r);
            if constexpr (CRC) {
                uint32_t c0;
                if constexpr (NARROW)
                    c0 = crc32c0_low_word(crc_t, (uint32_t)r ^ (uint32_t)a.key64, a.khi);
                else
                    c0 = crc32c_u64(crc_t, 0u, (uint64_t)r ^ a.key64);
                const uint64_t h = ((uint64_t)c0 << 32) + (uint64_t)(c0 ^ a.k1);
                if constexpr (NARROW) return mod_u64_u32(h, b);
                else return h % b;
            } else if constexpr (NARROW) {
                return hash_narrow_bounded(r, b, a.key);
            } else {
                return hash_bounded(r, b, a.key);
            }
        };
        // final position: even, or a seed position (r < P0).  On 32-bit
        // positions, with P0 even, that is one unsigned compare: w = (r XOR 1)
        // - P0 has w's low bit set iff r is even, and rotating it right by one
        // maps the even r to [2^31, 2^32), the odd r >= P0 to [0, 2^31 - P0/2)
        // and the odd r < P0 (w wrapped) to [2^31 - P0/2, 2^31).
        auto stop = [&](R r) {
            if constexpr (NARROW) {
                const uint32_t w = (r ^ 1u) - P0;
                return ((w >> 1) | (w << 31)) >= stop_min;
            } else {
                return r < P0 || !((uint32_t)r & 1u);
            }
        };
        auto node = [&](R r) -> uint32_t {
            return r < P0 ? a.S[r] : (uint32_t)(a.n0 + divd((r - P0) >> 1));
        };

        const uint64_t off = tile * kTile;
        const uint32_t tn = tile_len(kTile, a.count - off);
        const uint64_t ibase = a.begin + off;
        const uint32_t tn2 = tile + 1 < t1 ? tile_len(kTile, a.count - off - kTile) : 0u;
        // 32-bit positions: the stage holds the final position r and the
        // flush maps it to its node, with every lane busy; 64-bit: the node.
        if constexpr (NARROW)
            chain_tile_next_until<kModelCarry>(stage, tn, tn2, lane, (R)(a.P0 + 2 * ibase + 1), hash, stop,
                                               [](R r) { return r; }, cc, coff);
        else
            chain_tile_next_until<kModelCarry>(stage, tn, tn2, lane, (R)(a.P0 + 2 * ibase + 1), hash, stop, node,
                                               cc, coff);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        uint32_t *out = a.edges + 2 * off;
        auto pair_at = [&](uint32_t j, uint32_t &u0, uint32_t &v0, uint32_t &u1, uint32_t &v1) {
            const uint2 s = *reinterpret_cast<const uint2 *>(stage + j);
            u0 = (uint32_t)(a.n0 + divd((R)(ibase + j)));
            u1 = (uint32_t)(a.n0 + divd((R)(ibase + j + 1)));
            if constexpr (NARROW) {
                v0 = node(s.x);
                v1 = node(s.y);
            } else {
                v0 = s.x;
                v1 = s.y;
            }
        };
        if (tn == kTile && vec16) {
            // full tile: kTile / 128 pairs per lane, no partial-pair checks
#pragma unroll 2
            for (uint32_t t = 0; t < kTile / (2 * kWave); t++) {
                const uint32_t j = 2 * lane + t * (2 * kWave);
                uint32_t u0, v0, u1, v1;
                pair_at(j, u0, v0, u1, v1);
                store_edges16(out + 2 * j, u0, v0, u1, v1);
            }
        } else {
            for (uint32_t j = 2 * lane; j < tn; j += 2 * kWave) {
                uint32_t u0, v0, u1, v1;
                pair_at(j, u0, v0, u1, v1);
                if (vec16)
                    store_pair<true>(out, j, tn, u0, v0, u1, v1);
                else
                    store_pair<false>(out, j, tn, u0, v0, u1, v1);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };

    for (uint64_t tile = t0; tile < t1; tile++) {
        if (a.div.pow2)
            run_tile(std::true_type{}, tile);
        else
            run_tile(std::false_type{}, tile);
    }
}

}  // namespace ba

// Host self-test of mod_u64_u32 (the same algorithm the CRC kernels run,
// with the reciprocal seed computed on the host): r[j] = x[j] mod b[j].
extern "C" int ba_host_mod64(const uint64_t *x, const uint32_t *b, uint32_t *r, uint64_t count)
{
    if (count && (!x || !b || !r)) return BA_EINVAL;
    for (uint64_t j = 0; j < count; j++)
        if (b[j] == 0) return BA_EINVAL;
    for (uint64_t j = 0; j < count; j++) r[j] = ba::mod_u64_u32(x[j], b[j]);
    return BA_OK;
}
