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
// held in LDS (8 KiB per block).
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

// x mod b for 1 <= b < 2^32, exact; there is no 64-by-32-bit division
// instruction.  Two steps, each with a quotient estimate in double precision:
// r1 = hi mod b, then (r1 * 2^32 + lo) mod b, whose quotient is below 2^32.
// With y within 2^-48 of 1/b (a 2^-23 seed refined twice by Newton's
// iteration), the estimate num * y is within 2^-17 of num / b: num converts
// exactly below 2^53, and above it b > num / 2^32 > 2^21 bounds the
// conversion's share of the error by 2^-21.  The truncated (and clamped)
// estimate is therefore q - 1, q or q + 1, and one signed correction of
// num - q_est * b gives the remainder.
__host__ __device__ __forceinline__ uint32_t mod_u64_u32(uint64_t x, uint32_t b)
{
    const double bd = (double)b;
#if defined(__HIP_DEVICE_COMPILE__)
    double y = (double)__builtin_amdgcn_rcpf((float)b);
#else
    double y = (double)(1.0f / (float)b);
#endif
    y = fma(fma(-bd, y, 1.0), y, y);
    y = fma(fma(-bd, y, 1.0), y, y);
    auto reduce = [&](uint64_t num) -> uint32_t {  // num < b * 2^32
        const double qd = (double)num * y;
        const uint32_t q = qd >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)qd;
        int64_t r = (int64_t)(num - (uint64_t)q * b);
        if (r < 0)
            r += b;
        else if (r >= (int64_t)b)
            r -= b;
        return (uint32_t)r;
    };
    const uint32_t r1 = reduce(x >> 32);
    return reduce(((uint64_t)r1 << 32) | (uint32_t)x);
}

enum : uint32_t { kModelNoLoops = 1, kModelCrc = 2 };

struct ModelArgs {
    HashKey key;
    uint32_t k1;       // crc32c(1, 0): the register-1 offset of the crc hash
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
template <bool CRC, bool NOLOOPS, bool NARROW>
__global__ __launch_bounds__(kGenBlock) void k_gen_model(ModelArgs a)
{
    using R = typename std::conditional<NARROW, uint32_t, uint64_t>::type;
    __shared__ uint32_t stage_all[kGenWaves][kTile];
    __shared__ uint32_t crc_t[CRC ? 8 : 1][256];
    if constexpr (CRC) {
        for (uint32_t j = threadIdx.x; j < 8 * 256; j += kGenBlock) crc_t[j / 256][j % 256] = kCrcTables.t[j / 256][j % 256];
        __syncthreads();
    }
    const uint32_t lane = __lane_id();
    const uint32_t wv = threadIdx.x / kWave;
    uint32_t *stage = stage_all[wv];
    const uint64_t wstride = (uint64_t)gridDim.x * kGenWaves;
    const R P0 = (R)a.P0;

    // floor(x / d) in the width of the launch
    auto divd = [&](R x) -> R {
        if constexpr (NARROW) return div32(x, a.div);
        else return div64(x, a.div);
    };
    // draw bound of the edge whose second endpoint sits at odd r >= P0
    auto bound = [&](R r) -> R {
        if constexpr (NOLOOPS) return P0 + 2 * (R)a.div.d * divd((r - P0) >> 1);  // (r-P0-1)/2 = edge index
        else return r;
    };
    auto hash = [&](R r) -> R {
        const R b = bound(r);
        if constexpr (CRC) {
            const uint32_t c0 = crc32c_u64(crc_t, 0u, (uint64_t)r ^ a.key64);
            const uint64_t h = ((uint64_t)c0 << 32) + (uint64_t)(c0 ^ a.k1);
            if constexpr (NARROW) return mod_u64_u32(h, b);
            else return h % b;
        } else if constexpr (NARROW) {
            return hash_narrow_bounded(r, b, a.key);
        } else {
            return hash_bounded(r, b, a.key);
        }
    };
    auto stop = [&](R r) { return r < P0 || !((uint32_t)r & 1u); };
    auto node = [&](R r) -> uint32_t { return r < P0 ? a.S[r] : (uint32_t)(a.n0 + divd((r - P0) >> 1)); };

    for (uint64_t tile = (uint64_t)blockIdx.x * kGenWaves + wv; tile < a.ntiles; tile += wstride) {
        const uint64_t off = tile * kTile;
        const uint32_t tn = (uint32_t)min((uint64_t)kTile, a.count - off);
        const uint64_t ibase = a.begin + off;
        chain_tile_until(stage, tn, lane, (R)(a.P0 + 2 * ibase + 1), hash, stop, node);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        uint32_t *out = a.edges + 2 * off;
        const bool vec16 = (((uintptr_t)out) & 15) == 0;
        for (uint32_t j = 2 * lane; j < tn; j += 2 * kWave) {
            const uint2 s = *reinterpret_cast<const uint2 *>(stage + j);
            const uint32_t u0 = (uint32_t)(a.n0 + divd((R)(ibase + j)));
            const uint32_t u1 = (uint32_t)(a.n0 + divd((R)(ibase + j + 1)));
            if (vec16)
                store_pair<true>(out, j, tn, u0, s.x, u1, s.y);
            else
                store_pair<false>(out, j, tn, u0, s.x, u1, s.y);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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
