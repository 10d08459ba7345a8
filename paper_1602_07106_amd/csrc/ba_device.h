// ba_device.h -- device arithmetic of the per-edge Barabasi-Albert generator
// for gfx950: the keyed position hash on 32-bit lanes and exact division.
//
// The hash maps a position r >= 1 of the edge array to a pseudorandom
// position in 0..r-1 (paper Section 2, the paragraph on reproducing random
// behaviour):
//
//     h(r) = umul64hi(fmix64(r XOR key), r),   key = seed * 0x9E3779B97F4A7C15
//
// fmix64 is the SplitMix64 output mix (Steele, Lea & Flood, OOPSLA 2014).
// CDNA VALUs are 32 bits wide, so every 64-bit quantity is a (lo, hi) pair of
// 32-bit registers and every product is built from 32x32 multiplies (the
// 32x32+64 -> 64 multiply-add, v_mad_u64_u32, and the 32-bit multiply-high).
// Two variants exist:
//   * narrow: r < 2^32.  The high word of r XOR key is then the high word of
//     the key, so the first xor-shift and half of the first multiply fold into
//     per-key constants, and the final high product needs 2 multiplies;
//   * wide:   any 64-bit r (4 multiplies for the high product).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ba {

constexpr uint64_t kPhi64 = 0x9E3779B97F4A7C15ull;
constexpr uint32_t kC1Lo = 0x1CE4E5B9u, kC1Hi = 0xBF58476Du;  // fmix64 multiplier 1
constexpr uint32_t kC2Lo = 0x133111EBu, kC2Hi = 0x94D049BBu;  // fmix64 multiplier 2

// Per-key constants of the hash (computed once on the host).
struct HashKey {
    uint32_t klo, khi;  // key
    uint32_t c1fold;    // narrow path: (khi ^ (khi >> 30)) * kC1Lo mod 2^32
};

inline HashKey make_hash_key(uint64_t seed)
{
    HashKey k;
    uint64_t key = seed * kPhi64;
    k.klo = (uint32_t)key;
    k.khi = (uint32_t)(key >> 32);
    k.c1fold = (k.khi ^ (k.khi >> 30)) * kC1Lo;
    return k;
}

// low 32 bits of (hi:lo) >> s, 0 < s < 32 (one v_alignbit_b32)
__device__ __forceinline__ uint32_t shr64_lo(uint32_t hi, uint32_t lo, uint32_t s)
{
    return __builtin_amdgcn_alignbit(hi, lo, s);
}

// 32x32 + 64 -> 64 (v_mad_u64_u32)
__device__ __forceinline__ uint64_t mad64(uint32_t a, uint32_t b, uint64_t c)
{
    return (uint64_t)a * (uint64_t)b + c;
}

// a * b + c mod 2^64, and whether it carried out of 64 bits: v_mad_u64_u32
// writes that carry to a lane mask, which the compiler's own lowering of
// the sum does not use (it recomputes it with a compare).
__device__ __forceinline__ uint64_t mad64_carry(uint32_t a, uint32_t b, uint64_t c, bool &carry)
{
    uint64_t d, mask;
    asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(d), "=s"(mask) : "v"(a), "v"(b), "v"(c));
    carry = __builtin_amdgcn_inverse_ballot_w64(mask);
    return d;
}

// fmix64 after its first xor-shift, on (lo, hi) halves: multiply by C1,
// xor-shift 27, multiply by C2, xor-shift 31.  `hi_c1` is the already
// accumulated high-word contribution of the first multiply's hi*C1lo term.
__device__ __forceinline__ void fmix_tail(uint32_t &lo, uint32_t &hi, uint32_t hi_c1)
{
    uint64_t p = mad64(lo, kC1Lo, 0);
    hi = (uint32_t)(p >> 32) + lo * kC1Hi + hi_c1;
    lo = (uint32_t)p;
    lo ^= shr64_lo(hi, lo, 27);
    hi ^= hi >> 27;
    p = mad64(lo, kC2Lo, 0);
    hi = (uint32_t)(p >> 32) + lo * kC2Hi + hi * kC2Lo;
    lo = (uint32_t)p;
    lo ^= shr64_lo(hi, lo, 31);
    hi ^= hi >> 31;
}

// umul64hi(fmix64(r XOR key), b) for r, b < 2^32: a value in 0..b-1.
__device__ __forceinline__ uint32_t hash_narrow_bounded(uint32_t r, uint32_t b, const HashKey &k)
{
    uint32_t lo = r ^ k.klo;                 // high word of r ^ key is khi
    lo ^= shr64_lo(k.khi, lo, 30);           // z ^= z >> 30, low word
    uint32_t hi = 0;                         // high word folded into c1fold
    fmix_tail(lo, hi, k.c1fold);
    // umul64hi(z, b) with b < 2^32: (hi*b + mulhi(lo, b)) >> 32
    uint32_t t = __umulhi(lo, b);
    return (uint32_t)(mad64(hi, b, t) >> 32);
}

// h(r) for r < 2^32.
__device__ __forceinline__ uint32_t hash_narrow(uint32_t r, const HashKey &k) { return hash_narrow_bounded(r, r, k); }

// umul64hi(fmix64(r XOR key), b) for any 64-bit r and b >= 1: a value in
// 0..b-1 (the draw bound b is r itself in the plain model).
__device__ __forceinline__ uint64_t hash_bounded(uint64_t r, uint64_t b, const HashKey &k)
{
    uint32_t lo = (uint32_t)r ^ k.klo, hi = (uint32_t)(r >> 32) ^ k.khi;
    lo ^= shr64_lo(hi, lo, 30);
    hi ^= hi >> 30;
    fmix_tail(lo, hi, hi * kC1Lo);
    // umul64hi((hi:lo), (b1:b0)) = hi*b1 + floor((hi*b0 + t) / 2^32), with
    // t = lo*b1 + mulhi(lo, b0) < 2^64.  hi*b0 + t can carry out of 64 bits;
    // the carry is bit 32 of that quotient, taken from the multiply-add's own
    // carry-out, so all of t is added at once and no 32-bit half has to be
    // copied into a fresh register pair.
    const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
    const uint64_t t = mad64(lo, b1, __umulhi(lo, b0));
    bool carry;
    const uint64_t w = mad64_carry(hi, b0, t, carry);
    return mad64(hi, b1, (w >> 32) | (carry ? (uint64_t)1 << 32 : 0));
}

// h(r) for any 64-bit r >= 1.
__device__ __forceinline__ uint64_t hash_wide(uint64_t r, const HashKey &k) { return hash_bounded(r, r, k); }

// Exact floor(x / d) for a fixed d >= 1 (Granlund & Montgomery, "Division by
// invariant integers using multiplication", PLDI 1994), with l = ceil(log2 d)
// for d not a power of 2 (a power of two is a plain shift by log2 d).  Every
// quotient the kernels take has a numerator one bit narrower than its word
// (edge indices and halved positions: below 2^31 when positions are below
// 2^32, below 2^63 always), so both widths use the round-up method for
// (N-1)-bit numerators, whose multiplier fits N bits:
//      m = floor(2^(N-1+l) / d) + 1 < 2^N,  floor(x / d) = mulhi(m, x) >> (l - 1)
// for x < 2^(N-1).  With e = m*d - 2^(N-1+l) in (0, d],
// x*m / 2^(N-1+l) = x/d + x*e / (d 2^(N-1+l)), and the second term is below
// 2^-l < 1/d, so the floor does not move.
struct Divider {
    uint32_t d;
    uint32_t pow2;   // 1 if d is a power of two
    uint32_t shift;  // log2 d (pow2) or l - 1
    uint32_t m32;    // m for N = 32 (x < 2^31)
    uint64_t m64;    // m for N = 64 (x < 2^63)
};

inline Divider make_divider(uint32_t d)
{
    Divider v{};
    v.d = d;
    if (d == 0) return v;  // never used to divide
    if ((d & (d - 1)) == 0) {
        v.pow2 = 1;
        v.shift = (uint32_t)__builtin_ctz(d);
        return v;
    }
    uint32_t l = 32 - (uint32_t)__builtin_clz(d - 1);  // ceil(log2 d), d >= 3
    v.shift = l - 1;
    v.m32 = (uint32_t)((((uint64_t)1 << (31 + l)) / d) + 1);
    v.m64 = (uint64_t)((((unsigned __int128)1 << (63 + l)) / d) + 1);
    return v;
}

__host__ __device__ __forceinline__ uint32_t mulhi32(uint32_t a, uint32_t b)
{
    return (uint32_t)(((uint64_t)a * b) >> 32);
}

__host__ __device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul64hi(a, b);
#else
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

// x < 2^31
__host__ __device__ __forceinline__ uint32_t div32(uint32_t x, const Divider &v)
{
    if (v.pow2) return x >> v.shift;
    return mulhi32(x, v.m32) >> v.shift;
}

// x < 2^63
__host__ __device__ __forceinline__ uint64_t div64(uint64_t x, const Divider &v)
{
    if (v.pow2) return x >> v.shift;
    return mulhi64(x, v.m64) >> v.shift;
}

}  // namespace ba
