// ba_degree.h -- full degree array of a generated graph on gfx950.
//
// deg[v] counts the positions of the edge array holding v (paper Section 2:
// E[2i] = floor(i/d) gives every node exactly d first endpoints; the rest are
// the second endpoints v_i).  Second endpoints land on random nodes, heavily
// skewed towards low IDs (E[deg v] ~ d*sqrt(n/v)).  Per-edge global atomics
// on gfx950 run at a fixed ~2.7e10 cache-line requests/s whatever the
// footprint, about 15x slower than generating the edges, so the counts go
// through a radix partition in HBM and finish as LDS histograms:
//
//   V  (in the generator): the tile flush also writes the second endpoints
//      alone, 4 bytes per edge, so the partition reads half the bytes of the
//      edge array.
//   P  (k_deg_part): persistent blocks read that list in 20K-edge
//      chunks, counting-sort the second endpoints of a chunk by 32768-node
//      sub-bucket (v >> 15) in LDS and append each sub-bucket's run of 16-bit
//      local indices to the block's own region for that sub-bucket.  Regions
//      are private per (block, sub-bucket), so no reservation atomics; a
//      block keeps its fill counters in LDS across its chunks.  At most 2048
//      sub-buckets fit the LDS tables, so larger graphs take several windows
//      of sub-buckets, each a pass over the edges.
//   T  (k_deg_tot): per sub-bucket, its entry total over all regions and its
//      number of count parts (about 2^20 entries each).
//   S  (k_deg_scan): exclusive scan of the parts.
//   H  (k_deg_hist): one block per part streams its regions into an LDS
//      histogram of 32768 counters and adds the counts to deg (plain
//      read-modify-write when a sub-bucket is a single part, atomics only for
//      the few heavy multi-part ones).  On a whole graph's first pass, where
//      deg[v] = d, a single part stores d + count without the read, unless a
//      region overflowed in the pass (a workspace flag).
//   tail (k_deg_tail): the targets after the last whole chunk, by global
//      atomics, launched after H so H's direct stores cannot overwrite them.
//
// Region capacities come from the mean-field Barabasi-Albert degree law
// (expected second endpoints of edges [B, B+C) on nodes [a, b)) with slack;
// entries beyond a capacity fall back to a direct global atomic, so the
// result never depends on the capacities, only the speed does.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace ba {

constexpr uint32_t kS2 = 15;                    // sub-bucket width of the partition kernel: 32768 nodes
constexpr uint32_t kSub = 1u << kS2;
constexpr uint32_t kWin = 2048;                 // sub-buckets per partition window
constexpr uint32_t kS16 = 16;                   // sub-bucket width of the fused generator: 65536 nodes
constexpr uint32_t kSub16 = 1u << kS16;
constexpr uint32_t kWin16 = 1024;               // its sub-buckets (one window: n <= 2^26)
constexpr uint32_t kPBlock = 1024;
constexpr uint32_t kPPer = 20;                  // edges per thread per chunk
constexpr uint32_t kPChunk = kPBlock * kPPer;   // 20480 edges per chunk
constexpr uint32_t kPBlocksMax = 1024;          // partition blocks a layout allows
constexpr uint32_t kHPartMin = 1u << 20;        // entries per count part, at least
constexpr uint32_t kHParts = 256;               // count parts a pass aims at (one per compute unit)
constexpr uint32_t kHBlock = 1024;
constexpr uint64_t kPieceMax = 1ull << 31;      // edges per pipeline pass
constexpr uint64_t kPieceMin = 1ull << 20;

__host__ __device__ inline uint64_t isqrt_u64(uint64_t x)
{
    uint64_t r = (uint64_t)sqrt((double)x);
    while (r * r > x) r--;
    while ((r + 1) * (r + 1) <= x) r++;
    return r;
}

// Expected number of edges among [B, B+C) whose second endpoint lies in
// [a, b): with t = i/d nodes present, a new edge hits node v with
// probability about 1/(2 sqrt(t v)) (mean-field BA degree d*sqrt(t/v) over
// 2td endpoints), i.e. lands in [a, b) with probability g(t) =
// (sqrt(min(b,t)) - sqrt(min(a,t))) / sqrt(t); integrate over t.
__host__ __device__ inline double expected_bucket_mass(uint64_t d, uint64_t B, uint64_t C, double a, double b)
{
    const double t0 = (double)B / (double)d, t1 = (double)(B + C) / (double)d;
    double G[2];
    for (int q = 0; q < 2; q++) {
        const double t = q ? t1 : t0;
        if (t <= a)
            G[q] = 0.0;
        else if (t <= b)
            G[q] = t - 2.0 * sqrt(a * t) + a;
        else
            G[q] = b - 2.0 * sqrt(a * b) + a + 2.0 * (sqrt(b) - sqrt(a)) * (sqrt(t) - sqrt(b));
    }
    return (double)d * (G[1] - G[0]);
}

// Capacity of one (block, sub-bucket) region when P blocks share an expected
// mass M: an even share plus slack.
__host__ __device__ inline uint32_t region_cap(double M, uint32_t P)
{
    const double e = M / (double)P;
    return (uint32_t)(1.15 * e + 8.0 * sqrt(e) + 64.0);
}

// Layout of one pass of the pipeline over C edges of a graph with n nodes
// partitioned by at most P blocks.
struct DegPlan {
    uint32_t NBsub, NW, P;
    uint32_t fused;  // n <= 2^26: the generator partitions its own targets into 65536-node sub-buckets
                     // (no target list); else the partition kernel, 32768-node sub-buckets in windows
    uint32_t S;      // sub-bucket shift: 16 (fused) or 15
    uint32_t H;      // entries per count part (target): a sub-bucket of t entries is counted by
                     // ceil(t / H) blocks, whose counts meet in deg by global atomics
    uint64_t n, C;
    uint64_t A;  // region entries reserved in the layout
    uint64_t o_V, o_rcap, o_off, o_fill, o_tot, o_parts, o_partoff, o_flag, o_L, bytes;
};

static inline uint64_t align256(uint64_t x) { return (x + 255) & ~(uint64_t)255; }

static inline DegPlan make_deg_plan(uint64_t n, uint64_t C, uint32_t P)
{
    DegPlan p{};
    p.n = n;
    p.C = C;
    p.P = P;
    p.fused = n <= ((uint64_t)kWin16 << kS16) ? 1u : 0u;
    p.S = p.fused ? kS16 : kS2;
    // Parts about as large as one compute unit's share of the pass: fewer
    // parts mean fewer global atomics when their counts meet (each part of
    // a sub-bucket adds its whole counter array), while no part may hold
    // much more than a unit's share, or it alone sets the histogram's time
    // (the lowest sub-buckets draw the most targets).
    p.H = (uint32_t)std::max<uint64_t>(kHPartMin, C / kHParts);
    p.NBsub = (uint32_t)((n + ((uint64_t)1 << p.S) - 1) >> p.S);
    if (p.NBsub == 0) p.NBsub = 1;
    p.NW = p.fused ? 1u : (p.NBsub + kWin - 1) / kWin;
    // sum of region_cap over sub-buckets and blocks is at most
    //   1.15 C + 8 sqrt(P NBsub C) + 64 P NBsub  (Cauchy-Schwarz), plus rounding
    p.A = C + C / 6 + 8 * isqrt_u64((uint64_t)P * p.NBsub * C) + 8 + 65ull * P * p.NBsub;
    uint64_t o = 0;
    p.o_V = o; o = align256(o + (p.fused ? 0 : 4 * C));
    p.o_rcap = o; o = align256(o + 4ull * p.NBsub);
    p.o_off = o; o = align256(o + 8ull * p.NBsub);
    p.o_fill = o; o = align256(o + 4ull * P * p.NBsub);
    p.o_tot = o; o = align256(o + 4ull * p.NBsub);
    p.o_parts = o; o = align256(o + 4ull * p.NBsub);
    p.o_partoff = o; o = align256(o + 4ull * (p.NBsub + 1));
    p.o_flag = o; o = align256(o + 4);
    p.o_L = o; o = align256(o + 2 * p.A);
    p.bytes = o;
    return p;
}

struct DegArgs {
    DegPlan p;
    uint64_t B, d;          // first edge of the pass, edges per node
    uint32_t *deg;
    unsigned char *ws;
    uint32_t g0;            // first sub-bucket of the window (partition kernel)
    double scale;           // capacity scale (1 normally)
    uint32_t fresh;         // deg[v] = d for every node and nothing of this pass added yet
};

__device__ __forceinline__ const uint32_t *ws_V(const DegArgs &a) { return (const uint32_t *)(a.ws + a.p.o_V); }
__device__ __forceinline__ uint32_t *ws_rcap(const DegArgs &a) { return (uint32_t *)(a.ws + a.p.o_rcap); }
__device__ __forceinline__ uint64_t *ws_off(const DegArgs &a) { return (uint64_t *)(a.ws + a.p.o_off); }
__device__ __forceinline__ uint32_t *ws_fill(const DegArgs &a) { return (uint32_t *)(a.ws + a.p.o_fill); }
__device__ __forceinline__ uint32_t *ws_tot(const DegArgs &a) { return (uint32_t *)(a.ws + a.p.o_tot); }
// set when a region overflowed in this pass (its entries went to deg by atomics)
__device__ __forceinline__ uint32_t *ws_flag(const DegArgs &a) { return (uint32_t *)(a.ws + a.p.o_flag); }
__device__ __forceinline__ uint32_t *ws_parts(const DegArgs &a) { return (uint32_t *)(a.ws + a.p.o_parts); }
__device__ __forceinline__ uint32_t *ws_partoff(const DegArgs &a) { return (uint32_t *)(a.ws + a.p.o_partoff); }
__device__ __forceinline__ uint16_t *ws_L(const DegArgs &a) { return (uint16_t *)(a.ws + a.p.o_L); }

__device__ __forceinline__ void deg_atomic_add(uint32_t *deg, uint64_t v, uint32_t c)
{
    __hip_atomic_fetch_add(deg + v, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Workgroup barrier that orders LDS only: global stores issued before it
// stay in flight (a full __syncthreads would wait for them to complete).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Block-wide exclusive scan of one value per thread (blockDim.x a multiple
// of 64, at most 1024); `sh` holds 16 words.
template <class T>
__device__ __forceinline__ T block_exclusive_scan(T x, T *sh, T *total)
{
    const uint32_t lane = __lane_id(), w = threadIdx.x / 64, nw = blockDim.x / 64;
    T incl = x;
    for (int o = 1; o < 64; o <<= 1) {
        const T y = __shfl_up(incl, o);
        if (lane >= (uint32_t)o) incl += y;
    }
    if (lane == 63) sh[w] = incl;
    lds_barrier();
    T base = 0, tot = 0;
    for (uint32_t q = 0; q < nw; q++) {
        if (q < w) base += sh[q];
        tot += sh[q];
    }
    lds_barrier();
    *total = tot;
    return base + incl - x;
}

// Region capacity of every sub-bucket (scaled for tests of the overflow
// path) and the offset of each sub-bucket's P regions (one block).
__global__ __launch_bounds__(1024) void k_deg_plan(DegArgs a)
{
    __shared__ uint64_t sh[16];
    const uint32_t N = a.p.NBsub;
    uint32_t *rcap = ws_rcap(a);
    uint64_t *off = ws_off(a);
    uint64_t carry = 0;
    if (threadIdx.x == 0) *ws_flag(a) = 0;
    for (uint32_t i0 = 0; i0 < N; i0 += 1024) {
        const uint32_t g = i0 + threadIdx.x;
        uint64_t x = 0;
        uint32_t cap = 0;
        if (g < N) {
            const double lo = (double)((uint64_t)g << a.p.S);
            const uint64_t hi = ((uint64_t)(g + 1) << a.p.S) < a.p.n ? ((uint64_t)(g + 1) << a.p.S) : a.p.n;
            const double M = N == 1 ? (double)a.p.C : expected_bucket_mass(a.d, a.B, a.p.C, lo, (double)hi);
            cap = (uint32_t)((double)region_cap(M, a.p.P) * a.scale);
            x = (uint64_t)cap * a.p.P;
        }
        uint64_t tot;
        const uint64_t ex = block_exclusive_scan<uint64_t>(x, sh, &tot);
        if (g < N) {
            uint64_t o = carry + ex;
            if (o > a.p.A) o = a.p.A;
            if (o + x > a.p.A) cap = (uint32_t)((a.p.A - o) / a.p.P);  // never past the layout
            rcap[g] = cap;
            off[g] = o;
        }
        carry += tot;
    }
}

// P: partition of second endpoints into per-(block, sub-bucket) regions,
// for sub-buckets g0 .. g0+kWin-1.
//
// Region slots are addressed relative to the window's first region in 32
// bits: a window spans at most sum(cap) * P <= 1.15 C + 8 sqrt(P kWin C) +
// 64 P kWin slots (Cauchy-Schwarz over its sub-buckets, capacity scale <= 1),
// under 3.2e9 for C <= kPieceMax, P <= kPBlocksMax.
__global__ __launch_bounds__(kPBlock) void k_deg_part(DegArgs a)
{
    constexpr uint32_t kOut = kWin << kS2;  // entry outside the window or past the chunk
    __shared__ uint32_t cnt[kWin + 64];    // per chunk: counts, then run starts; + 64 lane-private
                                           // counters that absorb entries outside the window
    __shared__ uint32_t fill[kWin];        // entries this block has sent to each region
    __shared__ uint32_t cap[kWin];         // region capacity
    __shared__ uint32_t rbase[kWin];       // this block's region start, window-relative
    __shared__ uint2 dl[kWin];             // per chunk: (slot of sorted entry 0, slot limit)
    __shared__ uint32_t stage[kPChunk];    // sorted (bin << 15 | local index)
    __shared__ uint32_t scan_sh[16];
    __shared__ uint32_t any_over;          // per chunk: some region of this block is full
    const uint32_t g0 = a.g0;
    const uint32_t nwin = min(kWin, a.p.NBsub - g0);
    const uint32_t blk = blockIdx.x, P = gridDim.x;
    const uint64_t wslot = ws_off(a)[g0];
    uint16_t *Lw = ws_L(a) + wslot;
    for (uint32_t b = threadIdx.x; b < kWin; b += kPBlock) {
        const uint32_t cp = b < nwin ? ws_rcap(a)[g0 + b] : 0u;
        fill[b] = 0;
        cap[b] = cp;
        rbase[b] = b < nwin ? (uint32_t)(ws_off(a)[g0 + b] - wslot + (uint64_t)blk * cp) : 0u;
    }

    // whole chunks only: the last C mod kPChunk targets go to k_deg_tail
    const uint64_t nchunks = a.p.C / kPChunk;
    const uint32_t lane = __lane_id(), wv = threadIdx.x / 64;
    const uint32_t wbase = wv * (kPPer * 64);
    // second endpoints: wave w reads targets e0 + (20*64) w + 64 q + lane
    // (64 consecutive 4-byte targets per load, issued back to back).  The
    // next chunk's loads are issued as soon as the current chunk has moved
    // to its own registers, so they have a whole chunk's time to arrive.
    uint32_t v[kPPer], vn[kPPer];
    auto load = [&](uint64_t ch) {
        const uint32_t *wsrc = ws_V(a) + ch * kPChunk + wbase + lane;
#pragma unroll
        for (uint32_t q = 0; q < kPPer; q++) vn[q] = wsrc[q * 64];
    };
    if ((uint64_t)blk < nchunks) load(blk);
    for (uint64_t ch = blk; ch < nchunks; ch += P) {
#pragma unroll
        for (uint32_t q = 0; q < kPPer; q++) v[q] = vn[q];
        if (ch + P < nchunks) load(ch + P);
        for (uint32_t b = threadIdx.x; b < kWin + 64; b += kPBlock) cnt[b] = 0;
#pragma unroll
        for (uint32_t q = 0; q < kPPer; q++) {
            const uint32_t r = (v[q] >> kS2) - g0;
            v[q] = r < nwin ? (r << kS2) | (v[q] & (kSub - 1)) : kOut;
        }
        lds_barrier();
        // counts; each entry keeps its rank within its bin (16 bits: a bin
        // holds at most kPChunk entries of a chunk), two ranks a register
        // (no branches, so the atomics issue back to back)
        uint32_t rk[kPPer / 2];
#pragma unroll
        for (uint32_t q = 0; q < kPPer; q += 2) {
            const uint32_t b0 = (v[q] >> kS2) + (v[q] == kOut ? lane : 0u);
            const uint32_t b1 = (v[q + 1] >> kS2) + (v[q + 1] == kOut ? lane : 0u);
            const uint32_t r0 = atomicAdd(&cnt[b0], 1u);
            const uint32_t r1 = atomicAdd(&cnt[b1], 1u);
            rk[q / 2] = (r0 & 0xFFFFu) | (r1 << 16);
        }
        if (threadIdx.x == 0) any_over = 0;
        lds_barrier();
        // exclusive scan over the window (two bins per thread), destinations
        const uint32_t c0 = cnt[2 * threadIdx.x], c1 = cnt[2 * threadIdx.x + 1];
        uint32_t total;
        const uint32_t s0 = block_exclusive_scan<uint32_t>(c0 + c1, scan_sh, &total);
#pragma unroll
        for (uint32_t h = 0; h < 2; h++) {
            const uint32_t b = 2 * threadIdx.x + h;
            const uint32_t c = h ? c1 : c0, st = h ? s0 + c0 : s0;
            if (c) {
                const uint32_t f = fill[b], cp = cap[b];
                const uint32_t room = f < cp ? cp - f : 0u;
                // region slot of sorted entry x is dst + x (mod 2^32), valid while x < lim
                dl[b] = make_uint2(rbase[b] + f - st, st + min(room, c));
                fill[b] = f + c;
                if (c > room) any_over = 1;
            }
            cnt[b] = st;  // start of the bin's run
        }
        lds_barrier();
        // scatter into sorted order: run start + rank, four starts read at a time
        static_assert(kPPer % 4 == 0, "scatter batches");
#pragma unroll
        for (uint32_t q0 = 0; q0 < kPPer; q0 += 4) {
            uint32_t st4[4];
#pragma unroll
            for (uint32_t j = 0; j < 4; j++) st4[j] = cnt[v[q0 + j] >> kS2];  // cnt[kWin] for outside entries
#pragma unroll
            for (uint32_t j = 0; j < 4; j++) {
                const uint32_t q = q0 + j;
                if (v[q] != kOut) stage[st4[j] + ((rk[q / 2] >> (16 * (q & 1))) & 0xFFFFu)] = v[q];
            }
        }
        lds_barrier();
        const bool over = any_over != 0;
        // sorted runs out: consecutive threads take consecutive sorted
        // entries, so a store covers a few runs of contiguous region slots
        for (uint32_t x0 = threadIdx.x; x0 < total; x0 += 4 * kPBlock) {
            uint32_t w[4];
            uint2 t[4];
#pragma unroll
            for (uint32_t u = 0; u < 4; u++) w[u] = x0 + u * kPBlock < total ? stage[x0 + u * kPBlock] : 0u;
#pragma unroll
            for (uint32_t u = 0; u < 4; u++) t[u] = dl[w[u] >> kS2];
            if (!over) {  // no region full in this chunk (the normal case)
#pragma unroll
                for (uint32_t u = 0; u < 4; u++)
                    if (x0 + u * kPBlock < total) Lw[t[u].x + x0 + u * kPBlock] = (uint16_t)(w[u] & (kSub - 1));
            } else {
                if (x0 == threadIdx.x && threadIdx.x == 0) *ws_flag(a) = 1;  // deg takes atomics before H
#pragma unroll
                for (uint32_t u = 0; u < 4; u++) {
                    const uint32_t x = x0 + u * kPBlock;
                    if (x < total) {
                        if (x < t[u].y)
                            Lw[t[u].x + x] = (uint16_t)(w[u] & (kSub - 1));
                        else
                            deg_atomic_add(a.deg, ((uint64_t)(g0 + (w[u] >> kS2)) << kS2) | (w[u] & (kSub - 1)),
                                           1u);
                    }
                }
            }
        }
        lds_barrier();
    }
    uint32_t *gfill = ws_fill(a) + (uint64_t)blk * a.p.NBsub + g0;
    for (uint32_t b = threadIdx.x; b < nwin; b += kPBlock) gfill[b] = fill[b];
}

// The last C mod kPChunk second endpoints of the pass (fewer than one
// partition chunk), counted with global atomics.
__global__ __launch_bounds__(256) void k_deg_tail(DegArgs a)
{
    const uint64_t e0 = a.p.C / kPChunk * kPChunk;
    const uint64_t e = e0 + (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < a.p.C) deg_atomic_add(a.deg, ws_V(a)[e], 1u);
}

// T: per sub-bucket total over its regions (capped fills) and part count.
__global__ __launch_bounds__(256) void k_deg_tot(DegArgs a)
{
    __shared__ uint32_t sh[4];
    const uint32_t g = blockIdx.x;
    const uint32_t cp = ws_rcap(a)[g];
    const uint32_t *fill = ws_fill(a);
    uint32_t s = 0;
    for (uint32_t p = threadIdx.x; p < a.p.P; p += 256) s += min(fill[(uint64_t)p * a.p.NBsub + g], cp);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (__lane_id() == 0) sh[threadIdx.x / 64] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t t = sh[0] + sh[1] + sh[2] + sh[3];
        ws_tot(a)[g] = t;
        uint32_t np = (uint32_t)(((uint64_t)t + a.p.H - 1) / a.p.H);
        if (np > a.p.P) np = a.p.P;
        ws_parts(a)[g] = np;
    }
}

// S: exclusive scan of the parts over all sub-buckets (one block of 1024).
__global__ __launch_bounds__(1024) void k_deg_scan(DegArgs a)
{
    __shared__ uint32_t sh[16];
    const uint32_t N = a.p.NBsub;
    const uint32_t *parts = ws_parts(a);
    uint32_t *off = ws_partoff(a);
    uint32_t carry = 0;
    for (uint32_t i0 = 0; i0 < N; i0 += 1024) {
        const uint32_t i = i0 + threadIdx.x;
        const uint32_t x = i < N ? parts[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan<uint32_t>(x, sh, &tot);
        if (i < N) off[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) off[N] = carry;
}

// H: one block per part (sub-bucket g, the regions of a contiguous range of
// partition blocks): LDS histogram, then the counts go to deg.
// The part of histogram block k: sub-bucket g, its number of parts np and the
// partition blocks p0 .. p1-1 whose regions the part holds; false past the
// last part.
struct HistPart {
    uint32_t g, np, p0, p1;
};
__device__ __forceinline__ bool hist_part(const DegArgs &a, uint32_t k, HistPart &h)
{
    const uint32_t N = a.p.NBsub;
    const uint32_t *poff = ws_partoff(a);
    if (k >= poff[N]) return false;
    uint32_t lo = 0, hi = N;  // sub-bucket g with poff[g] <= k < poff[g+1]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (poff[mid] <= k) lo = mid; else hi = mid;
    }
    h.g = lo;
    h.np = ws_parts(a)[lo];
    const uint32_t j = k - poff[lo], P = a.p.P;
    h.p0 = (uint32_t)((uint64_t)P * j / h.np);
    h.p1 = (uint32_t)((uint64_t)P * (j + 1) / h.np);
    return true;
}

// 16 bytes of region entries, read once: a non-temporal load, so the reads
// do not hold L2 lines that the other regions' reads could use.
__device__ __forceinline__ uint4 load_nt16(const uint4 *p)
{
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 x = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
    return make_uint4(x.x, x.y, x.z, x.w);
}

// Calls f(x) for every entry x (a 16-bit local index) of the regions the
// calling wave takes of a part: regions p0 + wv, p0 + wv + 16, ...  Lane j
// fetches the fill of the wave's j-th region up front (at most kPBlocksMax /
// 16 = 64 regions a wave), so no region waits on a load of its own length.
// A region is read in batches of up to four 16-byte loads per lane (8
// entries each, where aligned); its first batch also carries the unaligned
// head and the tail, one element per lane (each is shorter than 8 entries).
// The loads of the next batch, of this region or the next, are issued
// before the current batch's entries are visited, so the reads and the
// counting overlap.  Returns the wave's entry count.
template <class F>
__device__ __forceinline__ uint32_t hist_visit(const DegArgs &a, const HistPart &h, F f)
{
    constexpr uint32_t kHW = kHBlock / 64;  // waves of the block: a wave takes every kHW-th region
    static_assert(kPBlocksMax / kHW <= 64, "one region fill per lane");
    const uint32_t N = a.p.NBsub, g = h.g;
    const uint32_t cp = ws_rcap(a)[g];
    const uint64_t base = ws_off(a)[g];
    const uint32_t *fill = ws_fill(a);
    const uint16_t *L = ws_L(a);
    const uint32_t lane = __lane_id(), wv = threadIdx.x / 64;
    const uint32_t p00 = h.p0 + wv;
    const uint32_t pl = p00 + kHW * lane;
    const uint32_t nl = pl < h.p1 ? min(fill[(uint64_t)pl * N + g], cp) : 0u;
    const uint32_t nreg = p00 < h.p1 ? (h.p1 - p00 + kHW - 1) / kHW : 0u;  // the wave's regions
    if (nreg == 0) return 0;
    struct Region {
        const uint16_t *src;
        uint32_t n, head, nv;  // entries, unaligned head, whole 16-byte vectors after it
    };
    struct Batch {
        uint4 q[4];
        uint32_t hv, tv;  // first batch: a head and a tail element
    };
    auto region = [&](uint32_t jr) {
        Region R;
        R.n = (uint32_t)__builtin_amdgcn_readlane((int)nl, (int)jr);  // jr is wave-uniform
        R.src = L + base + (uint64_t)(p00 + kHW * jr) * cp;
        R.head = min(R.n, (uint32_t)((8 - (((uintptr_t)R.src >> 1) & 7)) & 7));
        R.nv = (R.n - R.head) / 8;
        return R;
    };
    auto load = [&](Batch &B, const Region &R, uint32_t b) {
        const uint4 *vs = reinterpret_cast<const uint4 *>(R.src + R.head);
#pragma unroll
        for (uint32_t k = 0; k < 4; k++) {
            const uint32_t t = lane + 64 * (4 * b + k);
            B.q[k] = t < R.nv ? load_nt16(vs + t) : make_uint4(0u, 0u, 0u, 0u);
        }
        if (b == 0) {
            const uint32_t x = R.head + R.nv * 8 + lane;
            B.hv = lane < R.head ? (uint32_t)R.src[lane] : 0u;
            B.tv = x < R.n ? (uint32_t)R.src[x] : 0u;
        }
    };
    auto visit8 = [&](const uint4 &q) {
        f(q.x & 0xFFFFu);
        f(q.x >> 16);
        f(q.y & 0xFFFFu);
        f(q.y >> 16);
        f(q.z & 0xFFFFu);
        f(q.z >> 16);
        f(q.w & 0xFFFFu);
        f(q.w >> 16);
    };
    auto visit = [&](const Batch &B, const Region &R, uint32_t b) {
#pragma unroll
        for (uint32_t k = 0; k < 4; k++)
            if (lane + 64 * (4 * b + k) < R.nv) visit8(B.q[k]);
        if (b == 0) {
            if (lane < R.head) f(B.hv);
            if (R.head + R.nv * 8 + lane < R.n) f(B.tv);
        }
    };
    Region cur = region(0);
    uint32_t total = cur.n, jr = 0, b = 0;
    Batch bc, bn;
    load(bc, cur, 0);
    for (;;) {
        // the batch after (jr, b): the region's next one, else the next region's first
        const uint32_t nb = cur.nv > 256 ? (cur.nv + 255) / 256 : 1u;
        Region nxt = cur;
        uint32_t jr2 = jr, b2 = b + 1;
        if (b2 == nb) {
            jr2 = jr + 1;
            b2 = 0;
            if (jr2 < nreg) nxt = region(jr2);
        }
        const bool more = jr2 < nreg;
        if (more) load(bn, nxt, b2);
        visit(bc, cur, b);
        if (!more) break;
        if (b2 == 0) total += nxt.n;
        cur = nxt;
        jr = jr2;
        b = b2;
        bc = bn;
    }
    return total;
}

__global__ __launch_bounds__(kHBlock) void k_deg_hist(DegArgs a)
{
    __shared__ uint32_t cnt[kSub];
    HistPart hp;
    if (!hist_part(a, blockIdx.x, hp)) return;
    const uint32_t g = hp.g, np = hp.np;
    for (uint32_t x = threadIdx.x; x < kSub; x += kHBlock) cnt[x] = 0;
    __syncthreads();
    hist_visit(a, hp, [&](uint32_t x) { atomicAdd(&cnt[x], 1u); });
    __syncthreads();
    const uint64_t vbase = (uint64_t)g << kS2;
    // deg[v] = d before this block for a single-part sub-bucket of a fresh
    // pass with no region overflow (the tail's atomics run after this kernel)
    const bool direct = a.fresh && *ws_flag(a) == 0;
    static_assert(kSub % (8 * kHBlock) == 0, "count write-back batches");
    for (uint32_t y0 = threadIdx.x; y0 < kSub; y0 += 8 * kHBlock) {
        uint32_t c[8];
#pragma unroll
        for (uint32_t u = 0; u < 8; u++) {
            const uint64_t v = vbase + y0 + u * kHBlock;
            c[u] = v < a.p.n ? cnt[y0 + u * kHBlock] : 0u;
        }
        if (np == 1 && direct) {  // the only block of this sub-bucket: d + count, no read
#pragma unroll
            for (uint32_t u = 0; u < 8; u++)
                if (c[u]) a.deg[vbase + y0 + u * kHBlock] = (uint32_t)a.d + c[u];
        } else if (np == 1) {  // the only block of this sub-bucket: plain read-modify-write, 8 reads in flight
            uint32_t old[8];
#pragma unroll
            for (uint32_t u = 0; u < 8; u++) old[u] = c[u] ? a.deg[vbase + y0 + u * kHBlock] : 0u;
#pragma unroll
            for (uint32_t u = 0; u < 8; u++)
                if (c[u]) a.deg[vbase + y0 + u * kHBlock] = old[u] + c[u];
        } else {
#pragma unroll
            for (uint32_t u = 0; u < 8; u++)
                if (c[u]) deg_atomic_add(a.deg, vbase + y0 + u * kHBlock, c[u]);
        }
    }
}

// H for the fused generator's 65536-node sub-buckets: the same streaming of
// a part's regions into an LDS histogram, with two 16-bit counters per LDS
// word (128 KiB; node 2y in the low half of word y, 2y+1 in the high half).
// Increments do not test for a wrap.  Instead the block sums its counters
// afterwards: a wrap of a low half carries one into the high half and loses
// 65536, a wrap of a high half loses 65536, so the sum equals the number of
// entries counted exactly when no counter wrapped.  When one did (a node
// with 65536 or more second endpoints in one part: never for the mean-field
// degrees of realistic graphs, but possible for tiny n and huge d) the block
// adds every entry of its part to deg by global atomics instead.
__global__ __launch_bounds__(kHBlock) void k_deg_hist16(DegArgs a)
{
    constexpr uint32_t kWords = kSub16 / 2;
    constexpr uint32_t kPer = kWords / kHBlock;  // counter words a thread writes back
    __shared__ uint32_t cnt[kWords];
    __shared__ uint32_t sh[16];
    __shared__ uint32_t counted;
    HistPart hp;
    if (!hist_part(a, blockIdx.x, hp)) return;
    for (uint32_t y = threadIdx.x; y < kWords; y += kHBlock) cnt[y] = 0;
    if (threadIdx.x == 0) counted = 0;
    __syncthreads();
    const uint32_t mine = hist_visit(a, hp, [&](uint32_t x) { atomicAdd(&cnt[x >> 1], 1u << ((x & 1u) << 4)); });
    if (__lane_id() == 0) atomicAdd(&counted, mine);  // mine is wave-uniform
    __syncthreads();
    uint32_t c[kPer], s = 0;
#pragma unroll
    for (uint32_t u = 0; u < kPer; u++) {
        c[u] = cnt[threadIdx.x + u * kHBlock];
        s += (c[u] & 0xFFFFu) + (c[u] >> 16);
    }
    uint32_t sum;
    (void)block_exclusive_scan<uint32_t>(s, sh, &sum);
    const uint64_t vbase = (uint64_t)hp.g << kS16;
    if (sum != counted) {  // some counter wrapped: this part's entries by global atomics
        hist_visit(a, hp, [&](uint32_t x) { deg_atomic_add(a.deg, vbase + x, 1u); });
        return;
    }
    // deg[v] = d before this block for a single-part sub-bucket of a fresh
    // pass with no region overflow
    const bool direct = a.fresh && *ws_flag(a) == 0;
    const uint64_t n = a.p.n;
#pragma unroll
    for (uint32_t u0 = 0; u0 < kPer; u0 += 8) {
        uint32_t old[16];
        if (hp.np == 1 && !direct) {  // plain read-modify-write, 16 reads in flight
#pragma unroll
            for (uint32_t u = 0; u < 8; u++) {
                const uint64_t v = vbase + 2 * (threadIdx.x + (u0 + u) * kHBlock);
                old[2 * u] = (c[u0 + u] & 0xFFFFu) && v < n ? a.deg[v] : 0u;
                old[2 * u + 1] = (c[u0 + u] >> 16) && v + 1 < n ? a.deg[v + 1] : 0u;
            }
        }
#pragma unroll
        for (uint32_t u = 0; u < 8; u++) {
            const uint64_t v = vbase + 2 * (threadIdx.x + (u0 + u) * kHBlock);
#pragma unroll
            for (uint32_t h = 0; h < 2; h++) {
                const uint32_t cv = h ? c[u0 + u] >> 16 : c[u0 + u] & 0xFFFFu;
                if (!cv || v + h >= n) continue;
                if (hp.np == 1 && direct)
                    a.deg[v + h] = (uint32_t)a.d + cv;  // the only block of this sub-bucket: d + count, no read
                else if (hp.np == 1)
                    a.deg[v + h] = old[2 * u + h] + cv;
                else
                    deg_atomic_add(a.deg, v + h, cv);
            }
        }
    }
}

}  // namespace ba
