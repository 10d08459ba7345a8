// ba_rates.hip -- issue-rate and store-rate microbenchmarks that price the
// integer-ALU roofline of the generator on gfx950 (built as libba_rates.so;
// used by bench.py --workload rates, not by the generator).
//
// The algorithmic work of one edge is counted in VALU instructions of a
// plain 32-bit lowering of the hash (a multiply class: 32-bit multiplies,
// the 32x32+64 multiply-add, alignbit and three-input add; and a simple
// class: xor, shift, add).  What one such instruction costs in lane-cycles
// is measured here: every lane runs kChains independent dependency chains
// of one instruction, so the issue rate, not the latency, is what the time
// shows.  The store rate is a plain 16-byte fill of a large buffer.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kChains = 8;

enum Op { kMulLo = 0, kMulHi = 1, kMad64 = 2, kAlignbit = 3, kAdd3 = 4, kXor = 5, kShr = 6, kAdd = 7, kOps = 8 };

template <int OP>
__device__ __forceinline__ void step(uint32_t &x, uint32_t c)
{
    if constexpr (OP == kMulLo) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(x) : "v"(c));
    if constexpr (OP == kMulHi) asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(x) : "v"(c));
    if constexpr (OP == kMad64) {
        uint64_t acc;
        asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, 0" : "=v"(acc) : "v"(x), "v"(c) : "vcc");
        x = (uint32_t)acc;  // the chain goes on through the low half
    }
    if constexpr (OP == kAlignbit) asm volatile("v_alignbit_b32 %0, %0, %1, 7" : "+v"(x) : "v"(c));
    if constexpr (OP == kAdd3) asm volatile("v_add3_u32 %0, %0, %1, %1" : "+v"(x) : "v"(c));
    if constexpr (OP == kXor) asm volatile("v_xor_b32 %0, %0, %1" : "+v"(x) : "v"(c));
    if constexpr (OP == kShr) asm volatile("v_lshrrev_b32 %0, 1, %0" : "+v"(x));
    if constexpr (OP == kAdd) asm volatile("v_add_u32 %0, %0, %1" : "+v"(x) : "v"(c));
}

template <int OP>
__global__ __launch_bounds__(256) void k_rate(uint32_t iters, uint32_t seed, uint32_t *sink)
{
    uint32_t x[kChains];
    const uint32_t c = seed | 1u;
#pragma unroll
    for (int j = 0; j < kChains; j++) x[j] = threadIdx.x * 7919u + j + seed;
    for (uint32_t it = 0; it < iters; it++) {
#pragma unroll
        for (int u = 0; u < 4; u++)
#pragma unroll
            for (int j = 0; j < kChains; j++) step<OP>(x[j], c);
    }
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < kChains; j++) r ^= x[j];
    if (r == 0x12345678u) sink[blockIdx.x] = r;  // keeps the chains live
}

__global__ __launch_bounds__(256) void k_fill16(uint4 *p, uint64_t n16, uint32_t value)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint4 w = make_uint4(value, value, value, value);
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n16; j += stride) p[j] = w;
}

template <int OP>
void launch(uint32_t blocks, uint32_t iters, uint32_t *sink, hipStream_t st)
{
    hipLaunchKernelGGL(k_rate<OP>, dim3(blocks), dim3(256), 0, st, iters, 0x9E3779B9u, sink);
}

}  // namespace

extern "C" {

// Instructions of the measured kind one lane issues per iteration.
int ba_rate_ops_per_iter(int op) { return op >= 0 && op < kOps ? 4 * kChains : 0; }

// Times one launch of the op's chains (blocks of 256 threads, `sink` a device
// buffer of `blocks` uint32) with HIP events on `stream`; *ms gets the
// duration.  Returns 0, or -1 for a bad op, or the hipError_t of a failure.
int ba_rate_run(int op, uint32_t blocks, uint32_t iters, uint32_t *sink, void *stream, float *ms)
{
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (op < 0 || op >= kOps || !sink || !ms) return -1;
    if (hipEventCreate(&e0) != hipSuccess) return (int)hipGetLastError();
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return (int)hipGetLastError();
    }
    (void)hipEventRecord(e0, st);
    switch (op) {
    case kMulLo: launch<kMulLo>(blocks, iters, sink, st); break;
    case kMulHi: launch<kMulHi>(blocks, iters, sink, st); break;
    case kMad64: launch<kMad64>(blocks, iters, sink, st); break;
    case kAlignbit: launch<kAlignbit>(blocks, iters, sink, st); break;
    case kAdd3: launch<kAdd3>(blocks, iters, sink, st); break;
    case kXor: launch<kXor>(blocks, iters, sink, st); break;
    case kShr: launch<kShr>(blocks, iters, sink, st); break;
    default: launch<kAdd>(blocks, iters, sink, st); break;
    }
    (void)hipEventRecord(e1, st);
    hipError_t e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    if (e == hipSuccess) e = hipGetLastError();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return e == hipSuccess ? 0 : (int)e;
}

// Times one 16-byte fill of n16 uint4 elements at p (device) on `stream`.
int ba_rate_fill(void *p, uint64_t n16, uint32_t blocks, void *stream, float *ms)
{
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (!p || !ms) return -1;
    if (hipEventCreate(&e0) != hipSuccess) return (int)hipGetLastError();
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return (int)hipGetLastError();
    }
    (void)hipEventRecord(e0, st);
    hipLaunchKernelGGL(k_fill16, dim3(blocks), dim3(256), 0, st, (uint4 *)p, n16, 0xA5A5A5A5u);
    (void)hipEventRecord(e1, st);
    hipError_t e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    if (e == hipSuccess) e = hipGetLastError();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return e == hipSuccess ? 0 : (int)e;
}

}  // extern "C"
