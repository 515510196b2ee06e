// alu_peak.hip -- issue-rate microbenchmarks of the integer instructions the
// keys kernel is built from, run on every compute unit: v_mad_u64_u32 (the
// 32 x 32 -> 64-bit product of a Philox round), v_bitop3_b32 (its three-way
// XOR) and whole Philox4x32-10 blocks (ten rounds of two of each).  They give
// the measured integer peak the keys kernel is compared against.
//
// Every lane keeps several independent dependency chains so that the
// instruction latency is hidden and the issue rate is what is measured; every
// chain's final value is stored, so no instruction can be dropped.
#include <hip/hip_runtime.h>

#include <cstdint>

#define PEAK_API extern "C" __attribute__((visibility("default")))

namespace {

constexpr int kChains = 8;

__device__ __forceinline__ uint64_t mad64(uint32_t x, uint32_t m, uint64_t add)
{
    uint64_t r, carry;
    asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(r), "=&s"(carry) : "v"(x), "s"(m), "v"(add));
    (void)carry;
    return r;
}

__device__ __forceinline__ uint32_t bitop3_xor(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm volatile("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// kChains independent chains acc <- x * m + acc, iters times.
__global__ __launch_bounds__(256) void mad_kernel(uint64_t *out, int iters, uint32_t m)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t acc[kChains];
    uint32_t x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        acc[c] = t + c;
        x[c] = t * 2654435761u + c;
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = mad64(x[c], m, acc[c]);
    }
    uint64_t s = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s ^= acc[c];
    out[t] = s;
}

// kChains independent chains acc <- acc ^ y ^ z, iters times.
__global__ __launch_bounds__(256) void bitop3_kernel(uint32_t *out, int iters, uint32_t y)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc[kChains], z[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        acc[c] = t + c;
        z[c] = t * 40503u + c;
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = bitop3_xor(acc[c], y, z[c]);
    }
    uint32_t s = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s ^= acc[c];
    out[t] = s;
}

// Philox4x32-10 blocks, kBlocks interleaved per lane: each round two
// v_mad_u64_u32 and two v_bitop3_b32 per block (the round key words come from
// scalar registers, as in the keys kernel).
constexpr int kBlocks = 4;

__global__ __launch_bounds__(256) void philox_kernel(uint32_t *out, int iters, uint32_t k0_in, uint32_t k1_in)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t sink = 0;
    for (int i = 0; i < iters; ++i) {
        uint32_t c0[kBlocks], c1[kBlocks], c2[kBlocks], c3[kBlocks];
#pragma unroll
        for (int b = 0; b < kBlocks; ++b) {
            c0[b] = t * kBlocks + b;
            c1[b] = static_cast<uint32_t>(i);
            c2[b] = t ^ (static_cast<uint32_t>(i) * 0x9E3779B9u);
            c3[b] = 0u;
        }
        uint32_t k0 = k0_in, k1 = k1_in;
#pragma unroll
        for (int r = 0; r < 10; ++r) {
#pragma unroll
            for (int b = 0; b < kBlocks; ++b) {
                const uint64_t pa = mad64(c0[b], 0xD2511F53u, 0);
                const uint64_t pb = mad64(c2[b], 0xCD9E8D57u, 0);
                const uint32_t n0 = bitop3_xor(static_cast<uint32_t>(pb >> 32), c1[b], k0);
                const uint32_t n2 = bitop3_xor(static_cast<uint32_t>(pa >> 32), c3[b], k1);
                c1[b] = static_cast<uint32_t>(pb);
                c3[b] = static_cast<uint32_t>(pa);
                c0[b] = n0;
                c2[b] = n2;
            }
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
#pragma unroll
        for (int b = 0; b < kBlocks; ++b) sink ^= c0[b] ^ c1[b] ^ c2[b] ^ c3[b];
    }
    out[t] = sink;
}

}  // namespace

// which: 0 v_mad_u64_u32, 1 v_bitop3_b32, 2 Philox4x32-10 blocks.  Runs `reps`
// timed launches of `grid` workgroups of 256 lanes, `iters` iterations each,
// after one untimed launch; ms[0] = the fastest launch's milliseconds and
// *units = instructions (0, 1) or Philox blocks (2) one launch performs.
// Returns 0 or a HIP error code.
PEAK_API int nzpeak_run(int which, int grid, int iters, int reps, double *ms, double *units)
{
    if (which < 0 || which > 2 || grid < 1 || iters < 1 || reps < 1 || !ms || !units) return -1;
    void *buf = nullptr;
    const size_t threads = static_cast<size_t>(grid) * 256;
    hipError_t e = hipMalloc(&buf, threads * 8);
    if (e != hipSuccess) return e;
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    double best = 1e30;
    for (int r = 0; r <= reps && e == hipSuccess; ++r) {
        (void)hipEventRecord(a, nullptr);
        if (which == 0)
            hipLaunchKernelGGL(mad_kernel, dim3(grid), dim3(256), 0, nullptr, static_cast<uint64_t *>(buf), iters,
                               0x9E3779B1u);
        else if (which == 1)
            hipLaunchKernelGGL(bitop3_kernel, dim3(grid), dim3(256), 0, nullptr, static_cast<uint32_t *>(buf), iters,
                               0x5BD1E995u);
        else
            hipLaunchKernelGGL(philox_kernel, dim3(grid), dim3(256), 0, nullptr, static_cast<uint32_t *>(buf), iters,
                               0x243F6A88u, 0x85A308D3u);
        (void)hipEventRecord(b, nullptr);
        e = hipEventSynchronize(b);
        float t = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
        if (r > 0 && t < best) best = t;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(buf);
    if (e != hipSuccess) return e;
    *ms = best;
    *units = static_cast<double>(threads) * iters * (which == 2 ? kBlocks : kChains);
    return 0;
}
