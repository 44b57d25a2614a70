// hrr_scan.hpp -- exclusive prefix sum of u32 counts on a gfx950 device, used
// by the eye ordering (bucket offsets) and by the device hierarchy build
// (radix-sort digit offsets, child slots of a level).
//
// Three stream-ordered launches: every block sums one chunk of kScanChunk
// counts, one block scans the chunk sums (1024 per step, any number of
// steps), and every block rescans its chunk from its chunk's base.  The
// output may be the input array (a block reads its whole chunk before it
// writes any of it).  The kernels have internal linkage, so every HIP source
// that includes this header carries its own copy.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hrr {
namespace scan {

constexpr uint32_t kScanChunk = 4096;   // 16 counts per thread of 256

// Inclusive scan of one value per lane over a wave of 64.
__device__ __forceinline__ uint32_t wave_inclusive(uint32_t x) {
    const uint32_t lane = threadIdx.x & 63u;
#pragma unroll
    for (uint32_t off = 1; off < 64u; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

// Inclusive scan of one value per thread over a block of 256 threads in
// thread order; *total receives the block's sum.  lds holds 4 words.
__device__ __forceinline__ uint32_t block_inclusive_256(uint32_t x, uint32_t* lds, uint32_t* total) {
    const uint32_t t = threadIdx.x, w = t >> 6;
    x = wave_inclusive(x);
    if ((t & 63u) == 63u) lds[w] = x;
    __syncthreads();
    uint32_t before = 0;
    for (uint32_t q = 0; q < w; ++q) before += lds[q];
    *total = lds[0] + lds[1] + lds[2] + lds[3];
    __syncthreads();
    return x + before;
}

static __global__ __launch_bounds__(256) void chunk_sums_kernel(const uint32_t* in, uint32_t n, uint32_t* sums) {
    __shared__ uint32_t lds[4];
    const uint32_t b = blockIdx.x * kScanChunk + threadIdx.x * 16u;
    uint32_t sum = 0;
    for (uint32_t q = 0; q < 16u; ++q) sum += b + q < n ? in[b + q] : 0u;
    uint32_t total;
    (void)block_inclusive_256(sum, lds, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

static __global__ __launch_bounds__(256) void chunk_bases_kernel(uint32_t* sums, uint32_t n_chunks) {
    __shared__ uint32_t lds[4];
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < n_chunks; b0 += 1024u) {
        const uint32_t b = b0 + threadIdx.x * 4u;
        uint32_t x[4], sum = 0;
        for (uint32_t q = 0; q < 4u; ++q) {
            x[q] = b + q < n_chunks ? sums[b + q] : 0u;
            sum += x[q];
        }
        uint32_t total;
        uint32_t run = carry + block_inclusive_256(sum, lds, &total) - sum;
        for (uint32_t q = 0; q < 4u; ++q) {
            if (b + q < n_chunks) sums[b + q] = run;
            run += x[q];
        }
        carry += total;
    }
}

static __global__ __launch_bounds__(256) void apply_kernel(const uint32_t* in, uint32_t* out, uint32_t n,
                                                           const uint32_t* sums) {
    __shared__ uint32_t lds[4];
    const uint32_t b = blockIdx.x * kScanChunk + threadIdx.x * 16u;
    uint32_t x[16], sum = 0;
    for (uint32_t q = 0; q < 16u; ++q) {
        x[q] = b + q < n ? in[b + q] : 0u;
        sum += x[q];
    }
    uint32_t total;
    uint32_t run = sums[blockIdx.x] + block_inclusive_256(sum, lds, &total) - sum;
    for (uint32_t q = 0; q < 16u; ++q) {
        if (b + q < n) out[b + q] = run;
        run += x[q];
    }
}

// Words of chunk sums an n-count scan needs.
static inline uint32_t chunk_count(uint32_t n) { return (n + kScanChunk - 1u) / kScanChunk; }

// out[i] = in[0] + ... + in[i - 1] (mod 2^32); sums holds chunk_count(n)
// words of scratch.  Launches nothing for n == 0.
static inline hipError_t exclusive_sum(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* sums,
                                       hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const uint32_t chunks = chunk_count(n);
    hipLaunchKernelGGL(chunk_sums_kernel, dim3(chunks), dim3(256), 0, stream, in, n, sums);
    hipLaunchKernelGGL(chunk_bases_kernel, dim3(1), dim3(256), 0, stream, sums, chunks);
    hipLaunchKernelGGL(apply_kernel, dim3(chunks), dim3(256), 0, stream, in, out, n, sums);
    return hipGetLastError();
}

}  // namespace scan
}  // namespace hrr
