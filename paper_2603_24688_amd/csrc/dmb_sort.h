// dmb_sort.h -- device-wide exclusive scan (the Morton sort itself is
// rocPRIM's radix sort).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dmb {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 4;                       // elements per thread
constexpr int kScanTile = kScanBlock * kScanItems;  // 1024

// Block-local exclusive scan (inputs TI, sums and outputs TO: 64-bit outputs
// for offsets that can pass 2^32); writes the block total to sums[blockIdx].
template <typename TI, typename TO>
__global__ __launch_bounds__(kScanBlock) void k_scan_block(const TI* __restrict__ in, TO* __restrict__ out,
                                                           TO* __restrict__ sums, int64_t n)
{
    __shared__ TO wsum[kScanBlock / 64];
    int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
    TO v[kScanItems];
    TO t = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? TO(in[base + k]) : TO(0);
        t += v[k];
    }
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    TO x = t;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        TO y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    TO woff = 0;
    for (int w = 0; w < wid; ++w) woff += wsum[w];
    TO run = woff + x - t;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == kScanBlock - 1) {
        TO tot = 0;
        for (int w = 0; w < kScanBlock / 64; ++w) tot += wsum[w];
        sums[blockIdx.x] = tot;
    }
}

template <typename TO>
__global__ __launch_bounds__(kScanBlock) void k_scan_add(TO* __restrict__ out, const TO* __restrict__ sums, int64_t n)
{
    TO add = sums[blockIdx.x];
    int64_t base = int64_t(blockIdx.x) * kScanTile + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + int64_t(k) * kScanBlock;
        if (i < n) out[i] += add;
    }
}

}  // namespace dmb
