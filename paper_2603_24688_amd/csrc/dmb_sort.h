// dmb_sort.h -- device-wide exclusive scan and one-pass stable counting
// sort by an 8-bit digit (64-bit keys, 32-bit payload): the Morton sort of
// small species and the ordering of work items.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dmb {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 4;                       // elements per thread
constexpr int kScanTile = kScanBlock * kScanItems;  // 1024

// Block-local exclusive scan (inputs TI, sums and outputs TO: 64-bit outputs
// for offsets that can pass 2^32); writes the block total to sums[blockIdx].
// Inputs at or past n_in read as 0 (so that out[n_in] can hold the total).
template <typename TI, typename TO>
__global__ __launch_bounds__(kScanBlock) void k_scan_block(const TI* __restrict__ in, TO* __restrict__ out,
                                                           TO* __restrict__ sums, int64_t n, int64_t n_in)
{
    __shared__ TO wsum[kScanBlock / 64];
    int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
    TO v[kScanItems];
    TO t = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n_in) ? TO(in[base + k]) : TO(0);
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

// Adds to block b's tile the totals of blocks 0 .. b-1, which the block sums
// itself (for up to kScanOwnMax blocks), so the block totals need no scan of
// their own.
constexpr int64_t kScanOwnMax = 4096;

template <typename TO>
__global__ __launch_bounds__(kScanBlock) void k_scan_add_own(TO* __restrict__ out, const TO* __restrict__ sums,
                                                             int64_t n)
{
    __shared__ TO part[kScanBlock / 64];
    const int b = int(blockIdx.x);
    if (b == 0) return;
    TO acc = 0;
    for (int k = int(threadIdx.x); k < b; k += kScanBlock) acc += sums[k];
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    TO add = 0;
    for (int w = 0; w < kScanBlock / 64; ++w) add += part[w];
    const int64_t base = int64_t(b) * kScanTile + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + int64_t(k) * kScanBlock;
        if (i < n) out[i] += add;
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

// ---------------------------------------------------------------------------
// Stable LSD radix sort, 8-bit digits.  Each block owns kSortTile
// consecutive keys; per-block digit counts are scanned digit-major so the
// scatter keeps the input order of equal digits.
constexpr int kSortBlock = 256;
constexpr int kSortRounds = 16;
constexpr int kSortTile = kSortBlock * kSortRounds;  // 4096

__global__ __launch_bounds__(kSortBlock) void k_sort_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                                          uint32_t* __restrict__ table, int nblocks)
{
    __shared__ uint32_t hist[256];
    hist[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = int64_t(blockIdx.x) * kSortTile;
    uint32_t dg[kSortRounds];
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {    // all loads in flight before the first count
        int64_t i = base + int64_t(r) * kSortBlock + threadIdx.x;
        dg[r] = i < n ? uint32_t(keys[i] >> shift) & 255u : 256u;
    }
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r)
        if (dg[r] < 256u) atomicAdd(&hist[dg[r]], 1u);
    __syncthreads();
    table[int64_t(threadIdx.x) * nblocks + blockIdx.x] = hist[threadIdx.x];
}

__global__ __launch_bounds__(kSortBlock) void k_sort_scatter(const uint64_t* __restrict__ keys_in,
                                                             const uint32_t* __restrict__ vals_in,
                                                             uint64_t* __restrict__ keys_out,
                                                             uint32_t* __restrict__ vals_out, int64_t n, int shift,
                                                             const uint32_t* __restrict__ table, int nblocks)
{
    __shared__ uint32_t boff[256];
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[kSortBlock / 64][256];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    boff[tid] = table[int64_t(tid) * nblocks + blockIdx.x];
    run[tid] = 0;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int64_t base = int64_t(blockIdx.x) * kSortTile;
    uint64_t kr[kSortRounds];
    uint32_t vr[kSortRounds];
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {    // the block's keys and values, all loads in flight at once
        const int64_t i = base + int64_t(r) * kSortBlock + tid;
        kr[r] = i < n ? keys_in[i] : 0ull;
        vr[r] = i < n ? vals_in[i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
#pragma unroll
        for (int w = 0; w < kSortBlock / 64; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        int64_t i = base + int64_t(r) * kSortBlock + tid;
        bool valid = i < n;
        uint64_t key = kr[r];
        uint32_t val = vr[r];
        uint32_t d = uint32_t(key >> shift) & 255u;
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t bal = __ballot(valid && ((d >> b) & 1u));
            m &= ((d >> b) & 1u) ? bal : ~bal;
        }
        int rank = __popcll(m & lt);
        if (valid && rank == 0) wcnt[wid][d] = uint32_t(__popcll(m));
        __syncthreads();
        if (valid) {
            uint32_t pre = 0;
            for (int w = 0; w < wid; ++w) pre += wcnt[w][d];
            uint32_t pos = boff[d] + run[d] + pre + uint32_t(rank);
            keys_out[pos] = key;
            vals_out[pos] = val;
        }
        __syncthreads();
        uint32_t tot = 0;
#pragma unroll
        for (int w = 0; w < kSortBlock / 64; ++w) tot += wcnt[w][tid];
        run[tid] += tot;
        __syncthreads();
    }
}

}  // namespace dmb
