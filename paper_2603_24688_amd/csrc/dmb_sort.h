// dmb_sort.h -- device-wide exclusive scan and a stable LSD radix sort of
// 64-bit keys with 32-bit payloads: the Morton sort of both species and the
// ordering of work items.
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
// Onesweep LSD radix sort (Adinets & Merrill, "Onesweep: A Faster Least
// Significant Digit Radix Sort for GPUs", 2022): 8-bit digits of 64-bit keys
// with 32-bit payloads, stable.  One kernel histograms every digit pass in a
// single read of the keys (and clears the look-back state); then one kernel
// per pass: each block takes the next tile of kOsTile keys from an atomic
// counter, publishes its per-digit counts, finds the counts of all earlier
// tiles by decoupled look-back, ranks its keys stably in LDS and writes them
// out digit by digit (coalesced runs).  Tiles are numbered in the order
// blocks start, so a look-back only ever waits on tiles whose blocks are
// already running and publish their counts before they look back
// themselves; the wait is still bounded (kOsSpinMax polls, then an error
// flag is raised and the pass ends).
constexpr int kOsBlock = 512;
constexpr int kOsItems = 8;
constexpr int kOsTile = kOsBlock * kOsItems;   // 4096 keys per tile
constexpr int kOsMaxPasses = 8;
constexpr uint64_t kOsAgg = 1ull << 62;        // status: this tile's own count is available
constexpr uint64_t kOsInc = 2ull << 62;        // status: count of this and all earlier tiles
constexpr uint64_t kOsCount = (1ull << 62) - 1;
constexpr uint32_t kOsSpinMax = 1u << 24;

struct OsArgs {
    int64_t n;
    int passes, lo_bit;                 // digit p covers key bits [lo_bit + 8p, lo_bit + 8p + 8)
    uint32_t* hist;                     // [passes][256] global digit counts
    unsigned long long* status;         // [passes][ntile][256] look-back words
    uint32_t* tile_ctr;                 // [passes] tile counters
    uint32_t* err;                      // raised if a look-back wait gave up
    int64_t ntile;
};

// Global digit histograms of all passes; also clears the look-back state.
constexpr int kOsHistBlock = 256;
__global__ __launch_bounds__(kOsHistBlock) void k_os_hist(const uint64_t* __restrict__ keys, OsArgs a)
{
    __shared__ uint32_t h[kOsMaxPasses][256];
    for (int p = 0; p < a.passes; ++p) h[p][threadIdx.x] = 0u;
    __syncthreads();
    const int64_t stride = int64_t(gridDim.x) * kOsHistBlock;
    for (int64_t i = int64_t(blockIdx.x) * kOsHistBlock + threadIdx.x; i < a.n; i += stride) {
        const uint64_t k = keys[i];
        for (int p = 0; p < a.passes; ++p) atomicAdd(&h[p][uint32_t(k >> (a.lo_bit + 8 * p)) & 255u], 1u);
    }
    __syncthreads();
    for (int p = 0; p < a.passes; ++p)
        if (h[p][threadIdx.x]) atomicAdd(&a.hist[p * 256 + threadIdx.x], h[p][threadIdx.x]);
    const int64_t nst = int64_t(a.passes) * a.ntile * 256;
    for (int64_t i = int64_t(blockIdx.x) * kOsHistBlock + threadIdx.x; i < nst; i += stride) a.status[i] = 0ull;
}

// Exclusive scan of one value per digit held by threads 0..255 of the block
// (every thread of the block calls it; threads >= 256 pass 0 and get 0).
__device__ __forceinline__ uint32_t os_block_excl(uint32_t v, uint32_t* ws)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63 && w < 4) ws[w] = x;
    __syncthreads();
    uint32_t off = 0;
    for (int k = 0; k < w && k < 4; ++k) off += ws[k];
    __syncthreads();
    return off + x - v;
}

__global__ __launch_bounds__(kOsBlock) void k_os_pass(const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                      uint64_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                      OsArgs a, int pass)
{
    constexpr int kW = kOsBlock / 64;          // waves; wave w owns keys [w, w + 1) * kOsTile / kW of the tile
    __shared__ uint64_t sk[kOsTile];
    __shared__ uint32_t sv[kOsTile];
    __shared__ uint32_t hist[256], tstart[256], wcnt[kW][256];
    __shared__ uint64_t gbase[256];    // global position of this tile's first key of each digit
    __shared__ uint32_t ws[4];
    __shared__ uint32_t s_tile;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int shift = a.lo_bit + 8 * pass;
    const bool dig = tid < 256;                // threads 0..255 own one digit each
    if (tid == 0) s_tile = atomicAdd(&a.tile_ctr[pass], 1u);
    for (int k = tid; k < 256 * (kW + 1); k += kOsBlock) (k < 256 ? hist[k] : wcnt[k / 256 - 1][k % 256]) = 0u;
    __syncthreads();
    const int64_t tile = int64_t(s_tile);
    const int64_t base = tile * kOsTile;
    const int64_t wbase = base + int64_t(wid) * (kOsTile / kW);
    uint64_t kr[kOsItems];
    uint32_t vr[kOsItems];
#pragma unroll
    for (int r = 0; r < kOsItems; ++r) {       // round r: 64 consecutive keys of the wave's chunk
        const int64_t i = wbase + int64_t(r) * 64 + lane;
        kr[r] = i < a.n ? kin[i] : 0ull;
        vr[r] = i < a.n ? vin[i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kOsItems; ++r)
        if (wbase + int64_t(r) * 64 + lane < a.n) atomicAdd(&hist[uint32_t(kr[r] >> shift) & 255u], 1u);
    __syncthreads();
    // publish this tile's counts, then look back for the counts of all earlier tiles
    unsigned long long* st = a.status + (int64_t(pass) * a.ntile) * 256;
    const uint32_t mine = dig ? hist[tid] : 0u;
    if (dig && tile == 0) {
        __hip_atomic_store(&st[tid], kOsInc | mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if (dig) {
        __hip_atomic_store(&st[tile * 256 + tid], kOsAgg | mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // stable ranks within the wave's chunk, wave-private counts (no block barrier per round)
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    uint32_t rk[kOsItems];
#pragma unroll
    for (int r = 0; r < kOsItems; ++r) {
        const bool valid = wbase + int64_t(r) * 64 + lane < a.n;
        const uint32_t d = uint32_t(kr[r] >> shift) & 255u;
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bal = __ballot(valid && ((d >> b) & 1u));
            m &= ((d >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t before = valid ? wcnt[wid][d] : 0u;
        rk[r] = before + uint32_t(__popcll(m & lt));
        // the first lane of each digit group adds the group; a wave's LDS operations
        // complete in issue order, so the next round reads the updated count
        if (valid && (m & lt) == 0ull) wcnt[wid][d] = before + uint32_t(__popcll(m));
    }
    uint64_t excl = 0;
    if (dig && tile > 0) {
        int64_t t = tile - 1;
        uint32_t spins = 0;
        for (;;) {
            const uint64_t s = __hip_atomic_load(&st[t * 256 + tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (s & kOsInc) { excl += s & kOsCount; break; }
            if (s & kOsAgg) { excl += s & kOsCount; --t; spins = 0; continue; }
            if (++spins > kOsSpinMax) { atomicOr(a.err, 1u); break; }
            __builtin_amdgcn_s_sleep(1);
        }
        __hip_atomic_store(&st[tile * 256 + tid], kOsInc | (excl + mine), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // digit starts: global (digits below d over all keys + this digit in earlier tiles), in the tile,
    // and per wave (earlier waves' keys of the digit)
    const uint32_t g = dig ? a.hist[pass * 256 + tid] : 0u;
    const uint32_t gex = os_block_excl(g, ws);
    const uint32_t tex = os_block_excl(mine, ws);
    if (dig) {
        gbase[tid] = uint64_t(gex) + excl;
        tstart[tid] = tex;
        uint32_t acc = tex;
#pragma unroll
        for (int w = 0; w < kW; ++w) {
            const uint32_t cw = wcnt[w][tid];
            wcnt[w][tid] = acc;            // becomes the wave's first tile position of the digit
            acc += cw;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kOsItems; ++r) {
        if (wbase + int64_t(r) * 64 + lane < a.n) {
            const uint32_t d = uint32_t(kr[r] >> shift) & 255u;
            const uint32_t pos = wcnt[wid][d] + rk[r];
            sk[pos] = kr[r];
            sv[pos] = vr[r];
        }
    }
    __syncthreads();
    // write out in tile order: consecutive threads of one digit write consecutive positions
    const int64_t cnt = a.n - base < kOsTile ? a.n - base : kOsTile;
    for (int i = tid; i < int(cnt); i += kOsBlock) {
        const uint64_t k = sk[i];
        const uint32_t d = uint32_t(k >> shift) & 255u;
        const uint64_t pos = gbase[d] + uint64_t(i - int(tstart[d]));
        if (pos < uint64_t(a.n)) {
            kout[pos] = k;
            vout[pos] = sv[i];
        }
    }
}

}  // namespace dmb
