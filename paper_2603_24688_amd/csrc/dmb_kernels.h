// dmb_kernels.h -- gfx950 kernels of the DM-gas pair step: Morton cells,
// tiles and candidate lists, the gas mean-field pass, the DM Monte Carlo pass
// and the partner resolve.  See dmb.h for the operation each entry computes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

#include "../../include/dmb.h"
#include "dmb_device.h"
#include "dmb_mlp.h"

namespace dmb {

constexpr int kTile = 64;        // particles per tile (one wavefront)
constexpr int kXcd = 8;          // XCDs per MI355X; blockIdx round-robins over them
constexpr double kMsunG = 1.988409870698051e33;
constexpr double kKpcCm = 3.0856775814913673e21;
constexpr double kCKms = 299792.458;
constexpr double kMpG = 1.67262192369e-24;
enum { kRatesExact = 0, kRatesQuad = 1, kRatesMlp = 2, kRatesClosure = 3 };
constexpr int kMaxQuadNodes = 64;
constexpr int kMlpPassWaves = 4;     // independent waves per block of the network gas pass

// Integration window of rate_quad for K nodes: the wide window reaches 1e-10
// from K = 32 on; below K = 24 the narrow one is the cheaper choice at the
// 1e-3 level (K = 12 suffices there).
__host__ __device__ inline void quad_window(int K, double* hw, double* bmin)
{
    *hw = K >= 24 ? 8.5 : 5.5;
    *bmin = K >= 24 ? 11.0 : 7.0;
}

// Ordering of the LDS staging of one wave.  With one wave per block this is
// the block barrier; blocks of several independent waves order each wave's
// own LDS traffic (a wave's LDS operations complete in issue order).
template <int W>
__device__ __forceinline__ void stage_sync()
{
    if constexpr (W == 1) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

__device__ __forceinline__ int lane_id() { return int(threadIdx.x & 63); }

// Lane moves of the data-parallel primitives (DPP), all within registers.
// CTRL 0x111/0x112/0x114/0x118 = row_shr 1/2/4/8: lane i takes lane i - d of
// its row of 16; 0x142 = row_bcast:15: every lane of row r takes lane 16r - 1;
// 0x143 = row_bcast:31: every lane takes lane 31.  ROWS masks the rows that
// receive; lanes without a source and rows outside ROWS read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v)
{
    return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), CTRL, ROWS, 0xF, true));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_move(float v)
{
    return __uint_as_float(dpp_u32<CTRL, ROWS>(__float_as_uint(v)));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move(double v)
{
    const uint64_t b = uint64_t(__double_as_longlong(v));
    const uint64_t lo = dpp_u32<CTRL, ROWS>(uint32_t(b)), hi = dpp_u32<CTRL, ROWS>(uint32_t(b >> 32));
    return __longlong_as_double((long long)((hi << 32) | lo));
}

template <int CTRL, int ROWS, typename T>
__device__ __forceinline__ T dpp_take_add(T v, bool take)
{
    const T t = dpp_move<CTRL, ROWS>(v);
    return take ? v + t : v;
}
template <int CTRL, int ROWS, typename T>
__device__ __forceinline__ T dpp_take_max(T v, bool take)
{
    const T t = dpp_move<CTRL, ROWS>(v);
    return take && t > v ? t : v;
}
template <int CTRL, int ROWS, typename T>
__device__ __forceinline__ T dpp_take_min(T v, bool take)
{
    const T t = dpp_move<CTRL, ROWS>(v);
    return take && t < v ? t : v;
}

// Segmented inclusive scan upward over the wave: segments are runs of
// consecutive lanes, `lo` the first lane of this lane's run.  f(ctrl, rows,
// take) is called for up to six steps (four row shifts, then the two row
// broadcasts); folding the moved copies in where `take` holds leaves every
// lane with the combination of lanes [lo, lane] in a fixed order, so the
// run's total sits in its last lane.  A step that no lane takes is skipped
// (a wave-uniform branch): short runs cost only the first steps.
template <typename F>
__device__ __forceinline__ void seg_scan_up(int lane, int lo, F&& f)
{
    using std::integral_constant;
    const int row0 = lane & ~15;
    const int lr = max(lo, row0);   // first lane of the run within this lane's row
    bool tk = lane - 1 >= lr;
    if (__ballot(tk)) f(integral_constant<int, 0x111>(), integral_constant<int, 0xF>(), tk);
    tk = lane - 2 >= lr;
    if (__ballot(tk)) f(integral_constant<int, 0x112>(), integral_constant<int, 0xF>(), tk);
    tk = lane - 4 >= lr;
    if (__ballot(tk)) f(integral_constant<int, 0x114>(), integral_constant<int, 0xF>(), tk);
    tk = lane - 8 >= lr;
    if (__ballot(tk)) f(integral_constant<int, 0x118>(), integral_constant<int, 0xF>(), tk);
    tk = (lane & 16) != 0 && lo < row0;
    if (__ballot(tk)) f(integral_constant<int, 0x142>(), integral_constant<int, 0xA>(), tk);
    tk = lane >= 32 && lo <= 31;
    if (__ballot(tk)) f(integral_constant<int, 0x143>(), integral_constant<int, 0xC>(), tk);
}

// Inclusive prefix sum over the wave's lanes (v >= 0), in registers: four
// row shifts, then the row broadcasts carry row totals upward.
__device__ __forceinline__ int wave_incl_scan(int v)
{
    uint32_t u = uint32_t(v);
    u += dpp_u32<0x111, 0xF>(u);
    u += dpp_u32<0x112, 0xF>(u);
    u += dpp_u32<0x114, 0xF>(u);
    u += dpp_u32<0x118, 0xF>(u);
    u += dpp_u32<0x142, 0xA>(u);
    u += dpp_u32<0x143, 0xC>(u);
    return int(u);
}

// Value of lane j (wave-uniform j), read into a scalar register.
__device__ __forceinline__ float lane_get(float v, int j)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}

// Inclusive prefix maximum over the wave's lanes of values >= 0 (0 acts as
// "nothing yet"), in registers.
__device__ __forceinline__ uint32_t wave_incl_umax(uint32_t u)
{
    u = max(u, dpp_u32<0x111, 0xF>(u));
    u = max(u, dpp_u32<0x112, 0xF>(u));
    u = max(u, dpp_u32<0x114, 0xF>(u));
    u = max(u, dpp_u32<0x118, 0xF>(u));
    u = max(u, dpp_u32<0x142, 0xA>(u));
    u = max(u, dpp_u32<0x143, 0xC>(u));
    return u;
}

// ---------------------------------------------------------------------------
// Bounding cube for Morton keys.
__global__ __launch_bounds__(256) void k_bbox_partial(const double* __restrict__ pos, int64_t n,
                                                      double* __restrict__ part)
{
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        for (int a = 0; a < 3; ++a) {
            double v = pos[3 * i + a];
            lo[a] = fmin(lo[a], v);
            hi[a] = fmax(hi[a], v);
        }
    __shared__ double s[6][4];
    for (int a = 0; a < 3; ++a) {
        for (int d = 32; d >= 1; d >>= 1) {
            lo[a] = fmin(lo[a], __shfl_xor(lo[a], d));
            hi[a] = fmax(hi[a], __shfl_xor(hi[a], d));
        }
    }
    int w = threadIdx.x >> 6;
    if (lane_id() == 0)
        for (int a = 0; a < 3; ++a) { s[a][w] = lo[a]; s[3 + a][w] = hi[a]; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int a = 0; a < 3; ++a) {
            double l = s[a][0], h = s[3 + a][0];
            for (int k = 1; k < 4; ++k) { l = fmin(l, s[a][k]); h = fmax(h, s[3 + a][k]); }
            part[6 * blockIdx.x + a] = l;
            part[6 * blockIdx.x + 3 + a] = h;
        }
    }
}

// Scalars the host reads after a build stage, gathered into one buffer so
// that one copy brings them back: a 4- or 8-byte value, or the maximum of n
// binary64 values (h maxima).  A null source reads as 0.  One block.
constexpr int kReadbackMax = 8;
struct ReadbackArgs {
    const void* src[kReadbackMax];
    int64_t n[kReadbackMax];      // -4: uint32 value, -8: uint64 value, n >= 0: max of n doubles
    int cnt;
};

__global__ __launch_bounds__(256) void k_readback(ReadbackArgs a, uint64_t* __restrict__ dst)
{
    __shared__ double red[256];
    for (int i = 0; i < a.cnt; ++i) {
        const int64_t n = a.n[i];
        if (n < 0) {
            if (threadIdx.x == 0) {
                uint64_t v = 0;
                if (a.src[i]) v = n == -8 ? *static_cast<const uint64_t*>(a.src[i]) : *static_cast<const uint32_t*>(a.src[i]);
                dst[i] = v;
            }
            continue;
        }
        const double* x = static_cast<const double*>(a.src[i]);
        double m = 0.0;
        if (x)
            for (int64_t k = threadIdx.x; k < n; k += 256) m = fmax(m, x[k]);
        red[threadIdx.x] = m;
        __syncthreads();
        for (int w = 128; w >= 1; w >>= 1) {
            if (int(threadIdx.x) < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
            __syncthreads();
        }
        if (threadIdx.x == 0) dst[i] = uint64_t(__double_as_longlong(red[0]));
        __syncthreads();
    }
}

// cube[0..2] = origin, cube[3] = 2^21 / side (quantisation scale).  One wave.
__global__ __launch_bounds__(64) void k_bbox_final(const double* __restrict__ part, int nparts,
                                                   const double* __restrict__ boxL, double* __restrict__ cube)
{
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a) { lo[a] = 1e300; hi[a] = -1e300; }
    for (int k = lane_id(); k < nparts; k += 64)
        for (int a = 0; a < 3; ++a) {
            lo[a] = fmin(lo[a], part[6 * k + a]);
            hi[a] = fmax(hi[a], part[6 * k + 3 + a]);
        }
    for (int a = 0; a < 3; ++a)
        for (int d = 32; d >= 1; d >>= 1) {
            lo[a] = fmin(lo[a], __shfl_xor(lo[a], d));
            hi[a] = fmax(hi[a], __shfl_xor(hi[a], d));
        }
    if (lane_id() != 0) return;
    bool periodic = boxL[0] > 0.0;
    double side = 0.0;
    for (int a = 0; a < 3; ++a) {
        if (periodic) { lo[a] = 0.0; hi[a] = boxL[a]; }
        side = fmax(side, hi[a] - lo[a]);
    }
    side = side > 0.0 ? side * (1.0 + 1e-9) + 1e-300 : 1.0;
    for (int a = 0; a < 3; ++a) cube[a] = lo[a];
    cube[3] = 2097152.0 / side;
}

__device__ __forceinline__ uint64_t spread21(uint64_t x)
{
    x &= 0x1fffffull;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

// Morton key of each particle (input order), plus a packed copy of its
// position (wrapped into [0, L) when periodic) and h, so that the gather into
// Morton order (in k_subtile_write) reads one 32-byte record per particle.
__global__ __launch_bounds__(256) void k_morton(const double* __restrict__ pos, const double* __restrict__ h, int64_t n,
                                                const double* __restrict__ cube, const double* __restrict__ boxL,
                                                uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                double4* __restrict__ rec)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t q[3];
    double p[3];
    for (int a = 0; a < 3; ++a) {
        double x = pos[3 * i + a];
        if (boxL[a] > 0.0) x -= boxL[a] * floor(x / boxL[a]);
        p[a] = x;
        double f = (x - cube[a]) * cube[3];
        f = fmin(fmax(f, 0.0), 2097151.0);
        q[a] = uint64_t(f);
    }
    keys[i] = spread21(q[0]) | (spread21(q[1]) << 1) | (spread21(q[2]) << 2);
    vals[i] = uint32_t(i);
    rec[i] = make_double4(p[0], p[1], p[2], h[i]);
}

__global__ __launch_bounds__(256) void k_active_flags(const uint32_t* __restrict__ perm, int64_t n,
                                                      const uint8_t* __restrict__ active, uint32_t* __restrict__ flag)
{
    int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k > n) return;
    flag[k] = (k < n) ? (active ? (active[perm[k]] != 0 ? 1u : 0u) : 1u) : 0u;
}

__global__ __launch_bounds__(256) void k_compact(const uint32_t* __restrict__ flag, const uint32_t* __restrict__ off,
                                                 int64_t n, uint32_t* __restrict__ own)
{
    int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k < n && flag[k]) own[off[k]] = uint32_t(k);
}

// Tile bounds: one wave per tile of 64 consecutive entries of `list`
// (identity when list == nullptr).  box = {lo xyz, hi xyz}, hmax.
__global__ __launch_bounds__(64) void k_tile_bounds(const uint32_t* __restrict__ list, int64_t n,
                                                    const double* __restrict__ sx, const double* __restrict__ sy,
                                                    const double* __restrict__ sz, const double* __restrict__ sh,
                                                    double* __restrict__ box, double* __restrict__ hmax)
{
    int64_t t = blockIdx.x;
    int64_t k = t * kTile + lane_id();
    bool v = k < n;
    int64_t p = v ? (list ? int64_t(list[k]) : k) : 0;
    double x = v ? sx[p] : 1e300, y = v ? sy[p] : 1e300, z = v ? sz[p] : 1e300;
    double X = v ? sx[p] : -1e300, Y = v ? sy[p] : -1e300, Z = v ? sz[p] : -1e300;
    double hh = v ? sh[p] : 0.0;
    // minima / maxima over the wave in registers; totals at lane 63
    seg_scan_up(lane_id(), 0, [&](auto ctl, auto rows, bool take) {
        constexpr int C = decltype(ctl)::value, R = decltype(rows)::value;
        x = dpp_take_min<C, R>(x, take); y = dpp_take_min<C, R>(y, take); z = dpp_take_min<C, R>(z, take);
        X = dpp_take_max<C, R>(X, take); Y = dpp_take_max<C, R>(Y, take); Z = dpp_take_max<C, R>(Z, take);
        hh = dpp_take_max<C, R>(hh, take);
    });
    if (lane_id() == 63) {
        box[6 * t + 0] = x; box[6 * t + 1] = y; box[6 * t + 2] = z;
        box[6 * t + 3] = X; box[6 * t + 4] = Y; box[6 * t + 5] = Z;
        hmax[t] = hh;
    }
}

// Binary32 copy of a node's bounds for the candidate search, rounded
// outward: q[0] = (box lo, max h), q[1] = (box hi, 0), q[2] = (support lo, 0),
// q[3] = (support hi, 0).
__device__ __forceinline__ void write_node_q(float4* q, const double b[6], double hm, const double u[6])
{
    q[0] = make_float4(__double2float_rd(b[0]), __double2float_rd(b[1]), __double2float_rd(b[2]), __double2float_ru(hm));
    q[1] = make_float4(__double2float_ru(b[3]), __double2float_ru(b[4]), __double2float_ru(b[5]), 0.f);
    q[2] = make_float4(__double2float_rd(u[0]), __double2float_rd(u[1]), __double2float_rd(u[2]), 0.f);
    q[3] = make_float4(__double2float_ru(u[3]), __double2float_ru(u[4]), __double2float_ru(u[5]), 0.f);
}

// Super-tile bounds over 64 consecutive tiles: box, max h, support box.
__global__ __launch_bounds__(64) void k_super_bounds(int64_t ntile, const double* __restrict__ tbox,
                                                     const double* __restrict__ th, const double* __restrict__ tsup,
                                                     double* __restrict__ box, double* __restrict__ hmax,
                                                     double* __restrict__ sup, float4* __restrict__ q)
{
    int64_t s = blockIdx.x;
    int64_t t = s * kTile + lane_id();
    bool v = t < ntile;
    double b[6], u[6];
    for (int a = 0; a < 3; ++a) {
        b[a] = v ? tbox[6 * t + a] : 1e300;
        b[3 + a] = v ? tbox[6 * t + 3 + a] : -1e300;
        u[a] = v ? tsup[6 * t + a] : 1e300;
        u[3 + a] = v ? tsup[6 * t + 3 + a] : -1e300;
    }
    double hh = v ? th[t] : 0.0;
    seg_scan_up(lane_id(), 0, [&](auto ctl, auto rows, bool take) {
        constexpr int C = decltype(ctl)::value, R = decltype(rows)::value;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            b[a] = dpp_take_min<C, R>(b[a], take);
            b[3 + a] = dpp_take_max<C, R>(b[3 + a], take);
            u[a] = dpp_take_min<C, R>(u[a], take);
            u[3 + a] = dpp_take_max<C, R>(u[3 + a], take);
        }
        hh = dpp_take_max<C, R>(hh, take);
    });
    if (lane_id() == 63) {
        for (int a = 0; a < 6; ++a) { box[6 * s + a] = b[a]; sup[6 * s + a] = u[a]; }
        hmax[s] = hh;
        write_node_q(q + 4 * s, b, hh, u);
    }
}

// Sub-tiles of the "other" role: each chunk of 64 Morton-consecutive
// particles is cut wherever two neighbours in the order differ at a Morton
// level coarser than the chunk's median neighbour level minus one, so that a
// chunk straddling a coarse cell boundary becomes several compact boxes.
// Returns the mask of lanes that start a sub-tile.  `lo_bit` masks key bits
// the sort did not order.
__device__ __forceinline__ uint64_t subtile_cuts(const uint64_t* __restrict__ keys, int64_t n, int lo_bit,
                                                 int cut_delta, int64_t c)
{
    const int lane = lane_id();
    const int64_t k = c * kTile + lane;
    const bool valid = k < n;
    const int m = int(min<int64_t>(kTile, n - c * kTile));
    const uint64_t key = valid ? (keys[k] >> lo_bit) : 0ull;
    const uint64_t prev = __shfl_up(key, 1);
    int lvl = 22;
    if (valid && lane > 0) {
        uint64_t x = (prev ^ key) << lo_bit;       // differing sorted bits, in place
        lvl = x == 0ull ? 21 : (__clzll((long long)x) - 1) / 3;
    }
    // median neighbour level over lanes 1..m-1
    int med = 0;
    const int need = m / 2;
    for (int t = 21; t >= 0; --t) {
        int cntt = __popcll(__ballot(valid && lane > 0 && lvl >= t));
        if (cntt >= need) { med = t; break; }
    }
    return __ballot(valid && (lane == 0 || lvl < med - cut_delta));
}

// cnt[c] = number of sub-tiles of chunk c.
__global__ __launch_bounds__(64) void k_subtile_count(const uint64_t* __restrict__ keys, int64_t n, int lo_bit,
                                                      int cut_delta, uint32_t* __restrict__ cnt)
{
    const uint64_t cm = subtile_cuts(keys, n, lo_bit, cut_delta, blockIdx.x);
    if (lane_id() == 0) cnt[blockIdx.x] = uint32_t(__popcll(cm));
}

// Support box of one particle coordinate: [x - h, x + h] widened by a few
// units in the last place, so that it holds the exact interval.
__device__ __forceinline__ double sup_lo(double x, double h) { const double v = x - h; return v - 4e-16 * fabs(v); }
__device__ __forceinline__ double sup_hi(double x, double h) { const double v = x + h; return v + 4e-16 * fabs(v); }

// Starts, counts and bounds of the sub-tiles of chunk c at off[c]...: box,
// max h and support box (union of the particles' [x - h, x + h]), each a
// segmented reduction over the sub-tile's run of lanes.  Also writes the
// chunk's sorted SoA position and h, gathered from the packed records.
__global__ __launch_bounds__(64) void k_subtile_write(const uint64_t* __restrict__ keys, int64_t n, int lo_bit,
                                                      int cut_delta, const uint32_t* __restrict__ off,
                                                      uint32_t* __restrict__ sub_start, uint32_t* __restrict__ sub_cnt,
                                                      const uint32_t* __restrict__ perm,
                                                      const double4* __restrict__ rec, double* __restrict__ sx,
                                                      double* __restrict__ sy, double* __restrict__ sz,
                                                      double* __restrict__ sh, double* __restrict__ box,
                                                      double* __restrict__ hmax, double* __restrict__ sup,
                                                      float4* __restrict__ q)
{
    const int lane = lane_id();
    const int64_t c = blockIdx.x;
    const int64_t k = c * kTile + lane;
    const int m = int(min<int64_t>(kTile, n - c * kTile));
    const uint64_t cm = subtile_cuts(keys, n, lo_bit, cut_delta, c);
    const uint64_t above = lane == 63 ? 0ull : (cm >> (lane + 1));
    const int next = above ? lane + __ffsll((unsigned long long)above) : m;
    const bool valid = lane < m;
    // first lane of this lane's sub-tile (a run of lanes); lanes past the chunk end stand alone
    const uint64_t upto = cm & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
    const int lo = valid && upto ? 63 - __clzll(upto) : lane;
    const int64_t kk = valid ? k : c * kTile;
    const double4 r = rec[perm[kk]];
    if (valid) { sx[k] = r.x; sy[k] = r.y; sz[k] = r.z; sh[k] = r.w; }
    const double x3[3] = {r.x, r.y, r.z};
    const double hh = r.w;
    double b[6], u[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        b[a] = x3[a];
        b[3 + a] = x3[a];
        u[a] = sup_lo(x3[a], hh);
        u[3 + a] = sup_hi(x3[a], hh);
    }
    double hm = hh;
    // segmented minima / maxima over each run, in registers; totals at the run's last lane
    seg_scan_up(lane, lo, [&](auto ctl, auto rows, bool take) {
        constexpr int C = decltype(ctl)::value, R = decltype(rows)::value;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            b[a] = dpp_take_min<C, R>(b[a], take);
            b[3 + a] = dpp_take_max<C, R>(b[3 + a], take);
            u[a] = dpp_take_min<C, R>(u[a], take);
            u[3 + a] = dpp_take_max<C, R>(u[3 + a], take);
        }
        hm = dpp_take_max<C, R>(hm, take);
    });
    if (valid && lane == next - 1) {
        const uint64_t lt = lo == 0 ? 0ull : (~0ull >> (64 - lo));
        const int64_t idx = int64_t(off[c]) + __popcll(cm & lt);
        sub_start[idx] = uint32_t(c * kTile + lo);
        sub_cnt[idx] = uint32_t(next - lo);
#pragma unroll
        for (int a = 0; a < 6; ++a) { box[6 * idx + a] = b[a]; sup[6 * idx + a] = u[a]; }
        hmax[idx] = hm;
        write_node_q(q + 4 * idx, b, hm, u);
    }
}

// Squared gap between two boxes (minimum over periodic images).
__device__ __forceinline__ double box_gap2(const double* A, const double* B, const double* L)
{
    double g2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        double gap = fmax(0.0, fmax(B[a] - A[3 + a], A[a] - B[3 + a]));
        if (L[a] > 0.0) {
            double gp = fmax(0.0, fmax(B[a] + L[a] - A[3 + a], A[a] - B[3 + a] - L[a]));
            double gm = fmax(0.0, fmax(B[a] - L[a] - A[3 + a], A[a] - B[3 + a] + L[a]));
            gap = fmin(gap, fmin(gp, gm));
        }
        g2 += gap * gap;
    }
    return g2;
}

__device__ __forceinline__ bool boxes_near(const double* A, double ha, const double* B, double hb, const double* L)
{
    double reach = (ha + hb) * (1.0 + 1e-12);
    return box_gap2(A, B, L) < reach * reach;
}

// Owner box A (max h ha) against the support box Bs of some other particles:
// a pair can interact (|a - b| < h_a + h_b) only if a lies within h_a of b's
// support, so only if the gap is below ha.
__device__ __forceinline__ bool reach_near(const double* A, double ha, const double* Bs, const double* L)
{
    const double r = ha * (1.0 + 1e-12);
    return box_gap2(A, Bs, L) < r * r;
}

// Gap along one axis between [alo, ahi] and [blo, bhi] (minimum over the
// periodic images when L > 0).
__device__ __forceinline__ float axis_gap(float alo, float ahi, float blo, float bhi, float L)
{
    float g = fmaxf(0.f, fmaxf(blo - ahi, alo - bhi));
    if (L > 0.f) {
        const float gp = fmaxf(0.f, fmaxf(blo + L - ahi, alo - bhi - L));
        const float gm = fmaxf(0.f, fmaxf(blo - L - ahi, alo - bhi + L));
        g = fminf(g, fminf(gp, gm));
    }
    return g;
}

// Owner box (alo, ahi; ah = max h) against node q (write_node_q layout): both
// necessary conditions of some pair being within h_a + h_b, the Euclidean
// box gap below ah + max h of the node and the gap to the node's support box
// below ah.  Binary32 on outward-rounded bounds: the gaps' rounding is below
// 1e-5 of the reach, and `dL` (a few units in the last place of the box side)
// covers the rounding of the periodic image shifts.
__device__ __forceinline__ bool node_near(float4 alo, float4 ahi, float ah, const float4* __restrict__ q,
                                          const float L[3], float dL)
{
    const float4 lo = q[0], hi = q[1], slo = q[2], shi = q[3];
    const float g1x = axis_gap(alo.x, ahi.x, lo.x, hi.x, L[0]), g1y = axis_gap(alo.y, ahi.y, lo.y, hi.y, L[1]),
                g1z = axis_gap(alo.z, ahi.z, lo.z, hi.z, L[2]);
    const float g2x = axis_gap(alo.x, ahi.x, slo.x, shi.x, L[0]), g2y = axis_gap(alo.y, ahi.y, slo.y, shi.y, L[1]),
                g2z = axis_gap(alo.z, ahi.z, slo.z, shi.z, L[2]);
    const float r1 = fmaf(ah + lo.w, 1e-5f, ah + lo.w) + dL, r2 = fmaf(ah, 1e-5f, ah) + dL;
    return fmaf(g1x, g1x, fmaf(g1y, g1y, g1z * g1z)) < r1 * r1 && fmaf(g2x, g2x, fmaf(g2y, g2y, g2z * g2z)) < r2 * r2;
}

// Candidate search, in three steps.  (1) k_cand: candidate other super-tiles
// (64 consecutive sub-tiles) of each owner tile, culled through two levels of
// binary32 nodes (64 super-tiles per mega-tile).  count mode: cnt[t] = number
// of candidates; write mode: the flat list of (owner tile, super-tile) pairs,
// tile t's at off[t]..., in mega, super-tile order.  (2) k_sub_masks: for
// every pair, the super-tile's sub-tiles that pass the same node check
// against the owner tile, as a 64-bit mask.  (3) k_expand: the masks' set
// bits become each tile's candidate sub-tile list (ascending within a pair).
// Splitting the levels keeps the per-tile work short: one owner tile whose
// box spans much of the domain no longer holds up a whole launch.
// Owner tiles come in groups of 64 consecutive tiles; a first count pass over
// the groups (union box, max h) keeps each group's candidate list, and a
// tile whose group list fits tests only that list's super-tiles.  The node
// test only passes more easily as the owner box grows and h rises, so the
// group list holds every candidate of its tiles, in the same ascending
// order as the full traversal gives.
struct CandArgs {
    int64_t nown_tile, ntile, nsuper, nmega;
    const double* obox; const double* oh;
    const float4* sq; const float4* mq;   // binary32 nodes (write_node_q): super-, mega-tiles
    double L[3];
    uint32_t* cnt;
    const uint64_t* off;          // candidate offsets can pass 2^32 at Milky-Way sizes
    uint32_t* cand;
    uint32_t* pad;                // [owner tiles][pad_cap]: the count pass keeps the first pad_cap candidates
    int pad_cap;
    uint32_t* maxcnt;             // largest count (count pass)
    uint32_t* ptile;              // write mode: owner tile of each pair
    const uint32_t* gcnt;         // per group of 64 owner tiles: candidate count (nullptr: no group lists)
    const uint32_t* glist;        // [groups][gcap]: the group's candidates, valid when gcnt <= gcap
    int gcap;
};

constexpr int kCandUnroll = 4;     // independent node tests in flight per lane

// Owner tile of block b in a grid of 8 ceil(n / 8) blocks: XCD b % 8 takes a
// contiguous range of tiles, so neighbouring tiles (which share most of their
// candidates) meet in one L2.  Returns -1 for the padding blocks.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t n)
{
    const int64_t per = (n + kXcd - 1) / kXcd;
    const int64_t t = (b % kXcd) * per + b / kXcd;
    return t < n ? t : -1;
}

// The near megas' super-tiles are tested kCandUnroll megas at a time (their
// node loads overlap).  The count pass also stores the first pad_cap
// candidates of each tile; the lists stay there when all fit, else the write
// pass copies the fitting ones and traverses again for the others.
template <bool WRITE>
__global__ __launch_bounds__(64) void k_cand(CandArgs a)
{
    const int64_t t = xcd_tile(blockIdx.x, a.nown_tile);
    if (t < 0) return;
    const int lane = lane_id();
    if (WRITE && a.cnt[t] <= uint32_t(a.pad_cap)) {
        const uint32_t n = a.cnt[t];
        const uint32_t* src = a.pad + t * int64_t(a.pad_cap);
        uint32_t* dst = a.cand + a.off[t];
        uint32_t* dt = a.ptile + a.off[t];
        for (uint32_t k = uint32_t(lane); k < n; k += 64) { dst[k] = src[k]; dt[k] = uint32_t(t); }
        return;
    }
    uint32_t* pad = a.pad + t * int64_t(a.pad_cap);
    const float4 alo = make_float4(__double2float_rd(a.obox[6 * t + 0]), __double2float_rd(a.obox[6 * t + 1]),
                                   __double2float_rd(a.obox[6 * t + 2]), 0.f);
    const float4 ahi = make_float4(__double2float_ru(a.obox[6 * t + 3]), __double2float_ru(a.obox[6 * t + 4]),
                                   __double2float_ru(a.obox[6 * t + 5]), 0.f);
    const float ah = __double2float_ru(a.oh[t]);
    const float Lf[3] = {__double2float_ru(a.L[0]), __double2float_ru(a.L[1]), __double2float_ru(a.L[2])};
    const float dL = 1e-6f * fmaxf(Lf[0], fmaxf(Lf[1], Lf[2]));
    uint32_t count = 0;
    const uint64_t base = WRITE ? a.off[t] : 0ull;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const uint32_t gn = a.gcnt ? a.gcnt[t / kTile] : ~0u;
    if (gn <= uint32_t(a.gcap)) {
        // the group's candidates, kCandUnroll rounds of 64 at a time
        const uint32_t* gl = a.glist + (t / kTile) * int64_t(a.gcap);
        for (uint32_t k0 = 0; k0 < gn; k0 += 64 * kCandUnroll) {
            bool ok[kCandUnroll], hit[kCandUnroll];
            int64_t sg[kCandUnroll];
            float4 nq[kCandUnroll][4];
#pragma unroll
            for (int u = 0; u < kCandUnroll; ++u) {     // loads first, all in flight
                const uint32_t k = k0 + uint32_t(u * 64 + lane);
                ok[u] = k < gn;
                sg[u] = ok[u] ? int64_t(gl[k]) : 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) nq[u][q] = a.sq[4 * sg[u] + q];
            }
#pragma unroll
            for (int u = 0; u < kCandUnroll; ++u) hit[u] = ok[u] && node_near(alo, ahi, ah, nq[u], Lf, dL);
#pragma unroll
            for (int u = 0; u < kCandUnroll; ++u) {
                const uint64_t b = __ballot(hit[u]);
                const uint32_t k = count + uint32_t(__popcll(b & lt));
                if (WRITE && hit[u]) { a.cand[base + k] = uint32_t(sg[u]); a.ptile[base + k] = uint32_t(t); }
                if (!WRITE && hit[u] && k < uint32_t(a.pad_cap)) pad[k] = uint32_t(sg[u]);
                count += uint32_t(__popcll(b));
            }
        }
    }
    for (int64_t m0 = 0; gn > uint32_t(a.gcap) && m0 < a.nmega; m0 += 64) {
        const int64_t mg = m0 + lane;
        const bool hm = mg < a.nmega && node_near(alo, ahi, ah, a.mq + 4 * mg, Lf, dL);
        uint64_t bm = __ballot(hm);
        while (bm) {
            int64_t mi[kCandUnroll];
            bool mv[kCandUnroll];
#pragma unroll
            for (int u = 0; u < kCandUnroll; ++u) {
                mv[u] = bm != 0ull;
                mi[u] = mv[u] ? m0 + __ffsll((unsigned long long)bm) - 1 : m0;
                bm &= bm - 1;
            }
            bool hit[kCandUnroll];
            int64_t sg[kCandUnroll];
            float4 nq[kCandUnroll][4];
#pragma unroll
            for (int u = 0; u < kCandUnroll; ++u) {     // loads first, all in flight
                sg[u] = mi[u] * kTile + lane;
                const int64_t si = sg[u] < a.nsuper ? sg[u] : 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) nq[u][k] = a.sq[4 * si + k];
            }
#pragma unroll
            for (int u = 0; u < kCandUnroll; ++u)
                hit[u] = mv[u] && sg[u] < a.nsuper && node_near(alo, ahi, ah, nq[u], Lf, dL);
#pragma unroll
            for (int u = 0; u < kCandUnroll; ++u) {
                const uint64_t b = __ballot(hit[u]);
                const uint32_t k = count + uint32_t(__popcll(b & lt));
                if (WRITE && hit[u]) { a.cand[base + k] = uint32_t(sg[u]); a.ptile[base + k] = uint32_t(t); }
                if (!WRITE && hit[u] && k < uint32_t(a.pad_cap)) pad[k] = uint32_t(sg[u]);
                count += uint32_t(__popcll(b));
            }
        }
    }
    if (!WRITE && lane == 0) {
        a.cnt[t] = count;
        // one word shared by every tile: skip the atomic unless it can raise it
        if (count > __hip_atomic_load(a.maxcnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(a.maxcnt, count);
    }
}

struct SubMaskArgs {
    int64_t npairs, ntile;
    const uint32_t* ptile; const uint32_t* psup;   // pairs: owner tile, candidate super-tile
    const double* obox; const double* oh;          // owner tiles
    const float4* tq;                              // sub-tile nodes (write_node_q layout)
    double L[3];
    const uint32_t* sub_cnt;                       // particles per sub-tile
    uint64_t* mask; uint32_t* pcnt; uint32_t* pw;  // per pair: sub-tile mask, its count and its particles
};

constexpr int kSubPairs = 4;       // pairs per wave, their node loads in flight together

__global__ __launch_bounds__(64) void k_sub_masks(SubMaskArgs a)
{
    const int lane = lane_id();
    const int64_t p0 = int64_t(blockIdx.x) * kSubPairs;
    const float Lf[3] = {__double2float_ru(a.L[0]), __double2float_ru(a.L[1]), __double2float_ru(a.L[2])};
    const float dL = 1e-6f * fmaxf(Lf[0], fmaxf(Lf[1], Lf[2]));
    float4 nq[kSubPairs][4];
    int64_t st[kSubPairs], tl[kSubPairs];
    int sc[kSubPairs];
#pragma unroll
    for (int u = 0; u < kSubPairs; ++u) {     // loads first, all in flight
        const int64_t p = p0 + u < a.npairs ? p0 + u : 0;
        tl[u] = a.ptile[p];
        st[u] = int64_t(a.psup[p]) * kTile + lane;
        const int64_t si = st[u] < a.ntile ? st[u] : 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) nq[u][k] = a.tq[4 * si + k];
        sc[u] = int(a.sub_cnt[si]);
    }
#pragma unroll
    for (int u = 0; u < kSubPairs; ++u) {
        const int64_t t = tl[u];
        const float4 alo = make_float4(__double2float_rd(a.obox[6 * t + 0]), __double2float_rd(a.obox[6 * t + 1]),
                                       __double2float_rd(a.obox[6 * t + 2]), 0.f);
        const float4 ahi = make_float4(__double2float_ru(a.obox[6 * t + 3]), __double2float_ru(a.obox[6 * t + 4]),
                                       __double2float_ru(a.obox[6 * t + 5]), 0.f);
        const bool hit = p0 + u < a.npairs && st[u] < a.ntile &&
                         node_near(alo, ahi, __double2float_ru(a.oh[t]), nq[u], Lf, dL);
        const uint64_t m = __ballot(hit);
        const int w = wave_incl_scan(hit ? sc[u] : 0);
        if (lane == 0 && p0 + u < a.npairs) {
            a.mask[p0 + u] = m;
            a.pcnt[p0 + u] = uint32_t(__popcll(m));
        }
        if (lane == 63 && p0 + u < a.npairs) a.pw[p0 + u] = uint32_t(w);
    }
}

// Candidate sub-tiles of pair p at soff[p]... (ascending).
__global__ __launch_bounds__(256) void k_expand(int64_t npairs, const uint32_t* __restrict__ psup,
                                                const uint64_t* __restrict__ mask, const uint64_t* __restrict__ soff,
                                                uint32_t* __restrict__ cand)
{
    const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= npairs) return;
    uint64_t m = mask[p];
    const uint32_t s0 = psup[p] * uint32_t(kTile);
    uint32_t* dst = cand + soff[p];
    for (int k = 0; m; ++k, m &= m - 1) dst[k] = s0 + uint32_t(__ffsll((unsigned long long)m) - 1);
}

// Per owner tile: its candidate sub-tile count, where its list starts and
// the particles of its candidates (poff: pair offsets per tile, soff and
// woff: sub-tile and particle offsets per pair).
__global__ __launch_bounds__(256) void k_tile_subs(int64_t nt, const uint64_t* __restrict__ poff,
                                                   const uint64_t* __restrict__ soff, const uint64_t* __restrict__ woff,
                                                   uint32_t* __restrict__ scnt, uint64_t* __restrict__ sbeg,
                                                   uint32_t* __restrict__ swt)
{
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t > nt) return;
    if (t == nt) { scnt[t] = 0u; return; }
    const uint64_t b = soff[poff[t]], e = soff[poff[t + 1]];
    sbeg[t] = b;
    scnt[t] = uint32_t(e - b);
    swt[t] = uint32_t(min<uint64_t>(woff[poff[t + 1]] - woff[poff[t]], 0xFFFFFFFFull));
}

// Work items: each tile's candidate list cut into equal pieces of at most
// `split` sub-tiles.  A small problem (fewer than `target` x `split` candidate
// sub-tiles in all, `total`) gets a smaller piece size, down to kItemMinSplit,
// so that about `target` items keep every compute unit busy.
constexpr uint32_t kItemMinSplit = 4;
__global__ __launch_bounds__(256) void k_item_count(const uint32_t* __restrict__ cnt, int64_t nt, uint32_t split,
                                                    const uint64_t* __restrict__ total, uint32_t target,
                                                    uint32_t* __restrict__ icnt)
{
    int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t > nt) return;
    uint32_t s = split;
    if (target > 0 && split > kItemMinSplit) {
        const uint64_t want = (*total + target - 1) / target;
        s = uint32_t(max<uint64_t>(kItemMinSplit, min<uint64_t>(split, want)));
    }
    icnt[t] = t < nt ? (cnt[t] + s - 1) / s : 0u;
}

// Item it: its tile t (binary search over item_off), and the piece of t's
// list (cnt[t] sub-tiles from beg[t]) it covers: piece k of n holds
// candidates [k cnt / n, (k + 1) cnt / n).  Also a sort key that orders the
// items by decreasing candidate particles (wt: per tile; the item takes its
// share of the tile's), so that a pass starts the largest ones first and
// ends on small ones.
__global__ __launch_bounds__(256) void k_item_write(const uint64_t* __restrict__ beg, const uint32_t* __restrict__ cnt,
                                                    const uint32_t* __restrict__ wt,
                                                    const uint32_t* __restrict__ item_off, int64_t nt, int64_t nitems,
                                                    uint32_t* __restrict__ it_tile, uint64_t* __restrict__ it_cb,
                                                    uint64_t* __restrict__ it_ce, uint64_t* __restrict__ it_key,
                                                    uint32_t* __restrict__ it_id)
{
    const int64_t it = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (it >= nitems) return;
    int64_t lo = 0, hi = nt;      // largest t with item_off[t] <= it
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (int64_t(item_off[mid]) <= it) lo = mid; else hi = mid;
    }
    const uint64_t n = item_off[lo + 1] - item_off[lo], k = uint64_t(it - int64_t(item_off[lo])), c = cnt[lo];
    const uint64_t cb = k * c / n, ce = (k + 1) * c / n;
    it_tile[it] = uint32_t(lo);
    it_cb[it] = beg[lo] + cb;
    it_ce[it] = beg[lo] + ce;
    // 8-bit key, 1/12 octave per step: 255 for an empty item, smaller for larger ones
    const double w = double(wt[lo]) * double(ce - cb) / double(max<uint64_t>(c, 1));
    it_key[it] = 255u - uint32_t(fmin(255.0, 12.0 * log2(w + 1.0)));
    it_id[it] = uint32_t(it);
}

// ---------------------------------------------------------------------------
// Per-step gathers into sorted order.
// Per-pair data of the other species of a pass, one 16-byte-aligned record
// per sorted particle, so that a pair's reads are a few wide loads from one
// base pointer.
template <typename Real> struct alignas(16) GasRec {   // gas, read by the DM pass and the resolve
    double Vx, Vy, Vz;            // velocity
    Real vs, K, crit;             // sqrt(2 u / 3), K_j, P threshold
    uint32_t perm;                // sorted position -> gas index
};
template <typename Real> struct alignas(16) OwnRate {  // active gas in owner-slot order, read by the gas pass
    Real i2;                      // 1 / (2 vs^2) (infinite for cold gas)
    Real a, b;                    // alpha_n/3 vs^{n+1}, alpha_n vs^{n+3}
    Real r;                       // mu_j / (m_chi + mu_j)
};
template <typename Real> struct alignas(16) DmRec {    // DM, read by the gas pass (other) and the DM pass (owner)
    double vx, vy, vz;            // velocity
    Real m;                       // mass
    Real dt;                      // timestep
};

struct GasGatherArgs {
    int64_t n;
    const uint32_t* perm;
    const double* vel; const double* mass; const double* u; const double* mu;
    double m_chi, sig_kpc2_cn, alpha_n;
    int n_pow;
    int rb;                       // Rao-Blackwellised DM sampling: the record carries 1/(2 vs^2) and K alpha_{n-2} vs^{n+1}
    double alpha_rb;              // alpha_{n-2}
    double* Vx; double* Vy; double* Vz;
    const uint32_t* flag; const uint32_t* flag_off;         // active flags and their exclusive scan (sorted order)
    void* orate;                  // OwnRate<Real>[n_own], owner-slot order
    void* rec;                    // GasRec<Real>[n]
};

template <typename Real>
__device__ __forceinline__ void gas_derived(double u, double mu, double m_chi, double alpha_n, int n_pow,
                                            Real* vs, Real* inv2s2, Real* ra, Real* rb, Real* rr, Real* crit)
{
    double s2 = 2.0 * u / 3.0;
    double s = sqrt(s2);
    *vs = Real(s);
    *inv2s2 = Real(s2 > 0.0 ? 1.0 / (2.0 * s2) : INFINITY);
    *ra = Real(alpha_n / 3.0 * pow(s, double(n_pow + 1)));
    *rb = Real(alpha_n * pow(s, double(n_pow + 3)));
    *rr = Real(mu / (m_chi + mu));
    double q = (m_chi + mu) / mu;
    *crit = Real(fmin(0.1, 1e-4 * q * q));
}

template <typename Real>
__global__ __launch_bounds__(256) void k_gather_gas(GasGatherArgs a)
{
    int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    uint32_t o = a.perm[k];
    a.Vx[k] = a.vel[3 * int64_t(o)];
    a.Vy[k] = a.vel[3 * int64_t(o) + 1];
    a.Vz[k] = a.vel[3 * int64_t(o) + 2];
    double mu = a.mu ? a.mu[o] : kMpG;
    Real vs, i2, ra, rb, rr, cr;
    gas_derived<Real>(a.u[o], mu, a.m_chi, a.alpha_n, a.n_pow, &vs, &i2, &ra, &rb, &rr, &cr);
    if (a.flag[k]) {
        OwnRate<Real> w;
        w.i2 = i2; w.a = ra; w.b = rb; w.r = rr;
        reinterpret_cast<OwnRate<Real>*>(a.orate)[a.flag_off[k]] = w;
    }
    const double Kd = a.mass[o] * kMsunG / mu * a.sig_kpc2_cn;
    GasRec<Real> r;
    r.Vx = a.vel[3 * int64_t(o)]; r.Vy = a.vel[3 * int64_t(o) + 1]; r.Vz = a.vel[3 * int64_t(o) + 2];
    r.vs = vs; r.K = Real(Kd); r.crit = cr; r.perm = o;
    if (a.rb) {
        const double s = sqrt(2.0 * a.u[o] / 3.0);
        r.vs = i2;
        if (s > 0.0) r.K = Real(Kd * a.alpha_rb * pow(s, double(a.n_pow + 1)));
    }
    reinterpret_cast<GasRec<Real>*>(a.rec)[k] = r;
}

struct DmGatherArgs {
    int64_t n;
    const uint32_t* perm;
    const double* vel; const double* mass; const double* dt;
    double dt_default;
    void* rec;                    // DmRec<Real>[n]
};

template <typename Real>
__global__ __launch_bounds__(256) void k_gather_dm(DmGatherArgs a)
{
    int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    uint32_t o = a.perm[k];
    DmRec<Real> r;
    r.vx = a.vel[3 * int64_t(o)]; r.vy = a.vel[3 * int64_t(o) + 1]; r.vz = a.vel[3 * int64_t(o) + 2];
    r.m = Real(a.mass[o]);
    r.dt = Real(a.dt ? a.dt[o] : a.dt_default);
    reinterpret_cast<DmRec<Real>*>(a.rec)[k] = r;
}

__global__ __launch_bounds__(256) void k_fill_out(int64_t n_gas, int64_t n_dm, double* dp, double* de, double* dv,
                                                  int32_t* partner, double* psum, double* pmax, uint64_t* counters,
                                                  uint32_t* queues, int nqueues)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n_gas) {
        dp[3 * i] = 0.0; dp[3 * i + 1] = 0.0; dp[3 * i + 2] = 0.0;
        de[i] = 0.0;
    }
    if (i < n_dm) {
        dv[3 * i] = 0.0; dv[3 * i + 1] = 0.0; dv[3 * i + 2] = 0.0;
        partner[i] = -1;
        if (psum) psum[i] = 0.0;
        if (pmax) pmax[i] = 0.0;
    }
    if (i < 8 && counters) counters[i] = 0ull;
    if (i < nqueues) queues[i] = 0u;
}

// ---------------------------------------------------------------------------
// Pair passes.  One wavefront per block owns a tile of 64 owners (lane =
// owner) and walks its candidate sub-tiles of the other species in chunks of
// up to 64.  Test phase: each owner is checked against every sub-tile box of
// the chunk; the particles ("slots") of the sub-tiles some owner reaches are
// packed into groups of 64 (a sub-tile may straddle two groups), and one
// group is tested against all 64 owners at once as a dense binary32 product
// on the matrix cores (below), giving one 64-bit hit mask over the slots per
// owner.  Evaluate phase: the group's hits, ordered owner-major, are decoded
// 64 at a time (lane = pair); each lane repeats the test exactly in binary64
// and evaluates the pair; an owner's terms form a contiguous run of lanes, so
// a segmented scan in registers leaves each run's total on its last lane,
// which the owner lane pulls.  No atomics touch physical quantities.
constexpr float kTestMargin = 1.0f + 4e-6f;
// Slack of the expanded binary32 test |a-b|^2 - (ha+hb)^2 = A + B - 2 (a.b + ha hb)
// with A = |a|^2 - ha^2, B = |b|^2 - hb^2, in offsets from the owner tile's
// centre: evaluated as a six-term dot product (any summation order) its
// rounding error stays below 20 eps32 S ~ 1.2e-6 S, S = |a|^2 + ha^2 + |b|^2 + hb^2;
// subtracting kTestSlack S makes the test accept every pair with
// d^2 - (ha+hb)^2 < 2.8e-6 S.  As (ha+hb)^2 <= 2 S, that holds every pair inside
// in exact arithmetic and every pair of the near-boundary band
// |d^2/(ha+hb)^2 - 1| <= 1e-6, so the binary64 recheck sees all of them.
constexpr float kTestSlack = 4e-6f;

struct PassGeom {
    const uint32_t* own;          // owner slot -> sorted position (owner species)
    int64_t n_own;
    const double* ox; const double* oy; const double* oz; const double* oh;   // owner sorted pos/h
    const double* obox;           // owner tile boxes
    const double* tx; const double* ty; const double* tz; const double* th;   // other sorted pos/h
    int64_t n_other;
    const double* tbox;           // other sub-tile boxes
    const double* thmax;          // other sub-tile max h
    const uint32_t* sub_start; const uint32_t* sub_cnt;                       // other sub-tiles
    const uint32_t* cand;         // candidate other sub-tiles
    const uint32_t* it_tile; const uint64_t* it_cb; const uint64_t* it_ce;
    const uint32_t* item_off;     // [owner tiles + 1] item ranges per owner tile
    const uint32_t* item_order;   // items in the order they are dealt (largest first)
    int64_t n_items;
    uint32_t* queue_ctr;          // [kXcd] work counters
    double L[3];
    uint64_t* counters;
    // pair export (the PAIRS variants of the passes only): every visited pair
    // d_ij < h_i + h_j as (owner sorted index, other sorted index)
    uint32_t* pairs; unsigned long long* pair_n; uint64_t pair_cap;
};

// Appends this lane's pair (owner sorted index o, other sorted index q) to the
// export list when `take`: one counter atomic per wave, lanes in order.
__device__ __forceinline__ void pair_export(const PassGeom& G, bool take, uint32_t o, uint32_t q)
{
    const uint64_t m = __ballot(take);
    if (m == 0ull) return;
    const int lane = lane_id();
    unsigned long long base = 0ull;
    if (lane == __ffsll((long long)m) - 1) base = atomicAdd(G.pair_n, (unsigned long long)__popcll(m));
    base = __shfl(base, __ffsll((long long)m) - 1);
    const uint64_t pos = base + uint64_t(__popcll(m & ((1ull << lane) - 1ull)));
    if (take && pos < G.pair_cap) {
        G.pairs[2 * pos] = o;
        G.pairs[2 * pos + 1] = q;
    }
}

// Per tile pair: image shift of the other tile and whether every pair of
// particles is then at its minimum image (else per-pair minimum image).
__device__ __forceinline__ void tile_pair_shift(const double* A, const double* B, const double* L, double sh[3],
                                                bool* clean)
{
    bool ok = true;
    for (int a = 0; a < 3; ++a) {
        sh[a] = 0.0;
        if (L[a] > 0.0) {
            double ca = 0.5 * (A[a] + A[3 + a]), cb = 0.5 * (B[a] + B[3 + a]);
            sh[a] = L[a] * rint((ca - cb) / L[a]);
            double lo = A[a] - (B[3 + a] + sh[a]), hi = A[3 + a] - (B[a] + sh[a]);
            if (!(lo > -0.5 * L[a] && hi < 0.5 * L[a])) ok = false;
        }
    }
    *clean = ok;
}

// Minimum image along one axis.  The image index is rounded from d times 1/L
// (the reciprocal is loop-invariant, so no division per pair); it can differ
// from rounding d/L only where d/L lies within a few units in the last place
// of a half-integer, i.e. for separations near L/2, which no pair reaches
// (h_i + h_j < L/2 is required), so every pair keeps its distance bit for bit.
__device__ __forceinline__ double min_image(double d, double L) { return L > 0.0 ? d - L * rint(d * (1.0 / L)) : d; }
__device__ __forceinline__ float min_image_f(float d, float L) { return L > 0.f ? d - L * rintf(d * (1.f / L)) : d; }

// d^2 of owner (a) and other (b, already shifted); explicit evaluation order
// shared by every pass and by the resolve.
__device__ __forceinline__ double pair_d2(double ax, double ay, double az, double bx, double by, double bz,
                                          bool clean, const double* L)
{
    double dx = ax - bx, dy = ay - by, dz = az - bz;
    if (!clean) { dx = min_image(dx, L[0]); dy = min_image(dy, L[1]); dz = min_image(dz, L[2]); }
    return fma(dx, dx, fma(dy, dy, dz * dz));
}

// Work items are dealt to the 8 XCDs in chunks of kXcdChunk consecutive
// items (XCD x takes chunks x, x+8, ...), so neighbouring items share an L2
// while every XCD samples the whole domain; within an XCD, blocks take the
// next item from an atomic counter.
constexpr int kXcdChunk = 32;

template <int W = 1>
__device__ __forceinline__ bool item_next(uint32_t* queue_ctr, int64_t n_items, int64_t* it)
{
    const int x = blockIdx.x % kXcd;
    if constexpr (W == 1) {
        __shared__ int64_t s_it;
        if (threadIdx.x == 0) {
            const int64_t k = int64_t(atomicAdd(&queue_ctr[x], 1u));
            s_it = (k / kXcdChunk) * (int64_t(kXcd) * kXcdChunk) + int64_t(x) * kXcdChunk + (k % kXcdChunk);
        }
        __syncthreads();
        *it = s_it;
        __syncthreads();
    } else {
        int64_t v = 0;
        if (lane_id() == 0) {
            const int64_t k = int64_t(atomicAdd(&queue_ctr[x], 1u));
            v = (k / kXcdChunk) * (int64_t(kXcd) * kXcdChunk) + int64_t(x) * kXcdChunk + (k % kXcdChunk);
        }
        *it = __shfl(v, 0);
    }
    return *it < n_items;
}


// Bits [b, e) of a wave-uniform mask, tested for any set bit (0 <= b <= e <= 64).
__device__ __forceinline__ bool any_bits(uint64_t m, int b, int e)
{
    const int n = e - b;
    const uint64_t w = n >= 64 ? ~0ull : (1ull << n) - 1ull;
    return n > 0 && ((m >> b) & w) != 0ull;
}

// Index of the r-th set bit (r < popcount(m)).
__device__ __forceinline__ int select_bit(uint64_t m, int r)
{
    uint32_t w = uint32_t(m);
    int base = 0;
    int c = __popc(w);
    if (r >= c) { r -= c; w = uint32_t(m >> 32); base = 32; }
    c = __popc(w & 0xFFFFu); if (r >= c) { r -= c; w >>= 16; base += 16; }
    c = __popc(w & 0xFFu);   if (r >= c) { r -= c; w >>= 8; base += 8; }
    c = __popc(w & 0xFu);    if (r >= c) { r -= c; w >>= 4; base += 4; }
    c = __popc(w & 0x3u);    if (r >= c) { r -= c; w >>= 2; base += 2; }
    c = int(w & 1u);         if (r >= c) { base += 1; }
    return base;
}

// Per-wave LDS of the test phase.
struct TestLds {
    uint32_t dsh[64];             // periodic image of each chunk sub-tile: shift / L per axis, a signed byte each
    int dbase[64];                // first sorted index of each chunk sub-tile; bit 31: every pair of the
                                  // sub-tile is at its tile-level image (clean)
    int dpre[64], dincl[64];      // exclusive / inclusive slot prefix over the reached sub-tiles
    int sj[64];                   // slot -> chunk sub-tile (prefix-max scratch)
    double px[64], py[64], pz[64], ph[64];   // slot particles: shifted position and h
    uint32_t pq[64];              // slot -> sorted index of the other particle; bit 31: the slot's sub-tile is clean
    uint64_t mask[64];            // per owner lane: hit mask over the group's slots
    int offs[65];                 // owner-major offsets of the group's hits
};

// Test-phase state of one wave (owner lane values and the chunk/group cursor).
struct PairTest {
    bool ov;
    float fx, fy, fz, fh;         // owner offset from the tile centre and h (binary32)
    uint64_t c0, ce;              // next chunk start, end of the item's candidate list
    uint64_t actA, actB;          // chunk sub-tiles reached by some owner of lanes 0-31 / 32-63
    int total, Ps;                // slots of the chunk, start of the next group
};

typedef float f32x16 __attribute__((ext_vector_type(16)));

// Slot loaded by lane L.  In v_mfma_f32_32x32x2_f32 lane L supplies row L%32
// of A for K index L/32, and receives column L%32, rows 8(r/4) + 4(L/32) + r%4
// (r = 0..15) of D.  Rows of the slot tile st are slots
// 32 st + 16 ((i/4)%2) + 4 (i/8) + i%4, so lane L loads the slot of row L%32
// in tile L/32 and its 16 results of tile st are slots 32 st + 16 (L/32) + r.
__device__ __forceinline__ int slot_of_lane(int L)
{
    const int i = L & 31;
    return (L & 32) | (((i >> 2) & 1) << 4) | ((i >> 3) << 2) | (i & 3);
}

// e = A^T B over the three K steps; sign bits of the 16 results shifted into m
// (first result ends in the lowest of the 16 new bits).
__device__ __forceinline__ uint32_t mfma_signs(const float a[3], const float b[3], uint32_t m)
{
    f32x16 d = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    d = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0], b[0], d, 0, 0, 0);
    d = __builtin_amdgcn_mfma_f32_32x32x2f32(a[1], b[1], d, 0, 0, 0);
    d = __builtin_amdgcn_mfma_f32_32x32x2f32(a[2], b[2], d, 0, 0, 0);
#pragma unroll
    for (int r = 15; r >= 0; --r) m = __builtin_amdgcn_alignbit(m, __float_as_uint(d[r]), 31);
    __builtin_amdgcn_sched_barrier(0);    // one 16-register accumulator live at a time
    return m;
}

// The two 32-lane halves exchanged in one instruction (v_permlane32_swap):
// lo = (x of lanes 0-31, y of lanes 0-31 moved to lanes 32-63),
// hi = (x of lanes 32-63 moved to lanes 0-31, y of lanes 32-63).
__device__ __forceinline__ void halves_swap(uint32_t x, uint32_t y, uint32_t* lo, uint32_t* hi)
{
    const auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
    *lo = r[0];
    *hi = r[1];
}

// Operands of the product for K components (2 step + half) of two 32-lane
// halves: lanes 0-31 supply their own components 2 step, lanes 32-63 their own
// 2 step + 1, each half also receiving the other half's.  out[t][step] =
// operand for tile t.
__device__ __forceinline__ void half_operands(const float c[6], float out[2][3])
{
#pragma unroll
    for (int step = 0; step < 3; ++step) {
        uint32_t lo, hi;
        halves_swap(__float_as_uint(c[2 * step]), __float_as_uint(c[2 * step + 1]), &lo, &hi);
        out[0][step] = __uint_as_float(lo);
        out[1][step] = __uint_as_float(hi);
    }
}

__device__ __forceinline__ void test_begin(PairTest& T, bool ov, float fx, float fy, float fz, float fh, uint64_t cb,
                                           uint64_t ce)
{
    T.ov = ov; T.fx = fx; T.fy = fy; T.fz = fz; T.fh = fh;
    T.c0 = cb; T.ce = ce;
    T.actA = T.actB = 0ull;
    T.total = 0; T.Ps = 0;
}

// Next chunk of up to 64 candidate sub-tiles: descriptors to LDS (lane = sub-tile),
// per-owner reach check against each box, slot prefix over the reached ones.
// Every owner/sub-tile pair the per-pair test can accept passes the reach check:
// each candidate offset q lies in the binary32 box [lo, hi] (same rounding,
// monotone), so gap <= |p - q|, and an accepted pair has
// gap^2 < (fh + hb)^2 + (kTestSlack + 20 eps32) (|p|^2 + fh^2 + Q2 + hb^2), Q2 >= |q|^2,
// which the reach 6e-6 (...) below covers.
template <int W>
__device__ __forceinline__ void test_chunk(PairTest& T, TestLds& S, const PassGeom& G, const double* A,
                                           const double cen[3])
{
    const int lane = lane_id();
    const int nch = int(min<uint64_t>(64, T.ce - T.c0));
    stage_sync<W>();    // the previous chunk's groups are done with the descriptors
    int cnt = 0;
    // lane j holds chunk sub-tile j: box lo (offsets from the owner-tile centre) and max h,
    // box hi and the sub-tile's share of the reach slack, 6e-6 (Q2 + hmax^2), or -1 when the
    // sub-tile is not clean; the owner loop below reads them lane by lane
    float4 blo = make_float4(0.f, 0.f, 0.f, 0.f), bhi = make_float4(0.f, 0.f, 0.f, 0.f);
    if (lane < nch) {
        const uint32_t ot = G.cand[T.c0 + lane];
        const double* B = G.tbox + 6 * int64_t(ot);
        double Bx[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) Bx[k] = B[k];
        double sh[3];
        bool clean;
        tile_pair_shift(A, Bx, G.L, sh, &clean);
        blo = make_float4(float(Bx[0] + sh[0] - cen[0]), float(Bx[1] + sh[1] - cen[1]), float(Bx[2] + sh[2] - cen[2]),
                          float(G.thmax[ot]));
        bhi = make_float4(float(Bx[3] + sh[0] - cen[0]), float(Bx[4] + sh[1] - cen[1]), float(Bx[5] + sh[2] - cen[2]),
                          -1.f);
        if (clean) {
            const float Q2 = fmaxf(blo.x * blo.x, bhi.x * bhi.x) + fmaxf(blo.y * blo.y, bhi.y * bhi.y) +
                             fmaxf(blo.z * blo.z, bhi.z * bhi.z);
            bhi.w = 6e-6f * (Q2 + blo.w * blo.w);
        }
        uint32_t pk = 0u;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (G.L[a] > 0.0) pk |= (uint32_t(int(rint(sh[a] / G.L[a]))) & 255u) << (8 * a);
        S.dsh[lane] = pk;
        S.dbase[lane] = int(uint32_t(G.sub_start[ot]) | (clean ? 0x80000000u : 0u));
        cnt = int(G.sub_cnt[ot]);
    }
    T.c0 += uint64_t(nch);
    // the boxes go through LDS (the slot table, free until the chunk's first group is staged):
    // every lane then reads box j with two broadcast loads instead of eight lane reads
    float4* s_blo = reinterpret_cast<float4*>(S.px);
    float4* s_bhi = reinterpret_cast<float4*>(S.pz);
    s_blo[lane] = blo;
    s_bhi[lane] = bhi;
    stage_sync<W>();
    float fx = T.fx, fy = T.fy, fz = T.fz, fh = T.fh;     // opaque copies: not hoisted out of the item loop
    asm volatile("" : "+v"(fx), "+v"(fy), "+v"(fz), "+v"(fh));
    const float ao = 6e-6f * (fx * fx + fy * fy + fz * fz + fh * fh);   // the owner's share of the slack
    uint64_t actA = 0ull, actB = 0ull;
    for (int j = 0; j < nch; ++j) {
        const float4 lo = s_blo[j];
        const float4 hi = s_bhi[j];
        bool near = T.ov;
        if (hi.w >= 0.f) {
            const float gx = fmaxf(0.f, fmaxf(lo.x - fx, fx - hi.x));
            const float gy = fmaxf(0.f, fmaxf(lo.y - fy, fy - hi.y));
            const float gz = fmaxf(0.f, fmaxf(lo.z - fz, fz - hi.z));
            const float gap2 = fmaf(gx, gx, fmaf(gy, gy, gz * gz));
            const float hs = fh + lo.w;
            const float reach2 = fmaf(hs, hs, ao + hi.w) * (1.f + 1e-5f);
            near = T.ov && gap2 < reach2;
        }
        const uint64_t om = __ballot(near);
        if (uint32_t(om)) actA |= 1ull << j;
        if (om >> 32) actB |= 1ull << j;
    }
    T.actA = actA; T.actB = actB;
    const bool act = ((actA | actB) >> lane) & 1ull;
    const int ca = act ? cnt : 0;
    const int incl = wave_incl_scan(ca);
    S.dpre[lane] = incl - ca;
    S.dincl[lane] = incl;
    T.total = __shfl(incl, 63);
    T.Ps = 0;
}

// Test the next group of slots against the tile's owners.  Returns the group's
// hit count (wave-uniform), -1 when the item's candidates are exhausted.
template <int W>
__device__ __forceinline__ int test_next(PairTest& T, TestLds& S, const PassGeom& G, const double* A,
                                         const double cen[3], const float Lf[3])
{
    const int lane = lane_id();
    while (T.Ps >= T.total) {
        if (T.c0 >= T.ce) return -1;
        test_chunk<W>(T, S, G, A, cen);
    }
    stage_sync<W>();    // the previous group's decode is done with the slot table
    // reached sub-tiles whose slots overlap [Ps, Ps + 64): a contiguous run, the first of which
    // may have begun in the previous group and the last may go on in the next (full groups)
    const bool act = ((T.actA | T.actB) >> lane) & 1ull;
    const int pre = S.dpre[lane], inc = S.dincl[lane];
    const bool mem = act && inc > T.Ps && pre < T.Ps + 64;
    const uint64_t gm = __ballot(mem);
    const int end = min(S.dincl[63 - __clzll(gm)], T.Ps + 64);
    const int ns = end - T.Ps;
    const bool tileA = (T.actA & gm) != 0ull, tileB = (T.actB & gm) != 0ull;
    S.sj[lane] = 0;
    stage_sync<W>();
    if (mem) S.sj[max(pre - T.Ps, 0)] = lane + 1;
    stage_sync<W>();
    const int jm = int(wave_incl_umax(uint32_t(S.sj[lane]))) - 1;
    // lane L loads slot s
    const int s = slot_of_lane(lane);
    const int j = __shfl(jm, s);
    const bool sv = s < ns;
    int cl = 1;
    float c[6] = {0.f, 0.f, 0.f, 0.f, 1.f, __builtin_inff()};
    if (sv) {
        const uint32_t db = uint32_t(S.dbase[j]);
        const int64_t q = int64_t(db & 0x7fffffffu) + (s - (S.dpre[j] - T.Ps));
        cl = int(db >> 31);
        const uint32_t pk = S.dsh[j];
        const double X = G.tx[q] + double(int8_t(pk)) * G.L[0], Y = G.ty[q] + double(int8_t(pk >> 8)) * G.L[1],
                     Z = G.tz[q] + double(int8_t(pk >> 16)) * G.L[2];
        const double Hh = G.th[q];
        S.px[s] = X; S.py[s] = Y; S.pz[s] = Z; S.ph[s] = Hh;
        S.pq[s] = uint32_t(q) | (cl ? 0x80000000u : 0u);
        const float qx = float(X - cen[0]), qy = float(Y - cen[1]), qz = float(Z - cen[2]), qh = float(Hh);
        const float p2 = qx * qx + qy * qy + qz * qz, h2 = qh * qh;
        c[0] = -2.f * qx; c[1] = -2.f * qy; c[2] = -2.f * qz; c[3] = -2.f * qh;
        c[5] = (p2 - h2) - kTestSlack * (p2 + h2);
    }
    // owner terms are rebuilt per group: opaque copies keep the compiler from
    // hoisting them (they would stay live through the evaluate phase)
    float fx = T.fx, fy = T.fy, fz = T.fz, fh = T.fh;
    asm volatile("" : "+v"(fx), "+v"(fy), "+v"(fz), "+v"(fh));
    const float ap2 = fx * fx + fy * fy + fz * fz, ah2 = fh * fh;
    uint64_t m = 0ull;
    if (__ballot(!cl) == 0ull) {
        // e(slot, owner) = [-2q, -2qh, 1, B] . [p, ph, A, 1] on the matrix cores
        const float oc[6] = {T.ov ? fx : 0.f, T.ov ? fy : 0.f, T.ov ? fz : 0.f, T.ov ? fh : 0.f,
                             T.ov ? (ap2 - ah2) - kTestSlack * (ap2 + ah2) : __builtin_inff(), 1.f};
        float a[2][3], b[2][3];
        half_operands(c, a);
        half_operands(oc, b);
        uint32_t w0 = 0u, w1 = 0u;
        if (tileA) {
            if (ns > 32) w0 = mfma_signs(a[1], b[0], w0);
            w0 = mfma_signs(a[0], b[0], w0);
        }
        if (tileB) {
            if (ns > 32) w1 = mfma_signs(a[1], b[1], w1);
            w1 = mfma_signs(a[0], b[1], w1);
        }
        // w_t: owner 32 t + L%32 against slots 16 (L/32) + r (low half) and
        // 32 + 16 (L/32) + r (high half); owner L keeps w_{L/32}, the partner
        // supplies the other 32 slots
        uint32_t lo16, hi16;
        halves_swap(w0, w1, &lo16, &hi16);
        const uint32_t mlo = (lo16 & 0xffffu) | (hi16 << 16), mhi = (lo16 >> 16) | (hi16 & 0xffff0000u);
        m = (uint64_t(mhi) << 32) | mlo;
    } else {
        // some sub-tile needs the per-pair minimum image: owner lanes walk the slots
        stage_sync<W>();
        const float A2 = (ap2 - ah2) - kTestSlack * (ap2 + ah2);
        const float mx2 = -2.f * fx, my2 = -2.f * fy, mz2 = -2.f * fz, mh2 = -2.f * fh;
#pragma unroll 1
        for (int t = 0; t < ns; ++t) {
            const float4 q = make_float4(float(S.px[t] - cen[0]), float(S.py[t] - cen[1]), float(S.pz[t] - cen[2]),
                                         float(S.ph[t]));
            bool hit;
            if (S.pq[t] >> 31) {
                const float p2 = q.x * q.x + q.y * q.y + q.z * q.z, h2 = q.w * q.w;
                const float tb = (p2 - h2) - kTestSlack * (p2 + h2);
                hit = fmaf(mx2, q.x, fmaf(my2, q.y, fmaf(mz2, q.z, fmaf(mh2, q.w, A2 + tb)))) < 0.f;
            } else {
                const float dx = min_image_f(fx - q.x, Lf[0]), dy = min_image_f(fy - q.y, Lf[1]),
                            dz = min_image_f(fz - q.z, Lf[2]), hs = fh + q.w;
                hit = fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < hs * hs * kTestMargin;
            }
            if (T.ov && hit) m |= 1ull << t;
        }
    }
    S.mask[lane] = m;
    const int tot = __popcll(m);
    const int incl = wave_incl_scan(tot);
    S.offs[lane] = incl - tot;
    const int H = __shfl(incl, 63);
    if (lane == 63) S.offs[64] = H;
    T.Ps = end;
    stage_sync<W>();
    return H;
}

// Evaluation of a group's hits.  The hits are owner-major: owner o's are
// ranks [offs[o], offs[o+1]) of the group, its slots the set bits of mask[o]
// in increasing order.  With R = ceil(H / 64) rounds, lane l takes the
// contiguous ranks [l R, min((l + 1) R, H)), one per round, and keeps a
// running partial sum for the owner it is on.  When it takes an owner's last
// hit of the group it adds the partial to the owner's row of the item sums
// (in LDS) and moves to the next owner with hits; a lane whose range ends
// inside an owner's hits leaves an open partial, and the open partials of
// the lanes that share an owner are summed across lanes (segmented scan, lane
// order) and added by the last of them.  Each owner's last hit lies in one
// lane and one round, so the in-round adds touch distinct rows; every sum is
// formed in a fixed order, independent of timing.
struct HitWalk {
    int o;                        // owner of the lane's next hit (64: none)
    uint64_t rem;                 // slots of owner o not taken yet (the lane's next hit is the lowest)
    int n;                        // hits of the lane's range
    uint64_t own;                 // owners with hits in the group (wave-uniform)
};

// First owner with hits after owner o (64: none).
__device__ __forceinline__ int next_owner(uint64_t own, int o)
{
    const uint64_t m = own & ~((2ull << o) - 1ull);   // o = 63: 2 << 63 wraps to 0, m = 0
    return m ? int(__builtin_ctzll(m)) : 64;
}

// Lane ranges of a group with H > 0 hits in R rounds.  The owner of rank
// l R is the owner with hits whose first rank is the largest one <= l R:
// owner o marks lane ceil(offs[o] / R), the first lane whose range starts at
// or after its first hit (the largest owner wins a shared lane), and a prefix
// maximum over the lanes carries the marks upward.
__device__ __forceinline__ void walk_begin(TestLds& S, int lane, int H, int R, HitWalk& w)
{
    const int k0 = lane * R;
    w.n = max(0, min(R, H - k0));
    const int lo = S.offs[lane], hi = S.offs[lane + 1];
    w.own = __ballot(hi > lo);
    S.sj[lane] = 0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (hi > lo) {
        const int l0 = (lo + R - 1) / R;
        if (l0 < 64) atomicMax(&S.sj[l0], lane + 1);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    w.o = int(wave_incl_umax(uint32_t(S.sj[lane]))) - 1;
    w.rem = 0ull;
    if (w.n > 0) {
        const uint64_t m = S.mask[w.o];
        w.rem = m & (~0ull << select_bit(m, k0 - S.offs[w.o]));
    }
}

// Runs of lanes with the same key (open partials: the owner; others a key of
// their own): the first lane of this lane's run, and whether it is the last.
__device__ __forceinline__ int run_first(int lane, int key, bool* last)
{
    const int kp = __shfl(key, max(lane - 1, 0)), kn = __shfl(key, min(lane + 1, 63));
    *last = lane == 63 || kn != key;
    const bool first = lane == 0 || kp != key;
    return int(wave_incl_umax(first ? uint32_t(lane + 1) : 0u)) - 1;
}

// ---------------------------------------------------------------------------
// Gas (mean-field) pass: owners = active gas, others = DM.
// Box of global work item `it` in a batched pass: box_items[b] is the first
// item of box b (box_items[nbox] = total).
__device__ __forceinline__ int box_of_item(const int64_t* __restrict__ box_items, int nbox, int64_t it)
{
    int lo = 0, hi = nbox - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (box_items[mid] <= it) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

struct GasPassArgs {
    PassGeom g;
    const double* Vx; const double* Vy; const double* Vz;     // gas, sorted
    const void* orate;            // OwnRate<Real>[n_own], owner-slot order
    const void* drec;             // DmRec<Real>, sorted DM (velocity, mass)
    const float4* gtab;
    const void* gl_x; const void* gl_w; int gl_k; double inv_alpha;   // quadrature rates (Real)
    double gl_hw, gl_bmin;        // quadrature window
    const MlpBlob* mlp;           // network weights (network rates)
    int mlp_nidx;                 // one-hot slot of n
    float mlp_c0A, mlp_c1A, mlp_c0B, mlp_c1B;   // base-function constants
    float mlp_kA, mlp_kB;                       // 3/alpha_n, 1/alpha_n
    double* part;                 // [n_items][64][gas_sums<RM>()]
    // direct output for owner tiles with a single work item
    const uint32_t* perm;         // gas sorted pos -> index
    const double* mass; const double* mu; const double* dt;
    const double* u;              // gas internal energy (closure: varsigma^2 = 2u/3)
    double dt_default, m_chi, sig_kpc2_cn, alpha_n;
    double* dp; double* de;
};

// Sums the gas pass keeps per owner: the per-pair mean field sums
// (sum M g A w, sum M g (w^2 A - r B)); the closure keeps the DM moments
// (sum M g w, sum M g |w|^2, sum M g).
template <int RM> constexpr int gas_sums() { return RM == kRatesClosure ? 5 : 4; }

// Per-gas Maxwellian closure (Appendix F rates applied per gas particle): the
// DM around the gas particle form one Maxwellian population of kernel-weighted
// density rho = sum M g, drift W = sum M g w / rho and 1-D dispersion
// s_X^2 = (sum M g |w|^2 / rho - |W|^2) / 3.  The two-population rates at
// vth^2 = varsigma^2 + s_X^2 give, per unit of M_j dt sigma-bar_0 c^-n / (m_X + mu),
//   momentum rho A(|W|; vth) W,
//   energy   rho [B (m_X s_X^2 - mu varsigma^2) / (m_X + mu) + A varsigma^2 |W|^2] / vth^2,
// the Maxwellian average of the per-pair terms of eq. gas-dVdt / gas-dTdt.
// With both populations cold (vth = 0) the energy takes its limit, the
// per-pair form |W|^2 A - mu / (m_X + mu) B at A = |W|^{n+1}, B = |W|^{n+3}.
template <int N>
__device__ __forceinline__ void closure_transfer(const double s[5], double vs2, double mu, double m_chi,
                                                 double alpha_n, double v[4])
{
    v[0] = 0.0; v[1] = 0.0; v[2] = 0.0; v[3] = 0.0;
    const double rho = s[4];
    if (!(rho > 0.0)) return;
    const double Wx = s[0] / rho, Wy = s[1] / rho, Wz = s[2] / rho;
    const double W2 = Wx * Wx + Wy * Wy + Wz * Wz;
    const double sx2 = fmax(0.0, (s[3] / rho - W2) / 3.0);
    const double vth2 = vs2 + sx2;
    if (!(vth2 > 0.0) && !(W2 > 0.0)) return;
    double A, E;
    if (vth2 > 0.0) {
        double FA, FB;
        rate_1f1<N, double>(W2 / (2.0 * vth2), &FA, &FB);
        const double vth = sqrt(vth2);
        A = alpha_n / 3.0 * pow(vth, double(N + 1)) * FA;
        const double B = alpha_n * pow(vth, double(N + 3)) * FB;
        E = (B * (m_chi * sx2 - mu * vs2) / (m_chi + mu) + A * vs2 * W2) / vth2;
    } else {
        A = pow_np1<N>(sqrt(W2));
        E = A * W2 * (1.0 - mu / (m_chi + mu));
    }
    v[0] = rho * A * Wx; v[1] = rho * A * Wy; v[2] = rho * A * Wz;
    v[3] = rho * E;
}

// Output of gas o from its summed terms: dp = M_j dt S x (momentum sums),
// dE = M_j dt S x (energy sum), S = sigma-bar_0 c^-n / (m_X + mu_j).
struct GasOutArgs {
    const double* mass; const double* mu; const double* dt; const double* u;
    double dt_default, m_chi, sig_kpc2_cn, alpha_n;
    double* dp; double* de;
};
template <int N, int RM>
__device__ __forceinline__ void gas_store(const GasOutArgs& a, uint32_t o, const double* acc)
{
    const double mu = a.mu ? a.mu[o] : kMpG;
    const double dtj = a.dt ? a.dt[o] : a.dt_default;
    const double sc = a.mass[o] * dtj * kMsunG / (a.m_chi + mu) * a.sig_kpc2_cn;
    double v[4];
    if constexpr (RM == kRatesClosure) {
        closure_transfer<N>(acc, 2.0 * a.u[o] / 3.0, mu, a.m_chi, a.alpha_n, v);
    } else {
        for (int k = 0; k < 4; ++k) v[k] = acc[k];
    }
    a.dp[3 * int64_t(o)] = sc * v[0];
    a.dp[3 * int64_t(o) + 1] = sc * v[1];
    a.dp[3 * int64_t(o) + 2] = sc * v[2];
    a.de[o] = sc * v[3];
}

template <int N, int RM>
__device__ __forceinline__ void gas_write_out(const GasPassArgs& a, uint32_t o, const double* acc)
{
    const GasOutArgs w{a.mass, a.mu, a.dt, a.u, a.dt_default, a.m_chi, a.sig_kpc2_cn, a.alpha_n, a.dp, a.de};
    gas_store<N, RM>(w, o, acc);
}

// Occupancy: the binary32 passes fit 128 VGPRs and < 10 KB of LDS per
// one-wave block, so four waves share each SIMD (16 blocks per CU).
template <typename Real, int N, bool EXACT_G, int RM, bool BATCH = false, bool PAIRS = false>
__global__ __launch_bounds__(RM == kRatesMlp ? 64 * kMlpPassWaves : 64, RM == kRatesMlp ? 2 : (sizeof(Real) == 4 ? 4 : (RM == kRatesExact ? 1 : 2)))
void k_pass_gas(
    GasPassArgs a0, const GasPassArgs* __restrict__ boxes, const int64_t* __restrict__ box_items, int nbox)
{
    // BATCH: one launch over the work items of all boxes; a0 holds the
    // shared queue and item total, boxes[b] the arguments of box b.
    // The network variant runs kMlpPassWaves independent waves per block so
    // that they share one LDS copy of the weights.
    constexpr int W = RM == kRatesMlp ? kMlpPassWaves : 1;
    static_assert(RM != kRatesMlp || sizeof(Real) == 4, "network rates run in binary32");
    __shared__ TestLds S_[W];
    __shared__ Real s_gx[kMaxQuadNodes], s_gw[kMaxQuadNodes];
    __shared__ double o_x_[W][64], o_y_[W][64], o_z_[W][64], o_h_[W][64], o_Vx_[W][64], o_Vy_[W][64], o_Vz_[W][64];
    constexpr int NS = gas_sums<RM>();
    __shared__ double osum_[W][64 * NS];
    __shared__ __align__(16) unsigned char s_mlp[RM == kRatesMlp ? kMlpInferBytes : 16];
    const int wv = W == 1 ? 0 : int(threadIdx.x) >> 6;
    TestLds& S = S_[wv];
    double* o_x = o_x_[wv]; double* o_y = o_y_[wv]; double* o_z = o_z_[wv]; double* o_h = o_h_[wv];
    double* o_Vx = o_Vx_[wv]; double* o_Vy = o_Vy_[wv]; double* o_Vz = o_Vz_[wv];
    const int lane = lane_id();
    if constexpr (RM == kRatesQuad || RM == kRatesMlp) {
        if (int(threadIdx.x) < a0.gl_k) {
            s_gx[threadIdx.x] = reinterpret_cast<const Real*>(a0.gl_x)[threadIdx.x];
            s_gw[threadIdx.x] = reinterpret_cast<const Real*>(a0.gl_w)[threadIdx.x];
        }
    }
    if constexpr (RM == kRatesMlp) {
        const uint4* src = reinterpret_cast<const uint4*>(a0.mlp);
        uint4* dst = reinterpret_cast<uint4*>(s_mlp);
        for (int k = int(threadIdx.x); k < int(kMlpInferBytes / 16); k += 64 * W) dst[k] = src[k];
        __syncthreads();
    }
    const Real inv_alpha = Real(a0.inv_alpha), q_hw = Real(a0.gl_hw), q_bmin = Real(a0.gl_bmin);
    int64_t it;
    uint64_t npairs = 0;
    int cur_b = 0;
    while (item_next<W>(a0.g.queue_ctr, a0.g.n_items, &it)) {
        int b = 0;
        if constexpr (BATCH) {
            b = box_of_item(box_items, nbox, it);
            it -= box_items[b];
            if (b != cur_b) {   // counters belong to the box: flush when the box changes
                for (int d = 32; d >= 1; d >>= 1) npairs += __shfl_xor(npairs, d);
                if (lane == 0 && npairs)
                    atomicAdd((unsigned long long*)&boxes[cur_b].g.counters[0], (unsigned long long)npairs);
                npairs = 0;
                cur_b = b;
            }
        }
        const GasPassArgs& a = BATCH ? boxes[b] : a0;
        const PassGeom& G = a.g;
        const float Lf[3] = {float(G.L[0]), float(G.L[1]), float(G.L[2])};
        it = G.item_order[it];
        const int64_t t = G.it_tile[it];
        const OwnRate<Real>* orate = reinterpret_cast<const OwnRate<Real>*>(a.orate) + t * kTile;
        const uint64_t cb = G.it_cb[it], ce = G.it_ce[it];
        const int64_t slot = t * kTile + lane;
        const bool ov = slot < G.n_own;
        const int64_t sp = ov ? int64_t(G.own[slot]) : 0;
        const double mx = ov ? G.ox[sp] : 0.0, my = ov ? G.oy[sp] : 0.0, mz = ov ? G.oz[sp] : 0.0;
        const double mh = ov ? G.oh[sp] : 0.0;
        stage_sync<W>();
        o_x[lane] = mx; o_y[lane] = my; o_z[lane] = mz; o_h[lane] = mh;
        o_Vx[lane] = ov ? a.Vx[sp] : 0.0; o_Vy[lane] = ov ? a.Vy[sp] : 0.0; o_Vz[lane] = ov ? a.Vz[sp] : 0.0;
        double A[6];
        for (int k = 0; k < 6; ++k) A[k] = G.obox[6 * t + k];
        const double cen[3] = {0.5 * (A[0] + A[3]), 0.5 * (A[1] + A[4]), 0.5 * (A[2] + A[5])};
        const float fx = float(mx - cen[0]), fy = float(my - cen[1]), fz = float(mz - cen[2]), fh = float(mh);
        // the item's per-owner sums (row = owner lane)
        double* osum = osum_[wv] + NS * lane;
        for (int k = 0; k < NS; ++k) osum[k] = 0.0;
        PairTest T;
        test_begin(T, ov, fx, fy, fz, fh, cb, ce);
        for (;;) {
            const int H = test_next<W>(T, S, G, A, cen, Lf);
            if (H < 0) break;
            if (H == 0) continue;
            const int R = (H + 63) >> 6;
            HitWalk hw;
            walk_begin(S, lane, H, R, hw);
            // per-pair terms and the lane's partial sums in binary64 (the overlap near contact is
            // far below the binary32 range; sums of terms that cancel keep their accuracy)
            double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0, p4 = 0.0;
            bool open = false;
            for (int r = 0; r < R; ++r) {
                const bool live = r < hw.n;
                const int o = live ? hw.o : 0;
                const int sl = live ? int(__builtin_ctzll(hw.rem)) : 0;
                double c0 = 0, c1 = 0, c2 = 0, c3 = 0, c4 = 0;
                if constexpr (RM == kRatesClosure) {
                    // the closure's DM moments: kernel-weighted mass, momentum and |w|^2
                    bool hit = false;
                    uint32_t e_o = 0u, e_q = 0u;
                    if (live) {
                        const uint32_t pqv = S.pq[sl];
                        const int64_t q = int64_t(pqv & 0x7fffffffu);
                        const DmRec<Real> r = reinterpret_cast<const DmRec<Real>*>(a.drec)[q];
                        const double qx = S.px[sl], qy = S.py[sl], qz = S.pz[sl], qh = S.ph[sl];
                        const double d2 = pair_d2(o_x[o], o_y[o], o_z[o], qx, qy, qz, (pqv >> 31) != 0u, G.L);
                        const double hs = o_h[o] + qh;
                        if constexpr (PAIRS) {
                            hit = d2 < hs * hs;
                            e_o = G.own[t * kTile + o];
                            e_q = uint32_t(q);
                        }
                        if (d2 < hs * hs) {
                            npairs++;
                            const double gg = EXACT_G ? double(overlap_g_exact<Real>(sqrt_real(Real(d2)), Real(qh), Real(o_h[o])))
                                                      : overlap_g_gas(a.gtab, d2, qh, o_h[o]);
                            const double wx = r.vx - o_Vx[o], wy = r.vy - o_Vy[o], wz = r.vz - o_Vz[o];
                            const double mg = double(r.m) * gg;
                            c0 = mg * wx; c1 = mg * wy; c2 = mg * wz;
                            c3 = mg * (wx * wx + wy * wy + wz * wz);
                            c4 = mg;
                        }
                    }
                    if constexpr (PAIRS) pair_export(G, hit, e_o, e_q);
                } else if constexpr (RM != kRatesMlp) {
                    bool hit = false;
                    uint32_t e_o = 0u, e_q = 0u;
                    if (live) {
                        const uint32_t pqv = S.pq[sl];
                        const int64_t q = int64_t(pqv & 0x7fffffffu);
                        // the pair's records, issued before the distance work that hides their latency
                        const DmRec<Real> r = reinterpret_cast<const DmRec<Real>*>(a.drec)[q];
                        const OwnRate<Real> orr = orate[o];
                        const double qx = S.px[sl], qy = S.py[sl], qz = S.pz[sl], qh = S.ph[sl];
                        const double d2 = pair_d2(o_x[o], o_y[o], o_z[o], qx, qy, qz, (pqv >> 31) != 0u, G.L);
                        const double hs = o_h[o] + qh;
                        if constexpr (PAIRS) {
                            hit = d2 < hs * hs;
                            e_o = G.own[t * kTile + o];
                            e_q = uint32_t(q);
                        }
                        if (d2 < hs * hs) {
                            npairs++;
                            const double gg = EXACT_G ? double(overlap_g_exact<Real>(sqrt_real(Real(d2)), Real(qh), Real(o_h[o])))
                                                      : overlap_g_gas(a.gtab, d2, qh, o_h[o]);
                            const Real wx = Real(r.vx - o_Vx[o]), wy = Real(r.vy - o_Vy[o]), wz = Real(r.vz - o_Vz[o]);
                            const Real w2 = wx * wx + wy * wy + wz * wz;
                            Real FA, FB, Ar, Br;
                            const Real i2 = orr.i2;
                            if (isinf(i2)) {  // cold gas: A = w^{n+1}, B = w^{n+3}
                                const Real wn = sqrt_real(w2);
                                Ar = pow_np1<N>(wn);
                                Br = Ar * w2;
                            } else {
                                if constexpr (RM == kRatesQuad)
                                    rate_quad<N, Real>(sqrt_real(Real(2) * w2 * i2), s_gx, s_gw, a0.gl_k, inv_alpha,
                                                       q_hw, q_bmin, &FA, &FB);
                                else
                                    rate_1f1<N, Real>(w2 * i2, &FA, &FB);
                                Ar = orr.a * FA;
                                Br = orr.b * FB;
                            }
                            const double mg = double(r.m) * gg;
                            const double mgA = mg * double(Ar);
                            c0 = mgA * double(wx); c1 = mgA * double(wy); c2 = mgA * double(wz);
                            c3 = mg * double(w2 * Ar - orr.r * Br);
                        }
                    }
                    if constexpr (PAIRS) pair_export(G, hit, e_o, e_q);
                } else {
                    // pair geometry per lane, then the network over the whole wave
                    bool live2 = false;
                    int64_t q = 0;
                    double gg = 0.0;
                    float wx = 0.f, wy = 0.f, wz = 0.f, w2 = 0.f, i2 = 0.f, u = 0.f, mq = 0.f;
                    OwnRate<float> orr{0.f, 0.f, 0.f, 0.f};
                    if (live) {
                        const uint32_t pqv = S.pq[sl];
                        q = int64_t(pqv & 0x7fffffffu);
                        const double qx = S.px[sl], qy = S.py[sl], qz = S.pz[sl], qh = S.ph[sl];
                        const double d2 = pair_d2(o_x[o], o_y[o], o_z[o], qx, qy, qz, (pqv >> 31) != 0u, G.L);
                        const double hs = o_h[o] + qh;
                        if (d2 < hs * hs) {
                            live2 = true;
                            npairs++;
                            gg = overlap_g_gas(a.gtab, d2, qh, o_h[o]);
                            const DmRec<float> r = reinterpret_cast<const DmRec<float>*>(a.drec)[q];
                            wx = float(r.vx - o_Vx[o]);
                            wy = float(r.vy - o_Vy[o]);
                            wz = float(r.vz - o_Vz[o]);
                            mq = r.m;
                            w2 = wx * wx + wy * wy + wz * wz;
                            orr = reinterpret_cast<const OwnRate<float>*>(orate)[o];
                            i2 = orr.i2;
                            u = isinf(i2) ? 0.f : sqrt_real(2.f * w2 * i2);
                        }
                    }
                    const bool net = live2 && !isinf(i2) && u <= kMlpUMax;
                    float yA = 0.f, yB = 0.f;
                    if (__ballot(net) != 0ull) {
                        // an opaque zero offset keeps the weight reads inside the loop
                        // (hoisted, they would pin ~90 registers for the kernel's lifetime)
                        int zoff = 0;
                        asm volatile("" : "+v"(zoff));
                        const MlpBlob* Wl = reinterpret_cast<const MlpBlob*>(s_mlp + zoff);
                        // the round's pairs occupy lanes 0 .. nlive-1 (the lanes whose range
                        // reaches round r): evaluate only the 16-column blocks that hold some
                        const int nlive = min((H - r + R - 1) / R, 64);
                        if (nlive > 32)
                            mlp_forward64<4, 4>(Wl, mlp_input(u), a0.mlp_nidx, &yA, &yB);
                        else if (nlive > 16)
                            mlp_forward64<2, 2>(Wl, mlp_input(u), a0.mlp_nidx, &yA, &yB);
                        else
                            mlp_forward64<1, 1>(Wl, mlp_input(u), a0.mlp_nidx, &yA, &yB);
                    }
                    if (live2) {
                        float Ar, Br;
                        if (isinf(i2)) {
                            Ar = pow_np1<N>(sqrt_real(w2));
                            Br = Ar * w2;
                        } else {
                            float FA, FB;
                            if (net) {
                                float bA, bB;
                                mlp_base<N>(u * u, a0.mlp_c0A, a0.mlp_c1A, a0.mlp_c0B, a0.mlp_c1B, &bA, &bB);
                                FA = a0.mlp_kA * bA * __expf(yA);
                                FB = a0.mlp_kB * bB * __expf(yB);
                            } else {
                                rate_quad<N, float>(u, s_gx, s_gw, a0.gl_k, inv_alpha, q_hw, q_bmin, &FA, &FB);
                            }
                            Ar = orr.a * FA;
                            Br = orr.b * FB;
                        }
                        const double mg = double(mq) * gg;
                        const double mgA = mg * double(Ar);
                        c0 = mgA * double(wx); c1 = mgA * double(wy); c2 = mgA * double(wz);
                        c3 = mg * double(w2 * Ar - orr.r * Br);
                    }
                }
                p0 += c0; p1 += c1; p2 += c2; p3 += c3;
                if constexpr (NS == 5) p4 += c4;
                if (live) hw.rem &= hw.rem - 1ull;
                const bool done = live && hw.rem == 0ull;
                if (live) open = !done;
                if (__ballot(done) != 0ull && done) {
                    // the owner's last hit of the group: its partial goes to the owner's row
                    double* q = osum_[wv] + NS * hw.o;
                    q[0] += p0; q[1] += p1; q[2] += p2; q[3] += p3;
                    if constexpr (NS == 5) q[4] += p4;
                    p0 = 0.0; p1 = 0.0; p2 = 0.0; p3 = 0.0; p4 = 0.0;
                    hw.o = next_owner(hw.own, hw.o);
                    hw.rem = hw.o < 64 ? S.mask[hw.o] : 0ull;
                }
            }
            // open partials: lanes whose range ended inside an owner's hits
            if (__ballot(open) != 0ull) {
                bool last;
                const int lo = run_first(lane, open ? hw.o : 64 + lane, &last);
                seg_scan_up(lane, lo, [&](auto ctl, auto rows, bool take) {
                    constexpr int C = decltype(ctl)::value, RW = decltype(rows)::value;
                    p0 = dpp_take_add<C, RW>(p0, take);
                    p1 = dpp_take_add<C, RW>(p1, take);
                    p2 = dpp_take_add<C, RW>(p2, take);
                    p3 = dpp_take_add<C, RW>(p3, take);
                    if constexpr (NS == 5) p4 = dpp_take_add<C, RW>(p4, take);
                });
                if (open && last) {
                    double* q = osum_[wv] + NS * hw.o;
                    q[0] += p0; q[1] += p1; q[2] += p2; q[3] += p3;
                    if constexpr (NS == 5) q[4] += p4;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        double acc[NS];
        for (int k = 0; k < NS; ++k) acc[k] = osum[k];
        if (G.item_off[t + 1] - G.item_off[t] == 1u) {
            if (ov) gas_write_out<N, RM>(a, a.perm[sp], acc);
        } else {
            double* P = a.part + (it * kTile + lane) * NS;
            for (int k = 0; k < NS; ++k) P[k] = acc[k];
        }
    }
    for (int d = 32; d >= 1; d >>= 1) npairs += __shfl_xor(npairs, d);
    uint64_t* cnt = BATCH ? boxes[cur_b].g.counters : a0.g.counters;
    if (lane == 0 && npairs) atomicAdd((unsigned long long*)&cnt[0], (unsigned long long)npairs);
}

// ---------------------------------------------------------------------------
// DM (Monte Carlo) pass: owners = active DM, others = gas.
struct DmPassArgs {
    PassGeom g;
    const void* drec;                                         // DmRec<Real>, sorted DM (velocity, mass, dt)
    const uint32_t* dm_perm;                                  // DM sorted pos -> index
    const double* Vx; const double* Vy; const double* Vz;     // gas, sorted
    const void* grec;                                         // GasRec<Real>, sorted gas
    const float4* gtab;
    uint32_t k0, k1, step, box;
    const uint32_t* step_off;     // nullable: device offset added to step (graph replays)
    double* part_p;               // [n_items][64]
    float* part_pm;               // [n_items][64]
    uint8_t* part_nb;             // [n_items][64] near-boundary flags
    // direct decision for owner tiles with a single work item
    double* psum_own; double* psum; double* pmax;
    uint32_t* scount; uint32_t* slist;
};

// P_ij for one (DM, gas) pair: one Maxwellian gas-velocity sample (Philox tag
// 0) and P = K_j g v_rel^{n+1} dt_i (eq. dm-update-prob).  `urel` returns
// v_i - v^B_ij.  Shared by the DM pass and the partner resolve so both see
// identical values.
template <typename Real, int N, bool EXACT_G>
__device__ __forceinline__ Real pair_P(double d2, double dh, double gh, double vx, double vy, double vz, double Vx,
                                       double Vy, double Vz, Real vs, Real K, Real dt, uint32_t i, uint32_t j,
                                       uint32_t step, uint32_t box, uint32_t k0, uint32_t k1, const float4* gtab,
                                       Real urel[3])
{
    U4 r = philox_block(i, j, step, kTagGasVel, box, k0, k1);
    Real g = EXACT_G ? overlap_g_exact<Real>(sqrt_real(Real(d2)), Real(dh), Real(gh))
                     : Real(overlap_g_table32(gtab, d2, dh, gh));
    Real z[3];
    normals3<Real>(r, z);
    urel[0] = Real(vx - Vx) - vs * z[0];
    urel[1] = Real(vy - Vy) - vs * z[1];
    urel[2] = Real(vz - Vz) - vs * z[2];
    Real vrel = sqrt_real(urel[0] * urel[0] + urel[1] * urel[1] + urel[2] * urel[2]);
    return K * g * pow_np1<N>(vrel) * dt;
}

// Rao-Blackwellised P_ij (an exact-in-law variant of the per-pair draw):
// the expectation of P_ij over the Maxwellian gas-velocity sample,
// K_j g dt_i E|w - vs z|^{n+1}, w = v_i - V_j.  E|u|^{n+1} for
// u ~ N(w, vs^2 I) is the B rate integral of power n - 2,
// alpha_{n-2} vs^{n+1} 1F1(-(n+1)/2, 3/2, -w^2/(2 vs^2)); the gas record
// carries i2 = 1/(2 vs^2) (infinite for cold gas, where E = |w|^{n+1}) and
// Kb = K_j alpha_{n-2} vs^{n+1}.  Shared by the DM pass and the resolve.
template <typename Real, int N, bool EXACT_G>
__device__ __forceinline__ Real pair_Pbar(double d2, double dh, double gh, double vx, double vy, double vz,
                                          double Vx, double Vy, double Vz, Real i2, Real Kb, Real dt,
                                          const float4* gtab)
{
    static_assert(N > -4, "the expectation diverges for n = -4");
    const Real g = EXACT_G ? overlap_g_exact<Real>(sqrt_real(Real(d2)), Real(dh), Real(gh))
                           : Real(overlap_g_table32(gtab, d2, dh, gh));
    const Real wx = Real(vx - Vx), wy = Real(vy - Vy), wz = Real(vz - Vz);
    const Real w2 = wx * wx + wy * wy + wz * wz;
    Real E;
    if (isinf(i2)) {
        E = pow_np1<N>(sqrt_real(w2));
    } else {
        Real FA, FB;
        rate_1f1<N - 2, Real>(w2 * i2, &FA, &FB);
        E = FB;
    }
    return Kb * g * E * dt;
}

// Decision of eq. dm-update-vels for one DM owner: U_i (tag 2) against P_i;
// scattering DM go to the resolve list.  Returns flags (scatter, P>=1,
// non-finite, near-decision) as bits 0..3.
__device__ __forceinline__ uint32_t dm_decide(uint32_t o, int64_t s, double P, float Pm, uint32_t step, uint32_t box,
                                              uint32_t k0, uint32_t k1, double* psum_own, double* psum, double* pmax,
                                              uint32_t* scount, uint32_t* slist)
{
    psum_own[s] = P;
    if (psum) psum[o] = P;
    if (pmax) pmax[o] = double(Pm);
    U4 r = philox_block(o, 0xFFFFFFFFu, step, kTagDecision, box, k0, k1);
    double U = u24<double>(r.x);
    uint32_t f = 0;
    if (!isfinite(P)) f |= 4u;
    if (P >= 1.0) f |= 2u;
    if (U < P) {
        uint32_t idx = atomicAdd(scount, 1u);
        slist[idx] = uint32_t(s);
        f |= 1u;
    } else if (fabs(P - U) <= 1e-6 * U) {
        f |= 8u;
    }
    return f;
}

template <typename Real, int N, bool EXACT_G, bool BATCH = false, bool PAIRS = false, bool RB = false>
__global__ __launch_bounds__(64, sizeof(Real) == 4 ? 4 : 3) void k_pass_dm(DmPassArgs a0, const DmPassArgs* __restrict__ boxes,
                                                   const int64_t* __restrict__ box_items, int nbox)
{
    __shared__ TestLds S;
    __shared__ double o_x[64], o_y[64], o_z[64], o_h[64], o_vx[64], o_vy[64], o_vz[64];
    __shared__ Real o_dt[64];
    __shared__ uint32_t o_id[64];
    __shared__ double osP[64];
    __shared__ Real osM[64];
    __shared__ int osNB[64];
    const int lane = lane_id();
    int64_t it;
    uint64_t npairs = 0, ncrit = 0, nnear = 0, nscat = 0, npge1 = 0, nnonf = 0, nneard = 0;
    int cur_b = 0;
    // counters belong to the box: flushed when the box changes and at the end
    auto flush = [&](uint64_t* counters) {
        for (int d = 32; d >= 1; d >>= 1) {
            npairs += __shfl_xor(npairs, d);
            ncrit += __shfl_xor(ncrit, d);
            nnear += __shfl_xor(nnear, d);
            nscat += __shfl_xor(nscat, d);
            npge1 += __shfl_xor(npge1, d);
            nnonf += __shfl_xor(nnonf, d);
            nneard += __shfl_xor(nneard, d);
        }
        if (lane == 0) {
            if (npairs) atomicAdd((unsigned long long*)&counters[1], (unsigned long long)npairs);
            if (nscat) atomicAdd((unsigned long long*)&counters[2], (unsigned long long)nscat);
            if (nnear) atomicAdd((unsigned long long*)&counters[3], (unsigned long long)nnear);
            if (nneard) atomicAdd((unsigned long long*)&counters[4], (unsigned long long)nneard);
            if (ncrit) atomicAdd((unsigned long long*)&counters[5], (unsigned long long)ncrit);
            if (npge1) atomicAdd((unsigned long long*)&counters[6], (unsigned long long)npge1);
            if (nnonf) atomicAdd((unsigned long long*)&counters[7], (unsigned long long)nnonf);
        }
        npairs = ncrit = nnear = nscat = npge1 = nnonf = nneard = 0;
    };
    while (item_next(a0.g.queue_ctr, a0.g.n_items, &it)) {
        int b = 0;
        if constexpr (BATCH) {
            b = box_of_item(box_items, nbox, it);
            it -= box_items[b];
            if (b != cur_b) {
                flush(boxes[cur_b].g.counters);
                cur_b = b;
            }
        }
        const DmPassArgs& a = BATCH ? boxes[b] : a0;
        const PassGeom& G = a.g;
        const float Lf[3] = {float(G.L[0]), float(G.L[1]), float(G.L[2])};
        const uint32_t step = a.step + (a.step_off ? *a.step_off : 0u);
        it = G.item_order[it];
        const int64_t t = G.it_tile[it];
        const uint64_t cb = G.it_cb[it], ce = G.it_ce[it];
        const int64_t slot = t * kTile + lane;
        const bool ov = slot < G.n_own;
        const int64_t sp = ov ? int64_t(G.own[slot]) : 0;
        const double mx = ov ? G.ox[sp] : 0.0, my = ov ? G.oy[sp] : 0.0, mz = ov ? G.oz[sp] : 0.0;
        const double mh = ov ? G.oh[sp] : 0.0;
        __syncthreads();
        o_x[lane] = mx; o_y[lane] = my; o_z[lane] = mz; o_h[lane] = mh;
        {
            DmRec<Real> orc{0.0, 0.0, 0.0, Real(0), Real(0)};
            if (ov) orc = reinterpret_cast<const DmRec<Real>*>(a.drec)[sp];
            o_vx[lane] = orc.vx; o_vy[lane] = orc.vy; o_vz[lane] = orc.vz;
            o_dt[lane] = orc.dt;
        }
        o_id[lane] = ov ? a.dm_perm[sp] : 0u;
        double A[6];
        for (int k = 0; k < 6; ++k) A[k] = G.obox[6 * t + k];
        const double cen[3] = {0.5 * (A[0] + A[3]), 0.5 * (A[1] + A[4]), 0.5 * (A[2] + A[5])};
        const float fx = float(mx - cen[0]), fy = float(my - cen[1]), fz = float(mz - cen[2]), fh = float(mh);
        // the item's per-owner sums (row = owner lane)
        osP[lane] = 0.0; osM[lane] = Real(0); osNB[lane] = 0;
        PairTest T;
        test_begin(T, ov, fx, fy, fz, fh, cb, ce);
        for (;;) {
            const int H = test_next<1>(T, S, G, A, cen, Lf);
            if (H < 0) break;
            if (H == 0) continue;
            const int R = (H + 63) >> 6;
            HitWalk hw;
            walk_begin(S, lane, H, R, hw);
            // the lane's partial sum of P_ij in the pair precision (binary32: at most 64 terms, a
            // relative error below 6 units of 2^-24), its maximum and near-boundary flag; the
            // owner rows accumulate the partials in binary64
            Real pP = 0, pM = 0;
            int pNB = 0;
            bool open = false;
            for (int r = 0; r < R; ++r) {
                const bool live = r < hw.n;
                const int o = live ? hw.o : 0;
                const int sl = live ? int(__builtin_ctzll(hw.rem)) : 0;
                bool hit = false;
                uint32_t e_o = 0u, e_q = 0u;
                if (live) {
                    const uint32_t pqv = S.pq[sl];
                    const int64_t q = int64_t(pqv & 0x7fffffffu);
                    // the pair's gas record, issued before the distance work that hides its latency
                    const GasRec<Real> r = reinterpret_cast<const GasRec<Real>*>(a.grec)[q];
                    const double qx = S.px[sl], qy = S.py[sl], qz = S.pz[sl], qh = S.ph[sl];
                    const double d2 = pair_d2(o_x[o], o_y[o], o_z[o], qx, qy, qz, (pqv >> 31) != 0u, G.L);
                    const double hs = o_h[o] + qh;
                    const double hs2 = hs * hs;
                    if constexpr (PAIRS) {
                        hit = d2 < hs2;
                        e_o = G.own[t * kTile + o];
                        e_q = uint32_t(q);
                    }
                    if (fabs(d2 - hs2) <= 1e-6 * hs2) pNB = 1;
                    if (d2 < hs2) {
                        npairs++;
                        Real P;
                        if constexpr (RB) {
                            P = pair_Pbar<Real, N, EXACT_G>(d2, o_h[o], qh, o_vx[o], o_vy[o], o_vz[o], r.Vx, r.Vy, r.Vz,
                                                            r.vs, r.K, o_dt[o], a.gtab);
                        } else {
                            Real urel[3];
                            P = pair_P<Real, N, EXACT_G>(d2, o_h[o], qh, o_vx[o], o_vy[o], o_vz[o], r.Vx, r.Vy, r.Vz,
                                                         r.vs, r.K, o_dt[o], o_id[o], r.perm, step, a.box, a.k0, a.k1,
                                                         a.gtab, urel);
                        }
                        pP += P;
                        pM = pM > P ? pM : P;
                        if (P >= r.crit) ncrit++;
                    }
                    hw.rem &= hw.rem - 1ull;
                }
                if constexpr (PAIRS) pair_export(G, hit, e_o, e_q);
                const bool done = live && hw.rem == 0ull;
                if (live) open = !done;
                if (__ballot(done) != 0ull && done) {
                    // the owner's last hit of the group: its partial goes to the owner's row
                    osP[hw.o] += double(pP);
                    osM[hw.o] = osM[hw.o] > pM ? osM[hw.o] : pM;
                    osNB[hw.o] |= pNB;
                    pP = 0; pM = 0; pNB = 0;
                    hw.o = next_owner(hw.own, hw.o);
                    hw.rem = hw.o < 64 ? S.mask[hw.o] : 0ull;
                }
            }
            // open partials: lanes whose range ended inside an owner's hits
            if (__ballot(open) != 0ull) {
                bool last;
                const int lo = run_first(lane, open ? hw.o : 64 + lane, &last);
                seg_scan_up(lane, lo, [&](auto ctl, auto rows, bool take) {
                    constexpr int C = decltype(ctl)::value, RW = decltype(rows)::value;
                    pP = dpp_take_add<C, RW>(pP, take);
                    pM = dpp_take_max<C, RW>(pM, take);
                    pNB |= int(dpp_u32<C, RW>(uint32_t(pNB))) & int(take);
                });
                if (open && last) {
                    osP[hw.o] += double(pP);
                    osM[hw.o] = osM[hw.o] > pM ? osM[hw.o] : pM;
                    osNB[hw.o] |= pNB;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const double accP = osP[lane];
        const Real accM = osM[lane];
        const int accNB = osNB[lane];
        if (G.item_off[t + 1] - G.item_off[t] == 1u) {
            if (ov) {
                if (accNB) nnear++;
                uint32_t f = dm_decide(o_id[lane], slot, accP, float(accM), step, a.box, a.k0, a.k1, a.psum_own,
                                       a.psum, a.pmax, a.scount, a.slist);
                nscat += f & 1u; npge1 += (f >> 1) & 1u; nnonf += (f >> 2) & 1u; nneard += (f >> 3) & 1u;
            }
        } else {
            a.part_p[it * kTile + lane] = accP;
            a.part_pm[it * kTile + lane] = float(accM);
            a.part_nb[it * kTile + lane] = uint8_t(accNB);
        }
    }
    flush(BATCH ? boxes[cur_b].g.counters : a0.g.counters);
}

// Exported pairs from sorted to input indices, as (DM index, gas index).
// owner_is_dm: the list came from the DM pass (owner = DM).
__global__ __launch_bounds__(256) void k_pairs_map(int64_t n, uint32_t* __restrict__ pairs,
                                                   const uint32_t* __restrict__ owner_perm,
                                                   const uint32_t* __restrict__ other_perm, bool owner_is_dm)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint32_t o = owner_perm[pairs[2 * k]], q = other_perm[pairs[2 * k + 1]];
    pairs[2 * k] = owner_is_dm ? o : q;
    pairs[2 * k + 1] = owner_is_dm ? q : o;
}

// ---------------------------------------------------------------------------
// Combine partials of owners whose tile was split into several work items
// (fixed item order) and apply owner factors; single-item tiles were written
// by the pass itself.
struct GasCombineArgs {
    int64_t n_own;
    const uint32_t* own; const uint32_t* perm;
    const uint32_t* item_off;     // [nown_tile + 1]
    const double* part;           // [n_items][64][gas_sums<RM>()]
    GasOutArgs out;
};

// One block per owner tile with several items; wave w sums the tile's items
// w, w + kCombineWaves, ... (lane = owner slot) and the wave sums are added in
// wave order, so the result does not depend on scheduling.
constexpr int kCombineWaves = 8;

template <int N, int RM>
__global__ __launch_bounds__(64 * kCombineWaves) void k_combine_gas(GasCombineArgs a)
{
    constexpr int NS = gas_sums<RM>();
    __shared__ double s_acc[kCombineWaves][64][NS];
    const int64_t t = blockIdx.x;
    const uint32_t i0 = a.item_off[t], i1 = a.item_off[t + 1];
    if (i1 - i0 <= 1u) return;
    const int w = int(threadIdx.x) >> 6, l = lane_id();
    double acc[NS];
    for (int c = 0; c < NS; ++c) acc[c] = 0.0;
#pragma unroll 4
    for (uint32_t it = i0 + uint32_t(w); it < i1; it += kCombineWaves) {
        const double* P = a.part + (int64_t(it) * kTile + l) * NS;
        for (int c = 0; c < NS; ++c) acc[c] += P[c];
    }
    for (int c = 0; c < NS; ++c) s_acc[w][l][c] = acc[c];
    __syncthreads();
    const int64_t s = t * kTile + l;
    if (w != 0 || s >= a.n_own) return;
    for (int v = 1; v < kCombineWaves; ++v)
        for (int c = 0; c < NS; ++c) acc[c] += s_acc[v][l][c];
    gas_store<N, RM>(a.out, a.perm[a.own[s]], acc);
}

struct DmCombineArgs {
    int64_t n_own;
    const uint32_t* own; const uint32_t* perm;
    const uint32_t* item_off;
    const double* part_p; const float* part_pm; const uint8_t* part_nb;
    uint32_t k0, k1, step, box;
    const uint32_t* step_off;     // nullable: device offset added to step
    double* psum_own;             // [n_own] P_i in owner-slot order
    double* psum; double* pmax;   // outputs (nullable)
    uint32_t* scount; uint32_t* slist;
    uint64_t* counters;
};

__global__ __launch_bounds__(64 * kCombineWaves) void k_combine_dm(DmCombineArgs a)
{
    __shared__ double s_p[kCombineWaves][64];
    __shared__ float s_m[kCombineWaves][64];
    __shared__ uint32_t s_nb[kCombineWaves][64];
    const int64_t t = blockIdx.x;
    const uint32_t i0 = a.item_off[t], i1 = a.item_off[t + 1];
    if (i1 - i0 <= 1u) return;
    const int w = int(threadIdx.x) >> 6, l = lane_id();
    double P = 0.0;
    float Pm = 0.f;
    uint32_t nb = 0;
#pragma unroll 4
    for (uint32_t it = i0 + uint32_t(w); it < i1; it += kCombineWaves) {
        P += a.part_p[int64_t(it) * kTile + l];
        Pm = fmaxf(Pm, a.part_pm[int64_t(it) * kTile + l]);
        nb |= a.part_nb[int64_t(it) * kTile + l];
    }
    s_p[w][l] = P; s_m[w][l] = Pm; s_nb[w][l] = nb;
    __syncthreads();
    if (w != 0) return;
    const int64_t s = t * kTile + l;
    uint32_t f = 0;
    nb = 0;
    if (s < a.n_own) {
        P = 0.0;
        Pm = 0.f;
        for (int v = 0; v < kCombineWaves; ++v) { P += s_p[v][l]; Pm = fmaxf(Pm, s_m[v][l]); nb |= s_nb[v][l]; }
        uint32_t o = a.perm[a.own[s]];
        f = dm_decide(o, s, P, Pm, a.step + (a.step_off ? *a.step_off : 0u), a.box, a.k0, a.k1, a.psum_own, a.psum,
                      a.pmax, a.scount, a.slist);
    }
    uint64_t b0 = __ballot(f & 1u), b1 = __ballot(f & 2u), b2 = __ballot(f & 4u), b3 = __ballot(f & 8u);
    uint64_t b4 = __ballot(nb != 0);
    if (l == 0) {
        if (b0) atomicAdd((unsigned long long*)&a.counters[2], (unsigned long long)__popcll(b0));
        if (b4) atomicAdd((unsigned long long*)&a.counters[3], (unsigned long long)__popcll(b4));
        if (b3) atomicAdd((unsigned long long*)&a.counters[4], (unsigned long long)__popcll(b3));
        if (b1) atomicAdd((unsigned long long*)&a.counters[6], (unsigned long long)__popcll(b1));
        if (b2) atomicAdd((unsigned long long*)&a.counters[7], (unsigned long long)__popcll(b2));
    }
}

// ---------------------------------------------------------------------------
// Partner resolve for the DM that scatter (eq. dm-update-vels: one draw from
// the mixture): the partner is the smallest gas index whose running sum of
// P_ij exceeds U_i.  The DM's pairs are enumerated once (candidate sub-tiles
// first filtered by a point-to-box test) with the same arithmetic as the DM
// pass and cached in LDS as (gas index, P_ij); a radix select over the gas
// index, 8 bits per pass, accumulates P_ij per digit as exact fixed-point
// integers (P * 2^64 split into two u64 halves), so the running sums are exact
// sums of the per-pair values and do not depend on accumulation order.  DM
// with more pairs than the cache recompute their pairs in every pass.
struct ResolveArgs {
    PassGeom g;                   // owners = DM, others = gas sub-tiles (as in the DM pass)
    const uint64_t* cand_beg; const uint32_t* cand_cnt;   // each owner tile's candidate list
    const void* drec; const uint32_t* dm_perm;
    const void* grec;                                         // GasRec<Real>, sorted gas
    const double* gas_vel; const double* gas_u; const double* gas_mu;   // raw gas inputs (partner kick)
    double m_chi;
    double aniso_g;               // Henyey-Greenstein asymmetry of the scattering angle (0: isotropic)
    const double* tilt_gl;        // Rao-Blackwellised draw: 16-point Gauss-Legendre nodes [16] and weights [16]
    const float4* gtab;
    uint32_t k0, k1, step, box;
    const uint32_t* step_off;     // nullable: device offset added to step
    int n_gas_bits;
    uint32_t n_gas;
    const uint32_t* scount; const uint32_t* slist;
    double* dv; int32_t* partner;
    uint64_t* counters;
};

__device__ __forceinline__ void fixed_split(double P, unsigned long long* hi, unsigned long long* lo)
{
    if (!(P >= 0.0)) { *hi = 0ull; *lo = 0ull; return; }
    if (!(P < 2147483648.0)) { *hi = 1ull << 63; *lo = 0ull; return; }
    double pd = P * 4294967296.0;
    double fl = floor(pd);
    *hi = (unsigned long long)fl;
    *lo = (unsigned long long)((pd - fl) * 4294967296.0);
}

// Rao-Blackwellised partner draw: the relative velocity of the chosen pair
// from the tilted law |u|^M N(u; w, vs^2 I), M = n + 1, by inversion of
// three uniforms (tag 5).  In units of vs, r = |u| has density proportional
// to r^{M+1} e^{-(r-a)^2/2} (1 - e^{-2ra})/(2a), a = |w|/vs (r^{M+2}
// e^{-r^2/2} at a = 0), which is the 3-D density integrated over directions;
// given r, c = cos(u, w) has density ~ e^{rac} on [-1, 1].  The radial CDF
// is integrated on 24 unit cells from max(0, a - 12) (16-point
// Gauss-Legendre per cell, one lane per cell); the cell that holds u0 is
// found counting from below for u0 <= 1/2 and from above otherwise (so the
// tails keep their relative accuracy), and the radius inside it by Newton
// steps held in a bisection bracket, each partial integral spread over 16
// lanes (one node each, butterfly sum).  Every lane of the wavefront follows
// the same iterates.  Binary64 in both precisions.
constexpr int kTiltCells = 24;

template <int M>
__device__ __forceinline__ double tilt_density(double a, double r)
{
    if (!(r > 0.0)) return 0.0;
    const double sh = a > 0.0 ? -expm1(-2.0 * r * a) / (2.0 * a) : r;
    double p = 1.0;
#pragma unroll
    for (int k = 0; k < M + 1; ++k) p *= r;
    return p * exp(-0.5 * (r - a) * (r - a)) * sh;
}

template <int M>
__device__ double tilt_cell(double a, double x0, double x1, const double* gl)
{
    const double c = 0.5 * (x0 + x1), h = 0.5 * (x1 - x0);
    double s = 0.0;
    for (int k = 0; k < 16; ++k) s += gl[16 + k] * tilt_density<M>(a, c + h * gl[k]);
    return s * h;
}

// all 64 lanes of one wavefront call and all return the radius; gl in LDS
template <int M>
__device__ double tilted_radius(double a, double u0, const double* gl, double* s_cell, int lane)
{
    const double lo = fmax(0.0, a - 0.5 * kTiltCells);
    if (lane < kTiltCells) s_cell[lane] = tilt_cell<M>(a, lo + lane, lo + lane + 1.0, gl);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int kn = lane & 15;
    const double xk = gl[kn], wk = gl[16 + kn];
    double Z = 0.0;
    for (int k = 0; k < kTiltCells; ++k) Z += s_cell[k];
    const bool upper = u0 > 0.5;
    double T = (upper ? 1.0 - u0 : u0) * Z, cum = 0.0;
    int cl = upper ? kTiltCells - 1 : 0;
    if (!upper) {
        while (cl < kTiltCells - 1 && cum + s_cell[cl] < T) cum += s_cell[cl++];
    } else {
        while (cl > 0 && cum + s_cell[cl] < T) cum += s_cell[cl--];
    }
    T -= cum;
    const double x0 = lo + cl, x1 = x0 + 1.0;
    double bl = x0, bh = x1;
    const double fr = s_cell[cl] > 0.0 ? fmin(fmax(T / s_cell[cl], 0.0), 1.0) : 0.5;
    double r = upper ? x1 - fr : x0 + fr;
    for (int it = 0; it < 64; ++it) {
        // lower: F(r) = int_x0^r - T (increasing); upper: F(r) = T - int_r^x1 (increasing)
        const double xa = upper ? r : x0, xb = upper ? x1 : r;
        const double c = 0.5 * (xa + xb), h = 0.5 * (xb - xa);
        double I = wk * tilt_density<M>(a, c + h * xk);
        I += __shfl_xor(I, 8);
        I += __shfl_xor(I, 4);
        I += __shfl_xor(I, 2);
        I += __shfl_xor(I, 1);
        I *= h;
        const double F = upper ? T - I : I - T;
        if (F < 0.0) bl = r; else bh = r;
        const double g = tilt_density<M>(a, r);
        double rn = g > 0.0 ? r - F / g : 0.5 * (bl + bh);
        if (!(rn > bl && rn < bh)) rn = 0.5 * (bl + bh);
        const bool done = fabs(rn - r) <= 4e-15 * rn || !(bh - bl > 4e-15 * bh);
        r = rn;
        if (done) break;
    }
    return r;
}

// The elastic kick of eq. scatter_chi for DM oid scattering off gas j with
// relative velocity u = v_i - v_B: |u| is kept and its direction redrawn
// (tag 1 of the pair: isotropic, or the Henyey-Greenstein angle about u), the
// DM taking mu_j/(m_chi + mu_j) of the change.  Writes dv and the partner.
template <typename Real>
__device__ void scatter_kick(const ResolveArgs& a, uint32_t oid, uint32_t j, uint32_t step, Real ux, Real uy,
                             Real uz)
{
    const double muj = a.gas_mu ? a.gas_mu[j] : kMpG;
    const Real rr = Real(muj / (a.m_chi + muj));
    const Real vrel = sqrt_real(ux * ux + uy * uy + uz * uz);
    double dvx = 0.0, dvy = 0.0, dvz = 0.0;
    if (vrel > Real(0)) {
        U4 r2 = philox_block(oid, j, step, kTagDir, a.box, a.k0, a.k1);
        Real sp_, cp_;
        sincos_turns(u24<Real>(r2.y), &sp_, &cp_);
        Real iv = Real(1) / vrel;
        Real f = rr * vrel;
        Real n[3];
        if (a.aniso_g == 0.0) {
            // isotropic: the new direction directly, cos theta about the z axis
            const Real ct = Real(2) * u24<Real>(r2.x) - Real(1);
            const Real st = sqrt_real(fmax(Real(0), Real(1) - ct * ct));
            n[0] = st * cp_; n[1] = st * sp_; n[2] = ct;
        } else {
            // cos theta from p(Omega), about the incoming relative velocity
            const Real uh[3] = {ux * iv, uy * iv, uz * iv};
            Real ct, st;
            hg_angle(Real(a.aniso_g), u24<Real>(r2.x), &ct, &st);
            Real e1[3], e2[3];
            orthonormal_frame(uh, e1, e2);
            for (int k = 0; k < 3; ++k) n[k] = ct * uh[k] + st * (cp_ * e1[k] + sp_ * e2[k]);
        }
        dvx = double(f * (n[0] - ux * iv));
        dvy = double(f * (n[1] - uy * iv));
        dvz = double(f * (n[2] - uz * iv));
    }
    a.dv[3 * int64_t(oid)] = dvx;
    a.dv[3 * int64_t(oid) + 1] = dvy;
    a.dv[3 * int64_t(oid) + 2] = dvz;
    a.partner[oid] = int32_t(j);
}

constexpr int kResolveThreads = 1024; // sixteen wavefronts per scattering DM (the first 256 threads own the histogram bins)
constexpr int kResolveList = 2048;    // candidate sub-tiles kept per scattering DM after the point test
constexpr int kResolvePairs = 8192;   // pairs cached per scattering DM (LDS)

template <typename Real, int N, bool EXACT_G, bool RB = false>
__global__ __launch_bounds__(kResolveThreads) void k_resolve(ResolveArgs a)
{
    __shared__ unsigned long long hhi[256], hlo[256];

    __shared__ uint32_t s_list[kResolveList];
    __shared__ uint32_t s_pre[kResolveList + 1];
    __shared__ uint32_t s_gid[kResolvePairs];
    __shared__ double s_P[kResolvePairs];
    __shared__ uint32_t s_nrel, s_npairs, s_sel;
    __shared__ int s_near, s_found, s_lastnz;
    __shared__ unsigned __int128 s_cum[256], s_selb, s_sela;
    __shared__ unsigned long long s_run[kResolveThreads];
    static_assert(kResolveThreads >= 256 && kResolveThreads % 256 == 0, "thread t < 256 owns histogram bin t");
    const bool bin_owner = threadIdx.x < 256;
    const PassGeom& G = a.g;
    const int tid = threadIdx.x;
    const uint32_t step = a.step + (a.step_off ? *a.step_off : 0u);
    const uint32_t nsc = *a.scount;
    uint32_t nnearD = 0;

    for (uint32_t e = blockIdx.x; e < nsc; e += gridDim.x) {
        const int64_t s = a.slist[e];
        const int64_t sp = G.own[s];
        const int64_t t = s / kTile;
        const double mx = G.ox[sp], my = G.oy[sp], mz = G.oz[sp], mh = G.oh[sp];
        const DmRec<Real> orc = reinterpret_cast<const DmRec<Real>*>(a.drec)[sp];
        const double mvx = orc.vx, mvy = orc.vy, mvz = orc.vz;
        const Real mdt = orc.dt;
        const uint32_t oid = a.dm_perm[sp];
        U4 rd = philox_block(oid, 0xFFFFFFFFu, step, kTagDecision, a.box, a.k0, a.k1);
        const unsigned __int128 Ufix = (unsigned __int128)(2ull * (rd.x >> 8) + 1ull) << 39;
        double A[6];
        for (int k = 0; k < 6; ++k) A[k] = G.obox[6 * t + k];
        const uint64_t cb = a.cand_beg[t], ce = cb + a.cand_cnt[t];
        if (tid == 0) { s_nrel = 0; s_npairs = 0; }
        __syncthreads();
        // candidate sub-tiles this DM can reach (point-to-box gap < h_i + max h of the sub-tile)
        const double P6[6] = {mx, my, mz, mx, my, mz};
        for (uint64_t c = cb + tid; c < ce; c += kResolveThreads) {
            const uint32_t ot = G.cand[c];
            if (boxes_near(P6, mh, G.tbox + 6 * int64_t(ot), G.thmax[ot], G.L)) {
                const uint32_t pos = atomicAdd(&s_nrel, 1u);
                if (pos < uint32_t(kResolveList)) s_list[pos] = ot;
            }
        }
        __syncthreads();
        const uint32_t nrel = s_nrel;
        const bool use_list = nrel <= uint32_t(kResolveList);
        const uint32_t nl = use_list ? nrel : uint32_t(ce - cb);
        // prefix sums of particle counts over the kept sub-tiles (nl <= kResolveList):
        // counts loaded in parallel, each thread sums a contiguous run, the
        // run totals are scanned in LDS
        if (use_list) {
            for (uint32_t q = tid; q < nl; q += kResolveThreads) s_pre[q] = G.sub_cnt[s_list[q]];
            __syncthreads();
            const uint32_t per = (nl + kResolveThreads - 1) / kResolveThreads;
            const uint32_t q0 = min(nl, uint32_t(tid) * per), q1 = min(nl, q0 + per);
            uint32_t run = 0;
            for (uint32_t q = q0; q < q1; ++q) run += s_pre[q];
            s_run[tid] = run;
            __syncthreads();
            for (int d = 1; d < kResolveThreads; d <<= 1) {
                const unsigned long long y = tid >= d ? s_run[tid - d] : 0ull;
                __syncthreads();
                s_run[tid] += y;
                __syncthreads();
            }
            uint32_t acc = uint32_t(s_run[tid]) - run;
            for (uint32_t q = q0; q < q1; ++q) {
                const uint32_t v = s_pre[q];
                s_pre[q] = acc;
                acc += v;
            }
            if (tid == kResolveThreads - 1) s_pre[nl] = uint32_t(s_run[tid]);
        }
        __syncthreads();
        // Pairs of this DM, enumerated over the flattened particles of the kept
        // sub-tiles (all wavefronts of the block in parallel).  Without a list (too many
        // candidates) every candidate sub-tile is walked by one wavefront.
        auto for_pairs = [&](auto&& fn) {
            auto visit = [&](uint32_t ot, int kk) {
                double sh[3];
                bool clean;
                tile_pair_shift(A, G.tbox + 6 * int64_t(ot), G.L, sh, &clean);
                if (kk < int(G.sub_cnt[ot])) {
                    const int64_t k = int64_t(G.sub_start[ot]) + kk;
                    const double px = G.tx[k] + sh[0], py = G.ty[k] + sh[1], pz = G.tz[k] + sh[2];
                    const double d2 = pair_d2(mx, my, mz, px, py, pz, clean, G.L);
                    const double hs = mh + G.th[k];
                    if (d2 < hs * hs) {
                        const GasRec<Real> r = reinterpret_cast<const GasRec<Real>*>(a.grec)[k];
                        const uint32_t gid = r.perm;
                        double P;
                        if constexpr (RB) {
                            P = double(pair_Pbar<Real, N, EXACT_G>(d2, mh, G.th[k], mvx, mvy, mvz, r.Vx, r.Vy, r.Vz,
                                                                   r.vs, r.K, mdt, a.gtab));
                        } else {
                            Real urel[3];
                            P = double(pair_P<Real, N, EXACT_G>(d2, mh, G.th[k], mvx, mvy, mvz, r.Vx, r.Vy, r.Vz, r.vs,
                                                                r.K, mdt, oid, gid, step, a.box, a.k0, a.k1, a.gtab,
                                                                urel));
                        }
                        fn(gid, P);
                    }
                }
            };
            if (use_list) {
                const uint32_t np = s_pre[nl];
                for (uint32_t pos = tid; pos < np; pos += kResolveThreads) {
                    uint32_t lo = 0, hi = nl;  // largest q with s_pre[q] <= pos
                    while (hi - lo > 1) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (s_pre[mid] <= pos) lo = mid; else hi = mid;
                    }
                    visit(s_list[lo], int(pos - s_pre[lo]));
                }
            } else {
                const int w = tid >> 6, lane = tid & 63;
                for (uint32_t q = w; q < nl; q += kResolveThreads / 64) visit(G.cand[cb + q], lane);
            }
        };
        for_pairs([&](uint32_t gid, double P) {
            const uint32_t pos = atomicAdd(&s_npairs, 1u);
            if (pos < uint32_t(kResolvePairs)) { s_gid[pos] = gid; s_P[pos] = P; }
        });
        __syncthreads();
        const uint32_t npairs = s_npairs;
        const bool cached = npairs <= uint32_t(kResolvePairs);
        const int npass = (a.n_gas_bits + 7) / 8;
        uint32_t prefix = 0;
        unsigned __int128 below = 0;
        for (int ps = 0; ps < npass; ++ps) {
            const int shft = 8 * (npass - 1 - ps);
            hhi[tid & 255] = 0ull;
            hlo[tid & 255] = 0ull;
            __syncthreads();
            auto add = [&](uint32_t gid, double P) {
                if ((uint64_t(gid) >> (shft + 8)) == uint64_t(prefix)) {
                    unsigned long long hi, lo;
                    fixed_split(P, &hi, &lo);
                    const int dg = (gid >> shft) & 255u;
                    atomicAdd(&hhi[dg], hi);
                    atomicAdd(&hlo[dg], lo);
                }
            };
            if (cached) {
                for (uint32_t q = tid; q < npairs; q += kResolveThreads) add(s_gid[q], s_P[q]);
            } else {
                for_pairs(add);
            }
            // the selected bin: the first whose running sum (from `below`) passes
            // U_i, by an inclusive scan over the 256 bins (thread = bin)
            if (tid == 0) { s_found = 0; s_lastnz = -1; }
            __syncthreads();
            const int bt = tid & 255;
            const unsigned __int128 v = ((unsigned __int128)hhi[bt] << 32) + (unsigned __int128)hlo[bt];
            if (bin_owner) {
                s_cum[tid] = v;
                if (v != 0) atomicMax(&s_lastnz, tid);
            }
            __syncthreads();
            for (int d = 1; d < 256; d <<= 1) {
                const unsigned __int128 y = bin_owner && tid >= d ? s_cum[tid - d] : (unsigned __int128)0;
                __syncthreads();
                if (bin_owner) s_cum[tid] += y;
                __syncthreads();
            }
            const unsigned __int128 incl = below + s_cum[bt], excl = incl - v;
            if (bin_owner && excl <= Ufix && incl > Ufix) {      // unique: running sums increase, empty bins cannot pass
                s_found = 1;
                s_sel = uint32_t(tid);
                s_selb = excl;
                s_sela = incl;
            }
            __syncthreads();
            if (tid == 0 && !s_found) {   // rounding guard: keep the largest index with P > 0
                s_sel = uint32_t(s_lastnz < 0 ? 0 : s_lastnz);
                s_selb = below;
                s_sela = below + s_cum[255];
            }
            __syncthreads();
            below = s_selb;
            if (tid == 0 && ps == npass - 1) {
                // running sums adjacent to U_i (relative 1e-6 band)
                double Ud = double(Ufix) * 0x1p-64, Sb = double(s_selb) * 0x1p-64, Sa = double(s_sela) * 0x1p-64;
                s_near = (fabs(Sb - Ud) <= 1e-6 * Ud || fabs(Sa - Ud) <= 1e-6 * Ud) ? 1 : 0;
            }
            __syncthreads();
            prefix = (prefix << 8) | s_sel;
            __syncthreads();
        }
        if (tid == 0) {
            const uint32_t j = prefix < a.n_gas ? prefix : a.n_gas - 1u;
            nnearD += uint32_t(s_near);
            if constexpr (RB) {
                a.partner[oid] = int32_t(j);   // the kick follows in k_rb_kick
            } else {
                // the partner's gas-velocity sample from the same uniforms as its P_ij (tag 0),
                // and the kick, in binary64 in either precision: one thread per scattering DM
                const double vs = sqrt(2.0 * a.gas_u[j] / 3.0);
                U4 r = philox_block(oid, j, step, kTagGasVel, a.box, a.k0, a.k1);
                double z[3];
                normals3<double>(r, z);
                const double ux = (mvx - a.gas_vel[3 * int64_t(j)]) - vs * z[0];
                const double uy = (mvy - a.gas_vel[3 * int64_t(j) + 1]) - vs * z[1];
                const double uz = (mvz - a.gas_vel[3 * int64_t(j) + 2]) - vs * z[2];
                scatter_kick<double>(a, oid, j, step, ux, uy, uz);
            }
        }
        __syncthreads();
    }
    if (tid == 0 && nnearD) atomicAdd((unsigned long long*)&a.counters[4], (unsigned long long)nnearD);
}

// Kicks of the Rao-Blackwellised scheme, after k_resolve has chosen the
// partners: one wavefront per scattering DM draws the relative velocity of
// its pair from the tilted law (tag 5: radius, cosine to w, azimuth),
// u = vs r (c e + s (cos phi e1 + sin phi e2)), e = w/|w| (the z axis if
// w = 0; cold gas: u = w), and applies the kick, all in binary64.
template <typename Real, int N>
__global__ __launch_bounds__(64) void k_rb_kick(ResolveArgs a)
{
    __shared__ double s_cell[kTiltCells];
    __shared__ double s_gl[32];
    const int lane = int(threadIdx.x);
    if (lane < 32) s_gl[lane] = a.tilt_gl[lane];
    __syncthreads();
    const uint32_t step = a.step + (a.step_off ? *a.step_off : 0u);
    const uint32_t nsc = *a.scount;
    for (uint32_t e = blockIdx.x; e < nsc; e += gridDim.x) {
        const int64_t sp = a.g.own[a.slist[e]];
        const DmRec<Real> orc = reinterpret_cast<const DmRec<Real>*>(a.drec)[sp];
        const uint32_t oid = a.dm_perm[sp];
        const uint32_t j = uint32_t(a.partner[oid]);
        const double wx = orc.vx - a.gas_vel[3 * int64_t(j)], wy = orc.vy - a.gas_vel[3 * int64_t(j) + 1];
        const double wz = orc.vz - a.gas_vel[3 * int64_t(j) + 2];
        const double vsd = sqrt(2.0 * a.gas_u[j] / 3.0);
        const double wn = sqrt(wx * wx + wy * wy + wz * wz);
        double ud[3] = {wx, wy, wz};
        if (vsd > 0.0) {
            const U4 rt = philox_block(oid, j, step, kTagTilt, a.box, a.k0, a.k1);
            const double trad = tilted_radius<N + 1>(wn / vsd, u24<double>(rt.x), s_gl, s_cell, lane);
            const double kap = trad * wn / vsd;
            const double u1 = u24<double>(rt.y), u2 = u24<double>(rt.z);
            const double omc = kap > 0.0 ? -log1p(u1 * expm1(-2.0 * kap)) / kap : 2.0 * u1;
            const double cc = 1.0 - omc, ss = sqrt(fmax(0.0, omc * (2.0 - omc)));
            double ev[3] = {0.0, 0.0, 1.0}, e1[3], e2[3];
            if (wn > 0.0) { ev[0] = wx / wn; ev[1] = wy / wn; ev[2] = wz / wn; }
            orthonormal_frame(ev, e1, e2);
            double sp2, cp2;
            sincos_turns(u2, &sp2, &cp2);
            for (int k = 0; k < 3; ++k) ud[k] = vsd * trad * (cc * ev[k] + ss * (cp2 * e1[k] + sp2 * e2[k]));
        }
        // the kick in binary64 in either precision: the drawn u already is, and for a forward
        // Henyey-Greenstein angle n' - u/|u| is a difference of nearly equal unit vectors
        if (lane == 0) scatter_kick<double>(a, oid, j, step, ud[0], ud[1], ud[2]);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// ---------------------------------------------------------------------------
// Time loop (dmb_run): after each interaction step the DM take their kicks
// and the gas its momentum and internal-energy transfers (all computed from
// start-of-step states), then both species drift with their new velocities
// (kick, then drift), wrapped into [0, L) in a periodic box.
struct RunArgs {
    int64_t n_gas, n_dm;
    double* gpos; double* gvel; double* gu; const double* gmass; const double* gmu;
    double* dpos; double* dvel; const double* dmass;
    const double* dp_gas; const double* de_gas; const double* dv_dm; const double* p_max;
    const uint64_t* counters;
    double L[3];
    double m_chi;
    const double* dt;             // device: this step's dt
};

__global__ __launch_bounds__(256) void k_run_apply(RunArgs a)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const double dt = *a.dt;
    if (k < a.n_gas) {
        const double im = 1.0 / a.gmass[k];
        for (int c = 0; c < 3; ++c) {
            const double v = a.gvel[3 * k + c] + a.dp_gas[3 * k + c] * im;
            a.gvel[3 * k + c] = v;
            double x = a.gpos[3 * k + c] + v * dt;
            if (a.L[c] > 0.0) x -= a.L[c] * floor(x / a.L[c]);
            a.gpos[3 * k + c] = x;
        }
        a.gu[k] += a.de_gas[k] * im;
    } else if (k < a.n_gas + a.n_dm) {
        const int64_t i = k - a.n_gas;
        for (int c = 0; c < 3; ++c) {
            const double v = a.dvel[3 * i + c] + a.dv_dm[3 * i + c];
            a.dvel[3 * i + c] = v;
            double x = a.dpos[3 * i + c] + v * dt;
            if (a.L[c] > 0.0) x -= a.L[c] * floor(x / a.L[c]);
            a.dpos[3 * i + c] = x;
        }
    }
}

// Active sets of one step of a hierarchical-timestep run: particle i of
// species s (0 gas, 1 DM) is active iff its tag-3 uniform is below frac.
enum : uint32_t { kTagActive = 3u };
__global__ __launch_bounds__(256) void k_run_active(int64_t n_gas, int64_t n_dm, uint8_t* __restrict__ gact,
                                                    uint8_t* __restrict__ dact, uint32_t step, uint32_t box,
                                                    uint32_t k0, uint32_t k1, double frac)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n_gas + n_dm) return;
    const bool gas = k < n_gas;
    const uint32_t i = uint32_t(gas ? k : k - n_gas);
    const U4 r = philox_block(i, gas ? 0u : 1u, step, kTagActive, box, k0, k1);
    const uint8_t a = u24<double>(r.x) < frac ? 1u : 0u;
    if (gas) gact[i] = a;
    else dact[i] = a;
}

// Per-step diagnostics: fixed-order reductions (per-block partial sums, then
// one block adds the blocks in order), binary64.  Partial layout per block:
constexpr int kRunDiagBlocks = 256;
enum : int {
    kRdM = 0, kRdP = 1, kRdE = 4, kRdV1 = 5, kRdV2 = 8, kRdV3 = 11, kRdV4 = 14,    // DM (v moments unweighted)
    kRgM = 17, kRgP = 18, kRgE = 21, kRgU = 22, kRgV1 = 23, kRgV2 = 26,              // gas
    kRPmax = 29, kRCrit = 30, kRN = 31
};

__global__ __launch_bounds__(256) void k_run_diag_partial(RunArgs a, double* __restrict__ part)
{
    __shared__ double red[kRN][4];
    double acc[kRN];
    for (int q = 0; q < kRN; ++q) acc[q] = 0.0;
    acc[kRCrit] = 0.1;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n_dm; i += stride) {
        const double m = a.dmass[i];
        acc[kRdM] += m;
        for (int c = 0; c < 3; ++c) {
            const double v = a.dvel[3 * i + c], v2 = v * v;
            acc[kRdP + c] += m * v;
            acc[kRdE] += 0.5 * m * v2;
            acc[kRdV1 + c] += v;
            acc[kRdV2 + c] += v2;
            acc[kRdV3 + c] += v2 * v;
            acc[kRdV4 + c] += v2 * v2;
        }
        if (a.p_max) acc[kRPmax] = fmax(acc[kRPmax], a.p_max[i]);
    }
    for (int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < a.n_gas; j += stride) {
        const double m = a.gmass[j], u = a.gu[j];
        acc[kRgM] += m;
        acc[kRgU] += u;
        acc[kRgE] += m * u;
        for (int c = 0; c < 3; ++c) {
            const double v = a.gvel[3 * j + c];
            acc[kRgP + c] += m * v;
            acc[kRgE] += 0.5 * m * v * v;
            acc[kRgV1 + c] += v;
            acc[kRgV2 + c] += v * v;
        }
        // the criterion of eq. prob_criterion for this gas particle's pairs
        const double mu = a.gmu ? a.gmu[j] : kMpG, q = (a.m_chi + mu) / mu;
        acc[kRCrit] = fmin(acc[kRCrit], fmin(0.1, 1e-4 * q * q));
    }
    // block reduction in a fixed order: lanes by a butterfly, then waves in order
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int q = 0; q < kRN; ++q) {
        double v = acc[q];
        for (int d = 32; d >= 1; d >>= 1) {
            const double o = __shfl_xor(v, d);
            v = q == kRPmax ? fmax(v, o) : (q == kRCrit ? fmin(v, o) : v + o);
        }
        if (lane == 0) red[q][w] = v;
    }
    __syncthreads();
    if (threadIdx.x < kRN) {
        const int q = threadIdx.x;
        double v = red[q][0];
        for (int k = 1; k < 4; ++k) v = q == kRPmax ? fmax(v, red[q][k]) : (q == kRCrit ? fmin(v, red[q][k]) : v + red[q][k]);
        part[int64_t(blockIdx.x) * kRN + q] = v;
    }
}

// Diagnostics row (layout of the DMB_D_* indices) and the next dt.
struct RunDiagArgs {
    int64_t n_gas, n_dm;
    const double* part; int nblocks;
    const uint64_t* counters;
    double* row;                  // device row of the diagnostics
    double* dt;                   // device: this step's dt (in), next step's dt (out when control != 0)
    double* time;                 // device: elapsed time (advanced by this step's dt)
    int control; double dt_max, safety;
    int first;                    // row of the initial state: no counters, no step
};

__global__ __launch_bounds__(64) void k_run_diag_final(RunDiagArgs a)
{
    __shared__ double tot[kRN];
    if (threadIdx.x < kRN) {
        const int q = threadIdx.x;
        double v = q == kRCrit ? 0.1 : 0.0;
        for (int b = 0; b < a.nblocks; ++b) {
            const double x = a.part[int64_t(b) * kRN + q];
            v = q == kRPmax ? fmax(v, x) : (q == kRCrit ? fmin(v, x) : v + x);
        }
        tot[q] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double* r = a.row;
    const double nd = double(a.n_dm), ng = double(a.n_gas);
    const double dt = *a.dt;
    if (!a.first) *a.time += dt;
    r[DMB_D_TIME] = *a.time;
    r[DMB_D_DT] = a.first ? 0.0 : dt;
    for (int c = 0; c < 3; ++c) {
        r[DMB_D_P_DM + c] = tot[kRdP + c];
        r[DMB_D_P_GAS + c] = tot[kRgP + c];
        r[DMB_D_V_DM + c] = tot[kRdM] > 0.0 ? tot[kRdP + c] / tot[kRdM] : 0.0;
        r[DMB_D_V_GAS + c] = tot[kRgM] > 0.0 ? tot[kRgP + c] / tot[kRgM] : 0.0;
    }
    r[DMB_D_E_DM] = tot[kRdE];
    r[DMB_D_E_GAS] = tot[kRgE];
    // 1-D dispersions about the (unweighted) mean; gas: thermal 2u/3 plus the bulk spread / 3
    double s2d = 0.0, jb = 0.0, s2g = 0.0;
    if (a.n_dm > 0) {
        for (int c = 0; c < 3; ++c) {
            const double m1 = tot[kRdV1 + c] / nd, m2 = tot[kRdV2 + c] / nd, m3 = tot[kRdV3 + c] / nd,
                         m4 = tot[kRdV4 + c] / nd;
            const double c2 = m2 - m1 * m1;
            const double c3 = m3 - 3.0 * m1 * m2 + 2.0 * m1 * m1 * m1;
            const double c4 = m4 - 4.0 * m1 * m3 + 6.0 * m1 * m1 * m2 - 3.0 * m1 * m1 * m1 * m1;
            s2d += c2 / 3.0;
            if (c2 > 0.0) {
                const double S = c3 / (c2 * sqrt(c2)), K = c4 / (c2 * c2);
                jb = fmax(jb, (S * S + 0.25 * (K - 3.0) * (K - 3.0)) / 6.0);   // no sample-size factor (App. F)
            }
        }
    }
    if (a.n_gas > 0) {
        double spread = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double m1 = tot[kRgV1 + c] / ng;
            spread += tot[kRgV2 + c] / ng - m1 * m1;
        }
        s2g = (2.0 / 3.0) * (tot[kRgU] / ng) + spread / 3.0;
    }
    r[DMB_D_S2_DM] = s2d;
    r[DMB_D_S2_GAS] = s2g;
    r[DMB_D_JB_DM] = jb;
    r[DMB_D_SCATTERS] = a.first ? 0.0 : double(a.counters[DMB_C_SCATTERS]);
    r[DMB_D_CRIT_VIOL] = a.first ? 0.0 : double(a.counters[DMB_C_CRIT_VIOL]);
    r[DMB_D_P_MAX] = a.first ? 0.0 : tot[kRPmax];
    r[DMB_D_PAIRS] = a.first ? 0.0 : double(a.counters[DMB_C_PAIRS_DM]);
    r[DMB_D_PAIRS_GAS] = a.first ? 0.0 : double(a.counters[DMB_C_PAIRS_GAS]);
    // eq. prob_criterion: the next step keeps every P_ij below safety x the criterion
    double next = dt;
    if (a.control && !a.first) {
        next = a.dt_max;
        if (tot[kRPmax] > 0.0) next = fmin(next, dt * a.safety * tot[kRCrit] / tot[kRPmax]);
    }
    *a.dt = next;
}

// ---------------------------------------------------------------------------
// Overlap table (Appendix D), built on the device from the exact overlap (the
// regions and envelopes are described above overlap_g_table).
// Shell ratio QA(rho, eta) = H(1 + eta - eta rho, eta) / (eta^3 rho^8).
__device__ double gtab_qa(double rho, double eta)
{
    if (rho <= 0.5) {   // one polynomial piece of the Appendix D integral, in closed form
        const double dl = 1.0 + eta - eta * rho;
        return 512.0 / (kPi * dl) * (1.0 / 1120.0 - (1.0 + eta) * rho / 2520.0 + eta * rho * rho / 6300.0);
    }
    auto q = [rho](double e) {
        const double r2 = rho * rho, r4 = r2 * r2;
        return overlap_H_exact(1.0 + e - e * rho, e) / (e * e * e * r4 * r4);
    };
    if (eta > 0.0) return q(eta);
    // eta -> 0: quadratic extrapolation from eta = 1e-3, 2e-3, 3e-3 (QA is smooth in eta; much
    // closer to 0 the integration range shrinks to ~eta and rounding noise grows as 1/eta)
    return 3.0 * q(1e-3) - 3.0 * q(2e-3) + q(3e-3);
}

// Core ratio QB(delta, kappa) = H(delta, kappa (1 - delta)) / (1 - delta)^3.
__device__ double gtab_qb(double delta, double kappa)
{
    auto q = [kappa](double dl) {
        const double e = kappa * (1.0 - dl), t = 1.0 - dl;
        const double H = e > 0.0 ? overlap_H_exact(dl, e) : kernel_w(dl);
        return H / (t * t * t);
    };
    if (delta < 1.0 - 1e-9) return q(delta);
    return 3.0 * q(1.0 - 1e-3) - 3.0 * q(1.0 - 2e-3) + q(1.0 - 3e-3);   // delta -> 1: quadratic extrapolation
}

// Nodes in binary64, region-major: (Q, dQ/dx * dx, dQ/dy * dy) per node of
// the (kTabN + 1)^2 grid on [0,1]^2 (shell: x = rho/2, y = eta; core:
// x = delta, y = kappa).  Derivatives by fourth-order central differences,
// third-order one-sided at the grid edges, with step 1e-3: a smaller step
// would difference the rounding noise of the exact overlap at small eta.
constexpr int kTabNodesRegion = (kTabN + 1) * (kTabN + 1);
__global__ __launch_bounds__(256) void k_gtab_build(double* __restrict__ nodes)
{
    const int64_t id = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (id >= 2 * int64_t(kTabNodesRegion)) return;
    const int region = int(id / kTabNodesRegion), k = int(id % kTabNodesRegion);
    const int i = k % (kTabN + 1), j = k / (kTabN + 1);
    const double w = 1.0 / kTabN;
    const double x = i * w, y = j * w;
    auto Q = [region](double xx, double yy) { return region == 0 ? gtab_qa(2.0 * xx, yy) : gtab_qb(xx, yy); };
    const double st = 1e-3;
    auto deriv = [&](bool along_x) {
        const double v = along_x ? x : y;
        auto at = [&](double t) { return along_x ? Q(t, y) : Q(x, t); };
        if (v - 2.0 * st < 0.0)
            return (-11.0 * at(v) + 18.0 * at(v + st) - 9.0 * at(v + 2.0 * st) + 2.0 * at(v + 3.0 * st)) / (6.0 * st);
        if (v + 2.0 * st > 1.0)
            return (11.0 * at(v) - 18.0 * at(v - st) + 9.0 * at(v - 2.0 * st) - 2.0 * at(v - 3.0 * st)) / (6.0 * st);
        return (8.0 * (at(v + st) - at(v - st)) - (at(v + 2.0 * st) - at(v - 2.0 * st))) / (12.0 * st);
    };
    nodes[3 * id] = Q(x, y);
    nodes[3 * id + 1] = deriv(true) * w;
    nodes[3 * id + 2] = deriv(false) * w;
}

// Cell coefficients of the table interpolant from the four corner nodes
// (layout in the comment above overlap_g_table).
__global__ __launch_bounds__(256) void k_gtab_cells(const double* __restrict__ nodes, float4* __restrict__ tab)
{
    const int64_t id = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (id >= int64_t(kTabCells)) return;
    const int region = int(id / kTabCellsRegion), k = int(id % kTabCellsRegion);
    const int i = k % kTabN, j = k / kTabN;
    const double* rn = nodes + 3 * int64_t(region) * kTabNodesRegion;
    auto node = [&](int ii, int jj, int c) { return rn[3 * (int64_t(jj) * (kTabN + 1) + ii) + c]; };
    // Hermite along x on the two y rows: r(a) = R[0] + R[1] a + R[2] a^2 + R[3] a^3
    double R0[4], R1[4];
    for (int row = 0; row < 2; ++row) {
        const double v0 = node(i, j + row, 0), d0 = node(i, j + row, 1);
        const double v1 = node(i + 1, j + row, 0), d1 = node(i + 1, j + row, 1);
        double* R = row == 0 ? R0 : R1;
        R[0] = v0;
        R[1] = d0;
        R[2] = 3.0 * (v1 - v0) - 2.0 * d0 - d1;
        R[3] = 2.0 * (v0 - v1) + d0 + d1;
    }
    // y-derivative, linear along x
    const double E0[2] = {node(i, j, 2), node(i + 1, j, 2) - node(i, j, 2)};
    const double E1[2] = {node(i, j + 1, 2), node(i + 1, j + 1, 2) - node(i, j + 1, 2)};
    // Hermite along y: Q = r0 + e0 b + (3 (r1 - r0) - 2 e0 - e1) b^2 + (2 (r0 - r1) + e0 + e1) b^3
    double P2[4], P3[4];
    for (int c = 0; c < 4; ++c) {
        P2[c] = 3.0 * (R1[c] - R0[c]) - (c < 2 ? 2.0 * E0[c] + E1[c] : 0.0);
        P3[c] = 2.0 * (R0[c] - R1[c]) + (c < 2 ? E0[c] + E1[c] : 0.0);
    }
    float4* cc = tab + 4 * id;
    cc[0] = make_float4(float(R0[0]), float(R0[1]), float(R0[2]), float(R0[3]));
    cc[1] = make_float4(float(P2[0]), float(P2[1]), float(P2[2]), float(P2[3]));
    cc[2] = make_float4(float(P3[0]), float(P3[1]), float(P3[2]), float(P3[3]));
    cc[3] = make_float4(float(E0[0]), float(E0[1]), 0.f, 0.f);
}

template <typename Real>
__global__ __launch_bounds__(256) void k_overlap_eval(int64_t n, const double* d, const double* h1, const double* h2,
                                                      const float4* tab, bool exact, double* out)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double g;
    if (d[i] >= h1[i] + h2[i]) g = 0.0;
    else if (exact) g = double(overlap_g_exact<Real>(Real(d[i]), Real(h1[i]), Real(h2[i])));
    else g = overlap_g_table(tab, d[i] * d[i], h1[i], h2[i]);
    out[i] = g;
}

template <typename Real, int N, int RM>
__global__ __launch_bounds__(256) void k_rates_eval(int64_t n, const double* w, const double* vs, double alpha_n,
                                                    const void* gl_x, const void* gl_w, int gl_k, double hw,
                                                    double bmin, double* A, double* B)
{
    __shared__ Real s_gx[kMaxQuadNodes], s_gw[kMaxQuadNodes];
    if constexpr (RM == kRatesQuad) {
        if (int(threadIdx.x) < gl_k) {
            s_gx[threadIdx.x] = reinterpret_cast<const Real*>(gl_x)[threadIdx.x];
            s_gw[threadIdx.x] = reinterpret_cast<const Real*>(gl_w)[threadIdx.x];
        }
        __syncthreads();
    }
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = vs[i];
    Real w2 = Real(w[i] * w[i]);
    if (s <= 0.0) {
        Real wn = sqrt_real(w2);
        Real Ar = pow_np1<N>(wn);
        A[i] = double(Ar);
        B[i] = double(Ar * w2);
        return;
    }
    Real i2 = Real(1.0 / (2.0 * s * s));
    Real ra = Real(alpha_n / 3.0 * pow(s, double(N + 1))), rb = Real(alpha_n * pow(s, double(N + 3)));
    Real FA, FB;
    if constexpr (RM == kRatesQuad)
        rate_quad<N, Real>(sqrt_real(Real(2) * w2 * i2), s_gx, s_gw, gl_k, Real(1.0 / alpha_n), Real(hw), Real(bmin),
                           &FA, &FB);
    else
        rate_1f1<N, Real>(w2 * i2, &FA, &FB);
    A[i] = double(ra * FA);
    B[i] = double(rb * FB);
}

// The same values from the network, with the arithmetic of the network gas
// pass (binary32; quadrature for u > kMlpUMax; cold gas exact).
struct MlpRatesArgs {
    int64_t n; const double* w; const double* vs; double alpha_n;
    const MlpBlob* mlp; int nidx; float c0A, c1A, c0B, c1B, kA, kB;
    const float* gl_x; const float* gl_w; int gl_k; double hw, bmin;
    double* A; double* B;
};

template <int N>
__global__ __launch_bounds__(256) void k_rates_eval_mlp(MlpRatesArgs a)
{
    __shared__ float s_gx[kMaxQuadNodes], s_gw[kMaxQuadNodes];
    if (int(threadIdx.x) < a.gl_k) {
        s_gx[threadIdx.x] = a.gl_x[threadIdx.x];
        s_gw[threadIdx.x] = a.gl_w[threadIdx.x];
    }
    __syncthreads();
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool ok = i < a.n;
    const double s = ok ? a.vs[i] : 1.0;
    const float w2 = ok ? float(a.w[i] * a.w[i]) : 0.f;
    const bool cold = !(s > 0.0);
    const float i2 = cold ? INFINITY : float(1.0 / (2.0 * s * s));
    const float u = cold ? 0.f : sqrt_real(2.f * w2 * i2);
    const bool net = ok && !cold && u <= kMlpUMax;
    float yA = 0.f, yB = 0.f;
    mlp_forward64(a.mlp, mlp_input(u), a.nidx, &yA, &yB);
    if (!ok) return;
    float Ar, Br;
    if (cold) {
        Ar = pow_np1<N>(sqrt_real(w2));
        Br = Ar * w2;
    } else {
        const float ra = float(a.alpha_n / 3.0 * pow(s, double(N + 1))), rb = float(a.alpha_n * pow(s, double(N + 3)));
        float FA, FB;
        if (net) {
            float bA, bB;
            mlp_base<N>(u * u, a.c0A, a.c1A, a.c0B, a.c1B, &bA, &bB);
            FA = a.kA * bA * __expf(yA);
            FB = a.kB * bB * __expf(yB);
        } else {
            rate_quad<N, float>(u, s_gx, s_gw, a.gl_k, float(1.0 / a.alpha_n), float(a.hw), float(a.bmin), &FA, &FB);
        }
        Ar = ra * FA;
        Br = rb * FB;
    }
    a.A[i] = double(Ar);
    a.B[i] = double(Br);
}

__global__ __launch_bounds__(256) void k_philox_eval(int64_t n, const uint32_t* ctr, uint32_t k0, uint32_t k1,
                                                     uint32_t* out)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    U4 c{ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
    U4 r = philox4x32_10(c, k0, k1);
    out[4 * i] = r.x; out[4 * i + 1] = r.y; out[4 * i + 2] = r.z; out[4 * i + 3] = r.w;
}

}  // namespace dmb
