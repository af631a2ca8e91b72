// dmb_api.hip -- host side of the C ABI declared in include/dmb.h.
//
// Owns the device buffers (grow-only), validates arguments before enqueuing
// anything, and launches the kernels of dmb_kernels.h on the context stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/dmb.h"
#include "dmb_kernels.h"
#include "dmb_sort.h"

using namespace dmb;

namespace {

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    template <typename T> T* as() const { return reinterpret_cast<T*>(p); }
};

struct Species {
    int64_t n = 0, n_own = 0, ntile = 0, nsuper = 0, nmega = 0, nown_tile = 0, nchunk = 0;
    int sort_lo_bit = 0;
    DevBuf sub_ccnt, sub_coff, sub_start, sub_cnt;   // sub-tiles (other role): per-chunk counts/offsets, ranges
    DevBuf keys, keys2, vals, vals2;       // sort
    DevBuf sx, sy, sz, sh;                 // sorted position, h
    DevBuf flag, flag_off, own;            // active owners (sorted positions)
    DevBuf tbox, th, sbox, shh, mbox, mhh, obox, oh;  // sub-tiles, super-, mega-tiles, owner tiles
    DevBuf tsup, ssup, msup;               // support boxes (union of [x - h, x + h]) of sub-, super-, mega-tiles
    DevBuf tq, sq, mq;                     // binary32 candidate-search nodes of sub-, super-, mega-tiles
    DevBuf cube;                           // Morton cube
    DevBuf prec;                           // packed (x, y, z, h) in input order
    // per-step gathers (sorted order)
    DevBuf v0, v1, v2;                     // velocity components (double)
    DevBuf orate;                          // gas: OwnRate<Real> of the active gas, owner-slot order
    DevBuf rec;                            // per-pair records of this species as the other one (GasRec / DmRec)
    const uint32_t* perm = nullptr;        // = vals after the sort
};

struct Pairs {                             // candidate lists: owner tiles of A x sub-tiles of B
    // (owner tile, candidate super-tile) pairs: per-tile counts and offsets, the pairs, their sub-tile masks
    DevBuf cnt, off, psup, ptile, mask, pcnt, soff, pw, woff;
    DevBuf pad, maxcnt;                    // count-pass copy of the first pad_cap super-tiles per tile; largest count
    // groups of 64 owner tiles: bounds (box, h, support, nodes), candidate counts and lists, a spare max
    DevBuf gbox, gh, gsup, gq, gcnt, glist, gmax;
    // candidate sub-tiles: per-tile counts and starts, the lists, work items
    DevBuf scnt, beg, swt, cand, icnt, ioff, it_tile, it_cb, it_ce;
    DevBuf it_key, it_key2, it_id, it_ord;  // item order (largest first): sort keys, item ids, order
    int pad_cap = 128;                     // grown from the largest count seen
    int64_t npairs = 0, total = 0, nitems = 0;
};

// Grow-only scratch of one build + step (scans, radix sort, read-backs).
struct Scratch {
    DevBuf scan_tmp[4];
    DevBuf os_hist;                        // radix sort: digit counts of every pass, then tile counters
    DevBuf os_status;                      // radix sort: look-back words [passes][tiles][256]
    DevBuf bbox_part;
    DevBuf counters_local;
    DevBuf pair_cnt;                       // pair export counts [gas pass, DM pass]
    DevBuf rb_dev;                         // build-stage scalars for the host (one copy per stage)
};

// Cell structure and per-step buffers of one box (one periodic volume or
// open region).  The context keeps one for dmb_build_cells / dmb_interact_step
// and one per box of the batched calls.
struct Cells {
    Species gas, dm;
    Pairs gp, dp;                          // gas owners x DM tiles; DM owners x gas tiles
    DevBuf boxL;                           // periodic side lengths (device, 4 doubles)
    DevBuf part_gas, part_p, part_pm, part_nb, psum_own;
    DevBuf qctr, slist;
    int64_t built_ngas = -1, built_ndm = -1;
    const double* built_gas_pos = nullptr;
    const double* built_dm_pos = nullptr;
    double built_L[3] = {0, 0, 0};
};

}  // namespace

struct dmb_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cu = 256;
    DevBuf gtab;
    DevBuf tilt_gl;                        // 16-point Gauss-Legendre rule of the Rao-Blackwellised draw
    Cells cells;                           // single-box structure
    Cells* X = &cells;                     // structure the internal build / step functions act on
    std::vector<Cells*> boxes;             // batched boxes
    DevBuf bstep, bgeom, bitem;            // batched step: Philox step offset, per-box pass arguments, item offsets
    Scratch heap;                          // per-call scratch of the entry points that allocate
    Scratch* S = &heap;                    // scratch set in use (dmb_step_static swaps in its own)
    // the build runs the gas species' chain on a second stream beside the DM chain on the
    // caller's stream (fork and join by events); that chain has a scratch set of its own
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    Scratch heap2;
    Scratch* S2 = &heap2;
    DevBuf os_err;                         // radix sort: raised when a look-back wait gave up (sticky)
    // pair export (dmb_pair_list): destination lists, capacity
    uint32_t* pair_dst[2] = {nullptr, nullptr};
    int64_t pair_cap = 0;
    // static scratch (dmb_step_static): this device's copy of the file-scope array, and the
    // bump-carving state while a static call runs (arena != nullptr)
    DevBuf run_buf;                        // dmb_run: step outputs, diagnostics, dt
    double* run_dt_host = nullptr;         // pinned: the next step's dt
    char* static_ptr = nullptr;
    char* arena = nullptr;
    size_t arena_cap = 0, arena_off = 0;
    Cells static_cells;
    uint64_t* rb_host = nullptr;           // pinned
    bool pass_overlap = true;              // the two pair passes on two streams (dmb_set_pass_overlap)
    int split = 32;                        // candidate sub-tiles per work item of the DM pass (tunable);
                                           // the gas pass, whose partial sums cost more to combine, twice that
    int item_target_per_cu = 32;           // small problems: split candidate lists into about this many
                                           // work items per compute unit (0: always `split`)
    int item_share = 1;                    // boxes that share the chip in the build under way (batch)
    int subtile_delta = 1;                 // (tunable) sub-tile cut: Morton level below (median - delta)
    int group_cap = 1024;                  // candidate-search group list capacity (0: no group pass)
    int grid_pct = 100;                    // (tunable) persistent grid size, % of the resident maximum
    int batch_n = 0;                       // boxes of the last batch build
    DevBuf gl64, gl32;                     // Gauss-Legendre nodes [x | w] for the quadrature rates
    int gl_k = 0;
    // learned rate closure
    DevBuf mlp_p, mlp_m, mlp_v;            // binary32 master weights, Adam moments
    DevBuf mlp_blob;                       // packed bfloat16 weights (MlpBlob)
    DevBuf mlp_part, mlp_red, mlp_ts, mlp_loss, mlp_epoch, mlp_shuf;
    bool mlp_ready = false;
    hipStream_t train_stream = nullptr;
    // phase timing
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    struct Pending { int phase; hipEvent_t a, b; };
    std::vector<Pending> pending;
    double ph_ms[DMB_NPHASES] = {0};
    int64_t ph_calls[DMB_NPHASES] = {0};
    char err[512] = {0};
};

namespace {

dmb_status fail(dmb_ctx* c, dmb_status st, const char* fmt, ...)
{
    if (c) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(c->err, sizeof(c->err), fmt, ap);
        va_end(ap);
    }
    return st;
}

#define HIPCHK(ctx, call)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) return fail(ctx, DMB_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

dmb_status ensure(dmb_ctx* c, DevBuf& b, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    if (bytes <= b.cap) return DMB_OK;
    if (c->arena) {   // a static call: carve from the static scratch, never allocate
        const size_t off = (c->arena_off + 255) & ~size_t(255);
        if (off > c->arena_cap || bytes > c->arena_cap - off)
            return fail(c, DMB_ENOMEM, "static scratch of %zu bytes exhausted (%zu in use, %zu more requested)",
                        c->arena_cap, off, bytes);
        b.p = c->arena + off;
        b.cap = bytes;
        c->arena_off = off + bytes;
        return DMB_OK;
    }
    if (b.p) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return fail(c, DMB_EHIP, "sync before realloc: %s", hipGetErrorString(e));
        hipFree(b.p);
        b.p = nullptr;
        b.cap = 0;
    }
    size_t nb = bytes + bytes / 4 + 256;
    if (hipMalloc(&b.p, nb) != hipSuccess) {
        b.p = nullptr;
        return fail(c, DMB_ENOMEM, "hipMalloc(%zu) failed", nb);
    }
    b.cap = nb;
    return DMB_OK;
}

#define ENSURE(ctx, buf, bytes)                          \
    do {                                                 \
        dmb_status s_ = ensure(ctx, buf, (bytes));       \
        if (s_ != DMB_OK) return s_;                     \
    } while (0)

hipEvent_t ev_get(dmb_ctx* c)
{
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// RAII phase marker: records a start event now and a stop event on scope exit.
struct Phase {
    dmb_ctx* c;
    int ph;
    hipEvent_t a = nullptr;
    Phase(dmb_ctx* c_, int ph_) : c(c_), ph(ph_)
    {
        if (c->prof && (a = ev_get(c))) hipEventRecord(a, c->stream);
    }
    ~Phase()
    {
        if (!a) return;
        hipEvent_t b = ev_get(c);
        if (!b) { c->ev_pool.push_back(a); return; }
        hipEventRecord(b, c->stream);
        c->pending.push_back({ph, a, b});
    }
};

inline unsigned blocks_for(int64_t n, int bs) { return unsigned((n + bs - 1) / bs); }

// Exclusive scan of n values (TI in, TO out and partial sums) into out (out
// may equal in when the types agree); inputs from n_in on (n_in <= n) read
// as 0, so out[n_in] receives the total without touching in[n_in].
template <typename TI = uint32_t, typename TO = uint32_t>
dmb_status scan_excl(dmb_ctx* c, const TI* in, TO* out, int64_t n, int64_t n_in = -1, int level = 0)
{
    if (n <= 0) return DMB_OK;
    if (n_in < 0 || n_in > n) n_in = n;
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (level >= 4) return fail(c, DMB_EINVAL, "scan too large");
    ENSURE(c, c->S->scan_tmp[level], size_t(nb + 1) * sizeof(TO));
    TO* sums = c->S->scan_tmp[level].as<TO>();
    hipLaunchKernelGGL((k_scan_block<TI, TO>), dim3(unsigned(nb)), dim3(kScanBlock), 0, c->stream, in, out, sums, n,
                       n_in);
    if (nb > 1 && nb <= kScanOwnMax) {
        hipLaunchKernelGGL(k_scan_add_own<TO>, dim3(unsigned(nb)), dim3(kScanBlock), 0, c->stream, out,
                           (const TO*)sums, n);
    } else if (nb > 1) {
        dmb_status s = scan_excl<TO, TO>(c, sums, sums, nb, nb, level + 1);
        if (s != DMB_OK) return s;
        hipLaunchKernelGGL(k_scan_add<TO>, dim3(unsigned(nb)), dim3(kScanBlock), 0, c->stream, out, sums, n);
    }
    HIPCHK(c, hipGetLastError());
    return DMB_OK;
}

// Stable LSD radix sort of n (key, value) pairs by the key bits
// [lo_bit, lo_bit + 8 passes), ping-ponging between (ka, va) and (kb, vb);
// on return *ka, *va point at the sorted arrays.  A raised look-back error
// is reported by the next build's first read-back.
__global__ __launch_bounds__(256) void k_os_clear(uint32_t* __restrict__ w, int n)
{
    for (int i = int(threadIdx.x); i < n; i += 256) w[i] = 0u;
}

dmb_status radix_sort(dmb_ctx* c, uint64_t** ka, uint32_t** va, uint64_t** kb, uint32_t** vb, int64_t n, int lo_bit,
                      int passes)
{
    if (n <= 0 || passes <= 0) return DMB_OK;
    if (passes > kOsMaxPasses) return fail(c, DMB_EINVAL, "radix sort: %d passes", passes);
    const int64_t ntile = (n + kOsTile - 1) / kOsTile;
    const int nw = kOsMaxPasses * 256 + kOsMaxPasses;
    ENSURE(c, c->S->os_hist, size_t(nw) * 4);
    ENSURE(c, c->S->os_status, size_t(passes) * size_t(ntile) * 256 * 8);
    OsArgs a;
    a.n = n; a.passes = passes; a.lo_bit = lo_bit;
    a.hist = c->S->os_hist.as<uint32_t>();
    a.tile_ctr = a.hist + kOsMaxPasses * 256;
    a.status = c->S->os_status.as<unsigned long long>();
    a.err = c->os_err.as<uint32_t>();
    a.ntile = ntile;
    hipLaunchKernelGGL(k_os_clear, dim3(1), dim3(256), 0, c->stream, a.hist, nw);
    const int hb = int(std::min<int64_t>(2048, std::max<int64_t>(ntile, (int64_t(passes) * ntile * 256 + 4095) / 4096)));
    hipLaunchKernelGGL(k_os_hist, dim3(hb), dim3(kOsHistBlock), 0, c->stream, *ka, a);
    for (int p = 0; p < passes; ++p) {
        hipLaunchKernelGGL(k_os_pass, dim3(unsigned(ntile)), dim3(kOsBlock), 0, c->stream, *ka, *va, *kb, *vb, a, p);
        std::swap(*ka, *kb);
        std::swap(*va, *vb);
    }
    HIPCHK(c, hipGetLastError());
    return DMB_OK;
}

int bits_for(int64_t n)
{
    int b = 1;
    while ((int64_t(1) << b) < n) ++b;
    return b;
}

dmb_status check_particles(dmb_ctx* c, const dmb_particles* p, const char* name, bool gas)
{
    if (!p) return fail(c, DMB_EINVAL, "%s: null particle struct", name);
    if (p->n < 0) return fail(c, DMB_EINVAL, "%s: n < 0", name);
    if (p->n >= (int64_t(1) << 31)) return fail(c, DMB_ERANGE, "%s: n >= 2^31", name);
    if (p->n > 0 && (!p->pos || !p->h)) return fail(c, DMB_EINVAL, "%s: null pos or h", name);
    (void)gas;
    return DMB_OK;
}

// Morton sort + tiles + owner tiles + super tiles for one species.
dmb_status build_species(dmb_ctx* c, Species& S, const dmb_particles* p)
{
    S.n = p->n;
    if (S.n == 0) {
        S.n_own = S.ntile = S.nsuper = S.nmega = S.nown_tile = S.nchunk = 0;
        return DMB_OK;
    }
    const int64_t n = S.n;
    ENSURE(c, S.keys, n * 8); ENSURE(c, S.keys2, n * 8);
    ENSURE(c, S.vals, n * 4); ENSURE(c, S.vals2, n * 4);
    ENSURE(c, S.cube, 8 * sizeof(double));
    // bounding box (k_bbox_final takes [0, L) when L_x > 0, so the partial pass is skipped
    // then); enough blocks to fill the chip
    const bool periodic = c->X->built_L[0] > 0.0;
    const int nparts = periodic ? 0 : int(std::min<int64_t>(2048, (n + 1023) / 1024));
    ENSURE(c, c->S->bbox_part, std::max(nparts, 1) * 6 * sizeof(double));
    if (nparts > 0)
        hipLaunchKernelGGL(k_bbox_partial, dim3(nparts), dim3(256), 0, c->stream, p->pos, n, c->S->bbox_part.as<double>());
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(64), 0, c->stream, c->S->bbox_part.as<const double>(), nparts,
                       c->X->boxL.as<const double>(), S.cube.as<double>());
    ENSURE(c, S.prec, n * sizeof(double4));
    hipLaunchKernelGGL(k_morton, dim3(blocks_for(n, 256)), dim3(256), 0, c->stream, p->pos, p->h, n,
                       S.cube.as<const double>(), c->X->boxL.as<const double>(), S.keys.as<uint64_t>(),
                       S.vals.as<uint32_t>(), S.prec.as<double4>());
    // radix sort on the top bits that resolve ~2^6 particles per cell
    int need = std::min(63, std::max(24, 3 * ((bits_for(n) + 6 + 2) / 3)));
    int passes = (need + 7) / 8;
    // stable LSD radix sort of the keys' bits [63 - 8 passes, 63)
    const int lo_bit = std::max(0, 63 - 8 * passes);
    uint64_t *ka = S.keys.as<uint64_t>(), *kb = S.keys2.as<uint64_t>();
    uint32_t *va = S.vals.as<uint32_t>(), *vb = S.vals2.as<uint32_t>();
    {
        dmb_status s0 = radix_sort(c, &ka, &va, &kb, &vb, n, lo_bit, passes);
        if (s0 != DMB_OK) return s0;
    }
    S.sort_lo_bit = std::max(0, 63 - 8 * passes);
    // keep the sorted permutation in S.vals
    if (va != S.vals.as<uint32_t>()) {
        std::swap(S.vals, S.vals2);
        std::swap(S.keys, S.keys2);
    }
    S.perm = S.vals.as<const uint32_t>();
    // sorted position and h are gathered by k_subtile_write
    ENSURE(c, S.sx, n * 8); ENSURE(c, S.sy, n * 8); ENSURE(c, S.sz, n * 8); ENSURE(c, S.sh, n * 8);
    // owners (active subset, Morton order)
    ENSURE(c, S.flag, (n + 1) * 4); ENSURE(c, S.flag_off, (n + 1) * 4); ENSURE(c, S.own, n * 4);
    hipLaunchKernelGGL(k_active_flags, dim3(blocks_for(n + 1, 256)), dim3(256), 0, c->stream, S.perm, n, p->active,
                       S.flag.as<uint32_t>());
    dmb_status s = scan_excl(c, S.flag.as<const uint32_t>(), S.flag_off.as<uint32_t>(), n + 1);
    if (s != DMB_OK) return s;
    hipLaunchKernelGGL(k_compact, dim3(blocks_for(n, 256)), dim3(256), 0, c->stream, S.flag.as<const uint32_t>(),
                       S.flag_off.as<const uint32_t>(), n, S.own.as<uint32_t>());
    // sub-tile counts per 64-chunk (other role); totals are read back by the caller
    S.nchunk = (n + kTile - 1) / kTile;
    ENSURE(c, S.sub_ccnt, (S.nchunk + 1) * 4); ENSURE(c, S.sub_coff, (S.nchunk + 1) * 4);
    hipLaunchKernelGGL(k_subtile_count, dim3(unsigned(S.nchunk)), dim3(64), 0, c->stream,
                       S.keys.as<const uint64_t>(), n, S.sort_lo_bit, c->subtile_delta, S.sub_ccnt.as<uint32_t>());
    s = scan_excl(c, S.sub_ccnt.as<const uint32_t>(), S.sub_coff.as<uint32_t>(), S.nchunk + 1, S.nchunk);
    if (s != DMB_OK) return s;
    HIPCHK(c, hipGetLastError());
    return DMB_OK;
}

// Sub-tile ranges and bounds, super-tiles (needs the sub-tile count).
dmb_status build_subtiles(dmb_ctx* c, Species& S)
{
    if (S.n == 0) return DMB_OK;
    ENSURE(c, S.sub_start, S.ntile * 4); ENSURE(c, S.sub_cnt, S.ntile * 4);
    S.nsuper = (S.ntile + kTile - 1) / kTile;
    ENSURE(c, S.tbox, S.ntile * 48); ENSURE(c, S.th, S.ntile * 8); ENSURE(c, S.tsup, S.ntile * 48);
    ENSURE(c, S.sbox, S.nsuper * 48); ENSURE(c, S.shh, S.nsuper * 8); ENSURE(c, S.ssup, S.nsuper * 48);
    ENSURE(c, S.tq, S.ntile * 64); ENSURE(c, S.sq, S.nsuper * 64);
    hipLaunchKernelGGL(k_subtile_write, dim3(unsigned(S.nchunk)), dim3(64), 0, c->stream,
                       S.keys.as<const uint64_t>(), S.n, S.sort_lo_bit, c->subtile_delta,
                       S.sub_coff.as<const uint32_t>(), S.sub_start.as<uint32_t>(), S.sub_cnt.as<uint32_t>(),
                       S.perm, S.prec.as<const double4>(), S.sx.as<double>(), S.sy.as<double>(),
                       S.sz.as<double>(), S.sh.as<double>(), S.tbox.as<double>(), S.th.as<double>(),
                       S.tsup.as<double>(), S.tq.as<float4>());
    hipLaunchKernelGGL(k_super_bounds, dim3(unsigned(S.nsuper)), dim3(64), 0, c->stream, S.ntile,
                       S.tbox.as<const double>(), S.th.as<const double>(), S.tsup.as<const double>(),
                       S.sbox.as<double>(), S.shh.as<double>(), S.ssup.as<double>(), S.sq.as<float4>());
    S.nmega = (S.nsuper + kTile - 1) / kTile;
    ENSURE(c, S.mbox, S.nmega * 48); ENSURE(c, S.mhh, S.nmega * 8); ENSURE(c, S.msup, S.nmega * 48);
    ENSURE(c, S.mq, S.nmega * 64);
    hipLaunchKernelGGL(k_super_bounds, dim3(unsigned(S.nmega)), dim3(64), 0, c->stream, S.nsuper,
                       S.sbox.as<const double>(), S.shh.as<const double>(), S.ssup.as<const double>(),
                       S.mbox.as<double>(), S.mhh.as<double>(), S.msup.as<double>(), S.mq.as<float4>());
    HIPCHK(c, hipGetLastError());
    return DMB_OK;
}

// Owner tiles need n_own, known after a read-back.
dmb_status build_owner_tiles(dmb_ctx* c, Species& S)
{
    S.nown_tile = (S.n_own + kTile - 1) / kTile;
    if (S.nown_tile == 0) return DMB_OK;
    ENSURE(c, S.obox, S.nown_tile * 48); ENSURE(c, S.oh, S.nown_tile * 8);
    hipLaunchKernelGGL(k_tile_bounds, dim3(unsigned(S.nown_tile)), dim3(64), 0, c->stream, S.own.as<const uint32_t>(),
                       S.n_own, S.sx.as<const double>(), S.sy.as<const double>(), S.sz.as<const double>(),
                       S.sh.as<const double>(), S.obox.as<double>(), S.oh.as<double>());
    HIPCHK(c, hipGetLastError());
    return DMB_OK;
}

CandArgs cand_args(dmb_ctx* c, Species& A, Species& B, Pairs& P)
{
    CandArgs a;
    a.nown_tile = A.nown_tile; a.ntile = B.ntile; a.nsuper = B.nsuper; a.nmega = B.nmega;
    a.obox = A.obox.as<const double>(); a.oh = A.oh.as<const double>();
    a.sq = B.sq.as<const float4>(); a.mq = B.mq.as<const float4>();
    for (int k = 0; k < 3; ++k) a.L[k] = c->X->built_L[k];
    a.cnt = P.cnt.as<uint32_t>(); a.off = P.off.as<const uint64_t>(); a.cand = P.cand.as<uint32_t>();
    a.pad = P.pad.as<uint32_t>(); a.pad_cap = P.pad_cap; a.maxcnt = P.maxcnt.as<uint32_t>();
    a.cand = P.psup.as<uint32_t>(); a.ptile = P.ptile.as<uint32_t>();
    a.gcap = c->group_cap;
    a.gcnt = c->group_cap > 0 ? P.gcnt.as<const uint32_t>() : nullptr;
    a.glist = c->group_cap > 0 ? P.glist.as<const uint32_t>() : nullptr;
    return a;
}

dmb_status cand_count(dmb_ctx* c, Species& A, Species& B, Pairs& P)
{
    int64_t nt = A.nown_tile;
    ENSURE(c, P.cnt, (nt + 1) * 4); ENSURE(c, P.off, (nt + 1) * 8);
    ENSURE(c, P.icnt, (nt + 1) * 4); ENSURE(c, P.ioff, (nt + 1) * 4);
    ENSURE(c, P.scnt, (nt + 1) * 4); ENSURE(c, P.beg, (nt + 1) * 8);
    if (nt == 0 || B.ntile == 0) {
        HIPCHK(c, hipMemsetAsync(P.off.p, 0, (nt + 1) * 8, c->stream));
        HIPCHK(c, hipMemsetAsync(P.ioff.p, 0, (nt + 1) * 4, c->stream));
        return DMB_OK;
    }
    // the candidate copy kept by the count pass: at most kPadBytes in all
    constexpr int64_t kPadBytes = int64_t(3) << 30;
    P.pad_cap = int(std::max<int64_t>(0, std::min<int64_t>(P.pad_cap, kPadBytes / (4 * nt))));
    ENSURE(c, P.pad, std::max<int64_t>(1, nt * P.pad_cap) * 4);
    ENSURE(c, P.maxcnt, 4);
    HIPCHK(c, hipMemsetAsync(P.maxcnt.p, 0, 4, c->stream));
    // group lists: a count pass over groups of 64 owner tiles, their lists kept in glist
    if (c->group_cap > 0) {
        const int64_t ng = (nt + kTile - 1) / kTile;
        ENSURE(c, P.gbox, ng * 48); ENSURE(c, P.gh, ng * 8); ENSURE(c, P.gsup, ng * 48); ENSURE(c, P.gq, ng * 64);
        ENSURE(c, P.gcnt, ng * 4); ENSURE(c, P.glist, ng * c->group_cap * 4); ENSURE(c, P.gmax, 4);
        hipLaunchKernelGGL(k_super_bounds, dim3(unsigned(ng)), dim3(64), 0, c->stream, nt,
                           A.obox.as<const double>(), A.oh.as<const double>(), A.obox.as<const double>(),
                           P.gbox.as<double>(), P.gh.as<double>(), P.gsup.as<double>(), P.gq.as<float4>());
        CandArgs ga = cand_args(c, A, B, P);
        ga.nown_tile = ng; ga.obox = P.gbox.as<const double>(); ga.oh = P.gh.as<const double>();
        ga.cnt = P.gcnt.as<uint32_t>(); ga.pad = P.glist.as<uint32_t>(); ga.pad_cap = c->group_cap;
        ga.maxcnt = P.gmax.as<uint32_t>(); ga.gcnt = nullptr; ga.glist = nullptr;
        hipLaunchKernelGGL(k_cand<false>, dim3(unsigned((ng + kXcd - 1) / kXcd * kXcd)), dim3(64), 0, c->stream,
                           ga);
    }
    CandArgs a = cand_args(c, A, B, P);
    const unsigned grid = unsigned((nt + kXcd - 1) / kXcd * kXcd);
    hipLaunchKernelGGL(k_cand<false>, dim3(grid), dim3(64), 0, c->stream, a);
    dmb_status s = scan_excl<uint32_t, uint64_t>(c, P.cnt.as<const uint32_t>(), P.off.as<uint64_t>(), nt + 1, nt);
    if (s != DMB_OK) return s;
    HIPCHK(c, hipGetLastError());
    return DMB_OK;
}

// Pair list, sub-tile masks and counts, work-item counts (needs P.npairs).
dmb_status cand_subs(dmb_ctx* c, Species& A, Species& B, Pairs& P)
{
    int64_t nt = A.nown_tile;
    if (nt == 0 || B.ntile == 0 || P.npairs == 0) {
        if (nt > 0) {
            HIPCHK(c, hipMemsetAsync(P.scnt.p, 0, (nt + 1) * 4, c->stream));
            HIPCHK(c, hipMemsetAsync(P.ioff.p, 0, (nt + 1) * 4, c->stream));
        }
        return DMB_OK;
    }
    const int64_t np = P.npairs;
    ENSURE(c, P.psup, np * 4); ENSURE(c, P.ptile, np * 4);
    ENSURE(c, P.mask, np * 8); ENSURE(c, P.pcnt, (np + 1) * 4); ENSURE(c, P.soff, (np + 1) * 8);
    ENSURE(c, P.pw, (np + 1) * 4); ENSURE(c, P.woff, (np + 1) * 8); ENSURE(c, P.swt, (nt + 1) * 4);
    CandArgs a = cand_args(c, A, B, P);
    hipLaunchKernelGGL(k_cand<true>, dim3(unsigned((nt + kXcd - 1) / kXcd * kXcd)), dim3(64), 0, c->stream, a);
    SubMaskArgs m;
    m.npairs = np; m.ntile = B.ntile;
    m.ptile = P.ptile.as<const uint32_t>(); m.psup = P.psup.as<const uint32_t>();
    m.obox = A.obox.as<const double>(); m.oh = A.oh.as<const double>();
    m.tq = B.tq.as<const float4>();
    for (int k = 0; k < 3; ++k) m.L[k] = c->X->built_L[k];
    m.sub_cnt = B.sub_cnt.as<const uint32_t>();
    m.mask = P.mask.as<uint64_t>(); m.pcnt = P.pcnt.as<uint32_t>(); m.pw = P.pw.as<uint32_t>();
    hipLaunchKernelGGL(k_sub_masks, dim3(unsigned((np + kSubPairs - 1) / kSubPairs)), dim3(64), 0, c->stream, m);
    // candidate offsets in 64 bits (totals pass 2^32 at Milky-Way sizes)
    dmb_status s =
        scan_excl<uint32_t, uint64_t>(c, P.pcnt.as<const uint32_t>(), P.soff.as<uint64_t>(), np + 1, np);
    if (s != DMB_OK) return s;
    s = scan_excl<uint32_t, uint64_t>(c, P.pw.as<const uint32_t>(), P.woff.as<uint64_t>(), np + 1, np);
    if (s != DMB_OK) return s;
    hipLaunchKernelGGL(k_tile_subs, dim3(blocks_for(nt + 1, 256)), dim3(256), 0, c->stream, nt,
                       P.off.as<const uint64_t>(), P.soff.as<const uint64_t>(), P.woff.as<const uint64_t>(),
                       P.scnt.as<uint32_t>(), P.beg.as<uint64_t>(), P.swt.as<uint32_t>());
    hipLaunchKernelGGL(k_item_count, dim3(blocks_for(nt + 1, 256)), dim3(256), 0, c->stream,
                       P.scnt.as<const uint32_t>(), nt, uint32_t(&P == &c->X->gp ? 2 * c->split : c->split),
                       P.soff.as<const uint64_t>() + np,
                       uint32_t(int64_t(c->item_target_per_cu) * c->num_cu / std::max(1, c->item_share)),
                       P.icnt.as<uint32_t>());
    s = scan_excl(c, P.icnt.as<const uint32_t>(), P.ioff.as<uint32_t>(), nt + 1);
    if (s != DMB_OK) return s;
    HIPCHK(c, hipGetLastError());
    return DMB_OK;
}

// Candidate sub-tile lists and work items (needs P.total, P.nitems).
dmb_status cand_write(dmb_ctx* c, Species& A, Species& B, Pairs& P)
{
    int64_t nt = A.nown_tile;
    ENSURE(c, P.cand, std::max<int64_t>(P.total, 1) * 4);
    ENSURE(c, P.it_tile, std::max<int64_t>(P.nitems, 1) * 4);
    ENSURE(c, P.it_cb, std::max<int64_t>(P.nitems, 1) * 8);
    ENSURE(c, P.it_ce, std::max<int64_t>(P.nitems, 1) * 8);
    if (nt == 0 || B.ntile == 0 || P.total == 0) return DMB_OK;
    hipLaunchKernelGGL(k_expand, dim3(blocks_for(P.npairs, 256)), dim3(256), 0, c->stream, P.npairs,
                       P.psup.as<const uint32_t>(), P.mask.as<const uint64_t>(), P.soff.as<const uint64_t>(),
                       P.cand.as<uint32_t>());
    const int64_t ni = P.nitems;
    ENSURE(c, P.it_key, std::max<int64_t>(ni, 1) * 8); ENSURE(c, P.it_key2, std::max<int64_t>(ni, 1) * 8);
    ENSURE(c, P.it_id, std::max<int64_t>(ni, 1) * 4); ENSURE(c, P.it_ord, std::max<int64_t>(ni, 1) * 4);
    hipLaunchKernelGGL(k_item_write, dim3(blocks_for(ni, 256)), dim3(256), 0, c->stream, P.beg.as<const uint64_t>(),
                       P.scnt.as<const uint32_t>(), P.swt.as<const uint32_t>(), P.ioff.as<const uint32_t>(), nt, ni,
                       P.it_tile.as<uint32_t>(), P.it_cb.as<uint64_t>(), P.it_ce.as<uint64_t>(),
                       P.it_key.as<uint64_t>(), P.it_id.as<uint32_t>());
    uint64_t *ka = P.it_key.as<uint64_t>(), *kb = P.it_key2.as<uint64_t>();
    uint32_t *va = P.it_id.as<uint32_t>(), *vb = P.it_ord.as<uint32_t>();
    dmb_status s = radix_sort(c, &ka, &va, &kb, &vb, ni, 0, 1);   // one pass: the order lands in it_ord
    if (s != DMB_OK) return s;
    HIPCHK(c, hipGetLastError());
    return DMB_OK;
}

double alpha_n(int n) { return std::pow(2.0, 0.5 * (n + 5)) * std::tgamma(3.0 + 0.5 * n) / std::sqrt(kPi); }

bool n_supported(int n) { return n == -4 || n == -2 || n == 0 || n == 2; }

// K-point Gauss-Legendre nodes and weights on [-1, 1]: Newton iteration on the
// Legendre recurrence from the asymptotic initial guess.
void gauss_legendre(int K, double* x, double* w)
{
    for (int i = 0; i < K; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (K + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int j = 2; j <= K; ++j) {
                double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            if (K == 1) p0 = 1.0;
            dp = K * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int j = 2; j <= K; ++j) {
            double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
            p0 = p1;
            p1 = p2;
        }
        dp = K * (z * p1 - p0) / (z * z - 1.0);
        x[K - 1 - i] = z;
        w[K - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

dmb_status ensure_quad_nodes(dmb_ctx* c, int K)
{
    if (K == c->gl_k) return DMB_OK;
    ENSURE(c, c->gl64, 2 * kMaxQuadNodes * sizeof(double));
    ENSURE(c, c->gl32, 2 * kMaxQuadNodes * sizeof(float));
    double h64[2 * kMaxQuadNodes] = {0};
    float h32[2 * kMaxQuadNodes] = {0};
    gauss_legendre(K, h64, h64 + kMaxQuadNodes);
    for (int k = 0; k < 2 * kMaxQuadNodes; ++k) h32[k] = float(h64[k]);
    HIPCHK(c, hipMemcpyAsync(c->gl64.p, h64, sizeof(h64), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->gl32.p, h32, sizeof(h32), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->gl_k = K;
    return DMB_OK;
}

int quad_k(const dmb_params* p) { return p->quad_nodes == 0 ? 32 : p->quad_nodes; }

PassGeom geom(Cells& X, Species& A, Species& B, Pairs& P, uint64_t* counters)
{
    PassGeom g;
    g.own = A.own.as<const uint32_t>(); g.n_own = A.n_own;
    g.ox = A.sx.as<const double>(); g.oy = A.sy.as<const double>(); g.oz = A.sz.as<const double>();
    g.oh = A.sh.as<const double>(); g.obox = A.obox.as<const double>();
    g.tx = B.sx.as<const double>(); g.ty = B.sy.as<const double>(); g.tz = B.sz.as<const double>();
    g.th = B.sh.as<const double>(); g.n_other = B.n; g.tbox = B.tbox.as<const double>();
    g.thmax = B.th.as<const double>();
    g.sub_start = B.sub_start.as<const uint32_t>(); g.sub_cnt = B.sub_cnt.as<const uint32_t>();
    g.cand = P.cand.as<const uint32_t>();
    g.item_off = P.ioff.as<const uint32_t>();
    g.item_order = P.it_ord.as<const uint32_t>();
    g.it_tile = P.it_tile.as<const uint32_t>(); g.it_cb = P.it_cb.as<const uint64_t>();
    g.it_ce = P.it_ce.as<const uint64_t>(); g.n_items = P.nitems;
    g.queue_ctr = X.qctr.as<uint32_t>();
    for (int k = 0; k < 3; ++k) g.L[k] = X.built_L[k];
    g.counters = counters;
    g.pairs = nullptr; g.pair_n = nullptr; g.pair_cap = 0;
    return g;
}

// Persistent grid: as many blocks of `threads` as can be resident, capped by need.
int persist_blocks(dmb_ctx* c, const void* fn, int threads, int64_t want)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, 0) != hipSuccess || per_cu < 1) per_cu = 8;
    const int64_t full = std::max<int64_t>(8, (int64_t(c->num_cu) * per_cu * c->grid_pct / 100 / 8) * 8);
    return int(std::max<int64_t>(8, std::min<int64_t>(full, ((want + 7) / 8) * 8)));
}

double sig_kpc2_cn_of(const dmb_params* par)
{
    return par->sigma0_cm2 / (kKpcCm * kKpcCm) * std::pow(kCKms, -double(par->n_pow));
}

// Work enqueued inside an OnSide scope goes to the side stream with the side
// scratch set; fork() makes the side stream wait for the caller's stream so
// far, join() the caller's stream for the side stream.
struct OnSide {
    dmb_ctx* c;
    hipStream_t st;
    Scratch* sc;
    bool on;
    explicit OnSide(dmb_ctx* c_, bool on_ = true) : c(c_), st(c_->stream), sc(c_->S), on(on_)
    {
        if (on) { c->stream = c->side; c->S = c->S2; }
    }
    ~OnSide() { c->stream = st; c->S = sc; }
};

dmb_status fork(dmb_ctx* c)
{
    HIPCHK(c, hipEventRecord(c->ev_fork, c->stream));
    HIPCHK(c, hipStreamWaitEvent(c->side, c->ev_fork, 0));
    return DMB_OK;
}

dmb_status join(dmb_ctx* c)
{
    HIPCHK(c, hipEventRecord(c->ev_join, c->side));
    HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_join, 0));
    return DMB_OK;
}

// Runs a(gas side) on the side stream and b (DM side) on the caller's stream;
// both are enqueued before either status is checked, and the join comes first.
template <typename FA, typename FB>
dmb_status both(dmb_ctx* c, FA&& a, FB&& b)
{
    dmb_status s = fork(c);
    if (s != DMB_OK) return s;
    dmb_status sa;
    {
        OnSide on(c);
        sa = a();
    }
    dmb_status sb = b();
    dmb_status sj = join(c);
    if (sa != DMB_OK) return sa;
    if (sb != DMB_OK) return sb;
    return sj;
}

// Per-step gathers into Morton order and the clearing of outputs, counters
// and the box's queue counters (qctr: [0, 8) gas queue, [8, 16) DM queue,
// [16] scatter count).  Buffers are sized first; with `overlap` the gas
// gather runs on the side stream beside the DM gather (both are bound by
// the latency of their indexed reads).
template <typename Real, int RM>
dmb_status gather_and_fill(dmb_ctx* c, Cells& X, const dmb_particles* gas, const dmb_particles* dm,
                           const dmb_params* par, dmb_out* out, uint64_t* counters, bool overlap = false)
{
    Species& G = X.gas;
    Species& D = X.dm;
    const int rs = int(sizeof(Real));
    if (G.n > 0) {
        ENSURE(c, G.v0, G.n * 8); ENSURE(c, G.v1, G.n * 8); ENSURE(c, G.v2, G.n * 8);
        ENSURE(c, G.orate, std::max<int64_t>(G.n_own, 1) * rs * 4);
        ENSURE(c, G.rec, G.n * (sizeof(Real) == 4 ? sizeof(GasRec<float>) : sizeof(GasRec<double>)));
    }
    if (D.n > 0) ENSURE(c, D.rec, D.n * (sizeof(Real) == 4 ? sizeof(DmRec<float>) : sizeof(DmRec<double>)));
    ENSURE(c, X.qctr, (2 * kXcd + 4) * 4);
    if (X.gp.nitems > 0) ENSURE(c, X.part_gas, size_t(X.gp.nitems) * kTile * gas_sums<RM>() * 8);
    if (X.dp.nitems > 0) {
        ENSURE(c, X.part_p, size_t(X.dp.nitems) * kTile * 8);
        ENSURE(c, X.part_pm, size_t(X.dp.nitems) * kTile * 4);
        ENSURE(c, X.part_nb, size_t(X.dp.nitems) * kTile);
        ENSURE(c, X.psum_own, size_t(D.n_own) * 8);
        ENSURE(c, X.slist, size_t(D.n_own) * 4);
    }
    auto gas_gather = [&] {
        GasGatherArgs ga;
        ga.n = G.n; ga.perm = G.perm; ga.vel = gas->vel; ga.mass = gas->mass; ga.u = gas->u; ga.mu = gas->mu;
        ga.m_chi = par->m_chi_g; ga.sig_kpc2_cn = sig_kpc2_cn_of(par); ga.alpha_n = alpha_n(par->n_pow);
        ga.n_pow = par->n_pow;
        ga.rb = par->dm_sampling == DMB_SAMPLE_RB;
        ga.alpha_rb = ga.rb ? alpha_n(par->n_pow - 2) : 0.0;
        ga.Vx = G.v0.as<double>(); ga.Vy = G.v1.as<double>(); ga.Vz = G.v2.as<double>();
        ga.flag = G.flag.as<const uint32_t>(); ga.flag_off = G.flag_off.as<const uint32_t>();
        ga.orate = G.orate.p;
        ga.rec = G.rec.p;
        hipLaunchKernelGGL(k_gather_gas<Real>, dim3(blocks_for(G.n, 256)), dim3(256), 0, c->stream, ga);
    };
    const bool side = overlap && G.n > 0 && D.n > 0;
    if (side) {
        dmb_status s = fork(c);
        if (s != DMB_OK) return s;
        OnSide on(c);
        gas_gather();
    } else if (G.n > 0) {
        gas_gather();
    }
    if (D.n > 0) {
        DmGatherArgs da;
        da.n = D.n; da.perm = D.perm; da.vel = dm->vel; da.mass = dm->mass; da.dt = dm->dt;
        da.dt_default = par->dt;
        da.rec = D.rec.p;
        hipLaunchKernelGGL(k_gather_dm<Real>, dim3(blocks_for(D.n, 256)), dim3(256), 0, c->stream, da);
    }
    int64_t nfill = std::max<int64_t>(std::max<int64_t>(G.n, D.n), 2 * kXcd + 4);
    hipLaunchKernelGGL(k_fill_out, dim3(blocks_for(nfill, 256)), dim3(256), 0, c->stream, G.n, D.n, out->dp_gas,
                       out->de_gas, out->dv_dm, out->partner, out->p_sum, out->p_max, counters,
                       X.qctr.as<uint32_t>(), 2 * kXcd + 4);
    if (side) {
        dmb_status s = join(c);
        if (s != DMB_OK) return s;
    }
    HIPCHK(c, hipGetLastError());
    return DMB_OK;
}

template <typename Real, int N, int RM>
GasPassArgs gas_pass_args(dmb_ctx* c, Cells& X, const dmb_particles* gas, const dmb_params* par, dmb_out* out,
                          uint64_t* counters)
{
    Species& G = X.gas;
    Species& D = X.dm;
    GasPassArgs a;
    a.g = geom(X, G, D, X.gp, counters);
    a.Vx = G.v0.as<const double>(); a.Vy = G.v1.as<const double>(); a.Vz = G.v2.as<const double>();
    a.orate = G.orate.p;
    a.drec = D.rec.p;
    a.gtab = c->gtab.as<const float4>();
    const DevBuf& glb = sizeof(Real) == 8 ? c->gl64 : c->gl32;
    a.gl_x = glb.p;
    a.gl_w = glb.p ? static_cast<const char*>(glb.p) + kMaxQuadNodes * sizeof(Real) : nullptr;
    a.gl_k = c->gl_k;
    a.inv_alpha = 1.0 / alpha_n(par->n_pow);
    quad_window(c->gl_k, &a.gl_hw, &a.gl_bmin);
    a.mlp = nullptr;
    if constexpr (RM == kRatesMlp) {
        const double al = alpha_n(N);
        a.mlp = c->mlp_blob.as<const MlpBlob>();
        a.mlp_nidx = mlp_n_index(N);
        a.mlp_c0A = float(std::pow(al / 3.0, 4.0 / (N + 1)));
        a.mlp_c0B = float(std::pow(al, 4.0 / (N + 3)));
        a.mlp_c1A = float(kMlpC1[mlp_n_index(N)][0]);
        a.mlp_c1B = float(kMlpC1[mlp_n_index(N)][1]);
        a.mlp_kA = float(3.0 / al);
        a.mlp_kB = float(1.0 / al);
    }
    a.part = X.part_gas.as<double>();
    a.perm = G.perm; a.mass = gas->mass; a.mu = gas->mu; a.dt = gas->dt; a.u = gas->u; a.dt_default = par->dt;
    // the gas rates take the momentum-transfer cross section sigma-bar = (1 - g) sigma
    a.m_chi = par->m_chi_g; a.sig_kpc2_cn = sig_kpc2_cn_of(par) * (1.0 - par->aniso_g);
    a.alpha_n = alpha_n(par->n_pow);
    a.dp = out->dp_gas; a.de = out->de_gas;
    return a;
}

template <int N, int RM>
void combine_gas(dmb_ctx* c, Cells& X, const dmb_particles* gas, const dmb_params* par, dmb_out* out)
{
    Species& G = X.gas;
    GasCombineArgs cb;
    cb.n_own = G.n_own; cb.own = G.own.as<const uint32_t>(); cb.perm = G.perm;
    cb.item_off = X.gp.ioff.as<const uint32_t>(); cb.part = X.part_gas.as<const double>();
    cb.out = GasOutArgs{gas->mass, gas->mu, gas->dt, gas->u, par->dt, par->m_chi_g,
                        sig_kpc2_cn_of(par) * (1.0 - par->aniso_g), alpha_n(par->n_pow), out->dp_gas, out->de_gas};
    hipLaunchKernelGGL((k_combine_gas<N, RM>), dim3(unsigned((G.n_own + kTile - 1) / kTile)),
                       dim3(64 * kCombineWaves), 0, c->stream, cb);
}

DmPassArgs dm_pass_args(dmb_ctx* c, Cells& X, const dmb_params* par, dmb_out* out, uint64_t* counters,
                        const uint32_t* step_off)
{
    Species& G = X.gas;
    Species& D = X.dm;
    DmPassArgs a;
    a.g = geom(X, D, G, X.dp, counters);
    a.g.queue_ctr = X.qctr.as<uint32_t>() + kXcd;
    a.drec = D.rec.p; a.dm_perm = D.perm;
    a.Vx = G.v0.as<const double>(); a.Vy = G.v1.as<const double>(); a.Vz = G.v2.as<const double>();
    a.grec = G.rec.p;
    a.gtab = c->gtab.as<const float4>();
    a.k0 = uint32_t(par->seed); a.k1 = uint32_t(par->seed >> 32); a.step = par->step; a.box = par->box_id;
    a.step_off = step_off;
    a.part_p = X.part_p.as<double>(); a.part_pm = X.part_pm.as<float>(); a.part_nb = X.part_nb.as<uint8_t>();
    a.psum_own = X.psum_own.as<double>(); a.psum = out->p_sum; a.pmax = out->p_max;
    a.scount = X.qctr.as<uint32_t>() + 2 * kXcd; a.slist = X.slist.as<uint32_t>();
    return a;
}

template <typename Real, int N, bool RB>
void combine_dm_and_resolve(dmb_ctx* c, Cells& X, const DmPassArgs& a, const dmb_particles* gas,
                            const dmb_params* par, dmb_out* out, uint64_t* counters)
{
    constexpr bool kExact = sizeof(Real) == 8;
    Species& G = X.gas;
    Species& D = X.dm;
    DmCombineArgs cb;
    cb.n_own = D.n_own; cb.own = D.own.as<const uint32_t>(); cb.perm = D.perm;
    cb.item_off = X.dp.ioff.as<const uint32_t>(); cb.part_p = X.part_p.as<const double>();
    cb.part_pm = X.part_pm.as<const float>(); cb.part_nb = X.part_nb.as<const uint8_t>();
    cb.k0 = a.k0; cb.k1 = a.k1; cb.step = a.step; cb.box = a.box; cb.step_off = a.step_off;
    cb.psum_own = X.psum_own.as<double>(); cb.psum = out->p_sum; cb.pmax = out->p_max;
    cb.scount = a.scount; cb.slist = X.slist.as<uint32_t>(); cb.counters = counters;
    {
        Phase ph(c, DMB_PH_COMBINE_DM);
        hipLaunchKernelGGL(k_combine_dm, dim3(unsigned((D.n_own + kTile - 1) / kTile)), dim3(64 * kCombineWaves), 0,
                           c->stream, cb);
    }
    ResolveArgs r;
    r.g = a.g;
    r.cand_beg = X.dp.beg.as<const uint64_t>(); r.cand_cnt = X.dp.scnt.as<const uint32_t>();
    r.drec = a.drec; r.dm_perm = a.dm_perm;
    r.grec = a.grec;
    r.gas_vel = gas->vel; r.gas_u = gas->u; r.gas_mu = gas->mu; r.m_chi = par->m_chi_g;
    r.gtab = a.gtab; r.k0 = a.k0; r.k1 = a.k1; r.step = a.step; r.box = a.box; r.step_off = a.step_off;
    r.aniso_g = par->aniso_g;
    r.tilt_gl = c->tilt_gl.as<const double>();
    r.n_gas_bits = bits_for(std::max<int64_t>(G.n, 2));
    r.n_gas = uint32_t(G.n);
    r.scount = a.scount; r.slist = X.slist.as<const uint32_t>();
    r.dv = out->dv_dm; r.partner = out->partner; r.counters = counters;
    Phase ph(c, DMB_PH_RESOLVE);
    hipLaunchKernelGGL((k_resolve<Real, N, kExact, RB>), dim3(std::max(8, c->num_cu * 2)), dim3(kResolveThreads), 0,
                       c->stream, r);
    if constexpr (RB)
        hipLaunchKernelGGL((k_rb_kick<Real, N>), dim3(std::max(8, c->num_cu * 4)), dim3(64), 0, c->stream, r);
}

// The DM pair pass of one step (RB: Rao-Blackwellised sampling, expected
// P_ij); returns its arguments for the combine and resolve.
template <typename Real, int N, bool RB, bool PAIRS>
DmPassArgs dm_pass(dmb_ctx* c, Cells& X, const dmb_params* par, dmb_out* out, uint64_t* counters)
{
    constexpr bool kExact = sizeof(Real) == 8;
    DmPassArgs a = dm_pass_args(c, X, par, out, counters, nullptr);
    if constexpr (PAIRS) {
        a.g.pairs = c->pair_dst[1]; a.g.pair_cap = uint64_t(c->pair_cap);
        a.g.pair_n = c->S->pair_cnt.as<unsigned long long>() + 1;
    }
    const int nb = persist_blocks(c, (const void*)k_pass_dm<Real, N, kExact, false, PAIRS, RB>, 64, X.dp.nitems);
    Phase ph(c, DMB_PH_PASS_DM);
    hipLaunchKernelGGL((k_pass_dm<Real, N, kExact, false, PAIRS, RB>), dim3(nb), dim3(64), 0, c->stream, a,
                       (const DmPassArgs*)nullptr, (const int64_t*)nullptr, 0);
    return a;
}

// One interaction step of one box: gathers, then the DM pass, its combine,
// decisions and resolve on the caller's stream, and the gas pass and its
// combine on the side stream at the same time (disjoint outputs, queue words
// and counters); both persistent passes share the GPU and drain their own
// queues.  With pass overlap off, all of it runs in sequence on the caller's
// stream.
template <typename Real, int N, int RM, bool PAIRS = false>
dmb_status launch_step(dmb_ctx* c, const dmb_particles* gas, const dmb_particles* dm, const dmb_params* par,
                       dmb_out* out, uint64_t* counters)
{
    constexpr bool kExact = sizeof(Real) == 8;
    constexpr int kW = RM == kRatesMlp ? kMlpPassWaves : 1;
    Cells& X = *c->X;
    {
        Phase ph(c, DMB_PH_GATHER);
        dmb_status s = gather_and_fill<Real, RM>(c, X, gas, dm, par, out, counters, true);
        if (s != DMB_OK) return s;
    }
    bool rb = false;
    if constexpr (N > -4 && !PAIRS) rb = par->dm_sampling == DMB_SAMPLE_RB;
    const bool side = c->pass_overlap && X.gp.nitems > 0 && X.dp.nitems > 0;
    Scratch* const S0 = c->S;     // the pair-export counts live in the caller's scratch set
    if (side) {
        dmb_status s = fork(c);     // the side stream waits for the gathers only
        if (s != DMB_OK) return s;
    }
    // the DM pass is enqueued first, so its blocks are dispatched first
    DmPassArgs da;
    if (X.dp.nitems > 0) {
        if constexpr (N > -4 && !PAIRS) {
            if (rb) da = dm_pass<Real, N, true, false>(c, X, par, out, counters);
        }
        if (!rb) da = dm_pass<Real, N, false, PAIRS>(c, X, par, out, counters);
    }
    if (X.gp.nitems > 0) {
        OnSide on(c, side);
        GasPassArgs a = gas_pass_args<Real, N, RM>(c, X, gas, par, out, counters);
        if constexpr (PAIRS) {
            a.g.pairs = c->pair_dst[0]; a.g.pair_cap = uint64_t(c->pair_cap);
            a.g.pair_n = S0->pair_cnt.as<unsigned long long>();
        }
        const int nb = persist_blocks(c, (const void*)k_pass_gas<Real, N, kExact, RM, false, PAIRS>, 64 * kW,
                                      (X.gp.nitems + kW - 1) / kW);
        {
            Phase ph(c, DMB_PH_PASS_GAS);
            hipLaunchKernelGGL((k_pass_gas<Real, N, kExact, RM, false, PAIRS>), dim3(nb), dim3(64 * kW), 0, c->stream,
                               a, (const GasPassArgs*)nullptr, (const int64_t*)nullptr, 0);
        }
        Phase ph(c, DMB_PH_COMBINE_GAS);
        combine_gas<N, RM>(c, X, gas, par, out);
    }
    if (X.dp.nitems > 0) {
        if constexpr (N > -4 && !PAIRS) {
            if (rb) combine_dm_and_resolve<Real, N, true>(c, X, da, gas, par, out, counters);
        }
        if (!rb) combine_dm_and_resolve<Real, N, false>(c, X, da, gas, par, out, counters);
    }
    if (side) {
        dmb_status s = join(c);
        if (s != DMB_OK) return s;
    }
    HIPCHK(c, hipGetLastError());
    return DMB_OK;
}

// ---------------------------------------------------------------------------
// Batched boxes: per-box gathers, combines and resolves; each pair pass is one
// persistent launch over the work items of all boxes.  Arguments live in
// device arrays prepared by batch_prepare, so batch_enqueue launches kernels
// only (it can be captured in a graph).
struct BatchPlan {
    int nbox = 0;
    int64_t gas_items = 0, dm_items = 0;
    std::vector<GasPassArgs> ga;
    std::vector<DmPassArgs> da;
    int nb_gas = 0, nb_dm = 0;
    bool rb = false;                       // Rao-Blackwellised DM sampling
};

template <typename Real, int N, int RM>
dmb_status batch_prepare(dmb_ctx* c, int nbox, const dmb_particles* gas, const dmb_particles* dm,
                         const dmb_params* par, dmb_out* out, BatchPlan& P)
{
    constexpr bool kExact = sizeof(Real) == 8;
    constexpr int kW = RM == kRatesMlp ? kMlpPassWaves : 1;
    P.nbox = nbox;
    P.ga.resize(nbox);
    P.da.resize(nbox);
    std::vector<int64_t> gi(nbox + 1, 0), di(nbox + 1, 0);
    // global queues [0, 16) and the Philox step offset [16]
    ENSURE(c, c->bstep, 32 * sizeof(uint32_t));
    const uint32_t* step_off = c->bstep.as<const uint32_t>() + 2 * kXcd;
    for (int b = 0; b < nbox; ++b) {
        Cells& X = *c->boxes[b];
        // buffers the step writes (sized here so that enqueueing allocates nothing)
        if (X.gp.nitems > 0) ENSURE(c, X.part_gas, size_t(X.gp.nitems) * kTile * gas_sums<RM>() * 8);
        if (X.dp.nitems > 0) {
            ENSURE(c, X.part_p, size_t(X.dp.nitems) * kTile * 8);
            ENSURE(c, X.part_pm, size_t(X.dp.nitems) * kTile * 4);
            ENSURE(c, X.part_nb, size_t(X.dp.nitems) * kTile);
            ENSURE(c, X.psum_own, size_t(X.dm.n_own) * 8);
            ENSURE(c, X.slist, size_t(X.dm.n_own) * 4);
        }
        ENSURE(c, X.qctr, (2 * kXcd + 4) * 4);
        const int rs = int(sizeof(Real));
        Species& G = X.gas;
        Species& D = X.dm;
        if (G.n > 0) {
            ENSURE(c, G.v0, G.n * 8); ENSURE(c, G.v1, G.n * 8); ENSURE(c, G.v2, G.n * 8);
            ENSURE(c, G.orate, std::max<int64_t>(G.n_own, 1) * rs * 4);
            ENSURE(c, G.rec, G.n * (sizeof(Real) == 4 ? sizeof(GasRec<float>) : sizeof(GasRec<double>)));
        }
        if (D.n > 0) {
            ENSURE(c, D.rec, D.n * (sizeof(Real) == 4 ? sizeof(DmRec<float>) : sizeof(DmRec<double>)));
        }
        uint64_t* counters = out[b].counters;
        P.ga[b] = gas_pass_args<Real, N, RM>(c, X, gas + b, par + b, out + b, counters);
        P.da[b] = dm_pass_args(c, X, par + b, out + b, counters, step_off);
        gi[b + 1] = gi[b] + X.gp.nitems;
        di[b + 1] = di[b] + X.dp.nitems;
    }
    P.gas_items = gi[nbox];
    P.dm_items = di[nbox];
    const size_t argb = sizeof(GasPassArgs) + sizeof(DmPassArgs);
    ENSURE(c, c->bgeom, size_t(nbox) * argb + 256);
    ENSURE(c, c->bitem, size_t(2 * (nbox + 1)) * sizeof(int64_t));
    char* gdev = c->bgeom.as<char>();
    HIPCHK(c, hipMemcpyAsync(gdev, P.ga.data(), nbox * sizeof(GasPassArgs), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(gdev + size_t(nbox) * sizeof(GasPassArgs), P.da.data(), nbox * sizeof(DmPassArgs),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->bitem.p, gi.data(), (nbox + 1) * sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->bitem.as<int64_t>() + nbox + 1, di.data(), (nbox + 1) * sizeof(int64_t),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    P.nb_gas = persist_blocks(c, (const void*)k_pass_gas<Real, N, kExact, RM, true>, 64 * kW,
                              (P.gas_items + kW - 1) / kW);
    P.rb = false;
    if constexpr (N > -4) P.rb = par[0].dm_sampling == DMB_SAMPLE_RB;
    const void* dm_kernel = (const void*)k_pass_dm<Real, N, kExact, true>;
    if constexpr (N > -4)
        if (P.rb) dm_kernel = (const void*)k_pass_dm<Real, N, kExact, true, false, true>;
    P.nb_dm = persist_blocks(c, dm_kernel, 64, P.dm_items);
    return DMB_OK;
}

// The DM side of a batched step: one pass over all boxes' items, then the
// per-box combines and resolves.
template <typename Real, int N, bool RB>
void batch_dm_side(dmb_ctx* c, const dmb_particles* gas, const dmb_params* par, dmb_out* out, const BatchPlan& P,
                   const DmPassArgs* ddev, const int64_t* ditems)
{
    constexpr bool kExact = sizeof(Real) == 8;
    DmPassArgs a0 = P.da[0];
    a0.g.queue_ctr = c->bstep.as<uint32_t>() + kXcd;
    a0.g.n_items = P.dm_items;
    {
        Phase ph(c, DMB_PH_PASS_DM);
        hipLaunchKernelGGL((k_pass_dm<Real, N, kExact, true, false, RB>), dim3(P.nb_dm), dim3(64), 0, c->stream, a0,
                           ddev, ditems, P.nbox);
    }
    for (int b = 0; b < P.nbox; ++b)
        if (c->boxes[b]->dp.nitems > 0)
            combine_dm_and_resolve<Real, N, RB>(c, *c->boxes[b], P.da[b], gas + b, par + b, out + b, out[b].counters);
}

template <typename Real, int N, int RM>
dmb_status batch_enqueue(dmb_ctx* c, const dmb_particles* gas, const dmb_particles* dm, const dmb_params* par,
                         dmb_out* out, const BatchPlan& P)
{
    constexpr bool kExact = sizeof(Real) == 8;
    constexpr int kW = RM == kRatesMlp ? kMlpPassWaves : 1;
    const int nbox = P.nbox;
    const GasPassArgs* gdev = reinterpret_cast<const GasPassArgs*>(c->bgeom.p);
    const DmPassArgs* ddev = reinterpret_cast<const DmPassArgs*>(c->bgeom.as<char>() + size_t(nbox) * sizeof(GasPassArgs));
    const int64_t* gitems = c->bitem.as<const int64_t>();
    const int64_t* ditems = gitems + nbox + 1;
    for (int b = 0; b < nbox; ++b) {
        dmb_status s = gather_and_fill<Real, RM>(c, *c->boxes[b], gas + b, dm + b, par + b, out + b, out[b].counters);
        if (s != DMB_OK) return s;
    }
    hipLaunchKernelGGL(k_fill_out, dim3(1), dim3(256), 0, c->stream, int64_t(0), int64_t(0), (double*)nullptr,
                       (double*)nullptr, (double*)nullptr, (int32_t*)nullptr, (double*)nullptr, (double*)nullptr,
                       (uint64_t*)nullptr, c->bstep.as<uint32_t>(), 2 * kXcd);
    // as in the single-box step, the DM side (enqueued first) and the gas side run on two
    // streams, forked after the gathers and joined at the end (also inside a captured graph)
    const bool side = c->pass_overlap && P.gas_items > 0 && P.dm_items > 0;
    if (side) {
        dmb_status s = fork(c);
        if (s != DMB_OK) return s;
    }
    if (P.dm_items > 0) {
        bool done = false;
        if constexpr (N > -4) {
            if (P.rb) {
                batch_dm_side<Real, N, true>(c, gas, par, out, P, ddev, ditems);
                done = true;
            }
        }
        if (!done) batch_dm_side<Real, N, false>(c, gas, par, out, P, ddev, ditems);
    }
    if (P.gas_items > 0) {
        OnSide on(c, side);
        GasPassArgs a0 = P.ga[0];
        a0.g.queue_ctr = c->bstep.as<uint32_t>();
        a0.g.n_items = P.gas_items;
        {
            Phase ph(c, DMB_PH_PASS_GAS);
            hipLaunchKernelGGL((k_pass_gas<Real, N, kExact, RM, true>), dim3(P.nb_gas), dim3(64 * kW), 0, c->stream,
                               a0, gdev, gitems, nbox);
        }
        Phase ph(c, DMB_PH_COMBINE_GAS);
        for (int b = 0; b < nbox; ++b)
            if (c->boxes[b]->gp.nitems > 0) combine_gas<N, RM>(c, *c->boxes[b], gas + b, par + b, out + b);
    }
    if (side) {
        dmb_status s = join(c);
        if (s != DMB_OK) return s;
    }
    HIPCHK(c, hipGetLastError());
    return DMB_OK;
}

// nsteps steps of all boxes (Philox step = params.step + k), eagerly or as
// replays of one captured step.
template <typename Real, int N, int RM>
dmb_status batch_run(dmb_ctx* c, int nbox, const dmb_particles* gas, const dmb_particles* dm, const dmb_params* par,
                     dmb_out* out, int nsteps, bool graph)
{
    BatchPlan P;
    dmb_status s = batch_prepare<Real, N, RM>(c, nbox, gas, dm, par, out, P);
    if (s != DMB_OK) return s;
    uint32_t* step_off = c->bstep.as<uint32_t>() + 2 * kXcd;
    HIPCHK(c, hipMemsetAsync(step_off, 0, sizeof(uint32_t), c->stream));
    if (!graph) {
        for (int k = 0; k < nsteps; ++k) {
            if ((s = batch_enqueue<Real, N, RM>(c, gas, dm, par, out, P)) != DMB_OK) return s;
            hipLaunchKernelGGL(k_mlp_tick, dim3(1), dim3(1), 0, c->stream, step_off);
        }
        HIPCHK(c, hipGetLastError());
        return DMB_OK;
    }
    // capture needs a stream other than the legacy default one: use the
    // context's own non-blocking stream for the captured work when needed
    hipStream_t user = c->stream;
    HIPCHK(c, hipStreamSynchronize(user));
    if (!user) {
        if (!c->train_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->train_stream, hipStreamNonBlocking));
        c->stream = c->train_stream;
    }
    struct StreamRestore { dmb_ctx* c; hipStream_t s; ~StreamRestore() { c->stream = s; } } restore{c, user};
    const bool prof = c->prof;
    c->prof = false;                       // no event records inside the captured step
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    s = batch_enqueue<Real, N, RM>(c, gas, dm, par, out, P);
    hipLaunchKernelGGL(k_mlp_tick, dim3(1), dim3(1), 0, c->stream, step_off);
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    c->prof = prof;
    if (s != DMB_OK) { if (g) (void)hipGraphDestroy(g); return s; }
    if (e != hipSuccess) return fail(c, DMB_EHIP, "step capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(c, DMB_EHIP, "step graph: %s", hipGetErrorString(e));
    }
    hipError_t e2 = hipSuccess;
    {
        Phase ph(c, DMB_PH_PASS_GAS);     // whole replays are timed under the gas-pass slot when profiling
        for (int k = 0; k < nsteps && e == hipSuccess; ++k) e = hipGraphLaunch(ge, c->stream);
    }
    e2 = hipStreamSynchronize(c->stream);
    (void)hipGraphExecDestroy(ge);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess || e2 != hipSuccess)
        return fail(c, DMB_EHIP, "step replay: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    return DMB_OK;
}

template <typename Real, int RM>
dmb_status dispatch_n(dmb_ctx* c, const dmb_particles* gas, const dmb_particles* dm, const dmb_params* par,
                      dmb_out* out, uint64_t* counters)
{
    switch (par->n_pow) {
        case -4: return launch_step<Real, -4, RM>(c, gas, dm, par, out, counters);
        case -2: return launch_step<Real, -2, RM>(c, gas, dm, par, out, counters);
        case 0: return launch_step<Real, 0, RM>(c, gas, dm, par, out, counters);
        case 2: return launch_step<Real, 2, RM>(c, gas, dm, par, out, counters);
    }
    return fail(c, DMB_EINVAL, "n_pow %d not supported", par->n_pow);
}

template <typename Real>
dmb_status dispatch_rates(dmb_ctx* c, const dmb_particles* gas, const dmb_particles* dm, const dmb_params* par,
                          dmb_out* out, uint64_t* counters)
{
    if (par->rates == DMB_RATES_QUAD) {
        dmb_status s = ensure_quad_nodes(c, quad_k(par));
        if (s != DMB_OK) return s;
        return dispatch_n<Real, kRatesQuad>(c, gas, dm, par, out, counters);
    }
    if (par->rates == DMB_RATES_MLP) {
        if constexpr (sizeof(Real) == 4) {
            dmb_status s = ensure_quad_nodes(c, quad_k(par));
            if (s != DMB_OK) return s;
            return dispatch_n<float, kRatesMlp>(c, gas, dm, par, out, counters);
        } else {
            return fail(c, DMB_EINVAL, "network rates need DMB_FP32");
        }
    }
    if (par->rates == DMB_RATES_CLOSURE) return dispatch_n<Real, kRatesClosure>(c, gas, dm, par, out, counters);
    return dispatch_n<Real, kRatesExact>(c, gas, dm, par, out, counters);
}

template <typename Real, int RM>
dmb_status batch_dispatch_n(dmb_ctx* c, int nbox, const dmb_particles* gas, const dmb_particles* dm,
                            const dmb_params* par, dmb_out* out, int nsteps, bool graph)
{
    switch (par->n_pow) {
        case -4: return batch_run<Real, -4, RM>(c, nbox, gas, dm, par, out, nsteps, graph);
        case -2: return batch_run<Real, -2, RM>(c, nbox, gas, dm, par, out, nsteps, graph);
        case 0: return batch_run<Real, 0, RM>(c, nbox, gas, dm, par, out, nsteps, graph);
        case 2: return batch_run<Real, 2, RM>(c, nbox, gas, dm, par, out, nsteps, graph);
    }
    return fail(c, DMB_EINVAL, "n_pow %d not supported", par->n_pow);
}

template <typename Real>
dmb_status batch_dispatch_rates(dmb_ctx* c, int nbox, const dmb_particles* gas, const dmb_particles* dm,
                                const dmb_params* par, dmb_out* out, int nsteps, bool graph)
{
    if (par->rates == DMB_RATES_QUAD) {
        dmb_status s = ensure_quad_nodes(c, quad_k(par));
        if (s != DMB_OK) return s;
        return batch_dispatch_n<Real, kRatesQuad>(c, nbox, gas, dm, par, out, nsteps, graph);
    }
    if (par->rates == DMB_RATES_MLP) {
        if constexpr (sizeof(Real) == 4) {
            dmb_status s = ensure_quad_nodes(c, quad_k(par));
            if (s != DMB_OK) return s;
            return batch_dispatch_n<float, kRatesMlp>(c, nbox, gas, dm, par, out, nsteps, graph);
        } else {
            return fail(c, DMB_EINVAL, "network rates need DMB_FP32");
        }
    }
    if (par->rates == DMB_RATES_CLOSURE)
        return batch_dispatch_n<Real, kRatesClosure>(c, nbox, gas, dm, par, out, nsteps, graph);
    return batch_dispatch_n<Real, kRatesExact>(c, nbox, gas, dm, par, out, nsteps, graph);
}

// ---------------------------------------------------------------------------
// learned rate closure: host helpers
MlpConst mlp_const()
{
    MlpConst K;
    const int nv[4] = {-4, -2, 0, 2};
    for (int j = 0; j < 4; ++j) {
        const double al = alpha_n(nv[j]);
        K.lnA[j] = std::log(al / 3.0);
        K.lnB[j] = std::log(al);
        K.c0A[j] = std::pow(al / 3.0, 4.0 / (nv[j] + 1));
        K.c0B[j] = std::pow(al, 4.0 / (nv[j] + 3));
        K.inv_alpha[j] = 1.0 / al;
    }
    return K;
}

dmb_status mlp_alloc(dmb_ctx* c)
{
    ENSURE(c, c->mlp_p, kMlpParams * sizeof(float));
    ENSURE(c, c->mlp_m, kMlpParams * sizeof(float));
    ENSURE(c, c->mlp_v, kMlpParams * sizeof(float));
    ENSURE(c, c->mlp_blob, sizeof(MlpBlob));
    ENSURE(c, c->mlp_red, (kMlpParams + 1) * sizeof(float));
    return DMB_OK;
}

// Rebuild the packed weights from the binary32 master copy.
dmb_status mlp_repack(dmb_ctx* c, hipStream_t st)
{
    HIPCHK(c, hipMemsetAsync(c->mlp_blob.p, 0, sizeof(MlpBlob), st));
    hipLaunchKernelGGL(k_mlp_pack, dim3(blocks_for(kMlpParams, 256)), dim3(256), 0, st, c->mlp_p.as<const float>(),
                       c->mlp_blob.as<MlpBlob>());
    HIPCHK(c, hipGetLastError());
    return DMB_OK;
}

// Training samples (s, n index, targets) for n inputs x[n][4] and targets y[n][2].
dmb_status mlp_prep(dmb_ctx* c, int64_t n, const double* x, const double* y)
{
    ENSURE(c, c->mlp_ts, size_t(n) * sizeof(float4));
    hipLaunchKernelGGL(k_mlp_prep, dim3(blocks_for(n, 256)), dim3(256), 0, c->stream, n, x, y, c->mlp_ts.as<float4>());
    HIPCHK(c, hipGetLastError());
    return DMB_OK;
}

uint64_t splitmix64(uint64_t* s)
{
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t gcd64(uint64_t a, uint64_t b)
{
    while (b) { uint64_t t = a % b; a = b; b = t; }
    return a;
}

// Release the device buffers of one box.
void free_cells(Cells& X)
{
    auto fr = [](DevBuf& b) { if (b.p) (void)hipFree(b.p); b.p = nullptr; b.cap = 0; };
    for (Species* S : {&X.gas, &X.dm}) {
        DevBuf* all[] = {&S->keys, &S->keys2, &S->vals, &S->vals2, &S->sx, &S->sy, &S->sz, &S->sh, &S->flag,
                         &S->flag_off, &S->own, &S->tbox, &S->th, &S->sbox, &S->shh, &S->mbox, &S->mhh, &S->obox,
                         &S->oh, &S->cube, &S->v0, &S->v1, &S->v2, &S->orate, &S->rec, &S->sub_ccnt, &S->sub_coff, &S->sub_start, &S->sub_cnt, &S->tsup, &S->ssup,
                         &S->msup, &S->tq, &S->sq, &S->mq, &S->prec};
        for (DevBuf* b : all) fr(*b);
    }
    for (Pairs* P : {&X.gp, &X.dp}) {
        DevBuf* all[] = {&P->cnt, &P->off, &P->cand, &P->icnt, &P->ioff, &P->it_tile, &P->it_cb, &P->it_ce,
                         &P->pad, &P->maxcnt, &P->beg, &P->psup, &P->ptile, &P->mask, &P->pcnt, &P->soff,
                         &P->scnt, &P->pw, &P->woff, &P->swt, &P->it_key, &P->it_key2, &P->it_id,
                         &P->it_ord, &P->gbox, &P->gh, &P->gsup, &P->gq, &P->gcnt, &P->glist, &P->gmax};
        for (DevBuf* b : all) fr(*b);
    }
    DevBuf* rest[] = {&X.boxL, &X.part_gas, &X.part_p, &X.part_pm, &X.part_nb, &X.psum_own, &X.qctr, &X.slist};
    for (DevBuf* b : rest) fr(*b);
}

}  // namespace

namespace {
dmb_status build_cells_impl(dmb_ctx* c, const dmb_particles* gas, const dmb_particles* dm, const dmb_params* par);
}

// ===========================================================================
// Static scratch of dmb_step_static: one copy of this array per GPU the
// library is loaded on, held until the process ends.  Host code never uses
// the array's name as an address: dmb_create looks up each device's copy once
// (with that device current) and every later use goes through that pointer.
constexpr size_t kStaticScratchBytes = size_t(DMB_STATIC_SCRATCH_MIB) << 20;
constexpr int64_t kStaticMaxN = DMB_STATIC_MAX_N;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
char g_create_err[256] = "no error";   // message of the last failed dmb_create (no context exists then)

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// This device's address of `scratch` (the device must be current).
hipError_t static_scratch_of(int device, void** ptr)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}
}

extern "C" {

dmb_status dmb_create(dmb_ctx** out, int device, void* hip_stream)
{
    if (!out) return DMB_EINVAL;
    *out = nullptr;
    dmb_ctx* c = new (std::nothrow) dmb_ctx();
    if (!c) return DMB_ENOMEM;
    c->device = device;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    hipError_t he = hipSetDevice(device);
    if (he != hipSuccess) {
        snprintf(g_create_err, sizeof(g_create_err), "hipSetDevice(%d): %s", device, hipGetErrorString(he));
        delete c;
        return DMB_EHIP;
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
        c->num_cu = ncu;
    void* sp = nullptr;
    he = static_scratch_of(device, &sp);
    if (he != hipSuccess) {
        snprintf(g_create_err, sizeof(g_create_err), "static scratch of device %d: %s", device, hipGetErrorString(he));
        delete c;
        return DMB_EHIP;
    }
    c->static_ptr = static_cast<char*>(sp);
    he = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
    if (he != hipSuccess) {
        snprintf(g_create_err, sizeof(g_create_err), "build side stream: %s", hipGetErrorString(he));
        dmb_destroy(c);
        return DMB_EHIP;
    }
    he = hipHostMalloc(reinterpret_cast<void**>(&c->run_dt_host), sizeof(double));
    if (he == hipSuccess) he = hipHostMalloc(reinterpret_cast<void**>(&c->rb_host), kReadbackMax * sizeof(uint64_t));
    if (he != hipSuccess) {
        snprintf(g_create_err, sizeof(g_create_err), "pinned read-back buffer: %s", hipGetErrorString(he));
        dmb_destroy(c);
        return DMB_ENOMEM;
    }
    size_t tb = size_t(kTabCells) * 4 * sizeof(float4);
    const int64_t nnodes = 2 * int64_t(kTabNodesRegion);
    DevBuf nodes;
    if (ensure(c, c->gtab, tb) != DMB_OK || ensure(c, c->X->boxL, 4 * sizeof(double)) != DMB_OK ||
        ensure(c, c->os_err, sizeof(uint32_t)) != DMB_OK || ensure(c, c->tilt_gl, 32 * sizeof(double)) != DMB_OK ||
        ensure(c, nodes, size_t(nnodes) * 3 * sizeof(double)) != DMB_OK) {
        snprintf(g_create_err, sizeof(g_create_err), "%s", c->err);
        if (nodes.p) (void)hipFree(nodes.p);
        dmb_destroy(c);
        return DMB_ENOMEM;
    }
    double tilt_rule[32];
    gauss_legendre(16, tilt_rule, tilt_rule + 16);
    he = hipMemcpyAsync(c->tilt_gl.p, tilt_rule, sizeof(tilt_rule), hipMemcpyHostToDevice, c->stream);
    if (he != hipSuccess) {
        snprintf(g_create_err, sizeof(g_create_err), "node upload: %s", hipGetErrorString(he));
        (void)hipFree(nodes.p);
        dmb_destroy(c);
        return DMB_EHIP;
    }
    hipLaunchKernelGGL(k_os_clear, dim3(1), dim3(256), 0, c->stream, c->os_err.as<uint32_t>(), 1);
    hipLaunchKernelGGL(k_gtab_build, dim3(blocks_for(nnodes, 256)), dim3(256), 0, c->stream, nodes.as<double>());
    hipLaunchKernelGGL(k_gtab_cells, dim3(blocks_for(kTabCells, 256)), dim3(256), 0, c->stream,
                       nodes.as<const double>(), c->gtab.as<float4>());
    he = hipGetLastError();
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
    (void)hipFree(nodes.p);
    if (he != hipSuccess) {
        snprintf(g_create_err, sizeof(g_create_err), "overlap table build: %s", hipGetErrorString(he));
        dmb_destroy(c);
        return DMB_EHIP;
    }
    *out = c;
    return DMB_OK;
}

dmb_status dmb_destroy(dmb_ctx* c)
{
    if (!c) return DMB_EINVAL;
    hipSetDevice(c->device);
    if (c->stream) hipStreamSynchronize(c->stream);
    else hipDeviceSynchronize();
    if (c->side) hipStreamSynchronize(c->side);
    free_cells(c->cells);
    for (Cells* X : c->boxes) {
        free_cells(*X);
        delete X;
    }
    c->boxes.clear();
    auto fr = [](DevBuf& b) { if (b.p) hipFree(b.p); b.p = nullptr; b.cap = 0; };
    for (auto& b : c->heap.scan_tmp) fr(b);
    for (auto& b : c->heap2.scan_tmp) fr(b);
    DevBuf* side_bufs[] = {&c->heap2.os_hist, &c->heap2.os_status, &c->heap2.bbox_part, &c->heap2.counters_local,
                           &c->heap2.pair_cnt, &c->heap2.rb_dev};
    for (DevBuf* b : side_bufs) fr(*b);
    if (c->side) hipStreamDestroy(c->side);
    if (c->ev_fork) hipEventDestroy(c->ev_fork);
    if (c->ev_join) hipEventDestroy(c->ev_join);
    for (auto& p : c->pending) { c->ev_pool.push_back(p.a); c->ev_pool.push_back(p.b); }
    for (hipEvent_t e : c->ev_pool) hipEventDestroy(e);
    DevBuf* mlp[] = {&c->mlp_p, &c->mlp_m, &c->mlp_v, &c->mlp_blob, &c->mlp_part, &c->mlp_red, &c->mlp_ts,
                     &c->mlp_loss, &c->mlp_epoch, &c->mlp_shuf};
    for (DevBuf* b : mlp) fr(*b);
    if (c->train_stream) hipStreamDestroy(c->train_stream);
    DevBuf* rest[] = {&c->gl64, &c->gl32, &c->gtab, &c->tilt_gl, &c->heap.os_hist, &c->heap.os_status, &c->os_err,
                      &c->heap.bbox_part, &c->heap.counters_local, &c->heap.pair_cnt, &c->bstep, &c->bgeom,
                      &c->bitem, &c->heap.rb_dev};
    for (DevBuf* b : rest) fr(*b);
    if (c->rb_host) hipHostFree(c->rb_host);
    if (c->run_dt_host) hipHostFree(c->run_dt_host);
    fr(c->run_buf);
    delete c;
    return DMB_OK;
}

dmb_status dmb_set_stream(dmb_ctx* c, void* hip_stream)
{
    if (!c) return DMB_EINVAL;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    return DMB_OK;
}

const char* dmb_last_error(const dmb_ctx* c) { return c ? c->err : g_create_err; }

dmb_status dmb_build_stats(const dmb_ctx* c, int64_t* o)
{
    if (!c || !o) return DMB_EINVAL;
    const int64_t v[10] = {c->X->gas.n_own, c->X->dm.n_own, c->X->gas.ntile, c->X->dm.ntile, c->X->gas.nown_tile, c->X->dm.nown_tile,
                           c->X->gp.total, c->X->dp.total, c->X->gp.nitems, c->X->dp.nitems};
    for (int k = 0; k < 10; ++k) o[k] = v[k];
    return DMB_OK;
}

dmb_status dmb_set_pass_overlap(dmb_ctx* c, int32_t on)
{
    if (!c) return DMB_EINVAL;
    c->pass_overlap = on != 0;
    return DMB_OK;
}

dmb_status dmb_set_search_groups(dmb_ctx* c, int32_t cap)
{
    if (!c) return DMB_EINVAL;
    if (cap < 0 || cap > 65536) return fail(c, DMB_EINVAL, "dmb_set_search_groups: cap %d outside [0, 65536]", cap);
    c->group_cap = cap;
    return DMB_OK;
}

dmb_status dmb_profile_enable(dmb_ctx* c, int32_t on)
{
    if (!c) return DMB_EINVAL;
    c->prof = on != 0;
    return DMB_OK;
}

dmb_status dmb_profile_read(dmb_ctx* c, double* ms, int64_t* calls, int32_t reset)
{
    if (!c) return DMB_EINVAL;
    HIPCHK(c, hipSetDevice(c->device));
    for (auto& p : c->pending) {
        HIPCHK(c, hipEventSynchronize(p.b));
        float t = 0.f;
        HIPCHK(c, hipEventElapsedTime(&t, p.a, p.b));
        c->ph_ms[p.phase] += double(t);
        c->ph_calls[p.phase] += 1;
        c->ev_pool.push_back(p.a);
        c->ev_pool.push_back(p.b);
    }
    c->pending.clear();
    for (int k = 0; k < DMB_NPHASES; ++k) {
        if (ms) ms[k] = c->ph_ms[k];
        if (calls) calls[k] = c->ph_calls[k];
        if (reset) { c->ph_ms[k] = 0.0; c->ph_calls[k] = 0; }
    }
    return DMB_OK;
}

dmb_status dmb_build_cells(dmb_ctx* c, const dmb_particles* gas, const dmb_particles* dm, const dmb_params* par)
{
    if (!c) return DMB_EINVAL;
    if (!par) return fail(c, DMB_EINVAL, "null params");
    dmb_status s;
    if ((s = check_particles(c, gas, "gas", true)) != DMB_OK) return s;
    if ((s = check_particles(c, dm, "dm", false)) != DMB_OK) return s;
    bool periodic = par->box[0] > 0.0 || par->box[1] > 0.0 || par->box[2] > 0.0;
    if (periodic && !(par->box[0] > 0.0 && par->box[1] > 0.0 && par->box[2] > 0.0))
        return fail(c, DMB_EINVAL, "periodic box needs three positive sides");
    HIPCHK(c, hipSetDevice(c->device));
    c->X = &c->cells;
    return build_cells_impl(c, gas, dm, par);
}

}  // extern "C"

namespace {
// Scalars to bring back to the host in one copy (see k_readback).
struct Readback {
    ReadbackArgs a{};
    void u32(const void* p) { a.src[a.cnt] = p; a.n[a.cnt++] = -4; }
    void u64(const void* p) { a.src[a.cnt] = p; a.n[a.cnt++] = -8; }
    void dmax(const void* p, int64_t n) { a.src[a.cnt] = p; a.n[a.cnt++] = n; }
};

// Runs the gather, copies the values into pinned memory and waits for them.
dmb_status readback(dmb_ctx* c, const Readback& r, uint64_t* out)
{
    if (r.a.cnt == 0) return DMB_OK;
    ENSURE(c, c->S->rb_dev, kReadbackMax * sizeof(uint64_t));
    if (!c->rb_host) HIPCHK(c, hipHostMalloc(reinterpret_cast<void**>(&c->rb_host), kReadbackMax * sizeof(uint64_t)));
    hipLaunchKernelGGL(k_readback, dim3(1), dim3(256), 0, c->stream, r.a, c->S->rb_dev.as<uint64_t>());
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(c->rb_host, c->S->rb_dev.p, r.a.cnt * sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::memcpy(out, c->rb_host, r.a.cnt * sizeof(uint64_t));
    return DMB_OK;
}

// Cell structure of one box into c->X (arguments already checked).
dmb_status build_cells_impl(dmb_ctx* c, const dmb_particles* gas, const dmb_particles* dm, const dmb_params* par)
{
    dmb_status s;
    const bool periodic = par->box[0] > 0.0 || par->box[1] > 0.0 || par->box[2] > 0.0;
    ENSURE(c, c->X->boxL, 4 * sizeof(double));
    Phase ph(c, DMB_PH_BUILD);
    for (int k = 0; k < 3; ++k) c->X->built_L[k] = periodic ? par->box[k] : 0.0;
    double Lh[4] = {c->X->built_L[0], c->X->built_L[1], c->X->built_L[2], 0.0};
    HIPCHK(c, hipMemcpyAsync(c->X->boxL.p, Lh, sizeof(Lh), hipMemcpyHostToDevice, c->stream));
    Cells& X = *c->X;
    s = both(c, [&] { return build_species(c, X.gas, gas); }, [&] { return build_species(c, X.dm, dm); });
    if (s != DMB_OK) return s;
    // read back owner and sub-tile counts
    {
        Readback r;
        for (int sp = 0; sp < 2; ++sp) {
            Species& S = sp == 0 ? c->X->gas : c->X->dm;
            r.u32(S.n > 0 ? S.flag_off.as<uint32_t>() + S.n : nullptr);
            r.u32(S.n > 0 ? S.sub_coff.as<uint32_t>() + S.nchunk : nullptr);
        }
        r.u32(c->os_err.as<uint32_t>());
        uint64_t v[5];
        if ((s = readback(c, r, v)) != DMB_OK) return s;
        if (v[4] != 0) {
            hipLaunchKernelGGL(k_os_clear, dim3(1), dim3(256), 0, c->stream, c->os_err.as<uint32_t>(), 1);
            c->X->built_ngas = c->X->built_ndm = -1;
            return fail(c, DMB_EHIP, "radix sort: a look-back wait gave up");
        }
        c->X->gas.n_own = int64_t(v[0]);
        c->X->gas.ntile = int64_t(v[1]);
        c->X->dm.n_own = int64_t(v[2]);
        c->X->dm.ntile = int64_t(v[3]);
    }
    s = both(
        c,
        [&] {
            dmb_status t = build_subtiles(c, X.gas);
            return t == DMB_OK ? build_owner_tiles(c, X.gas) : t;
        },
        [&] {
            dmb_status t = build_subtiles(c, X.dm);
            return t == DMB_OK ? build_owner_tiles(c, X.dm) : t;
        });
    if (s != DMB_OK) return s;
    s = both(c, [&] { return cand_count(c, X.gas, X.dm, X.gp); }, [&] { return cand_count(c, X.dm, X.gas, X.dp); });
    if (s != DMB_OK) return s;
    uint64_t npairs[2] = {0, 0};
    uint32_t maxcnt[2] = {0, 0};
    double hmax[2] = {0, 0};
    {
        Readback r;
        for (int k = 0; k < 2; ++k) {
            Species& A = k == 0 ? c->X->gas : c->X->dm;
            Species& B = k == 0 ? c->X->dm : c->X->gas;
            Pairs& P = k == 0 ? c->X->gp : c->X->dp;
            r.u64(A.nown_tile > 0 ? P.off.as<uint64_t>() + A.nown_tile : nullptr);
            r.u32(A.nown_tile > 0 && B.ntile > 0 ? P.maxcnt.p : nullptr);
        }
        // largest h of each species from the super-tile maxima (periodic boxes)
        for (int sp = 0; sp < 2; ++sp) {
            Species& S = sp == 0 ? c->X->gas : c->X->dm;
            r.dmax(periodic && S.nsuper > 0 ? S.shh.p : nullptr, periodic ? S.nsuper : 0);
        }
        uint64_t v[6];
        if ((s = readback(c, r, v)) != DMB_OK) return s;
        for (int k = 0; k < 2; ++k) {
            npairs[k] = v[2 * k];
            maxcnt[k] = uint32_t(v[2 * k + 1]);
            std::memcpy(&hmax[k], &v[4 + k], sizeof(double));
        }
    }
    if (periodic) {
        double Lmin = std::min(par->box[0], std::min(par->box[1], par->box[2]));
        if (hmax[0] + hmax[1] >= 0.5 * Lmin) {
            c->X->built_ngas = c->X->built_ndm = -1;
            return fail(c, DMB_ERANGE, "max h_gas + max h_dm = %g >= L/2 = %g", hmax[0] + hmax[1], 0.5 * Lmin);
        }
    }
    c->X->gp.npairs = int64_t(npairs[0]);
    c->X->dp.npairs = int64_t(npairs[1]);
    s = both(c, [&] { return cand_subs(c, X.gas, X.dm, X.gp); }, [&] { return cand_subs(c, X.dm, X.gas, X.dp); });
    if (s != DMB_OK) return s;
    uint64_t tot[2] = {0, 0};
    uint32_t nit[2] = {0, 0};
    {
        Readback r;
        for (int k = 0; k < 2; ++k) {
            Species& A = k == 0 ? c->X->gas : c->X->dm;
            Pairs& P = k == 0 ? c->X->gp : c->X->dp;
            r.u64(A.nown_tile > 0 && P.npairs > 0 ? P.soff.as<uint64_t>() + P.npairs : nullptr);
            r.u32(A.nown_tile > 0 ? P.ioff.as<uint32_t>() + A.nown_tile : nullptr);
        }
        uint64_t v[4];
        if ((s = readback(c, r, v)) != DMB_OK) return s;
        for (int k = 0; k < 2; ++k) {
            tot[k] = v[2 * k];
            nit[k] = uint32_t(v[2 * k + 1]);
        }
    }
    c->X->gp.total = int64_t(tot[0]); c->X->gp.nitems = nit[0];
    c->X->dp.total = int64_t(tot[1]); c->X->dp.nitems = nit[1];
    s = both(c, [&] { return cand_write(c, X.gas, X.dm, X.gp); }, [&] { return cand_write(c, X.dm, X.gas, X.dp); });
    if (s != DMB_OK) return s;
    // later builds keep every candidate of (almost) every tile in the count pass
    for (int k = 0; k < 2; ++k) {
        Pairs& P = k == 0 ? c->X->gp : c->X->dp;
        if (int64_t(maxcnt[k]) > P.pad_cap) P.pad_cap = int(std::min<int64_t>(1 << 20, (int64_t(maxcnt[k]) * 5 / 4 + 63) / 64 * 64));
    }
    c->X->built_ngas = gas->n;
    c->X->built_ndm = dm->n;
    c->X->built_gas_pos = gas->pos;
    c->X->built_dm_pos = dm->pos;
    return DMB_OK;
}

// Argument checks shared by dmb_interact_step and dmb_pair_list.
dmb_status check_step(dmb_ctx* c, const dmb_particles* gas, const dmb_particles* dm, const dmb_params* par,
                      dmb_out* out)
{
    if (!par || !out) return fail(c, DMB_EINVAL, "null params or out");
    dmb_status s;
    if ((s = check_particles(c, gas, "gas", true)) != DMB_OK) return s;
    if ((s = check_particles(c, dm, "dm", false)) != DMB_OK) return s;
    if (gas->n != c->X->built_ngas || dm->n != c->X->built_ndm)
        return fail(c, DMB_ESTALE, "interact_step: sizes differ from the last build_cells");
    if (gas->n > 0 && (!gas->vel || !gas->mass || !gas->u))
        return fail(c, DMB_EINVAL, "gas: null vel, mass or u");
    if (dm->n > 0 && (!dm->vel || !dm->mass)) return fail(c, DMB_EINVAL, "dm: null vel or mass");
    if ((gas->n > 0 && (!out->dp_gas || !out->de_gas)) || (dm->n > 0 && (!out->dv_dm || !out->partner)))
        return fail(c, DMB_EINVAL, "null output array");
    if (!n_supported(par->n_pow)) return fail(c, DMB_EINVAL, "n_pow %d not supported", par->n_pow);
    if (par->rates != DMB_RATES_EXACT && par->rates != DMB_RATES_QUAD && par->rates != DMB_RATES_MLP &&
        par->rates != DMB_RATES_CLOSURE)
        return fail(c, DMB_EINVAL, "rates mode %d not supported", par->rates);
    if (par->rates == DMB_RATES_MLP && !c->mlp_ready)
        return fail(c, DMB_EINVAL, "network rates requested but no weights are loaded (dmb_mlp_init/set_params/train)");
    if (par->rates == DMB_RATES_MLP && par->precision != DMB_FP32)
        return fail(c, DMB_EINVAL, "network rates need DMB_FP32");
    if ((par->rates == DMB_RATES_QUAD || par->rates == DMB_RATES_MLP) &&
        (quad_k(par) < 4 || quad_k(par) > kMaxQuadNodes))
        return fail(c, DMB_EINVAL, "quad_nodes %d outside 4..%d", par->quad_nodes, kMaxQuadNodes);
    if (!(par->m_chi_g > 0.0) || !(par->sigma0_cm2 >= 0.0)) return fail(c, DMB_EINVAL, "bad m_chi or sigma0");
    if (!(std::fabs(par->aniso_g) < 1.0)) return fail(c, DMB_EINVAL, "aniso_g %g outside (-1, 1)", par->aniso_g);
    if (par->dm_sampling != DMB_SAMPLE_PAIR && par->dm_sampling != DMB_SAMPLE_RB)
        return fail(c, DMB_EINVAL, "dm_sampling %d not supported", par->dm_sampling);
    if (par->dm_sampling == DMB_SAMPLE_RB && par->n_pow <= -4)
        return fail(c, DMB_EINVAL, "Rao-Blackwellised sampling needs n_pow > -4 (the expectation diverges)");
    return DMB_OK;
}
}  // namespace

extern "C" {

dmb_status dmb_interact_step(dmb_ctx* c, const dmb_particles* gas, const dmb_particles* dm, const dmb_params* par,
                             dmb_out* out)
{
    if (!c) return DMB_EINVAL;
    c->X = &c->cells;
    dmb_status s0 = check_step(c, gas, dm, par, out);
    if (s0 != DMB_OK) return s0;
    HIPCHK(c, hipSetDevice(c->device));
    uint64_t* counters = out->counters;
    if (!counters) {
        ENSURE(c, c->S->counters_local, DMB_NCOUNTERS * 8);
        counters = c->S->counters_local.as<uint64_t>();
    }
    if (par->precision == DMB_FP64) return dispatch_rates<double>(c, gas, dm, par, out, counters);
    if (par->precision == DMB_FP32) return dispatch_rates<float>(c, gas, dm, par, out, counters);
    return fail(c, DMB_EINVAL, "precision %d not supported", par->precision);
}

dmb_status dmb_pair_list(dmb_ctx* c, const dmb_particles* gas, const dmb_particles* dm, const dmb_params* par,
                         dmb_out* out, int64_t cap, uint32_t* pairs_gas, uint32_t* pairs_dm, int64_t* counts)
{
    if (!c) return DMB_EINVAL;
    c->X = &c->cells;
    dmb_status s0 = check_step(c, gas, dm, par, out);
    if (s0 != DMB_OK) return s0;
    if (par->n_pow != 0 || par->rates != DMB_RATES_EXACT || par->dm_sampling != DMB_SAMPLE_PAIR)
        return fail(c, DMB_EINVAL, "pair_list: needs n_pow 0, DMB_RATES_EXACT and DMB_SAMPLE_PAIR");
    if (cap < 0 || (cap > 0 && (!pairs_gas || !pairs_dm)) || !counts)
        return fail(c, DMB_EINVAL, "pair_list: bad list arguments");
    if (par->precision != DMB_FP64 && par->precision != DMB_FP32)
        return fail(c, DMB_EINVAL, "precision %d not supported", par->precision);
    HIPCHK(c, hipSetDevice(c->device));
    uint64_t* counters = out->counters;
    if (!counters) {
        ENSURE(c, c->S->counters_local, DMB_NCOUNTERS * 8);
        counters = c->S->counters_local.as<uint64_t>();
    }
    ENSURE(c, c->S->pair_cnt, 2 * sizeof(unsigned long long));
    HIPCHK(c, hipMemsetAsync(c->S->pair_cnt.p, 0, 2 * sizeof(unsigned long long), c->stream));
    c->pair_dst[0] = pairs_gas; c->pair_dst[1] = pairs_dm; c->pair_cap = cap;
    dmb_status s = par->precision == DMB_FP64 ? launch_step<double, 0, kRatesExact, true>(c, gas, dm, par, out, counters)
                                              : launch_step<float, 0, kRatesExact, true>(c, gas, dm, par, out, counters);
    c->pair_dst[0] = c->pair_dst[1] = nullptr; c->pair_cap = 0;
    if (s != DMB_OK) return s;
    unsigned long long n[2] = {0ull, 0ull};
    HIPCHK(c, hipMemcpyAsync(n, c->S->pair_cnt.p, sizeof(n), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    Cells& X = *c->X;
    uint32_t* lists[2] = {pairs_gas, pairs_dm};
    for (int k = 0; k < 2; ++k) {
        counts[k] = int64_t(n[k]);
        const int64_t m = std::min<int64_t>(int64_t(n[k]), cap);
        if (m <= 0) continue;
        const bool owner_dm = k == 1;
        hipLaunchKernelGGL(k_pairs_map, dim3(blocks_for(m, 256)), dim3(256), 0, c->stream, m, lists[k],
                           owner_dm ? X.dm.perm : X.gas.perm, owner_dm ? X.gas.perm : X.dm.perm, owner_dm);
    }
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DMB_OK;
}

dmb_status dmb_run(dmb_ctx* c, const dmb_particles* gas, const dmb_particles* dm, const dmb_params* par0,
                   const dmb_run_cfg* cfg, double* diag)
{
    if (!c) return DMB_EINVAL;
    if (!par0 || !cfg || !diag) return fail(c, DMB_EINVAL, "run: null params, cfg or diag");
    if (cfg->nsteps < 0 || !(cfg->dt_max > 0.0) || !(cfg->safety > 0.0 && cfg->safety <= 1.0) ||
        !(cfg->active_frac >= 0.0 && cfg->active_frac <= 1.0))
        return fail(c, DMB_EINVAL, "run: nsteps %d, dt_max %g, safety %g, active_frac %g", cfg->nsteps, cfg->dt_max,
                    cfg->safety, cfg->active_frac);
    dmb_status s;
    if ((s = check_particles(c, gas, "gas", true)) != DMB_OK) return s;
    if ((s = check_particles(c, dm, "dm", false)) != DMB_OK) return s;
    if (gas->dt || dm->dt) return fail(c, DMB_EINVAL, "run: per-particle dt arrays are not supported");
    if ((gas->n > 0 && (!gas->vel || !gas->mass || !gas->u)) || (dm->n > 0 && (!dm->vel || !dm->mass)))
        return fail(c, DMB_EINVAL, "run: null vel, mass or u");
    HIPCHK(c, hipSetDevice(c->device));
    // per-run buffers: step outputs, diagnostics partials and rows, dt and time
    const int64_t ng = gas->n, nd = dm->n;
    ENSURE(c, c->run_buf, size_t(std::max<int64_t>(ng, 1)) * 32 + size_t(std::max<int64_t>(nd, 1)) * 56 +
                              size_t(kRunDiagBlocks) * kRN * 8 + size_t(cfg->nsteps + 1) * DMB_NDIAG * 8 + 64 +
                              DMB_NCOUNTERS * 8 + size_t(ng + nd) + 2048);
    char* b = c->run_buf.as<char>();
    auto take = [&b](size_t bytes) { char* p = b; b += (bytes + 255) & ~size_t(255); return p; };
    dmb_out out;
    out.dp_gas = reinterpret_cast<double*>(take(size_t(std::max<int64_t>(ng, 1)) * 24));
    out.de_gas = reinterpret_cast<double*>(take(size_t(std::max<int64_t>(ng, 1)) * 8));
    out.dv_dm = reinterpret_cast<double*>(take(size_t(std::max<int64_t>(nd, 1)) * 24));
    out.partner = reinterpret_cast<int32_t*>(take(size_t(std::max<int64_t>(nd, 1)) * 4));
    out.p_sum = nullptr;
    out.p_max = reinterpret_cast<double*>(take(size_t(std::max<int64_t>(nd, 1)) * 8));
    out.counters = reinterpret_cast<uint64_t*>(take(DMB_NCOUNTERS * 8));
    double* part = reinterpret_cast<double*>(take(size_t(kRunDiagBlocks) * kRN * 8));
    double* rows = reinterpret_cast<double*>(take(size_t(cfg->nsteps + 1) * DMB_NDIAG * 8));
    double* dtd = reinterpret_cast<double*>(take(16));
    double* timed = dtd + 1;
    uint8_t* gact = reinterpret_cast<uint8_t*>(take(size_t(std::max<int64_t>(ng, 1))));
    uint8_t* dact = reinterpret_cast<uint8_t*>(take(size_t(std::max<int64_t>(nd, 1))));
    // with drawn active sets the steps see the library's flag arrays
    dmb_particles gs = *gas, ds = *dm;
    if (cfg->active_frac > 0.0) {
        gs.active = gact;
        ds.active = dact;
    }
    double init[2] = {cfg->dt_max, 0.0};
    HIPCHK(c, hipMemcpyAsync(dtd, init, sizeof(init), hipMemcpyHostToDevice, c->stream));
    RunArgs ra;
    ra.n_gas = ng; ra.n_dm = nd;
    ra.gpos = const_cast<double*>(gas->pos); ra.gvel = const_cast<double*>(gas->vel);
    ra.gu = const_cast<double*>(gas->u); ra.gmass = gas->mass; ra.gmu = gas->mu;
    ra.dpos = const_cast<double*>(dm->pos); ra.dvel = const_cast<double*>(dm->vel); ra.dmass = dm->mass;
    ra.dp_gas = out.dp_gas; ra.de_gas = out.de_gas; ra.dv_dm = out.dv_dm; ra.p_max = out.p_max;
    ra.counters = out.counters;
    for (int k = 0; k < 3; ++k) ra.L[k] = par0->box[k];
    ra.m_chi = par0->m_chi_g;
    ra.dt = dtd;
    const unsigned nbd = unsigned(std::min<int64_t>(kRunDiagBlocks, std::max<int64_t>(1, (std::max(ng, nd) + 255) / 256)));
    RunDiagArgs da;
    da.n_gas = ng; da.n_dm = nd; da.part = part; da.nblocks = int(nbd); da.counters = out.counters;
    da.dt = dtd; da.time = timed; da.control = cfg->dt_control; da.dt_max = cfg->dt_max; da.safety = cfg->safety;
    auto diag_row = [&](int k) {
        hipLaunchKernelGGL(k_run_diag_partial, dim3(nbd), dim3(256), 0, c->stream, ra, part);
        da.row = rows + int64_t(k) * DMB_NDIAG;
        da.first = k == 0;
        hipLaunchKernelGGL(k_run_diag_final, dim3(1), dim3(64), 0, c->stream, da);
    };
    diag_row(0);
    dmb_params par = *par0;
    double dt = cfg->dt_max;
    for (int k = 0; k < cfg->nsteps; ++k) {
        par.step = par0->step + uint32_t(k);
        if (cfg->active_frac > 0.0)
            hipLaunchKernelGGL(k_run_active, dim3(blocks_for(ng + nd, 256)), dim3(256), 0, c->stream, ng, nd, gact,
                               dact, par.step, par.box_id, uint32_t(par.seed), uint32_t(par.seed >> 32),
                               cfg->active_frac);
        c->X = &c->cells;
        if ((s = build_cells_impl(c, &gs, &ds, &par)) != DMB_OK) return s;
        // the build waited on the stream, so the previous step's dt copy has landed
        if (cfg->dt_control && k > 0) dt = *c->run_dt_host;
        par.dt = dt;
        if ((s = check_step(c, &gs, &ds, &par, &out)) != DMB_OK) return s;
        if (par.precision == DMB_FP64) s = dispatch_rates<double>(c, &gs, &ds, &par, &out, out.counters);
        else if (par.precision == DMB_FP32) s = dispatch_rates<float>(c, &gs, &ds, &par, &out, out.counters);
        else s = fail(c, DMB_EINVAL, "precision %d not supported", par.precision);
        if (s != DMB_OK) return s;
        hipLaunchKernelGGL(k_run_apply, dim3(blocks_for(ng + nd, 256)), dim3(256), 0, c->stream, ra);
        diag_row(k + 1);
        // the next dt reaches the host with the next build's first read-back (same stream)
        HIPCHK(c, hipMemcpyAsync(c->run_dt_host, dtd, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(diag, rows, size_t(cfg->nsteps + 1) * DMB_NDIAG * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DMB_OK;
}

dmb_status dmb_step_static(dmb_ctx* c, const dmb_particles* gas, const dmb_particles* dm, const dmb_params* par,
                           dmb_out* out)
{
    if (!c) return DMB_EINVAL;
    if (!par || !out) return fail(c, DMB_EINVAL, "null params or out");
    dmb_status s;
    if ((s = check_particles(c, gas, "gas", true)) != DMB_OK) return s;
    if ((s = check_particles(c, dm, "dm", false)) != DMB_OK) return s;
    if (gas->n > kStaticMaxN || dm->n > kStaticMaxN)
        return fail(c, DMB_ERANGE, "step_static: n_gas %lld, n_dm %lld above the static limit %lld per species",
                    (long long)gas->n, (long long)dm->n, (long long)kStaticMaxN);
    const bool periodic = par->box[0] > 0.0 || par->box[1] > 0.0 || par->box[2] > 0.0;
    if (periodic && !(par->box[0] > 0.0 && par->box[1] > 0.0 && par->box[2] > 0.0))
        return fail(c, DMB_EINVAL, "periodic box needs three positive sides");
    if (par->rates != DMB_RATES_EXACT) return fail(c, DMB_EINVAL, "step_static: needs DMB_RATES_EXACT");
    if (c->prof) return fail(c, DMB_EINVAL, "step_static: phase timing is on (it creates events)");
    if (!c->static_ptr || !c->rb_host) return fail(c, DMB_EHIP, "step_static: no static scratch on this device");
    HIPCHK(c, hipSetDevice(c->device));
    // the static cell structure and scratch set, carved afresh from the static array
    Scratch fresh, fresh2;
    c->static_cells = Cells{};
    c->S = &fresh;
    c->S2 = &fresh2;
    c->X = &c->static_cells;
    c->arena = c->static_ptr;
    c->arena_cap = kStaticScratchBytes;
    c->arena_off = 0;
    s = build_cells_impl(c, gas, dm, par);
    if (s == DMB_OK) s = check_step(c, gas, dm, par, out);
    if (s == DMB_OK) {
        uint64_t* counters = out->counters;
        if (!counters && (s = ensure(c, c->S->counters_local, DMB_NCOUNTERS * 8)) == DMB_OK)
            counters = c->S->counters_local.as<uint64_t>();
        if (s == DMB_OK) {
            if (par->precision == DMB_FP64) s = dispatch_rates<double>(c, gas, dm, par, out, counters);
            else if (par->precision == DMB_FP32) s = dispatch_rates<float>(c, gas, dm, par, out, counters);
            else s = fail(c, DMB_EINVAL, "precision %d not supported", par->precision);
        }
    }
    c->arena = nullptr;
    c->arena_cap = c->arena_off = 0;
    c->S = &c->heap;
    c->S2 = &c->heap2;
    c->X = &c->cells;
    return s;
}

dmb_status dmb_sort_pairs(dmb_ctx* c, int64_t n, const uint64_t* keys_in, const uint32_t* vals_in, int32_t lo_bit,
                          int32_t passes, uint64_t* keys_out, uint32_t* vals_out)
{
    if (!c) return DMB_EINVAL;
    if (n < 0 || n >= (int64_t(1) << 31) || (n > 0 && (!keys_in || !vals_in || !keys_out || !vals_out)))
        return fail(c, DMB_EINVAL, "sort_pairs: bad arrays");
    if (passes < 1 || passes > kOsMaxPasses || lo_bit < 0 || lo_bit + 8 * passes > 64)
        return fail(c, DMB_EINVAL, "sort_pairs: bits [%d, %d) outside the key", lo_bit, lo_bit + 8 * passes);
    if (n == 0) return DMB_OK;
    HIPCHK(c, hipSetDevice(c->device));
    DevBuf kt, vt;
    dmb_status s = DMB_OK;
    if ((s = ensure(c, kt, size_t(n) * 8)) == DMB_OK && (s = ensure(c, vt, size_t(n) * 4)) == DMB_OK) {
        // the passes ping-pong between the output arrays and temporaries: start where the
        // last pass lands in the outputs
        uint64_t* k0 = (passes & 1) ? kt.as<uint64_t>() : keys_out;
        uint32_t* v0 = (passes & 1) ? vt.as<uint32_t>() : vals_out;
        uint64_t* k1 = (passes & 1) ? keys_out : kt.as<uint64_t>();
        uint32_t* v1 = (passes & 1) ? vals_out : vt.as<uint32_t>();
        if (hipMemcpyAsync(k0, keys_in, size_t(n) * 8, hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
            hipMemcpyAsync(v0, vals_in, size_t(n) * 4, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
            s = fail(c, DMB_EHIP, "sort_pairs: copy failed");
        if (s == DMB_OK) s = radix_sort(c, &k0, &v0, &k1, &v1, n, lo_bit, passes);
        uint32_t err = 0;
        if (s == DMB_OK && (hipMemcpyAsync(&err, c->os_err.p, 4, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
                            hipStreamSynchronize(c->stream) != hipSuccess))
            s = fail(c, DMB_EHIP, "sort_pairs: sync failed");
        if (s == DMB_OK && err) {
            hipLaunchKernelGGL(k_os_clear, dim3(1), dim3(256), 0, c->stream, c->os_err.as<uint32_t>(), 1);
            s = fail(c, DMB_EHIP, "radix sort: a look-back wait gave up");
        }
    }
    (void)hipStreamSynchronize(c->stream);
    if (kt.p) (void)hipFree(kt.p);
    if (vt.p) (void)hipFree(vt.p);
    return s;
}

dmb_status dmb_overlap_eval(dmb_ctx* c, int64_t n, const double* d, const double* h1, const double* h2,
                            int32_t precision, double* g_out)
{
    if (!c) return DMB_EINVAL;
    if (n < 0 || (n > 0 && (!d || !h1 || !h2 || !g_out))) return fail(c, DMB_EINVAL, "overlap_eval: bad args");
    if (n == 0) return DMB_OK;
    HIPCHK(c, hipSetDevice(c->device));
    if (precision == DMB_FP64)
        hipLaunchKernelGGL(k_overlap_eval<double>, dim3(blocks_for(n, 256)), dim3(256), 0, c->stream, n, d, h1, h2,
                           c->gtab.as<const float4>(), true, g_out);
    else
        hipLaunchKernelGGL(k_overlap_eval<float>, dim3(blocks_for(n, 256)), dim3(256), 0, c->stream, n, d, h1, h2,
                           c->gtab.as<const float4>(), false, g_out);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DMB_OK;
}

dmb_status dmb_rates_eval(dmb_ctx* c, int64_t n, const double* w, const double* vs, int32_t n_pow, int32_t precision,
                          int32_t rates, int32_t quad_nodes, double* A_out, double* B_out)
{
    if (!c) return DMB_EINVAL;
    if (n < 0 || (n > 0 && (!w || !vs || !A_out || !B_out))) return fail(c, DMB_EINVAL, "rates_eval: bad args");
    if (!n_supported(n_pow)) return fail(c, DMB_EINVAL, "n_pow %d not supported", n_pow);
    if (rates != DMB_RATES_EXACT && rates != DMB_RATES_QUAD && rates != DMB_RATES_MLP)
        return fail(c, DMB_EINVAL, "rates mode %d", rates);
    if (rates == DMB_RATES_MLP && !c->mlp_ready) return fail(c, DMB_EINVAL, "network rates: no weights loaded");
    const int K = quad_nodes == 0 ? 32 : quad_nodes;
    if (rates != DMB_RATES_EXACT && (K < 4 || K > kMaxQuadNodes)) return fail(c, DMB_EINVAL, "quad_nodes %d", quad_nodes);
    if (n == 0) return DMB_OK;
    HIPCHK(c, hipSetDevice(c->device));
    if (rates != DMB_RATES_EXACT) {
        dmb_status s = ensure_quad_nodes(c, K);
        if (s != DMB_OK) return s;
    }
    double al = alpha_n(n_pow);
    double hw = 0.0, bmin = 0.0;
    quad_window(K, &hw, &bmin);
    if (rates == DMB_RATES_MLP) {
        MlpRatesArgs m;
        m.n = n; m.w = w; m.vs = vs; m.alpha_n = al; m.mlp = c->mlp_blob.as<const MlpBlob>();
        m.nidx = mlp_n_index(n_pow);
        m.c0A = float(std::pow(al / 3.0, 4.0 / (n_pow + 1)));
        m.c0B = float(std::pow(al, 4.0 / (n_pow + 3)));
        m.c1A = float(kMlpC1[mlp_n_index(n_pow)][0]);
        m.c1B = float(kMlpC1[mlp_n_index(n_pow)][1]);
        m.kA = float(3.0 / al); m.kB = float(1.0 / al);
        m.gl_x = c->gl32.as<const float>(); m.gl_w = c->gl32.as<const float>() + kMaxQuadNodes; m.gl_k = K;
        m.hw = hw; m.bmin = bmin; m.A = A_out; m.B = B_out;
        dim3 g2(blocks_for(n, 256)), b2(256);
        switch (n_pow) {
            case -4: hipLaunchKernelGGL(k_rates_eval_mlp<-4>, g2, b2, 0, c->stream, m); break;
            case -2: hipLaunchKernelGGL(k_rates_eval_mlp<-2>, g2, b2, 0, c->stream, m); break;
            case 0: hipLaunchKernelGGL(k_rates_eval_mlp<0>, g2, b2, 0, c->stream, m); break;
            case 2: hipLaunchKernelGGL(k_rates_eval_mlp<2>, g2, b2, 0, c->stream, m); break;
        }
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return DMB_OK;
    }
    dim3 gr(blocks_for(n, 256)), bl(256);
    const void* x64 = c->gl64.p;
    const void* w64 = c->gl64.p ? static_cast<const char*>(c->gl64.p) + kMaxQuadNodes * 8 : nullptr;
    const void* x32 = c->gl32.p;
    const void* w32 = c->gl32.p ? static_cast<const char*>(c->gl32.p) + kMaxQuadNodes * 4 : nullptr;
#define RATES_CASE(NN)                                                                                              \
    case NN:                                                                                                        \
        if (rates == DMB_RATES_QUAD) {                                                                              \
            if (precision == DMB_FP64)                                                                              \
                hipLaunchKernelGGL((k_rates_eval<double, NN, kRatesQuad>), gr, bl, 0, c->stream, n, w, vs, al, x64, w64, K, hw, bmin, A_out, B_out); \
            else                                                                                                    \
                hipLaunchKernelGGL((k_rates_eval<float, NN, kRatesQuad>), gr, bl, 0, c->stream, n, w, vs, al, x32, w32, K, hw, bmin, A_out, B_out); \
        } else {                                                                                                    \
            if (precision == DMB_FP64)                                                                              \
                hipLaunchKernelGGL((k_rates_eval<double, NN, kRatesExact>), gr, bl, 0, c->stream, n, w, vs, al, x64, w64, K, hw, bmin, A_out, B_out); \
            else                                                                                                    \
                hipLaunchKernelGGL((k_rates_eval<float, NN, kRatesExact>), gr, bl, 0, c->stream, n, w, vs, al, x32, w32, K, hw, bmin, A_out, B_out); \
        }                                                                                                           \
        break;
    switch (n_pow) { RATES_CASE(-4) RATES_CASE(-2) RATES_CASE(0) RATES_CASE(2) }
#undef RATES_CASE
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DMB_OK;
}

dmb_status dmb_philox_eval(dmb_ctx* c, int64_t n, const uint32_t* ctr, uint64_t seed, uint32_t* out)
{
    if (!c) return DMB_EINVAL;
    if (n < 0 || (n > 0 && (!ctr || !out))) return fail(c, DMB_EINVAL, "philox_eval: bad args");
    if (n == 0) return DMB_OK;
    HIPCHK(c, hipSetDevice(c->device));
    hipLaunchKernelGGL(k_philox_eval, dim3(blocks_for(n, 256)), dim3(256), 0, c->stream, n, ctr, uint32_t(seed),
                       uint32_t(seed >> 32), out);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DMB_OK;
}

dmb_status dmb_mlp_labels(dmb_ctx* c, int64_t n, const double* x, int32_t quad_nodes, double* y)
{
    if (!c) return DMB_EINVAL;
    if (n < 0 || (n > 0 && (!x || !y))) return fail(c, DMB_EINVAL, "mlp_labels: bad args");
    const int K = quad_nodes == 0 ? 48 : quad_nodes;
    if (K < 4 || K > kMaxQuadNodes) return fail(c, DMB_EINVAL, "quad_nodes %d outside 4..%d", quad_nodes, kMaxQuadNodes);
    if (n == 0) return DMB_OK;
    HIPCHK(c, hipSetDevice(c->device));
    dmb_status s = ensure_quad_nodes(c, K);
    if (s != DMB_OK) return s;
    double hw, bmin;
    quad_window(K, &hw, &bmin);
    hipLaunchKernelGGL(k_mlp_labels, dim3(blocks_for(n, 256)), dim3(256), 0, c->stream, n, x, mlp_const(),
                       c->gl64.as<const double>(), c->gl64.as<const double>() + kMaxQuadNodes, K, hw, bmin, y);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DMB_OK;
}

dmb_status dmb_mlp_init(dmb_ctx* c, uint64_t seed)
{
    if (!c) return DMB_EINVAL;
    HIPCHK(c, hipSetDevice(c->device));
    dmb_status s = mlp_alloc(c);
    if (s != DMB_OK) return s;
    hipLaunchKernelGGL(k_mlp_init, dim3(blocks_for(kMlpParams, 256)), dim3(256), 0, c->stream, c->mlp_p.as<float>(),
                       uint32_t(seed), uint32_t(seed >> 32));
    HIPCHK(c, hipGetLastError());
    if ((s = mlp_repack(c, c->stream)) != DMB_OK) return s;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->mlp_ready = true;
    return DMB_OK;
}

dmb_status dmb_mlp_set_params(dmb_ctx* c, const float* params, int64_t count)
{
    if (!c) return DMB_EINVAL;
    if (!params || count != kMlpParams) return fail(c, DMB_EINVAL, "mlp_set_params: need %d values", kMlpParams);
    HIPCHK(c, hipSetDevice(c->device));
    dmb_status s = mlp_alloc(c);
    if (s != DMB_OK) return s;
    HIPCHK(c, hipMemcpyAsync(c->mlp_p.p, params, kMlpParams * sizeof(float), hipMemcpyHostToDevice, c->stream));
    if ((s = mlp_repack(c, c->stream)) != DMB_OK) return s;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->mlp_ready = true;
    return DMB_OK;
}

dmb_status dmb_mlp_get_params(dmb_ctx* c, float* params, int64_t count)
{
    if (!c) return DMB_EINVAL;
    if (!params || count != kMlpParams) return fail(c, DMB_EINVAL, "mlp_get_params: need %d values", kMlpParams);
    if (!c->mlp_ready) return fail(c, DMB_EINVAL, "mlp_get_params: no weights loaded");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipMemcpyAsync(params, c->mlp_p.p, kMlpParams * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DMB_OK;
}

dmb_status dmb_mlp_grad(dmb_ctx* c, int64_t n, const double* x, const double* y, float* grad, double* loss)
{
    if (!c) return DMB_EINVAL;
    if (n < 1 || !x || !y || !grad) return fail(c, DMB_EINVAL, "mlp_grad: bad args");
    if (!c->mlp_ready) return fail(c, DMB_EINVAL, "mlp_grad: no weights loaded");
    HIPCHK(c, hipSetDevice(c->device));
    dmb_status s = mlp_prep(c, n, x, y);
    if (s != DMB_OK) return s;
    const int64_t nblk = (n + kMlpWave - 1) / kMlpWave;
    ENSURE(c, c->mlp_part, size_t(nblk) * (kMlpParams + 1) * sizeof(float));
    MlpGradArgs g;
    g.ts = c->mlp_ts.as<const float4>(); g.n_total = n; g.batch = n; g.epoch = nullptr; g.shuffle = nullptr;
    g.step = 0; g.W = c->mlp_blob.as<const MlpBlob>(); g.part = c->mlp_part.as<float>();
    hipLaunchKernelGGL(k_mlp_grad, dim3(unsigned(nblk)), dim3(64), 0, c->stream, g);
    hipLaunchKernelGGL(k_mlp_reduce, dim3(blocks_for(kMlpParams + 1, 256)), dim3(256), 0, c->stream,
                       c->mlp_part.as<const float>(), int(nblk), c->mlp_red.as<float>());
    HIPCHK(c, hipGetLastError());
    std::vector<float> h(kMlpParams + 1);
    HIPCHK(c, hipMemcpyAsync(h.data(), c->mlp_red.p, h.size() * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::memcpy(grad, h.data(), kMlpParams * sizeof(float));
    if (loss) *loss = double(h[kMlpParams]);
    return DMB_OK;
}

dmb_status dmb_mlp_train(dmb_ctx* c, int64_t n, const double* x, const double* y, const dmb_mlp_train_cfg* cfg,
                         double* epoch_loss)
{
    if (!c) return DMB_EINVAL;
    if (!cfg || !x || !y) return fail(c, DMB_EINVAL, "mlp_train: null argument");
    if (cfg->epochs < 1 || cfg->batch < kMlpWave || cfg->batch % kMlpWave != 0 || n < cfg->batch)
        return fail(c, DMB_EINVAL, "mlp_train: need epochs >= 1, batch a positive multiple of 64, n >= batch");
    if (!(cfg->lr0 > 0.0) || !(cfg->lr_min >= 0.0) || !(cfg->beta1 >= 0.0 && cfg->beta1 < 1.0) ||
        !(cfg->beta2 >= 0.0 && cfg->beta2 < 1.0) || !(cfg->eps > 0.0))
        return fail(c, DMB_EINVAL, "mlp_train: bad optimiser settings");
    HIPCHK(c, hipSetDevice(c->device));
    dmb_status s;
    if (cfg->init) {
        if ((s = dmb_mlp_init(c, cfg->seed)) != DMB_OK) return s;
    } else if (!c->mlp_ready) {
        return fail(c, DMB_EINVAL, "mlp_train: no weights loaded and init == 0");
    }
    const int64_t S = n / cfg->batch, total = S * cfg->epochs, nblk = cfg->batch / kMlpWave;
    if ((s = mlp_prep(c, n, x, y)) != DMB_OK) return s;
    ENSURE(c, c->mlp_part, size_t(nblk) * (kMlpParams + 1) * sizeof(float));
    ENSURE(c, c->mlp_loss, size_t(total) * sizeof(float));
    ENSURE(c, c->mlp_epoch, sizeof(uint32_t));
    ENSURE(c, c->mlp_shuf, size_t(cfg->epochs) * 2 * sizeof(uint64_t));
    // one shuffle (an affine permutation of 0..n-1) per epoch
    std::vector<uint64_t> shuf(2 * size_t(cfg->epochs));
    uint64_t st = cfg->seed ^ 0x5DEECE66Dull;
    for (int e = 0; e < cfg->epochs; ++e) {
        uint64_t m = 1;
        if (n > 1) {
            do { m = 1 + splitmix64(&st) % uint64_t(n - 1); } while (gcd64(m, uint64_t(n)) != 1);
        }
        shuf[2 * e] = e == 0 && n == 1 ? 1 : m;
        shuf[2 * e + 1] = splitmix64(&st) % uint64_t(n);
    }
    HIPCHK(c, hipMemcpyAsync(c->mlp_shuf.p, shuf.data(), shuf.size() * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (!c->train_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->train_stream, hipStreamNonBlocking));
    hipStream_t ts = c->train_stream;
    HIPCHK(c, hipMemsetAsync(c->mlp_m.p, 0, kMlpParams * sizeof(float), ts));
    HIPCHK(c, hipMemsetAsync(c->mlp_v.p, 0, kMlpParams * sizeof(float), ts));
    HIPCHK(c, hipMemsetAsync(c->mlp_epoch.p, 0, sizeof(uint32_t), ts));
    MlpGradArgs g;
    g.ts = c->mlp_ts.as<const float4>(); g.n_total = n; g.batch = cfg->batch;
    g.epoch = c->mlp_epoch.as<const uint32_t>(); g.shuffle = c->mlp_shuf.as<const uint64_t>();
    g.W = c->mlp_blob.as<const MlpBlob>(); g.part = c->mlp_part.as<float>();
    MlpAdamArgs a;
    a.p = c->mlp_p.as<float>(); a.m = c->mlp_m.as<float>(); a.v = c->mlp_v.as<float>();
    a.part = c->mlp_part.as<const float>(); a.nblk = int(nblk); a.epoch = c->mlp_epoch.as<const uint32_t>();
    a.steps_per_epoch = S; a.total_steps = total;
    a.lr0 = float(cfg->lr0); a.lr_min = float(cfg->lr_min); a.beta1 = float(cfg->beta1); a.beta2 = float(cfg->beta2);
    a.eps = float(cfg->eps); a.W = c->mlp_blob.as<MlpBlob>(); a.loss = c->mlp_loss.as<float>();
    auto enqueue_epoch = [&]() {
        for (int64_t k = 0; k < S; ++k) {
            g.step = k;
            a.step = k;
            hipLaunchKernelGGL(k_mlp_grad, dim3(unsigned(nblk)), dim3(64), 0, ts, g);
            hipLaunchKernelGGL(k_mlp_adam, dim3(blocks_for(kMlpParams + 1, 256)), dim3(256), 0, ts, a);
        }
        hipLaunchKernelGGL(k_mlp_tick, dim3(1), dim3(1), 0, ts, c->mlp_epoch.as<uint32_t>());
    };
    if (cfg->use_graph) {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        HIPCHK(c, hipStreamBeginCapture(ts, hipStreamCaptureModeThreadLocal));
        enqueue_epoch();
        hipError_t e1 = hipStreamEndCapture(ts, &graph);
        if (e1 != hipSuccess) return fail(c, DMB_EHIP, "epoch capture: %s", hipGetErrorString(e1));
        e1 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e1 != hipSuccess) {
            hipGraphDestroy(graph);
            return fail(c, DMB_EHIP, "epoch graph: %s", hipGetErrorString(e1));
        }
        // one replay per epoch, each waited for before the next is launched
        hipError_t e2 = hipSuccess;
        for (int e = 0; e < cfg->epochs && e1 == hipSuccess && e2 == hipSuccess; ++e) {
            e1 = hipGraphLaunch(exec, ts);
            if (e1 == hipSuccess) e2 = hipStreamSynchronize(ts);
        }
        hipGraphExecDestroy(exec);
        hipGraphDestroy(graph);
        if (e1 != hipSuccess || e2 != hipSuccess)
            return fail(c, DMB_EHIP, "epoch replay: %s", hipGetErrorString(e1 != hipSuccess ? e1 : e2));
    } else {
        for (int e = 0; e < cfg->epochs; ++e) enqueue_epoch();
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipStreamSynchronize(ts));
    }
    if (epoch_loss) {
        std::vector<float> L(static_cast<size_t>(total));
        HIPCHK(c, hipMemcpy(L.data(), c->mlp_loss.p, L.size() * sizeof(float), hipMemcpyDeviceToHost));
        for (int e = 0; e < cfg->epochs; ++e) {
            double acc = 0.0;
            for (int64_t k = 0; k < S; ++k) acc += L[size_t(e) * S + k];
            epoch_loss[e] = acc / double(S);
        }
    }
    return DMB_OK;
}

dmb_status dmb_mlp_eval(dmb_ctx* c, int64_t n, const double* x, double* out)
{
    if (!c) return DMB_EINVAL;
    if (n < 0 || (n > 0 && (!x || !out))) return fail(c, DMB_EINVAL, "mlp_eval: bad args");
    if (!c->mlp_ready) return fail(c, DMB_EINVAL, "mlp_eval: no weights loaded");
    if (n == 0) return DMB_OK;
    HIPCHK(c, hipSetDevice(c->device));
    dmb_status s = ensure_quad_nodes(c, 48);
    if (s != DMB_OK) return s;
    double hw, bmin;
    quad_window(48, &hw, &bmin);
    hipLaunchKernelGGL(k_mlp_eval, dim3(blocks_for(n, 64)), dim3(64), 0, c->stream, n, x,
                       c->mlp_blob.as<const MlpBlob>(), mlp_const(), c->gl64.as<const double>(),
                       c->gl64.as<const double>() + kMaxQuadNodes, 48, hw, bmin, out);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DMB_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched boxes
namespace {
struct CellsGuard {          // restores the single-box structure as current
    dmb_ctx* c;
    ~CellsGuard() { c->X = &c->cells; }
};

dmb_status check_batch(dmb_ctx* c, int32_t nbox, const dmb_particles* gas, const dmb_particles* dm,
                       const dmb_params* par)
{
    if (nbox < 1 || nbox > 65536) return fail(c, DMB_EINVAL, "nbox %d outside 1..65536", nbox);
    if (!gas || !dm || !par) return fail(c, DMB_EINVAL, "null batch arrays");
    dmb_status s;
    for (int b = 0; b < nbox; ++b) {
        if ((s = check_particles(c, gas + b, "gas", true)) != DMB_OK) return s;
        if ((s = check_particles(c, dm + b, "dm", false)) != DMB_OK) return s;
        const dmb_params* p = par + b;
        const bool periodic = p->box[0] > 0.0 || p->box[1] > 0.0 || p->box[2] > 0.0;
        if (periodic && !(p->box[0] > 0.0 && p->box[1] > 0.0 && p->box[2] > 0.0))
            return fail(c, DMB_EINVAL, "box %d: periodic box needs three positive sides", b);
    }
    return DMB_OK;
}

dmb_status batch_build_all(dmb_ctx* c, int32_t nbox, const dmb_particles* gas, const dmb_particles* dm,
                           const dmb_params* par)
{
    CellsGuard guard{c};
    while (int(c->boxes.size()) < nbox) c->boxes.push_back(new Cells());
    struct ShareGuard { dmb_ctx* c; ~ShareGuard() { c->item_share = 1; } } share{c};
    c->item_share = nbox;
    for (int b = 0; b < nbox; ++b) {
        c->X = c->boxes[b];
        dmb_status s = build_cells_impl(c, gas + b, dm + b, par + b);
        if (s != DMB_OK) {
            c->batch_n = 0;
            char msg[512];
            snprintf(msg, sizeof(msg), "box %d: %s", b, c->err);
            return fail(c, s, "%s", msg);
        }
    }
    c->batch_n = nbox;
    return DMB_OK;
}

dmb_status batch_step_checked(dmb_ctx* c, int32_t nbox, const dmb_particles* gas, const dmb_particles* dm,
                              const dmb_params* par, dmb_out* out, int32_t nsteps, int32_t use_graph)
{
    if (nbox != c->batch_n) return fail(c, DMB_ESTALE, "batch_step: %d boxes, %d built", nbox, c->batch_n);
    if (!out) return fail(c, DMB_EINVAL, "null outputs");
    if (nsteps < 1) return fail(c, DMB_EINVAL, "nsteps < 1");
    const dmb_params& p0 = par[0];
    if (!n_supported(p0.n_pow)) return fail(c, DMB_EINVAL, "n_pow %d not supported", p0.n_pow);
    if (p0.rates != DMB_RATES_EXACT && p0.rates != DMB_RATES_QUAD && p0.rates != DMB_RATES_MLP &&
        p0.rates != DMB_RATES_CLOSURE)
        return fail(c, DMB_EINVAL, "rates mode %d not supported", p0.rates);
    if (p0.rates == DMB_RATES_MLP && (!c->mlp_ready || p0.precision != DMB_FP32))
        return fail(c, DMB_EINVAL, "network rates need loaded weights and DMB_FP32");
    if (p0.dm_sampling != DMB_SAMPLE_PAIR && p0.dm_sampling != DMB_SAMPLE_RB)
        return fail(c, DMB_EINVAL, "dm_sampling %d not supported", p0.dm_sampling);
    if (p0.dm_sampling == DMB_SAMPLE_RB && p0.n_pow <= -4)
        return fail(c, DMB_EINVAL, "Rao-Blackwellised sampling needs n_pow > -4 (the expectation diverges)");
    if ((p0.rates == DMB_RATES_QUAD || p0.rates == DMB_RATES_MLP) && (quad_k(&p0) < 4 || quad_k(&p0) > kMaxQuadNodes))
        return fail(c, DMB_EINVAL, "quad_nodes %d outside 4..%d", p0.quad_nodes, kMaxQuadNodes);
    for (int b = 0; b < nbox; ++b) {
        const dmb_params& p = par[b];
        if (p.n_pow != p0.n_pow || p.precision != p0.precision || p.rates != p0.rates ||
            quad_k(&p) != quad_k(&p0) || p.dm_sampling != p0.dm_sampling)
            return fail(c, DMB_EINVAL,
                        "box %d: n_pow, precision, rates, quad_nodes and dm_sampling must agree across boxes", b);
        if (!(p.m_chi_g > 0.0) || !(p.sigma0_cm2 >= 0.0)) return fail(c, DMB_EINVAL, "box %d: bad m_chi or sigma0", b);
        if (!(std::fabs(p.aniso_g) < 1.0)) return fail(c, DMB_EINVAL, "box %d: aniso_g %g outside (-1, 1)", b, p.aniso_g);
        const Cells& X = *c->boxes[b];
        if (gas[b].n != X.built_ngas || dm[b].n != X.built_ndm)
            return fail(c, DMB_ESTALE, "box %d: sizes differ from the last batch build", b);
        if (gas[b].n > 0 && (!gas[b].vel || !gas[b].mass || !gas[b].u))
            return fail(c, DMB_EINVAL, "box %d: gas: null vel, mass or u", b);
        if (dm[b].n > 0 && (!dm[b].vel || !dm[b].mass)) return fail(c, DMB_EINVAL, "box %d: dm: null vel or mass", b);
        if ((gas[b].n > 0 && (!out[b].dp_gas || !out[b].de_gas)) ||
            (dm[b].n > 0 && (!out[b].dv_dm || !out[b].partner)) || !out[b].counters)
            return fail(c, DMB_EINVAL, "box %d: null output array or counters", b);
    }
    if (p0.precision == DMB_FP64) return batch_dispatch_rates<double>(c, nbox, gas, dm, par, out, nsteps, use_graph != 0);
    if (p0.precision == DMB_FP32) return batch_dispatch_rates<float>(c, nbox, gas, dm, par, out, nsteps, use_graph != 0);
    return fail(c, DMB_EINVAL, "precision %d not supported", p0.precision);
}
}  // namespace

extern "C" {

dmb_status dmb_batch_build(dmb_ctx* c, int32_t nbox, const dmb_particles* gas, const dmb_particles* dm,
                           const dmb_params* par)
{
    if (!c) return DMB_EINVAL;
    dmb_status s = check_batch(c, nbox, gas, dm, par);
    if (s != DMB_OK) return s;
    HIPCHK(c, hipSetDevice(c->device));
    return batch_build_all(c, nbox, gas, dm, par);
}

dmb_status dmb_batch_step(dmb_ctx* c, int32_t nbox, const dmb_particles* gas, const dmb_particles* dm,
                          const dmb_params* par, dmb_out* out, int32_t nsteps, int32_t use_graph)
{
    if (!c) return DMB_EINVAL;
    dmb_status s = check_batch(c, nbox, gas, dm, par);
    if (s != DMB_OK) return s;
    HIPCHK(c, hipSetDevice(c->device));
    CellsGuard guard{c};
    return batch_step_checked(c, nbox, gas, dm, par, out, nsteps, use_graph);
}

dmb_status dmb_batch_tune(dmb_ctx* c, int32_t nbox, const dmb_particles* gas, const dmb_particles* dm,
                          const dmb_params* par, dmb_out* out, int64_t* choice)
{
    if (!c) return DMB_EINVAL;
    dmb_status s = check_batch(c, nbox, gas, dm, par);
    if (s != DMB_OK) return s;
    HIPCHK(c, hipSetDevice(c->device));
    CellsGuard guard{c};
    const int splits[3] = {32, 64, 128};
    const int deltas[3] = {0, 1, 2};
    const int grids[2] = {50, 100};
    const bool prof = c->prof;
    c->prof = false;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    double best = 1e300;
    int bs = c->split, bd = c->subtile_delta, bg = c->grid_pct;
    for (int sp : splits)
        for (int dl : deltas) {
            c->split = sp;
            c->subtile_delta = dl;
            if ((s = batch_build_all(c, nbox, gas, dm, par)) != DMB_OK) break;
            for (int gp : grids) {
                c->grid_pct = gp;
                if ((s = batch_step_checked(c, nbox, gas, dm, par, out, 1, 0)) != DMB_OK) break;   // warm-up
                (void)hipEventRecord(e0, c->stream);
                if ((s = batch_step_checked(c, nbox, gas, dm, par, out, 2, 0)) != DMB_OK) break;
                (void)hipEventRecord(e1, c->stream);
                (void)hipEventSynchronize(e1);
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (ms < best) { best = ms; bs = sp; bd = dl; bg = gp; }
            }
            if (s != DMB_OK) break;
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->prof = prof;
    c->split = bs;
    c->subtile_delta = bd;
    c->grid_pct = bg;
    if (s != DMB_OK) return s;
    if ((s = batch_build_all(c, nbox, gas, dm, par)) != DMB_OK) return s;
    if (choice) {
        choice[0] = bs;
        choice[1] = bd;
        choice[2] = bg;
        choice[3] = int64_t(best * 1000.0 / 2.0);   // microseconds per step
    }
    return DMB_OK;
}

}  // extern "C"
