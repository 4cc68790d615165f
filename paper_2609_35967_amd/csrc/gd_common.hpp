// gd_common.hpp -- internal definitions shared by the library's HIP sources:
// workspace layout, the device copy of the problem, the counter-based
// generator, double-double sums and wavefront reductions (wave64, gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gd.h"

namespace gd {

constexpr int kWave = 64;
constexpr int kXcd = 8;             // accelerator dies, each with its own L2
constexpr int kNBin = 128;          // controller bins: ilogb(m) in [-64, 63]
constexpr int kBinOff = 64;
constexpr int64_t kTicks = int64_t(1) << 30;  // ticks per collision step
constexpr int kSortTile = 4096;     // keys per radix-sort block
constexpr int kRedBlocks = 256;     // blocks of the bin reductions
constexpr int kMaxK = 256;
constexpr int kBucket = 4;          // particles per leaf bucket of the search tree
constexpr int kFan = 8;             // children per internal node of the search tree
constexpr int kMaxTreeLevels = 8;   // stored box levels (n <= 4 * 8^8 = 2^26 particles)
constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Device copy of gd_problem (passed by value to kernels).
struct DevProblem {
    int64_t n;
    int32_t k, kernel, push, nbin_min, erosion, grouping;
    int32_t periodic[3];
    double L[3];
    double rmax;
    double t0, m0, eps, dt_fn_max;
    double rho_s, s_min, v_frag;
    double GM, Sigma_g0, R0, p, q, h_g0, alpha, mu_mH, sigma_H2, s0, St0, r_in, r_out;
    int32_t drag, brownian, turbulence, caps;
    int32_t rates_fp32;
};

// Box of a node of the search tree, single precision rounded outward (lo
// down, hi up), so it always contains the exact box of its particles.
struct FBox {
    float lo[3];
    float hi[3];
};

// Device-resident header at the start of the workspace.
struct alignas(256) WsHeader {
    int32_t status;
    int32_t n_active;
    int32_t n_groups;
    int32_t pad0;
    double lo[3];
    double inv;                  // Morton scale 1024 / extent
    double hi[3];                // bounding box of the active particles: lo .. hi
    int32_t group_of[kNBin];     // plan: raw bin -> merged group (-1 empty)
    double gM[kNBin];            // plan: sum of M per merged group
    double scratch[16];
    int32_t xq[4][8];            // per-die work queues of the gather-heavy kernels
    int32_t heavy_n;             // sampling: particles handed to the wavefront-per-particle pass
    int32_t heavy_next;          // sampling: next of them to take
    int32_t knn_fb_n[2];         // neighbour search: queries the tile search handed back (two lists)
    int32_t mc_seg[kXcd];        // sampling: particles with an event, per die's segment of the list
    int32_t mc_next;             // sampling: next group of them to take
    int32_t heavy_n0;            // sampling: particles the screen sent straight to the wavefront pass (at the list's end)
    int32_t heavy_next0;         // sampling: next of those to take
};

// Workspace layout (byte offsets), identical on host and device.
struct Layout {
    size_t hdr, keys0, keys1, vals0, vals1, hist, red, pos4, boxes,
        snap, a, b, part, hint, heavy, mclist, stats, total;
    int64_t n;
    int32_t k;
    int32_t nsort_blocks;
    // implicit search tree: level l holds cnt[l] boxes (padded to a multiple
    // of kFan) starting at box index off[l]; level 0 = buckets of kBucket
    // slots, node i of level l >= 1 = children kFan*i .. kFan*i+7 of level l-1;
    // the root's children are the (<= kFan) boxes of the top level.  Levels
    // >= 1 sit at a common stride (the padded size of level 1), so that
    // off[l] = off1 + (l - 1) * stride1 is computed, not looked up.
    int32_t levels;
    int64_t lvl_cnt[kMaxTreeLevels];
    int64_t lvl_off[kMaxTreeLevels];
    int64_t off1, stride1;
};

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

__host__ inline Layout make_layout(int64_t n, int32_t k)
{
    Layout L{};
    L.n = n;
    L.k = k;
    L.nsort_blocks = int32_t((n + kSortTile - 1) / kSortTile);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
    const size_t nn = size_t(n > 0 ? n : 1);
    L.hdr = take(sizeof(WsHeader));
    L.keys0 = take(4 * nn);
    L.keys1 = take(4 * nn);
    L.vals0 = take(4 * nn);
    L.vals1 = take(4 * nn);
    L.hist = take(4 * size_t(256) * (L.nsort_blocks + 1));
    L.red = take(sizeof(double) * 8 * kRedBlocks);
    L.pos4 = take(32 * nn);
    {
        int64_t cnt = (int64_t(nn) + kBucket - 1) / kBucket;
        const int64_t pad0 = (cnt + kFan - 1) / kFan * kFan;
        const int64_t cnt1 = (cnt + kFan - 1) / kFan;
        L.off1 = pad0;
        L.stride1 = (cnt1 + kFan - 1) / kFan * kFan;  // the largest level >= 1
        int l = 0;
        for (;;) {
            L.lvl_cnt[l] = cnt;
            L.lvl_off[l] = l == 0 ? 0 : L.off1 + (l - 1) * L.stride1;
            ++l;
            if (cnt <= kFan || l == kMaxTreeLevels) break;
            cnt = (cnt + kFan - 1) / kFan;
        }
        L.levels = l;
        L.boxes = take(sizeof(FBox) * size_t(l == 1 ? pad0 : L.off1 + (l - 1) * L.stride1));
    }
    L.snap = take(32 * nn);
    L.a = take(8 * nn);
    L.b = take(8 * nn);
    L.part = take(sizeof(double) * 8 * kNBin * kRedBlocks);
    L.hint = take(8 * nn);
    L.heavy = take(24 * nn);  // sampling: (slot, events, time, mass) of deferred particles
    L.mclist = take(4 * ((nn + 255) / 256) * 256);  // sampling: particles with an event, a segment per die
#ifdef GD_KNN_STATS
    L.stats = take(32 * nn);
#endif
    L.total = o;
    return L;
}

// Workgroups are dealt to the XCDs (dies, each with its own L2) in turn.
// xcd_take() gives each wavefront one item of 64 consecutive particles: the
// items are split into kXcd contiguous Morton ranges, one per die, and a
// wavefront takes the next item of its die's range from that range's counter
// (slot x of `q`), so the Morton-near particles its lanes gather stay in one
// L2.  A die whose range is exhausted takes the next items of the following
// ranges, so spatial variations of cost cannot leave dies idle.  Every
// wavefront takes exactly one item whatever the hardware's dealing order,
// provided the grid holds exactly `nitems` wavefronts and the counters start
// at zero.  No LDS, no barrier.
enum { kQueueKnn = 0 };

__device__ inline int32_t xcd_range_lo(int x, int32_t nitems)
{
    return (nitems / kXcd) * x + (x < nitems % kXcd ? x : nitems % kXcd);
}

__device__ inline int32_t xcd_take(int32_t* q, int32_t nitems)
{
    int32_t got = -1;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        const int x0 = int(blockIdx.x % kXcd);
        for (int d = 0; d < kXcd && got < 0; ++d) {
            const int x = (x0 + d) % kXcd;
            const int32_t lo = xcd_range_lo(x, nitems), size = xcd_range_lo(x + 1, nitems) - lo;
            if (size <= 0) continue;
            const int32_t idx = atomicAdd(q + x, 1);
            if (idx < size) got = lo + idx;
        }
    }
    return __builtin_amdgcn_readfirstlane(got);
}

// Static form (no atomics): block `id` of `nb`, which the hardware deals to
// die x = id mod kXcd as its r-th, becomes block r of die x's contiguous
// range (a bijection for any nb).  The blocks of one run of a many-run grid
// are consecutive, so their local index splits the same way.
__device__ inline int64_t xcd_item(int64_t id, int64_t nb)
{
    const int64_t x = id % kXcd, r = id / kXcd;
    return (nb / kXcd) * x + (x < nb % kXcd ? x : nb % kXcd) + r;
}

// for short kernels of even cost: the grid's own blocks
__device__ inline int64_t xcd_block() { return xcd_item(blockIdx.x, gridDim.x); }

// ---------------------------------------------------------------------------
// Launches over many runs.  A kernel body takes its block as (index, count)
// within its own run's blocks: a one-run launch passes (blockIdx.x, gridDim.x)
// or the die-aware order; a many-run launch (one grid for every run) finds its
// run in a block map, run[g] for block g and b0[r] the first block of run r
// (runs with no blocks in a stage have b0[r] = b0[r + 1]), and reads that
// run's arguments from a table in device memory.  K is a struct with the
// argument type Args, the block size kThreads and the static device function
// body(const Args&, Blk).
struct Blk {
    int64_t id, n;
};

struct RunMap {
    const int32_t* run;
    const int32_t* b0;
    const int32_t* active;  // per-run flags read on the device (null: every run); a run whose flag is 0 skips the stage
};

template <class K>
__global__ __launch_bounds__(K::kThreads) void k_many(const typename K::Args* __restrict__ T, RunMap M)
{
    const int32_t r = M.run[blockIdx.x];
    if (M.active && !M.active[r]) return;
    const int32_t s = M.b0[r];
    // the run's arguments are read where they lie (uniform loads), not
    // copied: a copy indexed at run time would live in scratch memory
    K::body(T[r], Blk{int64_t(blockIdx.x) - s, int64_t(M.b0[r + 1] - s)});
}

// the counters a many-run interval clears before a stage (one block per run):
// the die queues and the two fallback counts of the search, or the list
// segment counts of sampling
struct ClearArgs {
    int32_t* a;
    int32_t na;
    int32_t* b;
    int32_t nb;
};

struct ClearCounters {
    using Args = ClearArgs;
    static constexpr int kThreads = 64;
    static __device__ __forceinline__ void body(const Args& A, Blk)
    {
        const int t = threadIdx.x;
        if (t < A.na) A.a[t] = 0;
        if (A.b && t < A.nb) A.b[t] = 0;
    }
};

template <typename T>
__host__ __device__ inline T* at(void* ws, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(ws) + off); }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw 2011): ten rounds of
// multiply-xor on words 0 and 2 with the Weyl-incremented key.
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c[0];
        const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2];
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0;
        const uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// The four uniforms of one event: (U_w in (0,1], U_p, U_c, U_f in [0,1)).
// Two generator calls with counters (id, interval, event, w), w = 0, 1.
__device__ inline void event_uniforms(uint64_t seed, uint32_t id, uint32_t iv, uint32_t e, double u[4])
{
    const double two53 = 1.0 / 9007199254740992.0;
    const uint32_t k0 = uint32_t(seed), k1 = uint32_t(seed >> 32);
#pragma unroll
    for (uint32_t w = 0; w < 2; ++w) {
        uint32_t c[4] = {id, iv, e, w};
        philox4x32_10(c, k0, k1);
        const uint64_t a = ((uint64_t(c[1]) << 32) | c[0]) >> 11;
        const uint64_t b = ((uint64_t(c[3]) << 32) | c[2]) >> 11;
        if (w == 0) {
            u[0] = double(a + 1) * two53;
            u[1] = double(b) * two53;
        } else {
            u[2] = double(a) * two53;
            u[3] = double(b) * two53;
        }
    }
}

__device__ inline int bin_of(double m)
{
    int b = ilogb(m);
    b = b < -kBinOff ? -kBinOff : b;
    b = b > kNBin - 1 - kBinOff ? kNBin - 1 - kBinOff : b;
    return b + kBinOff;
}

// ---------------------------------------------------------------------------
// Double-double accumulation (Knuth two-sum); the reductions of the
// controller are carried to ~2^-100 relative so that their final rounding
// matches the exactly rounded sum.
struct dd {
    double hi, lo;
};

__device__ inline dd dd_add(dd a, dd b)
{
    const double s = a.hi + b.hi;
    const double bb = s - a.hi;
    double e = (a.hi - (s - bb)) + (b.hi - bb);
    e = e + (a.lo + b.lo);
    const double h = s + e;
    return dd{h, e - (h - s)};
}

__device__ inline double shfl_xor_d(double v, int m)
{
    return __shfl_xor(v, m, kWave);
}

__device__ inline double wave_min_d(double v)
{
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) v = fmin(v, shfl_xor_d(v, m));
    return v;
}

__device__ inline double wave_max_d(double v)
{
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) v = fmax(v, shfl_xor_d(v, m));
    return v;
}

// Inclusive prefix sum over the 64 lanes by data-parallel-primitive moves
// (no LDS): shifts by 1, 2, 4, 8 within each row of 16 lanes, then lane 15 of
// each row added to the next row, then lane 31 to rows 2 and 3.  Lanes whose
// source lies outside the row (or that a row mask leaves out) add +0.
template <int CTRL, int ROWS>
__device__ inline double dpp_take(double x)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROWS, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROWS, 0xf, true);
    return __hiloint2double(hi, lo);
}

__device__ inline double wave_scan_incl(double x)
{
    x = x + dpp_take<0x111, 0xf>(x);  // row_shr:1
    x = x + dpp_take<0x112, 0xf>(x);  // row_shr:2
    x = x + dpp_take<0x114, 0xf>(x);  // row_shr:4
    x = x + dpp_take<0x118, 0xf>(x);  // row_shr:8
    x = x + dpp_take<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
    x = x + dpp_take<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
    return x;
}

__device__ inline double readlane_d(double x, int l)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                            __builtin_amdgcn_readlane(__double2loint(x), l));
}

// the double-double sum over the wavefront, in every lane: the DPP steps of
// wave_scan_incl with dd_add, then the last lane's prefix read across
template <int CTRL, int ROWS>
__device__ inline dd dd_step(dd v)
{
    return dd_add(v, dd{dpp_take<CTRL, ROWS>(v.hi), dpp_take<CTRL, ROWS>(v.lo)});
}

__device__ inline dd wave_sum_dd(dd v)
{
    v = dd_step<0x111, 0xf>(v);
    v = dd_step<0x112, 0xf>(v);
    v = dd_step<0x114, 0xf>(v);
    v = dd_step<0x118, 0xf>(v);
    v = dd_step<0x142, 0xa>(v);
    v = dd_step<0x143, 0xc>(v);
    return dd{readlane_d(v.hi, kWave - 1), readlane_d(v.lo, kWave - 1)};
}

// three such sums side by side (their steps interleave)
__device__ inline void wave_sum_dd3(dd& a, dd& b, dd& c)
{
    a = dd_step<0x111, 0xf>(a);
    b = dd_step<0x111, 0xf>(b);
    c = dd_step<0x111, 0xf>(c);
    a = dd_step<0x112, 0xf>(a);
    b = dd_step<0x112, 0xf>(b);
    c = dd_step<0x112, 0xf>(c);
    a = dd_step<0x114, 0xf>(a);
    b = dd_step<0x114, 0xf>(b);
    c = dd_step<0x114, 0xf>(c);
    a = dd_step<0x118, 0xf>(a);
    b = dd_step<0x118, 0xf>(b);
    c = dd_step<0x118, 0xf>(c);
    a = dd_step<0x142, 0xa>(a);
    b = dd_step<0x142, 0xa>(b);
    c = dd_step<0x142, 0xa>(c);
    a = dd_step<0x143, 0xc>(a);
    b = dd_step<0x143, 0xc>(b);
    c = dd_step<0x143, 0xc>(c);
    a = dd{readlane_d(a.hi, kWave - 1), readlane_d(a.lo, kWave - 1)};
    b = dd{readlane_d(b.hi, kWave - 1), readlane_d(b.lo, kWave - 1)};
    c = dd{readlane_d(c.hi, kWave - 1), readlane_d(c.lo, kWave - 1)};
}

__device__ inline void set_status(void* ws, int bits)
{
    atomicOr(&at<WsHeader>(ws, 0)->status, bits);
}

}  // namespace gd
