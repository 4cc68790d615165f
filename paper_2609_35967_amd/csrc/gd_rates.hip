// gd_rates.hip -- rates over the frozen neighbourhood and the interval plan
// (Sect. 2.5.1-2.5.3).
//
//  k_snapshot    derived snapshot of every particle: diameter s_j and grain
//                count N_j = M_j/m_j (the frozen properties neighbours read)
//  k_rates       one lane per particle: lambda*_ij over its slots in slot order,
//                lambda*_i, controller moments a_i = sum rate <J>, b_i = sum rate <J^2>
//  k_bin_reduce  per-block sums over ilogb(m) bins in double-double, grouped per
//                wavefront with ballots (deterministic order)
//  k_plan        merge bins, A_b, B_b, dt_req, dyadic dt_exe into the interval
//                state (one block)
#include "gd_common.hpp"
#include "gd_internal.hpp"
#include "gd_physics.hpp"

#include <algorithm>

namespace gd {

// packed snapshot of every particle: (m_j, s_j, N_j = M_j / m_j, 1 / m_j),
// one 32-byte record per neighbour gather
struct SnapArgs {
    DevProblem P;
    const double* m;
    const double* M;
    int64_t n;
    double4* snap;
};

struct Snapshot {
    using Args = SnapArgs;
    static constexpr int kThreads = 256;
    static __device__ __forceinline__ void body(const Args& A, Blk B)
    {
        const int64_t i = B.id * int64_t(blockDim.x) + threadIdx.x;
        if (i >= A.n) return;
        const double mi = A.m[i];
        const bool phys = A.P.kernel == GD_KERNEL_PHYSICAL;
        A.snap[i] = make_double4(mi, phys ? grain_size(A.P, mi) : 0.0, phys ? A.M[i] / mi : 0.0, 1.0 / mi);
    }
};

__global__ __launch_bounds__(256) void k_snapshot(SnapArgs A)
{
    Snapshot::body(A, Blk{int64_t(blockIdx.x), int64_t(gridDim.x)});
}

struct RatesArgs {
    DevProblem P;
    const int32_t* nbr;
    const int32_t* cnt;
    const double* dmax;
    const double* m;
    const double* x;
    const double* y;
    const double* z;
    const double4* snap;
    const double4* snap_own;  // the particle's own record: snap offset to the first own slot
    double* lam;
    double* lam_pair;
    double* a;
    double* b;
    void* ws;
    int64_t n_all;  // length of the snapshot: neighbour indices lie in [0, n_all)
};

constexpr int kGather = 4;  // neighbours whose slot and record loads are in flight together

// slots row[s0 .. s0+kGather) (those below cmax) and the snapshot records of
// the valid ones; invalid slots are left for the caller to flag
__device__ inline void gather_neighbours(const int32_t* row, int s0, int cmax, int64_t n, const double4* snap,
                                         int (&jj)[kGather], double4 (&rec)[kGather])
{
#pragma unroll
    for (int t = 0; t < kGather; ++t) jj[t] = s0 + t < cmax ? row[s0 + t] : -1;
#pragma unroll
    for (int t = 0; t < kGather; ++t) rec[t] = (jj[t] >= 0 && jj[t] < n) ? snap[jj[t]] : make_double4(0.0, 0.0, 0.0, 0.0);
}

struct Rates {
    using Args = RatesArgs;
    static constexpr int kThreads = 256;
    static __device__ __forceinline__ void body(const Args& A, Blk B);
};

__global__ __launch_bounds__(256) void k_rates(RatesArgs A)
{
    Rates::body(A, Blk{xcd_block(), int64_t(gridDim.x)});
}

__device__ __forceinline__ void Rates::body(const Args& A, Blk B)
{
    const int64_t i = B.id * int64_t(blockDim.x) + threadIdx.x;
    if (i >= A.P.n) return;
    const int k = A.P.k;
    const bool phys = A.P.kernel == GD_KERNEL_PHYSICAL;
    const int c = A.cnt[i];
    double lam = 0.0, sa = 0.0, sb = 0.0;
    if (c > 1) {
        QCtx q;
        query_ctx(A.P, A.x[i], A.y[i], A.z[i], A.dmax[i], q);
        const double mi = A.m[i];
        Own w;
        own_terms(A.P, q, mi, phys ? A.snap_own[i].y : 0.0, true, w);
        if (!(mi > 0.0) || !isfinite(mi)) set_status(A.ws, GD_DEV_NONFINITE);
        const int cmax = c < k ? c : k;
        // neighbours four at a time: their slots, then their records, in flight
        // together; the pairs are then taken in slot order as before
        for (int s0 = 0; s0 < cmax; s0 += kGather) {
            int jj[kGather];
            double4 rec[kGather];
            gather_neighbours(A.nbr + i * k, s0, cmax, A.n_all, A.snap, jj, rec);
#pragma unroll
            for (int t = 0; t < kGather; ++t) {
            const int s = s0 + t;
            if (s >= cmax) break;
            const int j = jj[t];
            if (j < 0 || j >= A.n_all) {
                set_status(A.ws, GD_DEV_INTERNAL);
                continue;
            }
            const double4 sn = rec[t];
            const double mj = sn.x;
            Pair o;
            pair_eval<true>(A.P, q, w, mj, phys ? sn.y : 0.0, phys ? sn.z : 0.0, sn.w, o);
            lam = lam + o.lam_star;
            if (A.lam_pair) A.lam_pair[i * k + s] = o.lam_star;
            double pa, pb;
            pair_moments(o, w, mj, pa, pb);
            sa = sa + pa;
            sb = sb + pb;
            }
        }
    }
    if (A.lam_pair)
        for (int s = (c > 1 ? c : 0); s < k; ++s) A.lam_pair[i * k + s] = 0.0;
    A.lam[i] = lam;
    A.a[i] = sa;
    A.b[i] = sb;
}

// The same pass with the single-precision pair form (gd_problem.rates_fp32):
// float pair terms, summed in FP64 in slot order.
struct RatesF32 {
    using Args = RatesArgs;
    static constexpr int kThreads = 256;
    static __device__ __forceinline__ void body(const Args& A, Blk B);
};

__global__ __launch_bounds__(256) void k_rates_f32(RatesArgs A)
{
    RatesF32::body(A, Blk{xcd_block(), int64_t(gridDim.x)});
}

__device__ __forceinline__ void RatesF32::body(const Args& A, Blk B)
{
    const int64_t i = B.id * int64_t(blockDim.x) + threadIdx.x;
    if (i >= A.P.n) return;
    const int k = A.P.k;
    const bool phys = A.P.kernel == GD_KERNEL_PHYSICAL;
    const int c = A.cnt[i];
    double lam = 0.0, sa = 0.0, sb = 0.0;
    if (c > 1) {
        QCtx q;
        query_ctx(A.P, A.x[i], A.y[i], A.z[i], A.dmax[i], q);
        QCtxF qf;
        query_ctx_f32(A.P, q, qf);
        const double mi = A.m[i];
        const float si = phys ? float(A.snap_own[i].y) : 0.0f;
        const float Sti = phys ? qf.stfac * si : 0.0f;
        const double rmi = 1.0 / mi;
        float mJf = 0.0f, mJ2f = 0.0f;
        if (phys) {
            double mJ, mJ2;
            frag_moments(A.snap_own[i].y, A.P.s_min, mJ, mJ2);
            mJf = float(mJ);
            mJ2f = float(mJ2);
        }
        if (!(mi > 0.0) || !isfinite(mi)) set_status(A.ws, GD_DEV_NONFINITE);
        const int cmax = c < k ? c : k;
        for (int s0 = 0; s0 < cmax; s0 += kGather) {
            int jj[kGather];
            double4 rec[kGather];
            gather_neighbours(A.nbr + i * k, s0, cmax, A.n_all, A.snap, jj, rec);
#pragma unroll
            for (int t = 0; t < kGather; ++t) {
            const int s = s0 + t;
            if (s >= cmax) break;
            const int j = jj[t];
            if (j < 0 || j >= A.n_all) {
                set_status(A.ws, GD_DEV_INTERNAL);
                continue;
            }
            const double4 sn = rec[t];
            PairF o;
            pair_eval_f32(A.P, qf, mi, rmi, si, Sti, sn.x, phys ? float(sn.y) : 0.0f, phys ? sn.z : 0.0, o);
            lam = lam + double(o.lam_star);
            if (A.lam_pair) A.lam_pair[i * k + s] = double(o.lam_star);
            float pa, pb;
            pair_moments_f32(o, mJf, mJ2f, pa, pb);
            sa = sa + double(pa);
            sb = sb + double(pb);
            }
        }
    }
    if (A.lam_pair)
        for (int s = (c > 1 ? c : 0); s < k; ++s) A.lam_pair[i * k + s] = 0.0;
    A.lam[i] = lam;
    A.a[i] = sa;
    A.b[i] = sb;
}

// ---------------------------------------------------------------------------
// Per-block bin sums.  mode 0 (plan): count, M, M a, M b over bin(m_snap).
// mode 1 (audit): M |ln(m_new/m_snap)|/3 over bin(m_snap).
// part[(blk * kNBin + bin) * 8 + f]: f = 0 count, (1,2) (3,4) (5,6) dd values.
constexpr int kRedWaves = 8;  // wavefronts per bin-reduction block

struct BinArgs {
    int mode;
    const double* msnap;
    const double* M;
    const double* va;
    const double* vb;
    int64_t n;
    double* part;
    void* ws;
};

// One step of a segmented inclusive double-double scan over the wavefront:
// a lane adds the value the DPP pattern brings it only when the source lane
// belongs to its own run (equal id; ids start at 1, so a lane with no
// source, which reads 0, adds nothing).  Runs must be contiguous in lane
// order; the steps are those of wave_scan_incl.
template <int CTRL, int ROWS>
__device__ inline void seg_step(dd& v, int id)
{
    const int oid = __builtin_amdgcn_update_dpp(0, id, CTRL, ROWS, 0xf, true);
    const dd s = dd_add(v, dd{dpp_take<CTRL, ROWS>(v.hi), dpp_take<CTRL, ROWS>(v.lo)});
    if (oid == id) v = s;
}

template <int NV>
__device__ inline void seg_scan(dd (&v)[NV], int id)
{
#pragma unroll
    for (int u = 0; u < NV; ++u) seg_step<0x111, 0xf>(v[u], id);
#pragma unroll
    for (int u = 0; u < NV; ++u) seg_step<0x112, 0xf>(v[u], id);
#pragma unroll
    for (int u = 0; u < NV; ++u) seg_step<0x114, 0xf>(v[u], id);
#pragma unroll
    for (int u = 0; u < NV; ++u) seg_step<0x118, 0xf>(v[u], id);
#pragma unroll
    for (int u = 0; u < NV; ++u) seg_step<0x142, 0xa>(v[u], id);
#pragma unroll
    for (int u = 0; u < NV; ++u) seg_step<0x143, 0xc>(v[u], id);
}

struct BinReduce {
    using Args = BinArgs;
    static constexpr int kThreads = kRedWaves * kWave;
    static __device__ __forceinline__ void body(const Args& A, Blk B);
};

__global__ __launch_bounds__(kRedWaves * kWave) void k_bin_reduce(BinArgs A)
{
    BinReduce::body(A, Blk{int64_t(blockIdx.x), int64_t(gridDim.x)});
}

__device__ __forceinline__ void BinReduce::body(const Args& A, Blk B)
{
    const int mode = A.mode;
    const double* __restrict__ msnap = A.msnap;
    const double* __restrict__ M = A.M;
    const double* __restrict__ va = A.va;
    const double* __restrict__ vb = A.vb;
    const int64_t n = A.n;
    double* __restrict__ part = A.part;
    void* ws = A.ws;
    __shared__ double acc[kRedWaves][kNBin][7];
    // a row of many bins in bin order: bin, run length and the three values
    // of each lane, per wavefront
    __shared__ int32_t sk[kRedWaves][kWave][2];
    __shared__ double sv[kRedWaves][kWave][3];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    for (int e = t; e < kRedWaves * kNBin * 7; e += kRedWaves * kWave) (&acc[0][0][0])[e] = 0.0;
    __syncthreads();
    const int64_t chunk = (n + B.n - 1) / B.n;
    const int64_t beg = B.id * chunk;
    const int64_t end = beg + chunk < n ? beg + chunk : n;
    bool range_bad = false;
    // wavefront w takes the rows of 64 slots w, w + kRedWaves, ... of the
    // block's range; the next row's operands are loaded before the current
    // row is reduced
    struct Row {
        double Mi, ms, a, b;
    };
    auto load = [&](int64_t i, Row& r) {
        const bool in = i < end;
        r.Mi = in ? M[i] : 0.0;
        r.ms = in ? msnap[i] : 1.0;
        r.a = in ? va[i] : 0.0;
        r.b = (in && mode == 0) ? vb[i] : 0.0;
    };
    const int64_t step = int64_t(kRedWaves) * kWave;
    int64_t rb = beg + int64_t(w) * kWave;
    Row cur;
    load(rb + lane, cur);
    for (; rb < end; rb += step) {
        Row nxt;
        load(rb + step + lane, nxt);
        const int64_t i = rb + lane;
        bool valid = i < end && cur.Mi > 0.0;
        double v0 = 0.0, v1 = 0.0, v2 = 0.0;
        int bin = 0;
        if (valid) {
            const double ms = cur.ms;
            bin = bin_of(ms);
            const int lb = ilogb(ms);
            range_bad = range_bad || lb < -kBinOff || lb > kNBin - 1 - kBinOff;
            if (mode == 0) {
                v0 = cur.Mi;
                v1 = cur.Mi * cur.a;
                v2 = cur.Mi * cur.b;
            } else {
                v0 = cur.Mi * (fabs(log(cur.a / ms)) / 3.0);
            }
        }
        // the lanes of the row grouped by bin, from one ballot per bit of the
        // bin: the lanes of my bin, how many of them come before me, and how
        // many lanes hold smaller bins (no lane is lost: invalid lanes take
        // key 255, after every bin)
        const int key = valid ? bin : 255;
        uint64_t same = ~uint64_t(0);
        int less = 0;
#pragma unroll
        for (int bit = 7; bit >= 0; --bit) {
            const uint64_t ones = __ballot((key >> bit) & 1);
            const bool mb = (key >> bit) & 1;
            if (mb) less += int(__popcll(same & ~ones));
            same &= mb ? ones : ~ones;
        }
        const int rank = int(__popcll(same & ((uint64_t(1) << lane) - 1)));
        const int run = int(__popcll(same));
        const uint64_t heads = __ballot(valid && rank == 0);
        if (__popcll(heads) > 1) {
            // several bins: the row in bin order through LDS, then one
            // segmented scan; the last lane of each bin's run adds the run
            const int pos = less + rank;
            sk[w][pos][0] = key;
            sk[w][pos][1] = rank == run - 1 ? run : 0;
            sv[w][pos][0] = v0;
            sv[w][pos][1] = v1;
            sv[w][pos][2] = v2;
            const int kb = sk[w][lane][0], last = sk[w][lane][1];
            dd sd[3] = {dd{sv[w][lane][0], 0.0}, dd{sv[w][lane][1], 0.0}, dd{sv[w][lane][2], 0.0}};
            if (mode == 0) {
                seg_scan<3>(sd, kb + 1);
            } else {
                dd s1[1] = {sd[0]};
                seg_scan<1>(s1, kb + 1);
                sd[0] = s1[0];
            }
            if (last > 0 && kb != 255) {
                double* a = acc[w][kb];
                a[0] += double(last);
#pragma unroll
                for (int u = 0; u < 3; ++u) {
                    if (u > 0 && mode != 0) break;
                    const dd x = dd_add(dd{a[1 + 2 * u], a[2 + 2 * u]}, sd[u]);
                    a[1 + 2 * u] = x.hi;
                    a[2 + 2 * u] = x.lo;
                }
            }
        } else {
            uint64_t rem = __ballot(valid);
            while (rem) {
                const int leader = __ffsll((unsigned long long)rem) - 1;
                const int bsel = __builtin_amdgcn_readlane(bin, leader);
                const bool mine = valid && bin == bsel;
                const uint64_t match = __ballot(mine);
                dd s0{mine ? v0 : 0.0, 0.0}, s1{0.0, 0.0}, s2{0.0, 0.0};
                if (mode == 0) {
                    s1 = dd{mine ? v1 : 0.0, 0.0};
                    s2 = dd{mine ? v2 : 0.0, 0.0};
                    wave_sum_dd3(s0, s1, s2);
                } else {
                    s0 = wave_sum_dd(s0);
                }
                if (lane == 0) {
                    double* a = acc[w][bsel];
                    a[0] += double(__popcll(match));
                    dd x = dd_add(dd{a[1], a[2]}, s0);
                    a[1] = x.hi;
                    a[2] = x.lo;
                    x = dd_add(dd{a[3], a[4]}, s1);
                    a[3] = x.hi;
                    a[4] = x.lo;
                    x = dd_add(dd{a[5], a[6]}, s2);
                    a[5] = x.hi;
                    a[6] = x.lo;
                }
                rem &= ~match;
            }
        }
        cur = nxt;
    }
    if (__ballot(range_bad) && lane == 0) set_status(ws, GD_DEV_MASS_RANGE);
    __syncthreads();
    for (int bin = t; bin < kNBin; bin += kRedWaves * kWave) {
        double* out = part + (B.id * kNBin + bin) * 8;
        double cnt = 0.0;
        dd x0{0.0, 0.0}, x1{0.0, 0.0}, x2{0.0, 0.0};
        for (int ww = 0; ww < kRedWaves; ++ww) {
            const double* a = acc[ww][bin];
            cnt += a[0];
            x0 = dd_add(x0, dd{a[1], a[2]});
            x1 = dd_add(x1, dd{a[3], a[4]});
            x2 = dd_add(x2, dd{a[5], a[6]});
        }
        out[0] = cnt;
        out[1] = x0.hi;
        out[2] = x0.lo;
        out[3] = x1.hi;
        out[4] = x1.lo;
        out[5] = x2.hi;
        out[6] = x2.lo;
    }
}

// ---------------------------------------------------------------------------
// Plan (Sect. 2.5.3): bins merged in ascending order until each holds >=
// nbin_min particles (a short last group joins the previous one);
// A_b = sum M a/sum M, B_b = sum M b/sum M;
// dt_req = min(dt_remain, dt_fn_max, eps C/A_b, (eps C)^2/B_b);
// dt_exe = dt_coll 2^-n, the largest aligned dyadic fraction <= dt_req.
constexpr int kPlanGroups = 8;  // block-partial groups summed in parallel

struct PlanArgs {
    DevProblem P;
    const double* part;
    int nblk;
    gd_interval* iv;
    WsHeader* h;
    void* ws;
};

struct Plan {
    using Args = PlanArgs;
    static constexpr int kThreads = kPlanGroups * kNBin;
    static __device__ __forceinline__ void body(const Args& A, Blk B);
};

__global__ __launch_bounds__(kPlanGroups * kNBin) void k_plan(PlanArgs A)
{
    Plan::body(A, Blk{0, 1});
}

__device__ __forceinline__ void Plan::body(const Args& A, Blk)
{
    const DevProblem& P = A.P;
    const double* __restrict__ part = A.part;
    const int nblk = A.nblk;
    gd_interval* iv = A.iv;
    WsHeader* h = A.h;
    __shared__ double pc[kPlanGroups][kNBin];
    __shared__ double ph[kPlanGroups][3][kNBin], pl[kPlanGroups][3][kNBin];
    __shared__ int32_t s_grp[kNBin];
    __shared__ int32_t s_ng;
    const int t = threadIdx.x, b = t % kNBin, gq = t / kNBin;
    {
        double c = 0.0;
        dd x0{0.0, 0.0}, x1{0.0, 0.0}, x2{0.0, 0.0};
#pragma unroll 4
        for (int blk = gq; blk < nblk; blk += kPlanGroups) {
            const double* a = part + (int64_t(blk) * kNBin + b) * 8;
            c += a[0];
            x0 = dd_add(x0, dd{a[1], a[2]});
            x1 = dd_add(x1, dd{a[3], a[4]});
            x2 = dd_add(x2, dd{a[5], a[6]});
        }
        pc[gq][b] = c;
        ph[gq][0][b] = x0.hi;
        pl[gq][0][b] = x0.lo;
        ph[gq][1][b] = x1.hi;
        pl[gq][1][b] = x1.lo;
        ph[gq][2][b] = x2.hi;
        pl[gq][2][b] = x2.lo;
    }
    __syncthreads();
    if (t < kNBin) {  // the groups combined in a fixed order: row 0 holds the bin totals
        double c = pc[0][t];
        dd x[3];
        for (int v = 0; v < 3; ++v) x[v] = dd{ph[0][v][t], pl[0][v][t]};
        for (int g = 1; g < kPlanGroups; ++g) {
            c += pc[g][t];
            for (int v = 0; v < 3; ++v) x[v] = dd_add(x[v], dd{ph[g][v][t], pl[g][v][t]});
        }
        pc[0][t] = c;
        for (int v = 0; v < 3; ++v) {
            ph[0][v][t] = x[v].hi;
            pl[0][v][t] = x[v].lo;
        }
    }
    __syncthreads();
    if (t == 0) {
        // merge rule in one ascending pass: a group opens at a non-empty bin
        // and closes once it holds nbin_min particles; a short open tail
        // joins the previous group (or is the only group).  Each group's sums
        // add its bins in ascending order.
        const double dt_coll = iv->dt_coll;
        const double Cf = iv->C;
        const int64_t ticks = iv->ticks;
        const double tick = ldexp(dt_coll, -30);
        double req = double(kTicks - ticks) * tick;
        if (P.dt_fn_max < req) req = P.dt_fn_max;
        const double eC = P.eps * Cf;
        auto finalize = [&](const dd (&x)[3], int g) {
            h->gM[g] = x[0].hi;
            const double A_ = x[0].hi > 0.0 ? x[1].hi / x[0].hi : 0.0;
            const double B_ = x[0].hi > 0.0 ? x[2].hi / x[0].hi : 0.0;
            if (A_ > 0.0) {
                const double tt = eC / A_;
                if (tt < req) req = tt;
            }
            if (B_ > 0.0) {
                const double tt = (eC * eC) / B_;
                if (tt < req) req = tt;
            }
        };
        int ng = 0, tail = -1;
        double acc = 0.0;
        bool open = false, has_pend = false;
        dd cur[3], pend[3];
        for (int bb = 0; bb < kNBin; ++bb) {
            s_grp[bb] = -1;
            if (pc[0][bb] == 0.0) continue;
            if (!open) {
                open = true;
                acc = 0.0;
                tail = bb;
                for (int v = 0; v < 3; ++v) cur[v] = dd{0.0, 0.0};
            }
            s_grp[bb] = ng;
            acc += pc[0][bb];
            for (int v = 0; v < 3; ++v) cur[v] = dd_add(cur[v], dd{ph[0][v][bb], pl[0][v][bb]});
            if (acc >= double(P.nbin_min)) {
                if (has_pend) finalize(pend, ng - 1);
                for (int v = 0; v < 3; ++v) pend[v] = cur[v];
                has_pend = true;
                ++ng;
                open = false;
            }
        }
        if (open) {
            if (has_pend) {
                for (int bb = tail; bb < kNBin; ++bb) {
                    if (pc[0][bb] == 0.0) continue;
                    s_grp[bb] = ng - 1;
                    for (int v = 0; v < 3; ++v) pend[v] = dd_add(pend[v], dd{ph[0][v][bb], pl[0][v][bb]});
                }
            } else {
                for (int v = 0; v < 3; ++v) pend[v] = cur[v];
                has_pend = true;
                ng = 1;
            }
        }
        if (has_pend) finalize(pend, ng - 1);
        int64_t size = kTicks;
        int nh = 0;
        for (nh = 0; nh <= 30; ++nh) {
            size = kTicks >> nh;
            if (double(size) * tick <= req && (ticks % size) == 0) break;
        }
        if (nh > 30) {
            size = 1;
            atomicOr(&h->status, GD_DEV_TICK_FLOOR);
        }
        h->n_groups = ng;
        iv->dt_req = req;
        iv->dt_exe = double(size) * tick;
        iv->exe_ticks = size;
        iv->n_groups = ng;
        h->scratch[0] = 0.0;  // event counter of the coming interval
        h->heavy_n = 0;       // and the sampling's deferred particles
        h->heavy_next = 0;
        h->heavy_n0 = 0;
        h->heavy_next0 = 0;
        s_ng = ng;
    }
    __syncthreads();
    if (t < kNBin) {
        h->group_of[t] = s_grp[t];
        if (t >= s_ng) h->gM[t] = 0.0;
    }
}

// The kRedBlocks block partials of each bin summed as a tree, one block per
// bin, into one row per bin (same layout as a block's partials): the plan and
// the audit then read a single row instead of looping over the blocks.
struct FoldArgs {
    const double* part;
    double* out;
    int nblk;  // partial rows written (the rest count as zero)
};

struct PartFold {
    using Args = FoldArgs;
    static constexpr int kThreads = kRedBlocks;
    static __device__ __forceinline__ void body(const Args& A, Blk B);
};

__global__ __launch_bounds__(kRedBlocks) void k_part_fold(FoldArgs A)
{
    PartFold::body(A, Blk{int64_t(blockIdx.x), int64_t(gridDim.x)});
}

__device__ __forceinline__ void PartFold::body(const Args& A, Blk B)
{
    __shared__ double c[kRedBlocks];
    __shared__ double hi[3][kRedBlocks], lo[3][kRedBlocks];
    const int b = int(B.id), t = threadIdx.x;
    double* __restrict__ out = A.out;
    const bool have = t < A.nblk;
    const double* a = A.part + (int64_t(have ? t : 0) * kNBin + b) * 8;
    c[t] = have ? a[0] : 0.0;
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        hi[v][t] = have ? a[1 + 2 * v] : 0.0;
        lo[v][t] = have ? a[2 + 2 * v] : 0.0;
    }
    __syncthreads();
    for (int w = kRedBlocks / 2; w > 0; w >>= 1) {
        if (t < w) {
            c[t] += c[t + w];
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                const dd x = dd_add(dd{hi[v][t], lo[v][t]}, dd{hi[v][t + w], lo[v][t + w]});
                hi[v][t] = x.hi;
                lo[v][t] = x.lo;
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        double* o = out + int64_t(b) * 8;
        o[0] = c[0];
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            o[1 + 2 * v] = hi[v][0];
            o[2 + 2 * v] = lo[v][0];
        }
        o[7] = 0.0;
    }
}

static_assert(kNBin * 8 <= 8 * kRedBlocks, "the folded rows fit the reduction scratch");

// fold the block partials `part` into the reduction scratch of the workspace
// (free outside the neighbour build); returns the folded rows
const double* launch_part_fold(const double* part, void* ws, const Layout& L, hipStream_t st)
{
    double* out = at<double>(ws, L.red);
    hipLaunchKernelGGL(k_part_fold, dim3(kNBin), dim3(kRedBlocks), 0, st, FoldArgs{part, out, kRedBlocks});
    return out;
}

// ---------------------------------------------------------------------------
void launch_bin_reduce(int mode, const double* msnap, const double* M, const double* va, const double* vb, int64_t n,
                       double* part, void* ws, hipStream_t st)
{
    hipLaunchKernelGGL(k_bin_reduce, dim3(kRedBlocks), dim3(kRedWaves * kWave), 0, st,
                       BinArgs{mode, msnap, M, va, vb, n, part, ws});
}

int launch_rates(const gd_problem* p, const gd_particles* s, const gd_neighbors* nb, gd_interval* iv, double* lam_i,
                 double* lam_pair, double* ab, void* ws, const Layout& L, hipStream_t st)
{
    const DevProblem P = to_dev(p);
    const int64_t n = p->n;
    const int g = int((n + 255) / 256);
    const double* m = s->m[s->cur];
    double4* snap = at<double4>(ws, L.snap);
    prof_mark(GD_PROF_RATES, 0, st);
    hipLaunchKernelGGL(k_snapshot, dim3(g), dim3(256), 0, st, SnapArgs{P, m, s->M, n, snap});
    RatesArgs A{};
    A.P = P;
    A.nbr = nb->nbr;
    A.cnt = nb->cnt;
    A.dmax = nb->dmax;
    A.m = m;
    A.x = s->x;
    A.y = s->y;
    A.z = s->z;
    A.snap = snap;
    A.lam = lam_i;
    A.lam_pair = lam_pair;
    A.a = ab ? ab : at<double>(ws, L.a);
    A.b = ab ? ab + n : at<double>(ws, L.b);
    A.ws = ws;
    A.n_all = n;
    A.snap_own = snap;
    if (p->rates_fp32) hipLaunchKernelGGL(k_rates_f32, dim3(g), dim3(256), 0, st, A);
    else hipLaunchKernelGGL(k_rates, dim3(g), dim3(256), 0, st, A);
    double* part = at<double>(ws, L.part);
    launch_bin_reduce(0, m, s->M, A.a, A.b, n, part, ws, st);
    const double* folded = launch_part_fold(part, ws, L, st);
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(kPlanGroups * kNBin), 0, st,
                       PlanArgs{P, folded, 1, iv, at<WsHeader>(ws, L.hdr), ws});
    prof_mark(GD_PROF_RATES, 1, st);
    return 0;
}

// Rates and plan of the slots [lo, hi) only (one spatial group): the particle's
// own arrays are addressed from lo, the snapshot (refreshed first when asked)
// covers every particle.  The executed interval is then held within 1/16 and
// 16 times the scheduled intervals sched[h] (0: none) of the groups h set in
// the group's interaction row (the lower limit wins a conflict), halved until
// aligned, and recorded in sched[g].
__global__ void k_group_clamp(gd_interval* iv, int g, int G, const unsigned long long* rows, int64_t* sched)
{
    if (threadIdx.x != 0) return;
    const unsigned long long row = rows[g];
    int64_t z_lo = 1, z_hi = kTicks;
    for (int h = 0; h < G; ++h) {
        const int64_t zh = sched[h];
        if (h == g || zh == 0 || !((row >> h) & 1ull)) continue;
        if (zh / 16 > z_lo) z_lo = zh / 16;
        if (16 * zh < z_hi) z_hi = 16 * zh;
    }
    if (z_hi < z_lo) z_hi = z_lo;
    const int64_t ticks = iv->ticks;
    int64_t z = iv->exe_ticks;
    if (z > z_hi) z = z_hi;
    if (z < z_lo) z = z_lo;
    while (z > 1 && ((ticks % z) != 0 || ticks + z > kTicks)) z >>= 1;
    iv->exe_ticks = z;
    iv->dt_exe = double(z) * ldexp(iv->dt_coll, -30);
    sched[g] = z;
}

int launch_rates_group(const gd_problem* p, const gd_particles* s, const gd_neighbors* nb, gd_interval* iv,
                       double* lam_i, int64_t lo, int64_t hi, int32_t group, int32_t n_groups, const uint64_t* rows,
                       int64_t* sched, bool snapshot, void* ws, const Layout& L, hipStream_t st)
{
    DevProblem P = to_dev(p);
    const int64_t n = p->n, cnt = hi - lo;
    const double* m = s->m[s->cur];
    double4* snap = at<double4>(ws, L.snap);
    prof_mark(GD_PROF_RATES, 0, st);
    if (snapshot)
        hipLaunchKernelGGL(k_snapshot, dim3(int((n + 255) / 256)), dim3(256), 0, st, SnapArgs{P, m, s->M, n, snap});
    P.n = cnt;
    RatesArgs A{};
    A.P = P;
    A.nbr = nb->nbr + lo * int64_t(p->k);
    A.cnt = nb->cnt + lo;
    A.dmax = nb->dmax + lo;
    A.m = m + lo;
    A.x = s->x + lo;
    A.y = s->y + lo;
    A.z = s->z + lo;
    A.snap = snap;
    A.snap_own = snap + lo;
    A.lam = lam_i + lo;
    A.lam_pair = nullptr;
    A.a = at<double>(ws, L.a) + lo;
    A.b = at<double>(ws, L.b) + lo;
    A.ws = ws;
    A.n_all = n;
    const int g = int((cnt + 255) / 256);
    if (cnt > 0) {
        if (p->rates_fp32) hipLaunchKernelGGL(k_rates_f32, dim3(g), dim3(256), 0, st, A);
        else hipLaunchKernelGGL(k_rates, dim3(g), dim3(256), 0, st, A);
    }
    double* part = at<double>(ws, L.part);
    launch_bin_reduce(0, m + lo, s->M + lo, A.a, A.b, cnt, part, ws, st);
    const double* folded = launch_part_fold(part, ws, L, st);
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(kPlanGroups * kNBin), 0, st,
                       PlanArgs{P, folded, 1, iv, at<WsHeader>(ws, L.hdr), ws});
    hipLaunchKernelGGL(k_group_clamp, dim3(1), dim3(64), 0, st, iv, int(group), int(n_groups),
                       reinterpret_cast<const unsigned long long*>(rows), sched);
    prof_mark(GD_PROF_RATES, 1, st);
    return 0;
}

// Rates and plan of every run as stages of one interval: snapshot, rates,
// the bin sums over n / red_div blocks per run (at most kRedBlocks), their
// fold and the plan.
void many_rates(ManyBuilder& B, const std::vector<ManyRun>& R, bool own_snapshot)
{
    const size_t nr = R.size();
    std::vector<SnapArgs> sn(nr);
    std::vector<RatesArgs> ra(nr);
    std::vector<BinArgs> bi(nr);
    std::vector<FoldArgs> fo(nr);
    std::vector<PlanArgs> pl(nr);
    std::vector<int64_t> nb(nr), nred(nr), nbin(nr, kNBin), one(nr, 1), f64(nr), f32(nr);
    for (size_t r = 0; r < nr; ++r) {
        const ManyRun& x = R[r];
        const gd_problem* p = &x.p;
        const gd_particles* s = &x.out;
        const DevProblem P = to_dev(p);
        const int64_t n = p->n;
        const double* m = s->m[s->cur];
        double4* snap = x.snap ? x.snap : at<double4>(x.ws, x.L.snap);
        sn[r] = SnapArgs{P, m, s->M, n, snap};
        RatesArgs& A = ra[r];
        A = RatesArgs{};
        A.P = P;
        A.nbr = x.nb.nbr;
        A.cnt = x.nb.cnt;
        A.dmax = x.nb.dmax;
        A.m = m;
        A.x = s->x;
        A.y = s->y;
        A.z = s->z;
        A.snap = snap;
        A.snap_own = x.snap ? snap + x.lo : snap;
        A.lam = x.lam_i;
        A.lam_pair = nullptr;
        A.a = at<double>(x.ws, x.L.a);
        A.b = at<double>(x.ws, x.L.b);
        A.ws = x.ws;
        A.n_all = x.n_all >= 0 ? x.n_all : n;
        nb[r] = cdiv(n, 256);
        f64[r] = p->rates_fp32 ? 0 : nb[r];
        f32[r] = p->rates_fp32 ? nb[r] : 0;
        nred[r] = std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, cdiv(n, B.tune.red_div)));
        double* part = at<double>(x.ws, x.L.part);
        double* folded = at<double>(x.ws, x.L.red);
        bi[r] = BinArgs{0, m, s->M, A.a, A.b, n, part, x.ws};
        fo[r] = FoldArgs{part, folded, int(nred[r])};
        pl[r] = PlanArgs{P, folded, 1, x.iv, at<WsHeader>(x.ws, x.L.hdr), x.ws};
    }
    if (own_snapshot) B.add<Snapshot>(sn, nb);
    B.add<Rates>(ra, f64);
    B.add<RatesF32>(ra, f32);
    B.add<BinReduce>(bi, nred);
    B.add<PartFold>(fo, nbin);
    B.add<Plan>(pl, one);
}

// the snapshot of a whole particle set as one step (one run; predicated by
// the builder's flags when set)
void many_snapshot(ManyBuilder& B, const gd_problem* p, const gd_particles* s, double4* snap)
{
    std::vector<SnapArgs> sn{SnapArgs{to_dev(p), s->m[s->cur], s->M, p->n, snap}};
    B.add<Snapshot>(sn, std::vector<int64_t>{cdiv(p->n, 256)});
}

// the audit's bin sums and their fold (mode 1 over m_snap, M, m_new), for
// the sampling stage's audit
void many_audit_sums(ManyBuilder& B, const std::vector<ManyRun>& R)
{
    const size_t nr = R.size();
    std::vector<BinArgs> bi(nr);
    std::vector<FoldArgs> fo(nr);
    std::vector<int64_t> nred(nr), nbin(nr, kNBin);
    for (size_t r = 0; r < nr; ++r) {
        const ManyRun& x = R[r];
        const gd_particles* s = &x.out;
        const int64_t n = x.p.n;
        nred[r] = std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, cdiv(n, B.tune.red_div)));
        double* part = at<double>(x.ws, x.L.part);
        bi[r] = BinArgs{1, s->m[s->cur], s->M, s->m[s->cur ^ 1], nullptr, n, part, x.ws};
        fo[r] = FoldArgs{part, at<double>(x.ws, x.L.red), int(nred[r])};
    }
    B.add<BinReduce>(bi, nred);
    B.add<PartFold>(fo, nbin);
}

}  // namespace gd
