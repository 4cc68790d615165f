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

namespace gd {

__global__ __launch_bounds__(256) void k_snapshot(DevProblem P, const double* __restrict__ m,
                                                  const double* __restrict__ M, int64_t n, double* __restrict__ s,
                                                  double* __restrict__ N)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    const double mi = m[i];
    s[i] = grain_size(P, mi);
    N[i] = M[i] / mi;
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
    const double* snap_s;
    const double* snap_N;
    double* lam;
    double* lam_pair;
    double* a;
    double* b;
    void* ws;
};

__global__ __launch_bounds__(256) void k_rates(RatesArgs A)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= A.P.n) return;
    const int k = A.P.k;
    const bool phys = A.P.kernel == GD_KERNEL_PHYSICAL;
    const int c = A.cnt[i];
    double lam = 0.0, sa = 0.0, sb = 0.0;
    const int32_t* row = A.nbr + i * k;
    if (c > 1) {
        QCtx q;
        query_ctx(A.P, A.x[i], A.y[i], A.z[i], A.dmax[i], q);
        const double mi = A.m[i];
        const double si = phys ? A.snap_s[i] : 0.0;
        const double Sti = phys ? q.stfac * si : 0.0;
        if (!(mi > 0.0) || !isfinite(mi)) set_status(A.ws, GD_DEV_NONFINITE);
        for (int s = 0; s < c && s < k; ++s) {
            const int j = row[s];
            if (j < 0 || j >= A.P.n) {
                set_status(A.ws, GD_DEV_INTERNAL);
                continue;
            }
            const double mj = A.m[j];
            const double sj = phys ? A.snap_s[j] : 0.0;
            const double Nj = phys ? A.snap_N[j] : 0.0;
            Pair o;
            pair_eval(A.P, q, mi, si, Sti, mj, sj, Nj, o);
            lam = lam + o.lam_star;
            if (A.lam_pair) A.lam_pair[i * k + s] = o.lam_star;
            double pa, pb;
            pair_moments(A.P, o, mi, si, mj, pa, pb);
            sa = sa + pa;
            sb = sb + pb;
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
__global__ __launch_bounds__(256) void k_bin_reduce(int mode, const double* __restrict__ msnap,
                                                    const double* __restrict__ M, const double* __restrict__ va,
                                                    const double* __restrict__ vb, int64_t n,
                                                    double* __restrict__ part, void* ws)
{
    __shared__ double acc[4][kNBin][7];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    for (int e = t; e < 4 * kNBin * 7; e += 256) (&acc[0][0][0])[e] = 0.0;
    __syncthreads();
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t beg = blockIdx.x * chunk;
    const int64_t end = beg + chunk < n ? beg + chunk : n;
    bool range_bad = false;
    for (int64_t base = beg; base < end; base += 256) {
        const int64_t i = base + t;
        bool valid = i < end;
        double Mi = 0.0, ms = 1.0, v0 = 0.0, v1 = 0.0, v2 = 0.0;
        int bin = 0;
        if (valid) {
            Mi = M[i];
            valid = Mi > 0.0;
        }
        if (valid) {
            ms = msnap[i];
            bin = bin_of(ms);
            const int lb = ilogb(ms);
            range_bad = range_bad || lb < -kBinOff || lb > kNBin - 1 - kBinOff;
            if (mode == 0) {
                v0 = Mi;
                v1 = Mi * va[i];
                v2 = Mi * vb[i];
            } else {
                v0 = Mi * (fabs(log(va[i] / ms)) / 3.0);
            }
        }
        uint64_t rem = __ballot(valid);
        while (rem) {
            const int leader = __ffsll((unsigned long long)rem) - 1;
            const int bsel = __shfl(bin, leader, 64);
            const bool mine = valid && bin == bsel;
            const uint64_t match = __ballot(mine);
            const dd s0 = wave_sum_dd(dd{mine ? v0 : 0.0, 0.0});
            dd s1{0.0, 0.0}, s2{0.0, 0.0};
            if (mode == 0) {
                s1 = wave_sum_dd(dd{mine ? v1 : 0.0, 0.0});
                s2 = wave_sum_dd(dd{mine ? v2 : 0.0, 0.0});
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
    if (__ballot(range_bad) && lane == 0) set_status(ws, GD_DEV_MASS_RANGE);
    __syncthreads();
    for (int bin = t; bin < kNBin; bin += 256) {
        double* out = part + (int64_t(blockIdx.x) * kNBin + bin) * 8;
        double cnt = 0.0;
        dd x0{0.0, 0.0}, x1{0.0, 0.0}, x2{0.0, 0.0};
        for (int ww = 0; ww < 4; ++ww) {
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
__global__ __launch_bounds__(kNBin) void k_plan(DevProblem P, const double* __restrict__ part, int nblk,
                                                gd_interval* iv, WsHeader* h, void* ws)
{
    __shared__ double cnt[kNBin];
    __shared__ double sM[kNBin][2], sA[kNBin][2], sB[kNBin][2];
    const int b = threadIdx.x;
    double c = 0.0;
    dd x0{0.0, 0.0}, x1{0.0, 0.0}, x2{0.0, 0.0};
    for (int blk = 0; blk < nblk; ++blk) {
        const double* a = part + (int64_t(blk) * kNBin + b) * 8;
        c += a[0];
        x0 = dd_add(x0, dd{a[1], a[2]});
        x1 = dd_add(x1, dd{a[3], a[4]});
        x2 = dd_add(x2, dd{a[5], a[6]});
    }
    cnt[b] = c;
    sM[b][0] = x0.hi;
    sM[b][1] = x0.lo;
    sA[b][0] = x1.hi;
    sA[b][1] = x1.lo;
    sB[b][0] = x2.hi;
    sB[b][1] = x2.lo;
    __syncthreads();
    if (b != 0) return;
    // merge rule
    int ng = 0;
    double acc = 0.0;
    bool open = false;
    for (int bb = 0; bb < kNBin; ++bb) {
        h->group_of[bb] = -1;
        if (cnt[bb] == 0.0) continue;
        if (!open) {
            open = true;
            acc = 0.0;
        }
        h->group_of[bb] = ng;
        acc += cnt[bb];
        if (acc >= double(P.nbin_min)) {
            ++ng;
            open = false;
        }
    }
    if (open) {
        if (ng > 0) {
            for (int bb = 0; bb < kNBin; ++bb)
                if (h->group_of[bb] == ng) h->group_of[bb] = ng - 1;
        } else {
            ng = 1;
        }
    }
    const double dt_coll = iv->dt_coll;
    const double Cf = iv->C;
    const int64_t ticks = iv->ticks;
    const double tick = ldexp(dt_coll, -30);
    double req = double(kTicks - ticks) * tick;
    if (P.dt_fn_max < req) req = P.dt_fn_max;
    const double eC = P.eps * Cf;
    for (int g = 0; g < ng; ++g) {
        dd m{0.0, 0.0}, a{0.0, 0.0}, bsum{0.0, 0.0};
        for (int bb = 0; bb < kNBin; ++bb) {
            if (h->group_of[bb] != g) continue;
            m = dd_add(m, dd{sM[bb][0], sM[bb][1]});
            a = dd_add(a, dd{sA[bb][0], sA[bb][1]});
            bsum = dd_add(bsum, dd{sB[bb][0], sB[bb][1]});
        }
        h->gM[g] = m.hi;
        const double A_ = m.hi > 0.0 ? a.hi / m.hi : 0.0;
        const double B_ = m.hi > 0.0 ? bsum.hi / m.hi : 0.0;
        if (A_ > 0.0) {
            const double tt = eC / A_;
            if (tt < req) req = tt;
        }
        if (B_ > 0.0) {
            const double tt = (eC * eC) / B_;
            if (tt < req) req = tt;
        }
    }
    for (int g = ng; g < kNBin; ++g) h->gM[g] = 0.0;
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
}

// ---------------------------------------------------------------------------
void launch_bin_reduce(int mode, const double* msnap, const double* M, const double* va, const double* vb, int64_t n,
                       double* part, void* ws, hipStream_t st)
{
    hipLaunchKernelGGL(k_bin_reduce, dim3(kRedBlocks), dim3(256), 0, st, mode, msnap, M, va, vb, n, part, ws);
}

int launch_rates(const gd_problem* p, const gd_particles* s, const gd_neighbors* nb, gd_interval* iv, double* lam_i,
                 double* lam_pair, double* ab, void* ws, const Layout& L, hipStream_t st)
{
    const DevProblem P = to_dev(p);
    const int64_t n = p->n;
    const int g = int((n + 255) / 256);
    const double* m = s->m[s->cur];
    double* snap_s = at<double>(ws, L.snap_s);
    double* snap_N = at<double>(ws, L.snap_N);
    prof_mark(GD_PROF_RATES, 0, st);
    if (p->kernel == GD_KERNEL_PHYSICAL)
        hipLaunchKernelGGL(k_snapshot, dim3(g), dim3(256), 0, st, P, m, s->M, n, snap_s, snap_N);
    RatesArgs A{};
    A.P = P;
    A.nbr = nb->nbr;
    A.cnt = nb->cnt;
    A.dmax = nb->dmax;
    A.m = m;
    A.x = s->x;
    A.y = s->y;
    A.z = s->z;
    A.snap_s = snap_s;
    A.snap_N = snap_N;
    A.lam = lam_i;
    A.lam_pair = lam_pair;
    A.a = ab ? ab : at<double>(ws, L.a);
    A.b = ab ? ab + n : at<double>(ws, L.b);
    A.ws = ws;
    hipLaunchKernelGGL(k_rates, dim3(g), dim3(256), 0, st, A);
    double* part = at<double>(ws, L.part);
    launch_bin_reduce(0, m, s->M, A.a, A.b, n, part, ws, st);
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(kNBin), 0, st, P, part, kRedBlocks, iv, at<WsHeader>(ws, L.hdr), ws);
    prof_mark(GD_PROF_RATES, 1, st);
    return 0;
}

}  // namespace gd
