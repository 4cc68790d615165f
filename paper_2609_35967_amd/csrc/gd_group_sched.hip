// gd_group_sched.hip -- the collision step of spatial groups (Sect. 2.5.3)
// with its scheduler on the device.
//
// The host form (the gd_*_group calls driven instant by instant) reads the
// scheduled sizes back at every instant.  Here each instant is one fixed
// sequence of launches over all groups, every stage predicated on flags that
// a one-thread kernel sets on the device:
//   instant   tau = the earliest end of the groups' intervals; the groups whose
//             interval ends at tau publish, those with tau < 2^30 start;
//   publish   each ending group's masses become the broadcast masses, and its
//             scheduled interval is over;
//   snapshot  of every particle, when some group starts;
//   rates, bin sums and plan of every starting group (the many-run stages);
//   clamp     the starting groups in ascending order: each request held within
//             1/16 .. 16 times the scheduled intervals of the groups it
//             interacts with (the lower limit wins a conflict), halved until
//             aligned; the interval gets the next number in planning order,
//             which keys its random numbers; its end is recorded;
//   sampling and audit of every starting group (the many-run stages).
// Once the step's 2^30 ticks are used, later instants do nothing, so the host
// can queue several and read one flag.  Each group is a run of the many-run
// form over its slots of the shared particle set, with its own workspace and
// interval state; the snapshot lives in one workspace for all.
#include "gd_common.hpp"
#include "gd_internal.hpp"

#include <algorithm>

namespace gd {

constexpr int kSchedGroups = 64;
constexpr int kSchedLog = 1 << 14;  // (group, start, ticks) of the intervals of one collision step

struct GroupSched {
    int64_t tau;
    int64_t next_iv;                // the next interval number (planning order)
    int64_t end[kSchedGroups];      // end tick of each group's current interval
    int64_t iv_of[kSchedGroups];    // number of each group's current interval
    int32_t start[kSchedGroups];    // starts an interval at tau
    int32_t pub[kSchedGroups];      // publishes at tau
    int32_t has[kSchedGroups];      // has had an interval in this step
    int32_t any;                    // some group starts at tau
    int32_t done;                   // the step's ticks are used
    int32_t n_log;
    int32_t overflow;
    int64_t log[kSchedLog][3];
};

__global__ void k_gs_begin(GroupSched* S, int G, int64_t first_iv, int64_t* sched)
{
    if (threadIdx.x != 0) return;
    S->tau = 0;
    S->next_iv = first_iv;
    for (int g = 0; g < G; ++g) {
        S->end[g] = 0;
        S->iv_of[g] = 0;
        S->start[g] = 0;
        S->pub[g] = 0;
        S->has[g] = 0;
        sched[g] = 0;
    }
    S->any = 0;
    S->done = 0;
    S->n_log = 0;
    S->overflow = 0;
}

__global__ void k_gs_instant(GroupSched* S, int G)
{
    if (threadIdx.x != 0) return;
    if (S->done) {
        for (int g = 0; g < G; ++g) {
            S->start[g] = 0;
            S->pub[g] = 0;
        }
        S->any = 0;
        return;
    }
    int64_t tau = kTicks;
    for (int g = 0; g < G; ++g) tau = S->end[g] < tau ? S->end[g] : tau;
    int any = 0;
    for (int g = 0; g < G; ++g) {
        S->pub[g] = (S->has[g] && S->end[g] == tau) ? 1 : 0;
        S->start[g] = (S->end[g] == tau && tau < kTicks) ? 1 : 0;
        any |= S->start[g];
    }
    S->any = any;
    S->tau = tau;
    if (tau >= kTicks) S->done = 1;
}

// the starting groups in ascending order (the ratio limits of a group read
// the scheduled sizes of the groups planned before it)
__global__ void k_gs_clamp(GroupSched* S, int G, gd_interval* ivs, const unsigned long long* rows, int64_t* sched)
{
    if (threadIdx.x != 0) return;
    const int64_t tau = S->tau;
    for (int g = 0; g < G; ++g) {
        if (!S->start[g]) continue;
        gd_interval* iv = ivs + g;
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
        S->end[g] = tau + z;
        S->has[g] = 1;
        S->iv_of[g] = S->next_iv;
        S->next_iv = S->next_iv + 1;
        if (S->n_log < kSchedLog) {
            S->log[S->n_log][0] = g;
            S->log[S->n_log][1] = tau;
            S->log[S->n_log][2] = z;
            S->n_log = S->n_log + 1;
        } else {
            S->overflow = 1;
        }
    }
}

// the broadcast of an ending group's masses; its scheduled interval is over
struct PublishArgs {
    double* dst;
    const double* src;
    int64_t n;
    int64_t* sched;
    int32_t group;
};

struct Publish {
    using Args = PublishArgs;
    static constexpr int kThreads = 256;
    static __device__ __forceinline__ void body(const Args& A, Blk B)
    {
        const int64_t i = B.id * int64_t(blockDim.x) + threadIdx.x;
        if (i < A.n) A.dst[i] = A.src[i];
        if (i == 0) A.sched[A.group] = 0;
    }
};

static void step_instant(char*, const ManyStep& s, hipStream_t st)
{
    hipLaunchKernelGGL(k_gs_instant, dim3(1), dim3(64), 0, st, reinterpret_cast<GroupSched*>(s.a0), int(s.a1));
}

struct ClampRef {
    GroupSched* S;
    int G;
    gd_interval* ivs;
    const unsigned long long* rows;
    int64_t* sched;
};

static void step_clamp(char* base, const ManyStep& s, hipStream_t st)
{
    const ClampRef& c = *reinterpret_cast<const ClampRef*>(reinterpret_cast<const char*>(s.a0));
    hipLaunchKernelGGL(k_gs_clamp, dim3(1), dim3(64), 0, st, c.S, c.G, c.ivs, c.rows, c.sched);
}

}  // namespace gd

using namespace gd;

struct gd_group_sched {
    int device;
    int32_t G;
    char* dev;          // the many-run tables
    GroupSched* S;      // the scheduler's device state
    int64_t* sched;
    std::vector<ManyStep> steps;
    ClampRef clamp;
};

extern "C" {

int32_t gd_group_sched_create(const gd_problem* p, const gd_particles* st, const gd_neighbors* nb,
                              const int32_t* group_lo, int32_t G, gd_interval* ivs, const uint64_t* rows,
                              int64_t* sched, double* lam_i, int32_t* n_events, void* const* ws, size_t ws_bytes,
                              void* snap_ws, uint64_t seed, gd_group_sched** out)
{
    if (!out) return GD_E_INVALID_ARG;
    *out = nullptr;
    if (!p || !st || !nb || !group_lo || !ivs || !rows || !sched || !lam_i || !ws || !snap_ws || G < 1 ||
        G > kSchedGroups)
        return GD_E_INVALID_ARG;
    if (p->n < 1 || p->k < 2 || p->k > kMaxK || st->cur < 0 || st->cur > 1 || !st->m[0] || !st->m[1] ||
        !nb->nbr || !nb->cnt || !nb->dmax)
        return GD_E_INVALID_ARG;
    if (group_lo[0] != 0) return GD_E_INVALID_ARG;
    for (int g = 0; g < G; ++g)
        if (group_lo[g + 1] <= group_lo[g] || group_lo[g + 1] > p->n || !ws[g]) return GD_E_INVALID_ARG;
    const Layout Lfull = make_layout(p->n, p->k);
    if (ws_bytes < Lfull.total) return GD_E_WORKSPACE;
    gd_group_sched* m = new gd_group_sched{};
    if (hipGetDevice(&m->device) != hipSuccess || hipMalloc(reinterpret_cast<void**>(&m->S), sizeof(GroupSched)) != hipSuccess) {
        delete m;
        return GD_E_HIP;
    }
    m->G = G;
    m->sched = sched;
    double4* snap = at<double4>(snap_ws, Lfull.snap);
    std::vector<ManyRun> R;
    const int k = p->k;
    for (int g = 0; g < G; ++g) {
        const int64_t lo = group_lo[g], n = group_lo[g + 1] - lo;
        ManyRun x{};
        x.p = *p;
        x.p.n = n;
        gd_particles s = *st;
        auto off = [&](double* a) { return a ? a + lo : a; };
        s.x = off(s.x);
        s.y = off(s.y);
        s.z = off(s.z);
        s.r = off(s.r);
        s.th = off(s.th);
        s.ph = off(s.ph);
        s.vr = off(s.vr);
        s.lth = off(s.lth);
        s.lph = off(s.lph);
        s.vz = off(s.vz);
        s.st_mid = off(s.st_mid);
        s.M = off(s.M);
        s.m[0] = off(s.m[0]);
        s.m[1] = off(s.m[1]);
        s.id = st->id + lo;
        x.in = s;
        x.out = s;
        x.nb = gd_neighbors{nb->nbr + lo * k, nb->cnt + lo, nb->dmax + lo, nullptr};
        x.iv = ivs + g;
        x.lam_i = lam_i + lo;
        x.n_events = n_events ? n_events + lo : nullptr;
        x.ws = ws[g];
        x.L = make_layout(n, k);
        x.seed = seed;
        x.lo = lo;
        x.n_all = p->n;
        x.snap = snap;
        x.interval_at = &m->S->iv_of[g];
        R.push_back(x);
    }
    ManyBuilder B;
    B.tune = gd_many_tuning{0, 256, 512, 2048, 768};  // the per-lane search is not used here
    GroupSched* S = m->S;
    B.add_raw(&step_instant, 0, reinterpret_cast<int64_t>(S), G);
    {
        std::vector<PublishArgs> pa(G);
        std::vector<int64_t> nbk(G);
        for (int g = 0; g < G; ++g) {
            const int64_t lo = group_lo[g], n = group_lo[g + 1] - lo;
            pa[g] = PublishArgs{st->m[st->cur] + lo, st->m[st->cur ^ 1] + lo, n, sched, g};
            nbk[g] = cdiv(n, 256);
        }
        B.active = S->pub;
        B.add<Publish>(pa, nbk);
    }
    B.active = &S->any;
    many_snapshot(B, p, st, snap);
    B.active = S->start;
    many_rates(B, R, false);
    m->clamp = ClampRef{S, G, ivs, reinterpret_cast<const unsigned long long*>(rows), sched};
    B.active = nullptr;
    B.add_raw(&step_clamp, 0, reinterpret_cast<int64_t>(&m->clamp), 0);
    B.active = S->start;
    many_sample(B, R);
    m->steps = B.steps;
    const size_t bytes = B.arena.size();
    if (hipMalloc(reinterpret_cast<void**>(&m->dev), bytes) != hipSuccess ||
        hipMemcpy(m->dev, B.arena.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(m->S);
        if (m->dev) (void)hipFree(m->dev);
        delete m;
        return GD_E_HIP;
    }
    *out = m;
    return GD_OK;
}

int32_t gd_group_sched_begin(gd_group_sched* m, int64_t first_interval, void* stream)
{
    if (!m || first_interval < 0) return GD_E_INVALID_ARG;
    hipLaunchKernelGGL(k_gs_begin, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream), m->S, m->G, first_interval,
                       m->sched);
    return hipGetLastError() == hipSuccess ? GD_OK : GD_E_HIP;
}

int32_t gd_group_sched_instants(gd_group_sched* m, int32_t count, void* stream)
{
    if (!m || count < 0) return GD_E_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (int32_t c = 0; c < count; ++c)
        for (const ManyStep& s : m->steps) s.fn(m->dev, s, st);
    return hipGetLastError() == hipSuccess ? GD_OK : GD_E_HIP;
}

int32_t gd_group_sched_read(gd_group_sched* m, void* stream, int32_t* done, int64_t* next_interval, int32_t* n_log,
                            int64_t* log, int32_t log_cap)
{
    if (!m || !done || !next_interval || !n_log || (log_cap > 0 && !log)) return GD_E_INVALID_ARG;
    if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return GD_E_HIP;
    int32_t head[4];
    int64_t nx;
    if (hipMemcpy(&nx, &m->S->next_iv, sizeof(nx), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(head, &m->S->done, sizeof(head), hipMemcpyDeviceToHost) != hipSuccess)
        return GD_E_HIP;
    *done = head[0];
    *n_log = head[2] ? -1 : head[1];
    *next_interval = nx;
    const int32_t nl = std::min<int32_t>(head[1], log_cap);
    if (nl > 0 && hipMemcpy(log, &m->S->log[0][0], sizeof(int64_t) * 3 * size_t(nl), hipMemcpyDeviceToHost) != hipSuccess)
        return GD_E_HIP;
    return GD_OK;
}

int32_t gd_group_sched_destroy(gd_group_sched* m)
{
    if (!m) return GD_OK;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(m->device);
    (void)hipFree(m->dev);
    (void)hipFree(m->S);
    (void)hipSetDevice(cur);
    delete m;
    return GD_OK;
}

}  // extern "C"
