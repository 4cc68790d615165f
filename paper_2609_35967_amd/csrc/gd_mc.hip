// gd_mc.hip -- Monte Carlo sampling of collision events against the frozen
// neighbourhood (Sect. 2.5.3) and the post-interval audit.
//
// One lane per particle.  The particle draws waiting times
// dt_w = -ln(U_w)/lambda*_i (Gillespie); an event happens iff dt_w fits in the
// rest of the interval.  Its partner is the first slot whose inclusive prefix of
// lambda*_ij exceeds U_p lambda*_i, its channel the first whose cumulative rate
// exceeds U_c lambda*_ij; the outcome (Sect. 2.5.2) updates only this particle,
// after which every lambda*_ij is recomputed from the new mass against the
// frozen neighbours.  lambda*_i of the start state comes from the rates pass
// (the same function of the same inputs), so particles without events never
// evaluate their pairs here.  Random numbers: Philox4x32-10 keyed by the seed,
// counters (id, interval, event, 0/1); every event uses both calls.
//
// Audit (a reading: the paper names what the audit monitors, not its rule):
// per merged controller bin the mass-weighted mean realised |ln(s'/s)|; if the
// largest exceeds 2 eps C, C halves (floor 0.25), else C grows by 1.25 (cap 1).
#include "gd_common.hpp"
#include "gd_internal.hpp"
#include "gd_physics.hpp"

#include <algorithm>

namespace gd {

struct McArgs {
    DevProblem P;
    const uint32_t* id;
    const int32_t* nbr;
    const int32_t* cnt;
    const double* dmax;
    const double* m;      // snapshot (frozen) masses
    const double* x;
    const double* y;
    const double* z;
    const double4* snap;  // packed (m, s, N, 0) of the frozen neighbourhood
    const double* lam_i;
    const gd_interval* iv;
    double* m_out;
    int32_t* n_events;
    int32_t* log;
    int32_t log_cap;
    uint64_t seed;
    uint32_t interval;
    int32_t interval_on_device;  // take the index from iv->n_intervals
    void* ws;
    unsigned long long* ev_counter;
    // particles still sampling after `budget` events are handed, at that
    // event boundary, to a pass that runs one wavefront per particle
    int32_t budget;
    struct Deferred* heavy;
    int32_t* heavy_n;
    int32_t* heavy_next;
    int64_t n_all;  // length of the snapshot: neighbour indices lie in [0, n_all)
    int32_t* list;       // particles with an event (screen -> event pass), a segment per die
    int32_t* list_seg;   // the segments' counts
    int32_t* list_next;  // the event pass's next group
    const int64_t* interval_at;  // when set: the interval index (a spatial group's number in planning order)
    const int32_t* active;       // when set and 0: the run has no interval now (its deferred list is skipped)
    // the screen sends a particle whose expected events lambda*_i dt_exe reach
    // early_events (0: none) straight to the wavefront-per-particle pass, to
    // entries n - 1, n - 2, ... of `heavy` (the event pass defers to entries
    // 0, 1, ...; no particle is in both), counted by heavy_n0, taken by
    // heavy_next0
    double early_events;
    int32_t* heavy_n0;
    int32_t* heavy_next0;
};

__device__ inline uint32_t mc_interval(const McArgs& A)
{
    if (A.interval_at) return uint32_t(*A.interval_at);
    return A.interval_on_device ? uint32_t(A.iv->n_intervals) : A.interval;
}

// a particle handed over after e events, at time t of the interval, with mass m
struct Deferred {
    int32_t i;
    int32_t e;
    double t;
    double m;
};

constexpr int kEventCap = 1 << 24;  // safety stop per particle and interval (status-flagged)
constexpr int kLaneEvents = 4;      // events a lane samples before handing its particle over
constexpr int kHeavyBlocks = 768;   // blocks (4 wavefronts each) of the wavefront-per-particle pass: 3 per SIMD
constexpr int kEventBlocks = 512;   // blocks (4 wavefronts each) of the event pass: two per SIMD
constexpr int kSmallList = 3072;    // at most this many particles with events: all to the wavefront pass
constexpr double kEarlyEvents = 64.0;  // expected events from which the screen sends a particle straight to that pass
constexpr int kEarlyBlocks = 256;      // blocks (4 wavefronts each) for those particles beside the event pass

template <int KP2>
__device__ inline double prefix_rates_f32(const McArgs& A, const QCtxF& q, const int32_t* row, int c, double mi,
                                          float si, float Sti, double (&pre)[KP2])
{
    const bool phys = A.P.kernel == GD_KERNEL_PHYSICAL;
    double li = 0.0;
#pragma unroll
    for (int s = 0; s < KP2; ++s) {
        if (s < c) {
            int j = row[s];
            if (j < 0 || j >= A.n_all) {
                set_status(A.ws, GD_DEV_INTERNAL);
                j = 0;
            }
            const double4 sn = A.snap[j];
            PairF o;
            pair_eval_f32(A.P, q, mi, 1.0 / mi, si, Sti, sn.x, phys ? float(sn.y) : 0.0f, phys ? sn.z : 0.0, o);
            li = li + double(o.lam_star);
        }
        pre[s] = li;
    }
    return li;
}

template <int KP2>
__device__ inline double prefix_rates(const McArgs& A, const QCtx& q, const int32_t* row, int c, const Own& w,
                                      double (&pre)[KP2])
{
    const bool phys = A.P.kernel == GD_KERNEL_PHYSICAL;
    double li = 0.0;
#pragma unroll
    for (int s = 0; s < KP2; ++s) {
        if (s < c) {
            int j = row[s];
            if (j < 0 || j >= A.n_all) {
                set_status(A.ws, GD_DEV_INTERNAL);
                j = 0;
            }
            const double4 sn = A.snap[j];
            Pair o;
            pair_eval(A.P, q, w, sn.x, phys ? sn.y : 0.0, phys ? sn.z : 0.0, sn.w, o);
            li = li + o.lam_star;
        }
        pre[s] = li;
    }
    return li;
}

// Sampling runs in two steps.  The screen (one lane per particle, few
// registers) draws each particle's first waiting time against lambda*_i of
// the rates pass: a particle without an event in the interval keeps its mass
// and is done; the others go, compacted, to a list.  The event pass then
// samples the listed particles, one lane each (up to kLaneEvents events,
// then the wavefront-per-particle pass), from a grid that strides over the
// list, so lanes without events never hold a wavefront's registers.  Its
// lanes redraw the first event's numbers (the same counters, so the same
// numbers).  For neighbourhoods beyond 64 (no prefix registers) the screen
// hands its particles straight to the wavefront-per-particle pass.
// The list has a segment per die: the blocks dealt to die x (block b with
// b % 8 == x, 256 particles each) fill segment x, which starts after the
// blocks of the dies before it, so that the count adds of one die go to its
// own counter.  One add per block.
__device__ inline int64_t seg_base(int x, int64_t nblocks)
{
    return ((nblocks / kXcd) * x + (x < nblocks % kXcd ? x : nblocks % kXcd)) * 256;
}

template <bool DIRECT_HEAVY>
struct McScreen {
    using Args = McArgs;
    static constexpr int kThreads = 256;
    static __device__ __forceinline__ void body(const Args& A, Blk B);
};

template <bool DIRECT_HEAVY>
__global__ __launch_bounds__(256) void k_mc_screen(McArgs A)
{
    McScreen<DIRECT_HEAVY>::body(A, Blk{int64_t(blockIdx.x), int64_t(gridDim.x)});
}

template <bool DIRECT_HEAVY>
__device__ __forceinline__ void McScreen<DIRECT_HEAVY>::body(const Args& A, Blk B)
{
    __shared__ int32_t s_w[4];
    __shared__ int32_t s_base;
    const int64_t i = B.id * int64_t(blockDim.x) + threadIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    bool ev = false, early = false;
    if (i < A.P.n) {
        const int c = A.cnt[i];
        const double m = A.m[i];
        const double li = A.lam_i[i];
        if (c > 1 && li > 0.0) {
            const uint32_t interval = mc_interval(A);
            double u[4];
            event_uniforms(A.seed, A.id[i], interval, 0u, u);
            ev = !(-log(u[0]) / li > A.iv->dt_exe);
            // many expected events: the whole interval in the wavefront pass
            // (the result is the same whichever pass samples a particle)
            early = !DIRECT_HEAVY && ev && A.early_events > 0.0 && li * A.iv->dt_exe >= A.early_events;
        }
        if (!ev) {
            A.m_out[i] = m;
            if (A.n_events) A.n_events[i] = 0;
            if (A.log)
                for (int f = 0; f < A.log_cap; ++f) A.log[i * A.log_cap + f] = -1;
        } else if ((DIRECT_HEAVY || early) && A.log) {
            for (int f = 0; f < A.log_cap; ++f) A.log[i * A.log_cap + f] = -1;
        }
    }
    if (!DIRECT_HEAVY) {  // the early ones, one add per wavefront that has any
        const uint64_t eb = __ballot(early);
        int32_t base = 0;
        if (lane == 0 && eb) base = atomicAdd(A.heavy_n0, int32_t(__popcll(eb)));
        base = __builtin_amdgcn_readfirstlane(base);
        if (early)
            A.heavy[A.P.n - 1 - (base + int32_t(__popcll(eb & ((uint64_t(1) << lane) - 1))))] =
                Deferred{int32_t(i), 0, 0.0, A.m[i]};
        ev = ev && !early;
    }
    const uint64_t bal = __ballot(ev);
    if (lane == 0) s_w[wv] = int32_t(__popcll(bal));
    __syncthreads();
    if (threadIdx.x == 0) {
        const int32_t tot = s_w[0] + s_w[1] + s_w[2] + s_w[3];
        int32_t b = 0;
        if (tot) b = atomicAdd(DIRECT_HEAVY ? A.heavy_n : &A.list_seg[B.id % kXcd], tot);
        s_base = b;
    }
    __syncthreads();
    if (ev) {
        int32_t at = s_base + int32_t(__popcll(bal & ((uint64_t(1) << lane) - 1)));
        for (int w = 0; w < wv; ++w) at += s_w[w];
        if (DIRECT_HEAVY) A.heavy[at] = Deferred{int32_t(i), 0, 0.0, A.m[i]};
        else A.list[seg_base(int(B.id % kXcd), B.n) + at] = int32_t(i);
    }
}

template <int KP2, bool F32>
__device__ inline int mc_particle(const McArgs& A, int64_t i)
{
    constexpr int KR = KP2;  // prefix registers
    int e = 0;
    if (i < A.P.n) {
        const int k = A.P.k;
        const bool phys = A.P.kernel == GD_KERNEL_PHYSICAL;
        const int c = A.cnt[i];
        double m = A.m[i];
        double li = A.lam_i[i];
        const double dt_exe = A.iv->dt_exe;
        const uint32_t interval = mc_interval(A);
        if (c > 1 && li > 0.0) {
            const uint32_t pid = A.id[i];
            const int32_t* row = A.nbr + i * k;
            QCtx q{};
            QCtxF qf{};
            Own own{};
            bool have_ctx = false, have_pre = false;
            double si = 0.0, Sti = 0.0;
            double pre[KR];
            double t = 0.0;
            for (;;) {
                if (!(li > 0.0)) break;
                if (e >= A.budget) {
                    // many events: the rest of this particle's interval runs
                    // in the wavefront-per-particle pass (li equals the prefix
                    // of the current mass, which that pass recomputes)
                    const int32_t slot = atomicAdd(A.heavy_n, 1);
                    A.heavy[slot] = Deferred{int32_t(i), e, t, m};
                    break;
                }
                if (e >= kEventCap) {
                    set_status(A.ws, GD_DEV_EVENT_CAP);
                    break;
                }
                double u[4];
                event_uniforms(A.seed, pid, interval, uint32_t(e), u);
                const double dtw = -log(u[0]) / li;
                if (dtw > dt_exe - t) break;
                t = t + dtw;
                if (!have_ctx) {
                    query_ctx(A.P, A.x[i], A.y[i], A.z[i], A.dmax[i], q);
                    if (F32) query_ctx_f32(A.P, q, qf);
                    have_ctx = true;
                }
                if (!have_pre) {
                    if (phys) {
                        si = grain_size(A.P, m);
                        Sti = F32 ? double(qf.stfac * float(si)) : q.stfac * si;
                    }
                    if (!F32) own_terms(A.P, q, m, si, false, own);
                    li = F32 ? prefix_rates_f32<KR>(A, qf, row, c, m, float(si), float(Sti), pre)
                             : prefix_rates<KR>(A, q, row, c, own, pre);
                    have_pre = true;
                }
                const double target = u[1] * li;
                int sel = c - 1;
                bool found = false;
#pragma unroll
                for (int s = 0; s < KR; ++s) {
                    const bool hit = !found && s < c - 1 && pre[s] > target;
                    sel = hit ? s : sel;
                    found = found || hit;
                }
                int j = row[sel];
                if (j < 0 || j >= A.n_all) j = 0;
                const double4 sn = A.snap[j];
                const double mj = sn.x;
                const double sj = phys ? sn.y : 0.0;
                Pair o;
                if (F32) {
                    PairF of;
                    pair_eval_f32(A.P, qf, m, 1.0 / m, float(si), float(Sti), mj, float(sj), phys ? sn.z : 0.0, of);
                    o.type = of.type;
                    o.r0 = of.r0;
                    o.r1 = of.r1;
                    o.lam_star = double(of.r0) + double(of.r1);
                    o.Ng = of.Ng;
                } else {
                    pair_eval(A.P, q, own, mj, sj, phys ? sn.z : 0.0, sn.w, o);
                }
                int ch = 0;
                if (o.type == kErosion) ch = (o.r0 > u[2] * o.lam_star) ? 0 : 1;
                double mnew;
                if (o.type == kStick) {
                    mnew = m + o.Ng * mj;
                } else if (o.type == kErosion) {
                    mnew = (ch == 0) ? m - o.Ng * mj : mj;
                } else {
                    const double a = sqrt(A.P.s_min);
                    const double w = a + u[3] * (sqrt(si) - a);
                    const double sn = w * w;
                    mnew = div_nr(kPi * A.P.rho_s * sn * sn * sn, 6.0);
                }
                if (A.log) {
                    if (e < A.log_cap) A.log[i * A.log_cap + e] = sel | (ch << 16) | (o.type << 24);
                    else set_status(A.ws, GD_DEV_LOG_OVERFLOW);
                }
                ++e;
                if (mnew != m) {
                    m = mnew;
                    have_pre = false;
                    if (phys) {
                        si = grain_size(A.P, m);
                        Sti = F32 ? double(qf.stfac * float(si)) : q.stfac * si;
                    }
                    if (!F32) own_terms(A.P, q, m, si, false, own);
                    li = F32 ? prefix_rates_f32<KR>(A, qf, row, c, m, float(si), float(Sti), pre)
                             : prefix_rates<KR>(A, q, row, c, own, pre);
                    have_pre = true;
                }
            }
        }
        A.m_out[i] = m;
        if (A.n_events) A.n_events[i] = e;
        if (A.log)
            for (int f = e; f < A.log_cap; ++f) A.log[i * A.log_cap + f] = -1;
    }
    return e;
}

// the listed particles, one lane each: the segments are read as one list;
// wavefront w takes entries 64 w .. 64 w + 63 first, then further groups of
// 64 from a counter until the list is exhausted (a wavefront with no first
// group touches no counter)
// the event pass's arguments: the sampling's and the screen's block count
// (the list's segments are laid out by it)
struct EventArgs {
    McArgs A;
    int64_t screen_blocks;
};

template <int KP2, bool F32>
struct McEvents {
    using Args = EventArgs;
    static constexpr int kThreads = 256;
    static __device__ __forceinline__ void body(const Args& E, Blk B);
};

template <int KP2, bool F32>
__global__ __launch_bounds__(256) void k_mc(EventArgs E)
{
    McEvents<KP2, F32>::body(E, Blk{int64_t(blockIdx.x), int64_t(gridDim.x)});
}

template <int KP2, bool F32>
__device__ __forceinline__ void McEvents<KP2, F32>::body(const Args& E, Blk B)
{
    const McArgs& A = E.A;
    const int64_t screen_blocks = E.screen_blocks;
    const int lane = threadIdx.x & 63;
    int32_t pre[kXcd + 1];
    pre[0] = 0;
#pragma unroll
    for (int x = 0; x < kXcd; ++x) pre[x + 1] = pre[x] + A.list_seg[x];
    const int32_t nl = pre[kXcd];
    const int32_t nw = int32_t(B.n * (blockDim.x / kWave));
    int32_t b = int32_t(B.id * (blockDim.x / kWave) + threadIdx.x / kWave) * kWave;
    if (nl <= kSmallList) {
        // few particles with events (a cold disk): each takes a wavefront of
        // the wavefront-per-particle pass at once, where its pairs are
        // evaluated side by side instead of one after another in a lane.
        // The grid strides over the list (a small grid covers less than it).
        for (int32_t t = b + lane; t < nl; t += nw * kWave) {
            int x = 0;
#pragma unroll
            for (int y = 1; y < kXcd; ++y) x += t >= pre[y] ? 1 : 0;
            const int32_t i = A.list[seg_base(x, screen_blocks) + (t - pre[x])];
            if (A.log)
                for (int f = 0; f < A.log_cap; ++f) A.log[i * A.log_cap + f] = -1;
            A.heavy[atomicAdd(A.heavy_n, 1)] = Deferred{i, 0, 0.0, A.m[i]};
        }
        return;
    }
    unsigned long long ev = 0;
    while (b < nl) {
        const int32_t t = b + lane;
        if (t < nl) {
            int x = 0;
#pragma unroll
            for (int y = 1; y < kXcd; ++y) x += t >= pre[y] ? 1 : 0;
            ev += (unsigned long long)mc_particle<KP2, F32>(A, A.list[seg_base(x, screen_blocks) + (t - pre[x])]);
        }
        int32_t nx = 0;
        if (lane == 0) nx = atomicAdd(A.list_next, kWave);
        b = nw * kWave + __builtin_amdgcn_readfirstlane(nx);
    }    // events of the interval, one atomic per wavefront
#pragma unroll
    for (int mk = 1; mk < 64; mk <<= 1) ev += __shfl_xor(ev, mk, 64);
    if (lane == 0 && ev) atomicAdd(A.ev_counter, ev);
}

// ---------------------------------------------------------------------------
// The rest of the interval of each deferred particle, one wavefront per
// particle.  Lane s < c holds neighbour slot s: the neighbour's terms that
// the frozen snapshot fixes for the whole interval are computed once, and
// per event the lane evaluates its pair for the particle's current mass and
// the outcome the event would have with that partner.  The prefix over the
// slots is a wavefront scan; the selection (first slot whose prefix exceeds
// the target) is a ballot, and the chosen lane's outcome is read across.
// The draws do not depend on the mass: lane L draws the numbers of event
// e0 + L, 64 events at a time, and each event reads its own from that lane.
// Wavefronts take particles from a counter until the list is exhausted.

// the numbers of events e0 .. e0 + 63 (lane L: event e0 + L): -ln U_w, U_p, U_c, U_f
struct Draws {
    double lw, up, uc, uf;
};

__device__ inline void draw64(const McArgs& A, uint32_t pid, uint32_t interval, uint32_t e0, int lane, Draws& d)
{
    double u[4];
    event_uniforms(A.seed, pid, interval, e0 + uint32_t(lane), u);
    d.lw = -log(u[0]);
    d.up = u[1];
    d.uc = u[2];
    d.uf = u[3];
}

// the rest of deferred particle `hidx` of the run described by A; returns the
// events it adds.  Lane s holds the pairs of slots s, s + 64, ... (R of
// them for neighbourhoods beyond 64).
template <int KP2, bool F32>
__device__ inline int run_deferred(const McArgs& A, int32_t hidx, int lane)
{
    constexpr int R = KP2 > kWave ? KP2 / kWave : 1;
    constexpr int W = KP2 < kWave ? KP2 : kWave;  // lanes holding slots
    const bool phys = A.P.kernel == GD_KERNEL_PHYSICAL;
    const double dt_exe = A.iv->dt_exe;
    const uint32_t interval = mc_interval(A);
    const Deferred H = A.heavy[hidx];
    const int64_t i = H.i;
    int e = H.e;
    double t = H.t, m = H.m;
    const int k = A.P.k;
    const int c = A.cnt[i];
    const uint32_t pid = A.id[i];
    QCtx q{};
    QCtxF qf{};
    query_ctx(A.P, A.x[i], A.y[i], A.z[i], A.dmax[i], q);
    if (F32) query_ctx_f32(A.P, q, qf);
    Nb nb[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int s = r * kWave + lane;
        const bool mine = s < c && lane < W;
        int j = mine ? A.nbr[i * k + s] : 0;
        if (mine && (j < 0 || j >= A.n_all)) set_status(A.ws, GD_DEV_INTERNAL);
        if (j < 0 || j >= A.n_all) j = 0;
        const double4 sn = A.snap[j];
        if (F32) {
            nb[r].mj = sn.x;
            nb[r].sj = phys ? sn.y : 0.0;
            nb[r].Nj = phys ? sn.z : 0.0;
        } else {
            nb_terms<true>(A.P, q, sn.x, phys ? sn.y : 0.0, phys ? sn.z : 0.0, sn.w, nb[r]);
        }
    }
    uint32_t e0 = uint32_t(e);
    Draws d;
    draw64(A, pid, interval, e0, lane, d);
    for (;;) {
        if (uint32_t(e) - e0 >= uint32_t(kWave)) {
            e0 = uint32_t(e);
            draw64(A, pid, interval, e0, lane, d);
        }
        const int L = int(uint32_t(e) - e0);
        const double lw = readlane_d(d.lw, L), up = readlane_d(d.up, L), uc = readlane_d(d.uc, L);
        // the pairs at the current mass, each with its outcome (a fragmentation
        // outcome does not depend on the partner and is made after the selection)
        double si = 0.0;
        Own w{};
        if (phys) si = grain_size(A.P, m);
        if (!F32) own_terms(A.P, q, m, si, false, w);
        const float Stf = F32 && phys ? qf.stfac * float(si) : 0.0f;
        double pre[R], mnew[R];
        int code[R];
        double carry = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            int type;
            double r0, lam, Ng;
            if (F32) {
                PairF of;
                pair_eval_f32(A.P, qf, m, 1.0 / m, float(si), Stf, nb[r].mj, float(nb[r].sj), nb[r].Nj, of);
                type = of.type;
                r0 = of.r0;
                lam = double(of.r0) + double(of.r1);  // the channel choice's total
                Ng = of.Ng;
                pre[r] = double(of.lam_star);         // the prefix adds the float rate
            } else {
                Pair o;
                pair_core<true>(A.P, q, w, nb[r], o);
                type = o.type;
                r0 = o.r0;
                lam = o.lam_star;
                Ng = o.Ng;
                pre[r] = o.lam_star;
            }
            const int ch = (type == kErosion && !(r0 > uc * lam)) ? 1 : 0;
            const double mj = nb[r].mj;
            mnew[r] = type == kStick ? m + Ng * mj : (ch == 0 ? m - Ng * mj : mj);
            code[r] = (ch << 16) | (type << 24);
            const double x = wave_scan_incl((r * kWave + lane < c && lane < W) ? pre[r] : 0.0);
            pre[r] = carry + x;
            carry = carry + readlane_d(x, kWave - 1);
        }
        const double li = carry;
        if (!(li > 0.0)) break;
        if (e >= kEventCap) {
            if (lane == 0) set_status(A.ws, GD_DEV_EVENT_CAP);
            break;
        }
        const double dtw = lw / li;
        if (dtw > dt_exe - t) break;
        t = t + dtw;
        const double target = up * li;
        // the first slot below c - 1 whose prefix exceeds the target, else c - 1
        int sel = c - 1;
#pragma unroll
        for (int r = R - 1; r >= 0; --r) {
            const uint64_t hit = __ballot(r * kWave + lane < c - 1 && pre[r] > target);
            if (hit) sel = r * kWave + int(__ffsll((unsigned long long)hit)) - 1;
        }
        const int sl = sel & (kWave - 1), sr = sel / kWave;
        int cd = 0;
        double mn = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (r == sr) {  // uniform: sel is the same in every lane
                cd = __builtin_amdgcn_readlane(code[r], sl);
                mn = readlane_d(mnew[r], sl);
            }
        }
        if ((cd >> 24) == kFrag) {
            const double uf = readlane_d(d.uf, L);
            const double a = sqrt(A.P.s_min);
            const double wf = a + uf * (sqrt(si) - a);
            const double sz = wf * wf;
            mn = div_nr(kPi * A.P.rho_s * sz * sz * sz, 6.0);
        }
        if (A.log && lane == 0) {
            if (e < A.log_cap) A.log[i * A.log_cap + e] = sel | cd;
            else set_status(A.ws, GD_DEV_LOG_OVERFLOW);
        }
        ++e;
        // (an unchanged mass recomputes the same rates: no branch around them)
        m = mn;
    }
    if (lane == 0) {
        A.m_out[i] = m;
        if (A.n_events) A.n_events[i] = e;
    }
    return e - H.e;
}

template <int KP2, bool F32>
__global__ __launch_bounds__(256) void k_mc_heavy(McArgs A)
{
    const int lane = threadIdx.x & 63;
    const int32_t nh = *A.heavy_n;
    unsigned long long ev_total = 0;
    // wavefront w takes entry w first, then entries nw, nw + 1, ... from the
    // counter (a wavefront with no first entry touches no counter)
    const int32_t nw = int32_t(gridDim.x * (blockDim.x / kWave));
    int32_t hidx = int32_t(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave);
    for (;;) {
        if (hidx >= nh) break;
        ev_total += (unsigned long long)run_deferred<KP2, F32>(A, hidx, lane);
        int32_t next = 0;
        if (lane == 0) next = atomicAdd(A.heavy_next, 1);
        hidx = nw + __builtin_amdgcn_readfirstlane(next);
    }
    if (lane == 0 && ev_total) atomicAdd(A.ev_counter, ev_total);
}

// The chains the screen sent early and the event pass, in one launch: the
// first kEarlyBlocks blocks (dispatched first) run the early chains (entries
// n - 1 - h of `heavy` for h < *heavy_n0; their wavefronts without one leave
// at once), the rest the event pass, so that the long chains run beside the
// event pass instead of after it.  The chains the event pass defers follow
// in k_mc_heavy.
template <int KP2, bool F32>
__global__ __launch_bounds__(256) void k_mc_fused(EventArgs E)
{
    if (blockIdx.x >= unsigned(kEarlyBlocks)) {
        McEvents<KP2, F32>::body(E, Blk{int64_t(blockIdx.x - unsigned(kEarlyBlocks)), int64_t(kEventBlocks)});
        return;
    }
    const McArgs& A = E.A;
    const int lane = threadIdx.x & 63;
    const int32_t nh = *A.heavy_n0;
    unsigned long long ev_total = 0;
    const int32_t nw = int32_t(kEarlyBlocks * (blockDim.x / kWave));
    int32_t h = int32_t(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave);
    for (;;) {
        if (h >= nh) break;
        ev_total += (unsigned long long)run_deferred<KP2, F32>(A, int32_t(A.P.n - 1 - h), lane);
        int32_t next = 0;
        if (lane == 0) next = atomicAdd(A.heavy_next0, 1);
        h = nw + __builtin_amdgcn_readfirstlane(next);
    }
    if (lane == 0 && ev_total) atomicAdd(A.ev_counter, ev_total);
}

// ---------------------------------------------------------------------------
// Many runs: a table in device memory holds, per slot, the sampling arguments
// of one run (written by its deferred call), after a 256-byte header whose
// first word counts the entries taken.  One launch runs the deferred
// particles of every slot: the global entry g is the slot's own entry
// g - (deferred particles of the slots before it).
constexpr size_t kTableHeader = 256;
constexpr int kMaxTableSlots = 4096;

__global__ void k_table_put(McArgs* dst, McArgs A)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = A;
}

template <int KP2, bool F32>
__global__ __launch_bounds__(256) void k_mc_heavy_batch(char* table, int32_t nbox)
{
    __shared__ int32_t s_pre[kMaxTableSlots];
    __shared__ int32_t s_total;
    const McArgs* T = reinterpret_cast<const McArgs*>(table + kTableHeader);
    int32_t* counter = reinterpret_cast<int32_t*>(table);
    const int t = threadIdx.x, lane = t & 63;
    for (int b = t; b < nbox; b += blockDim.x) s_pre[b] = (T[b].active && !*T[b].active) ? 0 : *T[b].heavy_n;
    __syncthreads();
    if (t < kWave) {  // exclusive prefix of the slots' counts, 64 at a time
        int32_t carry = 0;
        for (int c0 = 0; c0 < nbox; c0 += kWave) {
            const int32_t v = c0 + t < nbox ? s_pre[c0 + t] : 0;
            int32_t x = v;
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const int32_t y = __shfl_up(x, o, kWave);
                if (t >= o) x += y;
            }
            if (c0 + t < nbox) s_pre[c0 + t] = carry + x - v;
            carry += __shfl(x, kWave - 1, kWave);
        }
        if (t == 0) s_total = carry;
    }
    __syncthreads();
    const int32_t total = s_total;
    const int32_t nw = int32_t(gridDim.x * (blockDim.x / kWave));
    int32_t g = int32_t(blockIdx.x * (blockDim.x / kWave) + t / kWave);
    for (;;) {
        if (g >= total) break;
        // the last slot whose prefix is <= g (slots with no entries share a prefix)
        int lo = 0, hi = nbox - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_pre[mid] <= g) lo = mid;
            else hi = mid - 1;
        }
        const McArgs& A = T[lo];
        if (A.P.k > KP2 || (A.P.rates_fp32 != 0) != F32) {
            if (lane == 0) set_status(A.ws, GD_DEV_INTERNAL);
        } else {
            const int ev = run_deferred<KP2, F32>(A, g - s_pre[lo], lane);
            if (lane == 0 && ev) atomicAdd(A.ev_counter, (unsigned long long)ev);
        }
        int32_t next = 0;
        if (lane == 0) next = atomicAdd(counter, 1);
        g = nw + __builtin_amdgcn_readfirstlane(next);
    }
}

// ---------------------------------------------------------------------------
constexpr int kAuditGroups = 8;  // block-partial groups summed in parallel

struct AuditArgs {
    DevProblem P;
    const double* part;
    int nblk;
    gd_interval* iv;
    WsHeader* h;
};

struct Audit {
    using Args = AuditArgs;
    static constexpr int kThreads = kAuditGroups * kNBin;
    static __device__ __forceinline__ void body(const Args& A, Blk B);
};

__global__ __launch_bounds__(kAuditGroups * kNBin) void k_audit(AuditArgs A)
{
    Audit::body(A, Blk{0, 1});
}

__device__ __forceinline__ void Audit::body(const Args& A, Blk)
{
    const DevProblem& P = A.P;
    const double* __restrict__ part = A.part;
    const int nblk = A.nblk;
    gd_interval* iv = A.iv;
    WsHeader* h = A.h;
    __shared__ double sh[kAuditGroups][kNBin], sl[kAuditGroups][kNBin];
    __shared__ int32_t s_grp[kNBin];
    const int t = threadIdx.x, b = t % kNBin, gq = t / kNBin;
    {
        dd x{0.0, 0.0};
#pragma unroll 4
        for (int blk = gq; blk < nblk; blk += kAuditGroups) {
            const double* a = part + (int64_t(blk) * kNBin + b) * 8;
            x = dd_add(x, dd{a[1], a[2]});
        }
        sh[gq][b] = x.hi;
        sl[gq][b] = x.lo;
    }
    if (t < kNBin) s_grp[t] = h->group_of[t];
    __syncthreads();
    if (t < kNBin) {  // the groups combined in a fixed order
        dd x{sh[0][t], sl[0][t]};
        for (int g = 1; g < kAuditGroups; ++g) x = dd_add(x, dd{sh[g][t], sl[g][t]});
        sh[0][t] = x.hi;
        sl[0][t] = x.lo;
    }
    __syncthreads();
    if (t != 0) return;
    // groups are ascending runs of bins: one pass, each group's bins added in order
    double worst = 0.0;
    int g = -1;
    dd s{0.0, 0.0};
    auto close = [&]() {
        if (g >= 0 && h->gM[g] > 0.0) {
            const double r = s.hi / h->gM[g];
            if (r > worst) worst = r;
        }
    };
    for (int bb = 0; bb < kNBin; ++bb) {
        const int gb = s_grp[bb];
        if (gb < 0) continue;
        if (gb != g) {
            close();
            g = gb;
            s = dd{0.0, 0.0};
        }
        s = dd_add(s, dd{sh[0][bb], sl[0][bb]});
    }
    close();
    const double Cf = iv->C;
    const double thr = 2.0 * P.eps * Cf;
    iv->C = (worst > thr) ? fmax(0.25, 0.5 * Cf) : fmin(1.0, 1.25 * Cf);
    iv->audit_worst = worst;
    int64_t tk = iv->ticks + iv->exe_ticks;
    if (tk >= kTicks) tk = 0;
    iv->ticks = tk;
    iv->time = iv->time + iv->dt_exe;
    iv->n_intervals = iv->n_intervals + 1;
    iv->n_events = int64_t(*reinterpret_cast<const unsigned long long*>(&h->scratch[0]));
}

__global__ void k_interval_init(gd_interval* iv, double dt_coll)
{
    if (threadIdx.x != 0) return;
    iv->dt_coll = dt_coll;
    iv->dt_req = 0.0;
    iv->dt_exe = 0.0;
    iv->C = 1.0;
    iv->time = 0.0;
    iv->ticks = 0;
    iv->exe_ticks = 0;
    iv->n_intervals = 0;
    iv->n_events = 0;
    iv->audit_worst = 0.0;
    iv->n_groups = 0;
    iv->pad = 0;
}

void launch_interval_init(gd_interval* iv, double dt_coll, hipStream_t st)
{
    hipLaunchKernelGGL(k_interval_init, dim3(1), dim3(64), 0, st, iv, dt_coll);
}

static McArgs mc_args(const gd_problem* p, const gd_particles* s, const gd_neighbors* nb, gd_interval* iv,
                      const double* lam_i, uint64_t seed, uint32_t interval, bool interval_on_device,
                      int32_t* n_events, int32_t* log, int32_t log_cap, void* ws, const Layout& L)
{
    WsHeader* h = at<WsHeader>(ws, L.hdr);
    McArgs A{};
    A.P = to_dev(p);
    A.id = s->id;
    A.nbr = nb->nbr;
    A.cnt = nb->cnt;
    A.dmax = nb->dmax;
    A.m = s->m[s->cur];
    A.x = s->x;
    A.y = s->y;
    A.z = s->z;
    A.snap = at<double4>(ws, L.snap);
    A.lam_i = lam_i;
    A.iv = iv;
    A.m_out = s->m[s->cur ^ 1];
    A.n_events = n_events;
    A.log = log_cap > 0 ? log : nullptr;
    A.log_cap = log_cap;
    A.seed = seed;
    A.interval = interval;
    A.interval_on_device = interval_on_device ? 1 : 0;
    A.ws = ws;
    A.ev_counter = reinterpret_cast<unsigned long long*>(&h->scratch[0]);
    A.budget = kLaneEvents;
    A.heavy = at<Deferred>(ws, L.heavy);
    A.heavy_n = &h->heavy_n;
    A.heavy_next = &h->heavy_next;
    A.heavy_n0 = &h->heavy_n0;
    A.heavy_next0 = &h->heavy_next0;
    A.n_all = p->n;
    A.list = at<int32_t>(ws, L.mclist);
    A.list_seg = h->mc_seg;
    A.list_next = &h->mc_next;
    return A;
}

// the screen; false when it hands every particle with an event straight to
// the wavefront-per-particle pass (no event pass follows)
static bool launch_screen(const McArgs& A, const gd_problem* p, hipStream_t st)
{
    const int g = int((A.P.n + 255) / 256);
    static_assert(offsetof(WsHeader, mc_next) == offsetof(WsHeader, mc_seg) + kXcd * sizeof(int32_t),
                  "the segment counts and the next counter are cleared together");
    launch_fill_i32(A.list_seg, kXcd + 1, 0, st);
    if (p->k > 64) {  // no prefix registers: straight to the wavefront-per-particle pass
        hipLaunchKernelGGL(k_mc_screen<true>, dim3(g), dim3(256), 0, st, A);
        return false;
    }
    hipLaunchKernelGGL(k_mc_screen<false>, dim3(g), dim3(256), 0, st, A);
    return true;
}

static void launch_events(const McArgs& A, const gd_problem* p, hipStream_t st)
{
    const int g = int((A.P.n + 255) / 256);
    const dim3 eg(kEventBlocks), eb(256);
    if (A.early_events > 0.0) {  // with the early chains beside it
        const dim3 fg(kEarlyBlocks + kEventBlocks);
        const EventArgs E{A, int64_t(g)};
        if (p->rates_fp32) {
            if (p->k <= 32) hipLaunchKernelGGL((k_mc_fused<32, true>), fg, eb, 0, st, E);
            else hipLaunchKernelGGL((k_mc_fused<64, true>), fg, eb, 0, st, E);
        } else {
            if (p->k <= 32) hipLaunchKernelGGL((k_mc_fused<32, false>), fg, eb, 0, st, E);
            else hipLaunchKernelGGL((k_mc_fused<64, false>), fg, eb, 0, st, E);
        }
        return;
    }
    const EventArgs E{A, int64_t(g)};
    if (p->rates_fp32) {
        if (p->k <= 32) hipLaunchKernelGGL((k_mc<32, true>), eg, eb, 0, st, E);
        else hipLaunchKernelGGL((k_mc<64, true>), eg, eb, 0, st, E);
    } else {
        if (p->k <= 32) hipLaunchKernelGGL((k_mc<32, false>), eg, eb, 0, st, E);
        else hipLaunchKernelGGL((k_mc<64, false>), eg, eb, 0, st, E);
    }
}

static void launch_first(const McArgs& A, const gd_problem* p, hipStream_t st)
{
    if (launch_screen(A, p, st)) launch_events(A, p, st);
}

template <bool F32>
static void launch_heavy(const McArgs& A, int k, hipStream_t st)
{
    const dim3 g(kHeavyBlocks), b(256);
    if (k <= 32) hipLaunchKernelGGL((k_mc_heavy<32, F32>), g, b, 0, st, A);
    else if (k <= 64) hipLaunchKernelGGL((k_mc_heavy<64, F32>), g, b, 0, st, A);
    else if (k <= 128) hipLaunchKernelGGL((k_mc_heavy<128, F32>), g, b, 0, st, A);
    else hipLaunchKernelGGL((k_mc_heavy<256, F32>), g, b, 0, st, A);
}

static void launch_deferred(const McArgs& A, const gd_problem* p, hipStream_t st)
{
    if (p->rates_fp32) launch_heavy<true>(A, p->k, st);
    else launch_heavy<false>(A, p->k, st);
}

int launch_audit(const gd_problem* p, const gd_particles* s, gd_interval* iv, void* ws, const Layout& L, hipStream_t st)
{
    WsHeader* h = at<WsHeader>(ws, L.hdr);
    double* part = at<double>(ws, L.part);
    prof_mark(GD_PROF_AUDIT, 0, st);
    launch_bin_reduce(1, s->m[s->cur], s->M, s->m[s->cur ^ 1], nullptr, p->n, part, ws, st);
    const double* folded = launch_part_fold(part, ws, L, st);
    hipLaunchKernelGGL(k_audit, dim3(1), dim3(kAuditGroups * kNBin), 0, st, AuditArgs{to_dev(p), folded, 1, iv, h});
    prof_mark(GD_PROF_AUDIT, 1, st);
    return 0;
}

int launch_sample(const gd_problem* p, const gd_particles* s, const gd_neighbors* nb, gd_interval* iv,
                  const double* lam_i, uint64_t seed, uint32_t interval, bool interval_on_device, int32_t* n_events, int32_t* log,
                  int32_t log_cap, void* ws, const Layout& L, hipStream_t st, void* table, int32_t slot)
{
    McArgs A = mc_args(p, s, nb, iv, lam_i, seed, interval, interval_on_device, n_events, log, log_cap, ws, L);
    // (with a table the deferred particles wait for the launch over every
    // slot, so no chain starts early)
    if (!table) A.early_events = kEarlyEvents;
    prof_mark(GD_PROF_MC, 0, st);
    if (p->n > 0) launch_first(A, p, st);
    if (table) {
        // deferred particles are left to the launch over the whole table
        McArgs* dst = reinterpret_cast<McArgs*>(static_cast<char*>(table) + kTableHeader) + slot;
        hipLaunchKernelGGL(k_table_put, dim3(1), dim3(64), 0, st, dst, A);
        prof_mark(GD_PROF_MC, 1, st);
        return 0;
    }
    launch_deferred(A, p, st);
    prof_mark(GD_PROF_MC, 1, st);
    return launch_audit(p, s, iv, ws, L, st);
}

// Sampling and audit of the slots [lo, hi) only (one spatial group); the
// group's interval state supplies dt_exe and takes the audit.
int launch_sample_group(const gd_problem* p, const gd_particles* s, const gd_neighbors* nb, gd_interval* iv,
                        const double* lam_i, uint64_t seed, uint32_t interval, int64_t lo, int64_t hi,
                        int32_t* n_events, void* ws, const Layout& L, hipStream_t st)
{
    McArgs A = mc_args(p, s, nb, iv, lam_i, seed, interval, false, n_events, nullptr, 0, ws, L);
    const int64_t cnt = hi - lo;
    A.P.n = cnt;
    A.id = s->id + lo;
    A.nbr = nb->nbr + lo * int64_t(p->k);
    A.cnt = nb->cnt + lo;
    A.dmax = nb->dmax + lo;
    A.m = s->m[s->cur] + lo;
    A.x = s->x + lo;
    A.y = s->y + lo;
    A.z = s->z + lo;
    A.lam_i = lam_i + lo;
    A.m_out = s->m[s->cur ^ 1] + lo;
    A.n_events = n_events ? n_events + lo : nullptr;
    prof_mark(GD_PROF_MC, 0, st);
    if (cnt > 0) launch_first(A, p, st);
    launch_deferred(A, p, st);
    prof_mark(GD_PROF_MC, 1, st);
    WsHeader* h = at<WsHeader>(ws, L.hdr);
    double* part = at<double>(ws, L.part);
    DevProblem P = to_dev(p);
    P.n = cnt;
    prof_mark(GD_PROF_AUDIT, 0, st);
    launch_bin_reduce(1, s->m[s->cur] + lo, s->M + lo, s->m[s->cur ^ 1] + lo, nullptr, cnt, part, ws, st);
    const double* folded = launch_part_fold(part, ws, L, st);
    hipLaunchKernelGGL(k_audit, dim3(1), dim3(kAuditGroups * kNBin), 0, st, AuditArgs{P, folded, 1, iv, h});
    prof_mark(GD_PROF_AUDIT, 1, st);
    return 0;
}

size_t sample_table_bytes(int32_t nslot)
{
    return kTableHeader + sizeof(McArgs) * size_t(nslot);
}

int max_table_slots() { return kMaxTableSlots; }

int launch_sample_table(void* table, int32_t nslot, int32_t k, int32_t rates_fp32, hipStream_t st, int32_t nblocks)
{
    launch_fill_i32(static_cast<int32_t*>(table), 1, 0, st);
    char* tb = static_cast<char*>(table);
    const dim3 g(nblocks > 0 ? nblocks : kHeavyBlocks), b(256);
    if (rates_fp32) {
        if (k <= 32) hipLaunchKernelGGL((k_mc_heavy_batch<32, true>), g, b, 0, st, tb, nslot);
        else if (k <= 64) hipLaunchKernelGGL((k_mc_heavy_batch<64, true>), g, b, 0, st, tb, nslot);
        else if (k <= 128) hipLaunchKernelGGL((k_mc_heavy_batch<128, true>), g, b, 0, st, tb, nslot);
        else hipLaunchKernelGGL((k_mc_heavy_batch<256, true>), g, b, 0, st, tb, nslot);
    } else {
        if (k <= 32) hipLaunchKernelGGL((k_mc_heavy_batch<32, false>), g, b, 0, st, tb, nslot);
        else if (k <= 64) hipLaunchKernelGGL((k_mc_heavy_batch<64, false>), g, b, 0, st, tb, nslot);
        else if (k <= 128) hipLaunchKernelGGL((k_mc_heavy_batch<128, false>), g, b, 0, st, tb, nslot);
        else hipLaunchKernelGGL((k_mc_heavy_batch<256, false>), g, b, 0, st, tb, nslot);
    }
    return 0;
}

// Sampling and audit of every run as stages of one interval: clear the list
// counters, the screen, the per-lane event pass (k <= 64), the pass over the
// deferred particles of every run (one launch through a table of the runs'
// arguments, shaped for the largest k), then the audit's bin sums, fold and
// rule.  Draws take the interval index from each run's interval state.
static void many_table_step(char* base, const ManyStep& s, hipStream_t st)
{
    launch_sample_table(base + s.tab, int32_t(s.a0), int32_t(s.a1 >> 1), int32_t(s.a1 & 1), st, int32_t(s.nblocks));
}

void many_sample(ManyBuilder& B, const std::vector<ManyRun>& R)
{
    const size_t nr = R.size();
    std::vector<McArgs> ma(nr);
    std::vector<ClearArgs> clr(nr);
    std::vector<int64_t> one(nr, 1), nb(nr), scr_d(nr), scr_l(nr);
    int kmax = 1, f32 = 0;
    for (size_t r = 0; r < nr; ++r) {
        const ManyRun& x = R[r];
        ma[r] = mc_args(&x.p, &x.out, &x.nb, x.iv, x.lam_i, x.seed, 0u, true, x.n_events, nullptr, 0, x.ws, x.L);
        if (x.snap) ma[r].snap = x.snap;
        if (x.n_all >= 0) ma[r].n_all = x.n_all;
        ma[r].interval_at = x.interval_at;
        ma[r].active = B.active ? B.active + r : nullptr;
        clr[r] = ClearArgs{ma[r].list_seg, kXcd + 1, nullptr, 0};
        nb[r] = cdiv(x.p.n, 256);
        scr_d[r] = x.p.k > 64 ? nb[r] : 0;
        scr_l[r] = x.p.k > 64 ? 0 : nb[r];
        kmax = std::max(kmax, int(x.p.k));
        f32 = x.p.rates_fp32 ? 1 : 0;
    }
    B.add<ClearCounters>(clr, one);
    B.add<McScreen<true>>(ma, scr_d);
    B.add<McScreen<false>>(ma, scr_l);
    for (int cls = 0; cls < 2; ++cls) {
        std::vector<EventArgs> ev(nr);
        std::vector<int64_t> eb(nr, 0);
        bool any = false;
        for (size_t r = 0; r < nr; ++r) {
            const int k = R[r].p.k;
            ev[r] = EventArgs{ma[r], nb[r]};
            if (k <= 64 && (k <= 32) == (cls == 0)) {
                eb[r] = std::min<int64_t>(kEventBlocks, std::max<int64_t>(1, cdiv(R[r].p.n, B.tune.event_div)));
                any = true;
            }
        }
        if (!any) continue;
        if (cls == 0) {
            if (f32) B.add<McEvents<32, true>>(ev, eb);
            else B.add<McEvents<32, false>>(ev, eb);
        } else {
            if (f32) B.add<McEvents<64, true>>(ev, eb);
            else B.add<McEvents<64, false>>(ev, eb);
        }
    }
    // the deferred particles of every run: a table (256-byte header, then
    // the runs' arguments) in the arena
    std::vector<char> table(kTableHeader + sizeof(McArgs) * nr, 0);
    memcpy(table.data() + kTableHeader, ma.data(), sizeof(McArgs) * nr);
    const size_t tab = B.put_vec(table);
    ManyStep st{&many_table_step, tab, 0, 0, B.tune.heavy_blocks, int64_t(nr), int64_t(kmax) * 2 + f32};
    B.steps.push_back(st);
    many_audit_sums(B, R);
    std::vector<AuditArgs> au(nr);
    for (size_t r = 0; r < nr; ++r) {
        const ManyRun& x = R[r];
        au[r] = AuditArgs{to_dev(&x.p), at<double>(x.ws, x.L.red), 1, x.iv, at<WsHeader>(x.ws, x.L.hdr)};
    }
    B.add<Audit>(au, one);
}

}  // namespace gd
