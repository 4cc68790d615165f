// gd_internal.hpp -- launch functions of the library's kernels (host side).
#pragma once

#include <cstring>
#include <vector>

#include "gd_common.hpp"

namespace gd {

struct PermuteArgs {
    int64_t n;
    const uint32_t* perm;
    int32_t nd;
    const double* src[16];
    double* dst[16];
    const uint32_t* id_src;
    uint32_t* id_dst;
    double4* pos4;
    const double* hint_src;  // previous neighbour distance per input slot, or null
    double* hint_dst;        // into Morton order (0 when absent)
};

DevProblem to_dev(const gd_problem* p);
void prof_mark(int which, int after, hipStream_t st);

int launch_morton_sort(const gd_problem* p, const gd_particles* in, gd_particles* out, const double* hint, void* ws,
                       const Layout& L,
                       hipStream_t st);
void launch_fill_i32(int32_t* a, int64_t n, int32_t v, hipStream_t st);
int launch_knn(const gd_problem* p, const gd_neighbors* nb, void* ws, const Layout& L, hipStream_t st);
int launch_rates(const gd_problem* p, const gd_particles* s, const gd_neighbors* nb, gd_interval* iv, double* lam_i,
                 double* lam_pair, double* ab, void* ws, const Layout& L, hipStream_t st);
int launch_sample(const gd_problem* p, const gd_particles* s, const gd_neighbors* nb, gd_interval* iv,
                  const double* lam_i, uint64_t seed, uint32_t interval, bool interval_on_device, int32_t* n_events, int32_t* log,
                  int32_t log_cap, void* ws, const Layout& L, hipStream_t st, void* table, int32_t slot);
int launch_reshuffle(const gd_problem* p, const gd_neighbors* nb, uint64_t seed, uint32_t refresh, void* ws,
                     const Layout& L, hipStream_t st);
hipError_t reshuffle_static_table(int32_t** table);
int launch_reshuffle_static(const gd_problem* p, const gd_neighbors* nb, uint64_t seed, uint32_t refresh,
                            int32_t* table, hipStream_t st);
int launch_audit(const gd_problem* p, const gd_particles* s, gd_interval* iv, void* ws, const Layout& L, hipStream_t st);
size_t sample_table_bytes(int32_t nslot);
int max_table_slots();
int launch_sample_table(void* table, int32_t nslot, int32_t k, int32_t rates_fp32, hipStream_t st,
                        int32_t nblocks = 0);
int launch_push(const gd_problem* p, const gd_particles* s, const gd_interval* iv, double dt, void* ws,
                const Layout& L, hipStream_t st);
void launch_interval_init(gd_interval* iv, double dt_coll, hipStream_t st);
int launch_transport_dt(const gd_problem* p, const gd_particles* s, const gd_neighbors* nb, const gd_step_limits* lim,
                        gd_interval* iv, double* dt, void* ws, const Layout& L, hipStream_t st);
int launch_rates_group(const gd_problem* p, const gd_particles* s, const gd_neighbors* nb, gd_interval* iv,
                       double* lam_i, int64_t lo, int64_t hi, int32_t group, int32_t n_groups, const uint64_t* rows,
                       int64_t* sched, bool snapshot, void* ws, const Layout& L, hipStream_t st);
int launch_sample_group(const gd_problem* p, const gd_particles* s, const gd_neighbors* nb, gd_interval* iv,
                        const double* lam_i, uint64_t seed, uint32_t interval, int64_t lo, int64_t hi,
                        int32_t* n_events, void* ws, const Layout& L, hipStream_t st);
int max_groups();
int launch_group_interactions(const gd_problem* p, const gd_neighbors* nb, const int32_t* group_lo, int32_t G,
                              uint64_t* mask, hipStream_t st);
int launch_publish_group(const gd_particles* s, int64_t lo, int64_t hi, int64_t* sched, int32_t group,
                         hipStream_t st);
int launch_diffuse(const gd_problem* p, const gd_particles* s, double dt, uint64_t seed, uint32_t step,
                   hipStream_t st);
const double* launch_part_fold(const double* part, void* ws, const Layout& L, hipStream_t st);
void launch_bin_reduce(int mode, const double* msnap, const double* M, const double* va, const double* vb, int64_t n,
                       double* part, void* ws, hipStream_t st);

// ---------------------------------------------------------------------------
// Many runs stepped as one (gd_many_*): each stage of an interval is one
// launch over every run.  The recorders of each source append their stages'
// launches, for one parity of the state buffers, to a builder that collects
// the argument tables and block maps in one host arena, uploaded once.
struct ManyRun {
    gd_problem p;
    gd_particles in, out;  // the interval permutes `in` into `out`, then works on `out`
    gd_neighbors nb;
    gd_interval* iv;
    double* lam_i;
    int32_t* n_events;
    void* ws;
    Layout L;
    uint64_t seed;
    // a spatial group as a run: its arrays (out, nb, lam_i, n_events) start at
    // slot `lo` of one particle set of n_all slots, whose snapshot is `snap`
    // (null: the run's own, in its workspace); the sampling's interval index
    // is read from *interval_at when set
    int64_t lo = 0;
    int64_t n_all = -1;
    double4* snap = nullptr;
    const int64_t* interval_at = nullptr;
};

struct ManyStep;
using ManyFn = void (*)(char* base, const ManyStep& s, hipStream_t st);
struct ManyStep {
    ManyFn fn;
    size_t tab, run, b0;  // arena offsets of the argument table and the block map
    int64_t nblocks;
    int64_t a0, a1;       // step-specific values
    const int32_t* active = nullptr;  // per-run flags (device), or null
};

struct ManyBuilder {
    std::vector<char> arena;
    std::vector<ManyStep> steps;
    gd_many_tuning tune;

    size_t put(const void* p, size_t bytes)
    {
        const size_t at = (arena.size() + 255) & ~size_t(255);
        arena.resize(at + (bytes ? bytes : 1));
        if (bytes) memcpy(arena.data() + at, p, bytes);
        return at;
    }
    template <class A>
    size_t put_vec(const std::vector<A>& v)
    {
        return put(v.data(), v.size() * sizeof(A));
    }
    // block map of per-run block counts nb[r]
    int64_t map(const std::vector<int64_t>& nb, size_t& run_off, size_t& b0_off)
    {
        std::vector<int32_t> b0(nb.size() + 1, 0), run;
        for (size_t r = 0; r < nb.size(); ++r) {
            b0[r + 1] = b0[r] + int32_t(nb[r]);
            for (int64_t b = 0; b < nb[r]; ++b) run.push_back(int32_t(r));
        }
        run_off = put_vec(run);
        b0_off = put_vec(b0);
        return b0.back();
    }
    const int32_t* active = nullptr;  // flags the next added steps are predicated on
    template <class K>
    void add(const std::vector<typename K::Args>& tab, const std::vector<int64_t>& nb);
    void add_raw(ManyFn fn, size_t tab, int64_t a0, int64_t a1)
    {
        steps.push_back(ManyStep{fn, tab, 0, 0, 0, a0, a1, active});
    }
};

template <class K>
void many_launch(char* base, const ManyStep& s, hipStream_t st)
{
    if (s.nblocks <= 0) return;
    const RunMap M{reinterpret_cast<const int32_t*>(base + s.run), reinterpret_cast<const int32_t*>(base + s.b0),
                   s.active};
    hipLaunchKernelGGL(k_many<K>, dim3(unsigned(s.nblocks)), dim3(K::kThreads), 0, st,
                       reinterpret_cast<const typename K::Args*>(base + s.tab), M);
}

// (instantiated in the source that defines K's body)
template <class K>
void ManyBuilder::add(const std::vector<typename K::Args>& tab, const std::vector<int64_t>& nb)
{
    ManyStep s{&many_launch<K>, put_vec(tab), 0, 0, 0, 0, 0, active};
    s.nblocks = map(nb, s.run, s.b0);
    steps.push_back(s);
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

void many_sort(ManyBuilder& B, const std::vector<ManyRun>& R);
void many_knn(ManyBuilder& B, const std::vector<ManyRun>& R);
void many_rates(ManyBuilder& B, const std::vector<ManyRun>& R, bool own_snapshot = true);
void many_sample(ManyBuilder& B, const std::vector<ManyRun>& R);
void many_audit_sums(ManyBuilder& B, const std::vector<ManyRun>& R);
void many_snapshot(ManyBuilder& B, const gd_problem* p, const gd_particles* s, double4* snap);
void many_push(ManyBuilder& B, const std::vector<ManyRun>& R);

}  // namespace gd
