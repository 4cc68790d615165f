// gd_internal.hpp -- launch functions of the library's kernels (host side).
#pragma once

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
int launch_sample_table(void* table, int32_t nslot, int32_t k, int32_t rates_fp32, hipStream_t st);
int launch_push(const gd_problem* p, const gd_particles* s, const gd_interval* iv, double dt, void* ws,
                const Layout& L, hipStream_t st);
void launch_interval_init(gd_interval* iv, double dt_coll, hipStream_t st);
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

}  // namespace gd
