// gd_api.hip -- host side of the C ABI declared in include/gd.h: argument
// checks, workspace layout, launches on the caller's stream.  Allocates
// nothing; errors are returned as gd_status with a thread-local message.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "gd_common.hpp"
#include "gd_internal.hpp"

namespace gd {

static thread_local char g_err[512] = "";
static hipEvent_t g_prof[GD_PROF_COUNT][2] = {};

void prof_mark(int which, int after, hipStream_t st)
{
    hipEvent_t e = g_prof[which][after ? 1 : 0];
    if (e) (void)hipEventRecord(e, st);
}

static int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

DevProblem to_dev(const gd_problem* p)
{
    DevProblem d{};
    d.n = p->n;
    d.k = p->k;
    d.kernel = p->kernel;
    d.push = p->push;
    d.nbin_min = p->nbin_min > 0 ? p->nbin_min : (2 * p->k > 64 ? 2 * p->k : 64);
    d.erosion = p->erosion;
    d.grouping = p->grouping;
    for (int a = 0; a < 3; ++a) {
        d.periodic[a] = p->periodic[a];
        d.L[a] = p->L[a];
    }
    d.rmax = p->rmax;
    d.t0 = p->t0;
    d.m0 = p->m0;
    d.eps = p->eps;
    d.dt_fn_max = p->dt_fn_max;
    d.rho_s = p->rho_s;
    d.s_min = p->s_min;
    d.v_frag = p->v_frag;
    d.GM = p->GM;
    d.Sigma_g0 = p->Sigma_g0;
    d.R0 = p->R0;
    d.p = p->p;
    d.q = p->q;
    d.h_g0 = p->h_g0;
    d.alpha = p->alpha;
    d.mu_mH = p->mu_mH;
    d.sigma_H2 = p->sigma_H2;
    d.s0 = p->s0;
    d.St0 = p->St0;
    d.r_in = p->r_in;
    d.r_out = p->r_out;
    d.drag = p->drag;
    d.brownian = p->brownian;
    d.turbulence = p->turbulence;
    d.caps = p->caps;
    d.rates_fp32 = p->rates_fp32;
    return d;
}

static int check_problem(const gd_problem* p)
{
    if (!p) return fail(GD_E_INVALID_ARG, "problem is NULL");
    if (p->n < 0 || p->n >= (int64_t(1) << 31) - 1) return fail(GD_E_INVALID_ARG, "n = %lld out of range", (long long)p->n);
    if (p->k < 2 || p->k > kMaxK) return fail(GD_E_INVALID_ARG, "k = %d outside 2..%d", p->k, kMaxK);
    if (p->n * int64_t(p->k) >= (int64_t(1) << 31)) return fail(GD_E_UNSUPPORTED, "n * k must stay below 2^31");
    if (p->n > (int64_t(kBucket) << (3 * kMaxTreeLevels))) return fail(GD_E_UNSUPPORTED, "n must stay below 2^26");
    if (p->kernel < 0 || p->kernel > 3) return fail(GD_E_INVALID_ARG, "kernel = %d unknown", p->kernel);
    if (p->push < 0 || p->push > 2) return fail(GD_E_INVALID_ARG, "push = %d unknown", p->push);
    if (p->rates_fp32 != 0 && p->rates_fp32 != 1) return fail(GD_E_INVALID_ARG, "rates_fp32 must be 0 or 1");
    for (int a = 0; a < 3; ++a)
        if (p->periodic[a] && !(p->L[a] > 0.0)) return fail(GD_E_INVALID_ARG, "periodic axis %d needs L > 0", a);
    if (!(p->rmax > 0.0)) return fail(GD_E_INVALID_ARG, "rmax must be > 0 (INFINITY for none)");
    if (p->kernel != GD_KERNEL_PHYSICAL && (!(p->t0 > 0.0) || !(p->m0 > 0.0)))
        return fail(GD_E_INVALID_ARG, "dimensionless kernels need t0 > 0 and m0 > 0");
    if (p->kernel == GD_KERNEL_PHYSICAL &&
        (!(p->rho_s > 0.0) || !(p->GM > 0.0) || !(p->s0 > 0.0) || !(p->R0 > 0.0) || !(p->s_min > 0.0)))
        return fail(GD_E_INVALID_ARG, "physical kernel needs rho_s, GM, s0, R0, s_min > 0");
    return GD_OK;
}

static int check_ws(const gd_problem* p, void* ws, size_t ws_bytes, Layout& L)
{
    L = make_layout(p->n, p->k);
    if (!ws) return fail(GD_E_WORKSPACE, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(GD_E_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < L.total)
        return fail(GD_E_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
    return GD_OK;
}

static int check_state(const gd_problem* p, const gd_particles* s, bool need_other)
{
    if (!s) return fail(GD_E_INVALID_ARG, "particles is NULL");
    if (s->cur != 0 && s->cur != 1) return fail(GD_E_INVALID_ARG, "cur must be 0 or 1");
    if (!s->id || !s->x || !s->y || !s->z || !s->M || !s->m[s->cur])
        return fail(GD_E_INVALID_ARG, "id, x, y, z, M and m[cur] are required");
    if (need_other && !s->m[s->cur ^ 1]) return fail(GD_E_INVALID_ARG, "m[cur ^ 1] is required");
    if (p->push == GD_PUSH_GLOBAL && (!s->r || !s->th || !s->ph || !s->vr || !s->lth || !s->lph))
        return fail(GD_E_INVALID_ARG, "global push needs r, th, ph, vr, lth, lph");
    if (p->push == GD_PUSH_LOCAL && (!s->vz || !s->st_mid))
        return fail(GD_E_INVALID_ARG, "local push needs vz and st_mid");
    return GD_OK;
}

// `out` can receive the permutation of `in`: every array `in` provides, distinct
static int check_out(const gd_particles* in, const gd_particles* o)
{
    if (!o->id || !o->x || !o->y || !o->z || !o->M || !o->m[in->cur])
        return fail(GD_E_INVALID_ARG, "out needs id, x, y, z, M and m[cur]");
    const double* pairs[][2] = {{in->x, o->x}, {in->y, o->y}, {in->z, o->z}, {in->M, o->M},
                                {in->m[in->cur], o->m[in->cur]}, {in->r, o->r}, {in->th, o->th}, {in->ph, o->ph},
                                {in->vr, o->vr}, {in->lth, o->lth}, {in->lph, o->lph}, {in->vz, o->vz},
                                {in->st_mid, o->st_mid}};
    for (auto& pr : pairs) {
        if (pr[0] && !pr[1]) return fail(GD_E_INVALID_ARG, "out is missing an array that in provides");
        if (pr[0] && pr[0] == pr[1]) return fail(GD_E_INVALID_ARG, "in and out must not alias");
    }
    if (in->id == o->id) return fail(GD_E_INVALID_ARG, "in and out must not alias");
    return GD_OK;
}

static int check_nb(const gd_neighbors* nb)
{
    if (!nb || !nb->nbr || !nb->cnt || !nb->dmax) return fail(GD_E_INVALID_ARG, "neighbors nbr, cnt, dmax required");
    return GD_OK;
}

static int hip_ok(const char* what)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(GD_E_HIP, "%s: %s", what, hipGetErrorString(e));
    return GD_OK;
}

__global__ void k_copy_na(const WsHeader* h, int32_t* out)
{
    if (threadIdx.x == 0) *out = h->n_active;
}

__global__ void k_clear_status(WsHeader* h)
{
    if (threadIdx.x == 0) h->status = 0;
}

}  // namespace gd

using namespace gd;

extern "C" {

int32_t gd_workspace_size(const gd_problem* p, size_t* bytes)
{
    int rc = check_problem(p);
    if (rc) return rc;
    if (!bytes) return fail(GD_E_INVALID_ARG, "bytes is NULL");
    *bytes = make_layout(p->n, p->k).total;
    return GD_OK;
}

int32_t gd_workspace_init(const gd_problem* p, void* ws, size_t ws_bytes, void* stream)
{
    int rc = check_problem(p);
    if (rc) return rc;
    Layout L;
    rc = check_ws(p, ws, ws_bytes, L);
    if (rc) return rc;
    launch_fill_i32(at<int32_t>(ws, L.hdr), int64_t(sizeof(WsHeader) / 4), 0, static_cast<hipStream_t>(stream));
    return hip_ok("gd_workspace_init");
}

int32_t gd_interval_init(gd_interval* iv, double dt_coll, void* stream)
{
    if (!iv) return fail(GD_E_INVALID_ARG, "interval is NULL");
    if (!(dt_coll > 0.0)) return fail(GD_E_INVALID_ARG, "dt_coll must be > 0");
    launch_interval_init(iv, dt_coll, static_cast<hipStream_t>(stream));
    return hip_ok("gd_interval_init");
}

int32_t gd_build_neighbors(const gd_problem* p, const gd_particles* in, gd_particles* out, const gd_neighbors* nb,
                           void* ws, size_t ws_bytes, void* stream)
{
    int rc = check_problem(p);
    if (!rc) rc = check_state(p, in, false);
    if (!rc) rc = check_nb(nb);
    if (rc) return rc;
    if (!out) return fail(GD_E_INVALID_ARG, "out is NULL");
    gd_particles o = *out;
    o.cur = in->cur;
    rc = check_out(in, &o);
    if (rc) return rc;
    Layout L;
    rc = check_ws(p, ws, ws_bytes, L);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (p->n == 0) return GD_OK;
    launch_morton_sort(p, in, &o, nb->dmax, ws, L, st);
    out->cur = in->cur;
    launch_knn(p, nb, ws, L, st);
    if (nb->n_active) hipLaunchKernelGGL(k_copy_na, dim3(1), dim3(64), 0, st, at<WsHeader>(ws, L.hdr), nb->n_active);
    return hip_ok("gd_build_neighbors");
}

int32_t gd_collision_rates(const gd_problem* p, const gd_particles* s, const gd_neighbors* nb, gd_interval* iv,
                           double* lam_i, double* lam_pair, double* ab, void* ws, size_t ws_bytes, void* stream)
{
    int rc = check_problem(p);
    if (!rc) rc = check_state(p, s, false);
    if (!rc) rc = check_nb(nb);
    if (rc) return rc;
    if (!iv || !lam_i) return fail(GD_E_INVALID_ARG, "interval and lam_i are required");
    Layout L;
    rc = check_ws(p, ws, ws_bytes, L);
    if (rc) return rc;
    if (!(p->eps > 0.0) || !(p->dt_fn_max > 0.0)) return fail(GD_E_INVALID_ARG, "eps and dt_fn_max must be > 0");
    if (p->n == 0) return GD_OK;
    launch_rates(p, s, nb, iv, lam_i, lam_pair, ab, ws, L, static_cast<hipStream_t>(stream));
    return hip_ok("gd_collision_rates");
}

static int32_t sample_call(const gd_problem* p, const gd_particles* s, const gd_neighbors* nb, gd_interval* iv,
                           const double* lam_i, uint64_t seed, uint64_t interval_index, int32_t* n_events,
                           int32_t* log, int32_t log_cap, void* ws, size_t ws_bytes, void* stream, void* table,
                           size_t table_bytes, int32_t slot, const char* what)
{
    if (table && (slot < 0 || slot >= max_table_slots() || table_bytes < sample_table_bytes(slot + 1)))
        return fail(GD_E_INVALID_ARG, "%s: slot %d does not fit the table", what, slot);
    int rc = check_problem(p);
    if (!rc) rc = check_state(p, s, true);
    if (!rc) rc = check_nb(nb);
    if (rc) return rc;
    if (!iv || !lam_i) return fail(GD_E_INVALID_ARG, "interval and lam_i are required");
    const bool on_device = interval_index == GD_INTERVAL_ON_DEVICE;
    if (!on_device && (interval_index >> 32))
        return fail(GD_E_INVALID_ARG, "interval_index must be < 2^32 or GD_INTERVAL_ON_DEVICE");
    if (log_cap < 0 || (log_cap > 0 && !log)) return fail(GD_E_INVALID_ARG, "log_cap > 0 needs a log array");
    if (int64_t(log_cap) * p->n >= (int64_t(1) << 31)) return fail(GD_E_UNSUPPORTED, "n * log_cap must stay below 2^31");
    Layout L;
    rc = check_ws(p, ws, ws_bytes, L);
    if (rc) return rc;
    if (p->n == 0 && !table) return GD_OK;  // (a table slot is written even for no particles)
    launch_sample(p, s, nb, iv, lam_i, seed, on_device ? 0u : uint32_t(interval_index), on_device, n_events, log,
                  log_cap, ws, L, static_cast<hipStream_t>(stream), table, slot);
    return hip_ok(what);
}

int32_t gd_sample_collisions(const gd_problem* p, const gd_particles* s, const gd_neighbors* nb, gd_interval* iv,
                             const double* lam_i, uint64_t seed, uint64_t interval_index, int32_t* n_events,
                             int32_t* log, int32_t log_cap, void* ws, size_t ws_bytes, void* stream)
{
    return sample_call(p, s, nb, iv, lam_i, seed, interval_index, n_events, log, log_cap, ws, ws_bytes, stream,
                       nullptr, 0, 0, "gd_sample_collisions");
}

int32_t gd_reshuffle_neighbors(const gd_problem* p, const gd_neighbors* nb, uint64_t seed, uint32_t refresh,
                               void* ws, size_t ws_bytes, void* stream)
{
    int rc = check_problem(p);
    if (!rc) rc = check_nb(nb);
    if (rc) return rc;
    if (!nb->n_active) return fail(GD_E_INVALID_ARG, "neighbours: n_active is NULL");
    Layout L;
    rc = check_ws(p, ws, ws_bytes, L);
    if (rc) return rc;
    launch_reshuffle(p, nb, seed, refresh, ws, L, static_cast<hipStream_t>(stream));
    return hip_ok("gd_reshuffle_neighbors");
}

int32_t gd_reshuffle_neighbors_static(const gd_problem* p, const gd_neighbors* nb, uint64_t seed, uint32_t refresh,
                                      void* stream)
{
    int rc = check_problem(p);
    if (!rc) rc = check_nb(nb);
    if (rc) return rc;
    if (!nb->n_active) return fail(GD_E_INVALID_ARG, "neighbours: n_active is NULL");
    if (p->n > int64_t(GD_RESHUFFLE_STATIC_MAX))
        return fail(GD_E_INVALID_ARG, "gd_reshuffle_neighbors_static: n = %lld exceeds its fixed table of %d entries",
                    (long long)p->n, GD_RESHUFFLE_STATIC_MAX);
    int32_t* table = nullptr;
    const hipError_t e = reshuffle_static_table(&table);
    if (e != hipSuccess)
        return fail(GD_E_HIP, "gd_reshuffle_neighbors_static: device table address: %s", hipGetErrorString(e));
    launch_reshuffle_static(p, nb, seed, refresh, table, static_cast<hipStream_t>(stream));
    return hip_ok("gd_reshuffle_neighbors_static");
}

int32_t gd_sample_table_size(int32_t nslot, size_t* bytes)
{
    if (!bytes) return fail(GD_E_INVALID_ARG, "bytes is NULL");
    if (nslot < 1 || nslot > max_table_slots())
        return fail(GD_E_INVALID_ARG, "nslot must be in [1, %d]", max_table_slots());
    *bytes = sample_table_bytes(nslot);
    return GD_OK;
}

int32_t gd_sample_collisions_deferred(const gd_problem* p, const gd_particles* s, const gd_neighbors* nb,
                                      gd_interval* iv, const double* lam_i, uint64_t seed, uint64_t interval_index,
                                      int32_t* n_events, int32_t* log, int32_t log_cap, void* ws, size_t ws_bytes,
                                      void* table, size_t table_bytes, int32_t slot, void* stream)
{
    if (!table) return fail(GD_E_INVALID_ARG, "table is NULL");
    return sample_call(p, s, nb, iv, lam_i, seed, interval_index, n_events, log, log_cap, ws, ws_bytes, stream,
                       table, table_bytes, slot, "gd_sample_collisions_deferred");
}

int32_t gd_sample_table_run(void* table, size_t table_bytes, int32_t nslot, int32_t k, int32_t rates_fp32,
                            void* stream)
{
    if (!table) return fail(GD_E_INVALID_ARG, "table is NULL");
    if (nslot < 1 || nslot > max_table_slots() || table_bytes < sample_table_bytes(nslot))
        return fail(GD_E_INVALID_ARG, "nslot does not fit the table");
    if (k < 1 || k > kMaxK) return fail(GD_E_INVALID_ARG, "k must be in [1, %d]", kMaxK);
    if (rates_fp32 != 0 && rates_fp32 != 1) return fail(GD_E_INVALID_ARG, "rates_fp32 must be 0 or 1");
    launch_sample_table(table, nslot, k, rates_fp32, static_cast<hipStream_t>(stream));
    return hip_ok("gd_sample_table_run");
}

int32_t gd_sample_audit(const gd_problem* p, const gd_particles* s, gd_interval* iv, void* ws, size_t ws_bytes,
                        void* stream)
{
    int rc = check_problem(p);
    if (!rc) rc = check_state(p, s, true);
    if (rc) return rc;
    if (!iv) return fail(GD_E_INVALID_ARG, "interval is NULL");
    Layout L;
    rc = check_ws(p, ws, ws_bytes, L);
    if (rc) return rc;
    if (p->n == 0) return GD_OK;
    launch_audit(p, s, iv, ws, L, static_cast<hipStream_t>(stream));
    return hip_ok("gd_sample_audit");
}

int32_t gd_push(const gd_problem* p, const gd_particles* s, const gd_interval* iv, double dt, void* ws,
                size_t ws_bytes, void* stream)
{
    int rc = check_problem(p);
    if (!rc) rc = check_state(p, s, false);
    if (rc) return rc;
    if (!iv && !(dt >= 0.0)) return fail(GD_E_INVALID_ARG, "dt must be >= 0 when no interval is given");
    Layout L;
    rc = check_ws(p, ws, ws_bytes, L);
    if (rc) return rc;
    if (p->n == 0 || p->push == GD_PUSH_NONE) return GD_OK;
    launch_push(p, s, iv, dt, ws, L, static_cast<hipStream_t>(stream));
    return hip_ok("gd_push");
}

int32_t gd_diffuse(const gd_problem* p, const gd_particles* s, double dt, uint64_t seed, uint32_t step, void* stream)
{
    int rc = check_problem(p);
    if (rc) return rc;
    if (p->diffusion < 0 || p->diffusion > 2) return fail(GD_E_INVALID_ARG, "diffusion = %d unknown", p->diffusion);
    if (p->diffusion == GD_DIFFUSION_NONE) return GD_OK;
    if (!s) return fail(GD_E_INVALID_ARG, "particles is NULL");
    if (s->cur != 0 && s->cur != 1) return fail(GD_E_INVALID_ARG, "cur must be 0 or 1");
    if (!s->id || !s->x || !s->y || !s->z || !s->M || !s->r || !s->th || !s->ph || !s->vr || !s->lth || !s->lph)
        return fail(GD_E_INVALID_ARG, "diffusion needs id, x, y, z, M, r, th, ph, vr, lth, lph");
    if (!(p->St_diff >= 0.0)) return fail(GD_E_INVALID_ARG, "St_diff must be >= 0");
    if (p->St_diff == 0.0 && (!s->m[s->cur] || !(p->rho_s > 0.0) || !(p->s0 > 0.0)))
        return fail(GD_E_INVALID_ARG, "the local Stokes number needs m[cur], rho_s > 0 and s0 > 0");
    if (!(p->GM > 0.0) || !(p->R0 > 0.0) || !(p->h_g0 > 0.0) || !(p->alpha >= 0.0))
        return fail(GD_E_INVALID_ARG, "diffusion needs GM, R0, h_g0 > 0 and alpha >= 0");
    if (!(p->Sc[0] > 0.0) || (!p->vint && !(p->Sc[1] > 0.0)) || (!p->axisym && !(p->Sc[2] > 0.0)))
        return fail(GD_E_INVALID_ARG, "Schmidt number of a stepped direction must be > 0");
    if (!(dt >= 0.0) || !isfinite(dt)) return fail(GD_E_INVALID_ARG, "dt must be finite and >= 0");
    if (p->n == 0) return GD_OK;
    launch_diffuse(p, s, dt, seed, step, static_cast<hipStream_t>(stream));
    return hip_ok("gd_diffuse");
}

static int check_range(const gd_problem* p, int64_t lo, int64_t hi)
{
    if (lo < 0 || hi < lo || hi > p->n) return fail(GD_E_INVALID_ARG, "slot range [%lld, %lld) outside [0, %lld)",
                                                    (long long)lo, (long long)hi, (long long)p->n);
    return GD_OK;
}

int32_t gd_group_interactions(const gd_problem* p, const gd_neighbors* nb, const int32_t* group_lo, int32_t n_groups,
                              uint64_t* mask, void* stream)
{
    int rc = check_problem(p);
    if (!rc) rc = check_nb(nb);
    if (rc) return rc;
    if (n_groups < 1 || n_groups > max_groups())
        return fail(GD_E_INVALID_ARG, "n_groups = %d outside 1..%d", n_groups, max_groups());
    if (!group_lo || !mask) return fail(GD_E_INVALID_ARG, "group_lo and mask are required");
    if (group_lo[0] != 0) return fail(GD_E_INVALID_ARG, "group_lo[0] must be 0");
    for (int g = 0; g < n_groups; ++g)
        if (group_lo[g + 1] <= group_lo[g]) return fail(GD_E_INVALID_ARG, "groups must be non-empty and ascending");
    if (group_lo[n_groups] > p->n) return fail(GD_E_INVALID_ARG, "group_lo[n_groups] exceeds n");
    launch_group_interactions(p, nb, group_lo, n_groups, mask, static_cast<hipStream_t>(stream));
    return hip_ok("gd_group_interactions");
}

int32_t gd_collision_rates_group(const gd_problem* p, const gd_particles* s, const gd_neighbors* nb,
                                 gd_interval* iv, double* lam_i, int64_t lo, int64_t hi, int32_t group,
                                 int32_t n_groups, const uint64_t* rows, int64_t* sched, int32_t snapshot, void* ws,
                                 size_t ws_bytes, void* stream)
{
    int rc = check_problem(p);
    if (!rc) rc = check_state(p, s, false);
    if (!rc) rc = check_nb(nb);
    if (!rc) rc = check_range(p, lo, hi);
    if (rc) return rc;
    if (!iv || !lam_i) return fail(GD_E_INVALID_ARG, "interval and lam_i are required");
    if (n_groups < 1 || n_groups > max_groups() || group < 0 || group >= n_groups)
        return fail(GD_E_INVALID_ARG, "group %d of n_groups %d outside 0..%d", group, n_groups, max_groups() - 1);
    if (!rows || !sched) return fail(GD_E_INVALID_ARG, "rows and sched are required");
    Layout L;
    rc = check_ws(p, ws, ws_bytes, L);
    if (rc) return rc;
    if (p->n == 0) return GD_OK;
    launch_rates_group(p, s, nb, iv, lam_i, lo, hi, group, n_groups, rows, sched, snapshot != 0, ws, L,
                       static_cast<hipStream_t>(stream));
    return hip_ok("gd_collision_rates_group");
}

int32_t gd_sample_collisions_group(const gd_problem* p, const gd_particles* s, const gd_neighbors* nb,
                                   gd_interval* iv, const double* lam_i, uint64_t seed, uint64_t interval_index,
                                   int64_t lo, int64_t hi, int32_t* n_events, void* ws, size_t ws_bytes, void* stream)
{
    int rc = check_problem(p);
    if (!rc) rc = check_state(p, s, true);
    if (!rc) rc = check_nb(nb);
    if (!rc) rc = check_range(p, lo, hi);
    if (rc) return rc;
    if (!iv || !lam_i) return fail(GD_E_INVALID_ARG, "interval and lam_i are required");
    if (interval_index > 0xFFFFFFFFull) return fail(GD_E_INVALID_ARG, "interval_index must be below 2^32");
    Layout L;
    rc = check_ws(p, ws, ws_bytes, L);
    if (rc) return rc;
    if (p->n == 0) return GD_OK;
    launch_sample_group(p, s, nb, iv, lam_i, seed, uint32_t(interval_index), lo, hi, n_events, ws, L,
                        static_cast<hipStream_t>(stream));
    return hip_ok("gd_sample_collisions_group");
}

int32_t gd_publish_group(const gd_problem* p, const gd_particles* s, int64_t lo, int64_t hi, int64_t* sched,
                         int32_t group, void* stream)
{
    int rc = check_problem(p);
    if (!rc) rc = check_state(p, s, true);
    if (!rc) rc = check_range(p, lo, hi);
    if (rc) return rc;
    if (sched && (group < 0 || group >= max_groups())) return fail(GD_E_INVALID_ARG, "group %d out of range", group);
    launch_publish_group(s, lo, hi, sched, group, static_cast<hipStream_t>(stream));
    return hip_ok("gd_publish_group");
}

}  // extern "C"

struct gd_many {
    int device;
    int32_t nrun;
    int parity;
    char* dev;
    size_t bytes;
    std::vector<ManyStep> steps[2];
};

extern "C" {

int32_t gd_many_create(const gd_run* runs, int32_t nrun, const gd_many_tuning* tune, gd_many** out)
{
    if (!out) return fail(GD_E_INVALID_ARG, "gd_many_create: out is NULL");
    *out = nullptr;
    if (!runs || nrun < 1 || nrun > GD_MANY_MAX_RUNS)
        return fail(GD_E_INVALID_ARG, "gd_many_create: nrun = %d outside 1..%d", nrun, GD_MANY_MAX_RUNS);
    gd_many_tuning T{1, 256, 512, 2048, 768};
    if (tune) {
        if (tune->knn_tile < 0 || tune->knn_tile > 1 || tune->fallback_div < 0 || tune->event_div < 0 ||
            tune->red_div < 0 || tune->heavy_blocks < 0 || tune->heavy_blocks > 65536)
            return fail(GD_E_INVALID_ARG, "gd_many_create: tuning field out of range");
        T.knn_tile = tune->knn_tile;
        if (tune->fallback_div) T.fallback_div = tune->fallback_div;
        if (tune->event_div) T.event_div = tune->event_div;
        if (tune->red_div) T.red_div = tune->red_div;
        if (tune->heavy_blocks) T.heavy_blocks = tune->heavy_blocks;
    }
    std::vector<ManyRun> R[2];
    for (int32_t r = 0; r < nrun; ++r) {
        const gd_run& x = runs[r];
        int rc = check_problem(x.p);
        if (!rc && x.p->n < 1) rc = fail(GD_E_INVALID_ARG, "n must be >= 1");
        if (!rc) rc = check_state(x.p, x.a, true);
        if (!rc) rc = check_state(x.p, x.b, false);
        if (!rc) rc = check_nb(x.nb);
        if (!rc && (!x.iv || !x.lam_i)) rc = fail(GD_E_INVALID_ARG, "interval and lam_i are required");
        if (!rc && x.p->rates_fp32 != runs[0].p->rates_fp32) rc = fail(GD_E_INVALID_ARG, "runs differ in rates_fp32");
        Layout L;
        if (!rc) rc = check_ws(x.p, x.ws, x.ws_bytes, L);
        if (!rc) {  // each buffer can receive the other's permutation
            gd_particles a = *x.a, b = *x.b;
            b.cur = a.cur;
            rc = check_out(&a, &b);
            b.cur = a.cur ^ 1;
            a.cur = b.cur;
            if (!rc) rc = check_out(&b, &a);
        }
        if (rc) {
            char msg[sizeof(g_err)];
            snprintf(msg, sizeof(msg), "%s", g_err);
            return fail(rc, "gd_many_create: run %d: %s", r, msg);
        }
        for (int par = 0; par < 2; ++par) {
            ManyRun m{};
            m.p = *x.p;
            m.in = par ? *x.b : *x.a;
            m.out = par ? *x.a : *x.b;
            m.in.cur = x.a->cur ^ par;
            m.out.cur = m.in.cur;
            m.nb = *x.nb;
            m.iv = x.iv;
            m.lam_i = x.lam_i;
            m.n_events = x.n_events;
            m.ws = x.ws;
            m.L = L;
            m.seed = x.seed;
            R[par].push_back(m);
        }
    }
    ManyBuilder B;
    B.tune = T;
    std::vector<ManyStep> steps[2];
    for (int par = 0; par < 2; ++par) {
        B.steps.clear();
        many_sort(B, R[par]);
        many_knn(B, R[par]);
        many_rates(B, R[par]);
        many_sample(B, R[par]);
        many_push(B, R[par]);
        steps[par] = B.steps;
    }
    gd_many* m = new gd_many{};
    if (hipGetDevice(&m->device) != hipSuccess) {
        delete m;
        return fail(GD_E_HIP, "gd_many_create: no current device");
    }
    m->nrun = nrun;
    m->parity = 0;
    m->bytes = B.arena.size();
    if (hipMalloc(reinterpret_cast<void**>(&m->dev), m->bytes) != hipSuccess) {
        delete m;
        return fail(GD_E_HIP, "gd_many_create: hipMalloc of %zu bytes failed", B.arena.size());
    }
    if (hipMemcpy(m->dev, B.arena.data(), m->bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(m->dev);
        delete m;
        return fail(GD_E_HIP, "gd_many_create: upload of the tables failed");
    }
    m->steps[0] = steps[0];
    m->steps[1] = steps[1];
    *out = m;
    return GD_OK;
}

int32_t gd_many_interval(gd_many* m, void* stream)
{
    if (!m) return fail(GD_E_INVALID_ARG, "gd_many_interval: NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (const ManyStep& s : m->steps[m->parity]) s.fn(m->dev, s, st);
    m->parity ^= 1;
    return hip_ok("gd_many_interval");
}

int32_t gd_many_parity(const gd_many* m, int32_t* parity)
{
    if (!m || !parity) return fail(GD_E_INVALID_ARG, "gd_many_parity: NULL");
    *parity = m->parity;
    return GD_OK;
}

int32_t gd_many_destroy(gd_many* m)
{
    if (!m) return GD_OK;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(m->device);
    const hipError_t e = hipFree(m->dev);
    (void)hipSetDevice(cur);
    delete m;
    if (e != hipSuccess) return fail(GD_E_HIP, "gd_many_destroy: %s", hipGetErrorString(e));
    return GD_OK;
}

int32_t gd_transport_dt(const gd_problem* p, const gd_particles* s, const gd_neighbors* nb,
                        const gd_step_limits* lim, gd_interval* iv, double* dt, void* ws, size_t ws_bytes,
                        void* stream)
{
    int rc = check_problem(p);
    if (!rc) rc = check_state(p, s, false);
    if (!rc) rc = check_nb(nb);
    if (rc) return rc;
    if (!lim || !dt) return fail(GD_E_INVALID_ARG, "gd_transport_dt: limits and dt are required");
    if (!(lim->dt_max > 0.0) || !(lim->dt_out > 0.0) || !(lim->c_orb > 0.0) || !(lim->c_adv > 0.0) ||
        !(lim->c_diff > 0.0))
        return fail(GD_E_INVALID_ARG, "gd_transport_dt: limits must be positive");
    if (p->diffusion != 0 && (!s->r || !s->th)) return fail(GD_E_INVALID_ARG, "diffusion needs r and th");
    Layout L;
    rc = check_ws(p, ws, ws_bytes, L);
    if (rc) return rc;
    launch_transport_dt(p, s, nb, lim, iv, dt, ws, L, static_cast<hipStream_t>(stream));
    return hip_ok("gd_transport_dt");
}

int32_t gd_stream_create_cu_mask(const uint32_t* mask, int32_t mask_words, void** stream)
{
    if (!stream) return fail(GD_E_INVALID_ARG, "gd_stream_create_cu_mask: stream is NULL");
    *stream = nullptr;
    if (!mask || mask_words < 1) return fail(GD_E_INVALID_ARG, "gd_stream_create_cu_mask: empty mask");
    bool any = false;
    for (int32_t w = 0; w < mask_words; ++w) any = any || mask[w] != 0;
    if (!any) return fail(GD_E_INVALID_ARG, "gd_stream_create_cu_mask: no CU selected");
    hipStream_t st = nullptr;
    const hipError_t e = hipExtStreamCreateWithCUMask(&st, uint32_t(mask_words), mask);
    if (e != hipSuccess) return fail(GD_E_HIP, "gd_stream_create_cu_mask: %s", hipGetErrorString(e));
    *stream = st;
    return GD_OK;
}

int32_t gd_stream_destroy(void* stream)
{
    if (!stream) return GD_OK;
    const hipError_t e = hipStreamDestroy(static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(GD_E_HIP, "gd_stream_destroy: %s", hipGetErrorString(e));
    return GD_OK;
}

int32_t gd_status_read(void* ws, void* stream, int32_t* out)
{
    if (!ws || !out) return fail(GD_E_INVALID_ARG, "workspace and out are required");
    hipStream_t st = static_cast<hipStream_t>(stream);
    WsHeader* h = at<WsHeader>(ws, 0);
    int32_t v = 0;
    if (hipMemcpyAsync(&v, &h->status, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return hip_ok("gd_status_read");
    hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, st, h);
    *out = v;
    return hip_ok("gd_status_read");
}

int32_t gd_profile_events(int32_t which, void* before, void* after)
{
    if (which < 0 || which >= GD_PROF_COUNT) return fail(GD_E_INVALID_ARG, "which = %d unknown", which);
    g_prof[which][0] = static_cast<hipEvent_t>(before);
    g_prof[which][1] = static_cast<hipEvent_t>(after);
    return GD_OK;
}

const char* gd_last_error(void) { return g_err; }

const char* gd_version(void) { return "gd 0.1 (gfx950)"; }

}  // extern "C"
