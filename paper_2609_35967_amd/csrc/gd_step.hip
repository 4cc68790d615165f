// gd_step.hip -- the shared transport step of Sect. 2.6:
// dt = min(dt_max, dt_out, min_i dt_i) over the active particles, where dt_i
// is the most restrictive of the particle's local constraints: the orbital
// time c_orb / Omega_K, the drift time c_adv d_i / u_i over its neighbourhood
// radius d_i (u_i: speed relative to the local circular orbit, or |v_z| in
// the local column), and the diffusion time c_diff d_i^2 / D_i (D_i: the
// largest coefficient of the directions the diffusion step moves).  The
// paper names these constraints without their forms; this is the reading the
// library takes.  A streaming min-reduction: 64-88 bytes read per particle.
#include "gd_common.hpp"
#include "gd_internal.hpp"
#include "gd_physics.hpp"

#include <algorithm>

namespace gd {

struct StepArgs {
    DevProblem P;
    int32_t push, diffusion, vint, axisym;
    const double *x, *y, *r, *th, *vr, *lth, *lph, *vz, *m, *M, *d;
    double c_orb, c_adv, c_diff, St_diff;
    double Sc[3];
    double* red;
};

__device__ inline double local_dt(const StepArgs& A, int64_t i)
{
    const DevProblem& P = A.P;
    const double di = A.d[i];
    double t = INFINITY;
    if (A.push == GD_PUSH_GLOBAL) {
        const double R = sqrt(A.x[i] * A.x[i] + A.y[i] * A.y[i]);
        const double vK = sqrt(P.GM / R);
        t = fmin(t, A.c_orb / (vK / R));  // 1 / Omega_K = R / v_K
        const double vt = A.lth[i] / A.r[i];
        const double vp = A.lph[i] / R - vK;
        const double u = sqrt(A.vr[i] * A.vr[i] + vt * vt + vp * vp);
        if (di > 0.0 && u > 0.0) t = fmin(t, A.c_adv * di / u);
    } else if (A.push == GD_PUSH_LOCAL) {
        t = fmin(t, A.c_orb);
        const double u = fabs(A.vz[i]);
        if (di > 0.0 && u > 0.0) t = fmin(t, A.c_adv * di / u);
    }
    if (A.diffusion != 0 && di > 0.0) {
        double st, ct;
        sincos(A.th[i], &st, &ct);
        const double R = A.r[i] * st, Z = A.vint ? 0.0 : A.r[i] * ct;
        // nu = alpha h_g^2 R^2 Omega_K (no Z dependence); St at (R, Z), or the constant one
        const double lx = log(R / P.R0);
        const double hg2 = P.h_g0 * P.h_g0 * exp((P.q + 1.0) * lx);
        const double nu = P.alpha * hg2 * (R * R) * sqrt(P.GM / (R * R * R));
        double St = A.St_diff;
        if (!(St > 0.0)) {
            const double rr = sqrt(R * R + Z * Z);
            St = P.St0 / P.s0 * exp(-P.p * lx + (1.0 - R / rr) / hg2) * grain_size(P, A.m[i]);
        }
        double Sc = A.Sc[0];
        if (!A.vint) Sc = fmin(Sc, A.Sc[1]);
        if (!A.axisym) Sc = fmin(Sc, A.Sc[2]);
        const double D = nu / (Sc * (1.0 + St * St));
        if (D > 0.0) t = fmin(t, A.c_diff * (di * di) / D);
    }
    return t;
}

__global__ __launch_bounds__(256) void k_dt_partial(StepArgs A)
{
    __shared__ double s[4];
    double t = INFINITY;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < A.P.n; i += int64_t(gridDim.x) * blockDim.x)
        if (A.M[i] > 0.0) t = fmin(t, local_dt(A, i));
    t = wave_min_d(t);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) A.red[blockIdx.x] = fmin(fmin(s[0], s[1]), fmin(s[2], s[3]));
}

// min of the partials and the caps; the interval state (when given) takes
// dt_coll = dt / 2 for the coming step, at a collision-step boundary only
__global__ __launch_bounds__(64) void k_dt_final(const double* red, int nblk, double cap, double* out,
                                                 gd_interval* iv, void* ws)
{
    double t = INFINITY;
    for (int b = threadIdx.x; b < nblk; b += 64) t = fmin(t, red[b]);
    t = fmin(wave_min_d(t), cap);
    if (threadIdx.x != 0) return;
    *out = t;
    if (iv) {
        if (iv->ticks == 0) iv->dt_coll = 0.5 * t;
        else set_status(ws, GD_DEV_INTERNAL);
    }
}

int launch_transport_dt(const gd_problem* p, const gd_particles* s, const gd_neighbors* nb, const gd_step_limits* lim,
                        gd_interval* iv, double* dt, void* ws, const Layout& L, hipStream_t st)
{
    StepArgs A{};
    A.P = to_dev(p);
    A.push = p->push;
    A.diffusion = p->diffusion;
    A.vint = p->vint;
    A.axisym = p->axisym;
    A.x = s->x;
    A.y = s->y;
    A.r = s->r;
    A.th = s->th;
    A.vr = s->vr;
    A.lth = s->lth;
    A.lph = s->lph;
    A.vz = s->vz;
    A.m = s->m[s->cur];
    A.M = s->M;
    A.d = nb->dmax;
    A.c_orb = lim->c_orb;
    A.c_adv = lim->c_adv;
    A.c_diff = lim->c_diff;
    A.St_diff = p->St_diff;
    for (int a = 0; a < 3; ++a) A.Sc[a] = p->Sc[a];
    A.red = at<double>(ws, L.red);
    const int nblk = int(std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, (p->n + 255) / 256)));
    hipLaunchKernelGGL(k_dt_partial, dim3(nblk), dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(64), 0, st, A.red, nblk, fmin(lim->dt_max, lim->dt_out), dt, iv,
                       ws);
    return 0;
}

}  // namespace gd
