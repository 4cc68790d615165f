// gd_push.hip -- staggered semi-analytic push between intervals (Sect. 2.3.3).
//
// Drift-kick-drift.  The kick integrates the drag relaxation exactly for the
// force held at the drifted position: for dy/dt = -(y - y_g)/t_s + f,
//     y' = y E + (y_g + f t_s) G,   E = exp(-dt/t_s),  G = -expm1(-dt/t_s),
// which is the leapfrog kick when t_s -> infinity and the terminal velocity
// y_g + f t_s when dt >> t_s.  (The paper cites the method and states these
// limits without printing its steps; this step form is the reading used.)
//
//  local column: z, v_z; gravity -z (Omega = H = 1), gas at rest,
//                t_s = St_mid exp(z^2/2) (St inversely proportional to rho_g).
//  global:       y = (v_r, l_theta, l_phi); f_r = -GM/r^2 + l_th^2/r^3 +
//                l_ph^2/(r^3 sin^2 th), f_th = l_ph^2 cos th/(r^2 sin^3 th),
//                y_g = (0, 0, v_g,phi R); the l-terms of f use a half-kick
//                predictor.  The drift at fixed y is exact:
//                r = r0 + v_r t, u = t/(r0 r), th = th0 + l_th u,
//                ph = ph0 + l_ph sin(l_th u)/(l_th sin th0 sin th).
// One lane per particle; pure streaming over the state (bandwidth-bound).
#include "gd_common.hpp"
#include "gd_internal.hpp"
#include "gd_physics.hpp"

namespace gd {

struct LocalPushArgs {
    int64_t n;
    double* z;
    double* vz;
    const double* st;
    const double* M;
    const gd_interval* iv;
    double dt_host;
};

struct PushLocal {
    using Args = LocalPushArgs;
    static constexpr int kThreads = 256;
    static __device__ __forceinline__ void body(const Args& A, Blk B);
};

__global__ __launch_bounds__(256) void k_push_local(LocalPushArgs A)
{
    PushLocal::body(A, Blk{int64_t(blockIdx.x), int64_t(gridDim.x)});
}

__device__ __forceinline__ void PushLocal::body(const Args& A, Blk B)
{
    double* __restrict__ z = A.z;
    double* __restrict__ vz = A.vz;
    const double* __restrict__ st = A.st;
    const int64_t i = B.id * int64_t(blockDim.x) + threadIdx.x;
    if (i >= A.n) return;
    if (!(A.M[i] > 0.0)) return;
    const double dt = A.iv ? A.iv->dt_exe : A.dt_host;
    const double h = 0.5 * dt;
    const double v0 = vz[i];
    const double zs = z[i] + v0 * h;
    const double ts = st[i] * exp(0.5 * (zs * zs));
    const double r = dt / ts;
    const double E = exp(-r);
    const double G = -expm1(-r);
    const double v = v0 * E + (-zs) * ts * G;
    vz[i] = v;
    z[i] = zs + v * h;
}

__device__ inline double sinc_(double a)
{
    if (fabs(a) < 1e-4) return 1.0 - a * a / 6.0;
    return sin(a) / a;
}

__device__ inline void drift(double& r, double& th, double& ph, double vr, double lth, double lph, double tau)
{
    const double r0 = r, th0 = th;
    const double r1 = r0 + vr * tau;
    const double u = tau / (r0 * r1);
    const double a = lth * u;
    const double th1 = th0 + a;
    ph = ph + lph * u * sinc_(a) / (sin(th0) * sin(th1));
    r = r1;
    th = th1;
}

__device__ inline void forces(double GM, double r, double th, double lth, double lph, double& fr, double& fth)
{
    const double st = sin(th), ct = cos(th);
    const double r2 = r * r, r3 = r2 * r;
    fr = -GM / r2 + lth * lth / r3 + lph * lph / (r3 * (st * st));
    fth = lph * lph * ct / (r2 * (st * st * st));
}

struct PushArgs {
    DevProblem P;
    double *r, *th, *ph, *vr, *lth, *lph, *x, *y, *z, *M;
    const double* m;
    const gd_interval* iv;
    double dt_host;
};

struct PushGlobal {
    using Args = PushArgs;
    static constexpr int kThreads = 256;
    static __device__ __forceinline__ void body(const Args& A, Blk B);
};

__global__ __launch_bounds__(256) void k_push_global(PushArgs A)
{
    PushGlobal::body(A, Blk{int64_t(blockIdx.x), int64_t(gridDim.x)});
}

__device__ __forceinline__ void PushGlobal::body(const Args& A, Blk B)
{
    const int64_t i = B.id * int64_t(blockDim.x) + threadIdx.x;
    if (i >= A.P.n) return;
    if (!(A.M[i] > 0.0)) return;
    const DevProblem& P = A.P;
    const double dt = A.iv ? A.iv->dt_exe : A.dt_host;
    const double h = 0.5 * dt;
    double ri = A.r[i], ti = A.th[i], pi_ = A.ph[i];
    const double y0 = A.vr[i], y1 = A.lth[i], y2 = A.lph[i];
    drift(ri, ti, pi_, y0, y1, y2, h);
    double fr0, ft0;
    forces(P.GM, ri, ti, y1, y2, fr0, ft0);
    double n0, n1, n2;
    if (P.drag) {
        const double R = ri * sin(ti), Z = ri * cos(ti);
        Gas g;
        gas_at(P, R, Z, g);
        const double s = grain_size(P, A.m[i]);
        const double ts = g.stfac * s / g.OmK;
        const double lg = g.vgphi * R;
        const double rh = h / ts, rf = dt / ts;
        const double Eh = exp(-rh), Gh = -expm1(-rh);
        const double E = exp(-rf), G = -expm1(-rf);
        const double p1 = y1 * Eh + (ft0 * ts) * Gh;
        const double p2 = y2 * Eh + lg * Gh;
        double fr1, ft1;
        forces(P.GM, ri, ti, p1, p2, fr1, ft1);
        n0 = y0 * E + (fr1 * ts) * G;
        n1 = y1 * E + (ft1 * ts) * G;
        n2 = y2 * E + lg * G;
    } else {
        const double p1 = y1 + ft0 * h;
        double fr1, ft1;
        forces(P.GM, ri, ti, p1, y2, fr1, ft1);
        n0 = y0 + fr1 * dt;
        n1 = y1 + ft1 * dt;
        n2 = y2;
    }
    drift(ri, ti, pi_, n0, n1, n2, h);
    A.r[i] = ri;
    A.th[i] = ti;
    A.ph[i] = pi_;
    A.vr[i] = n0;
    A.lth[i] = n1;
    A.lph[i] = n2;
    const double st = sin(ti);
    A.x[i] = ri * st * cos(pi_);
    A.y[i] = ri * st * sin(pi_);
    A.z[i] = ri * cos(ti);
    if (ri < P.r_in || ri > P.r_out) A.M[i] = 0.0;
}

static PushArgs push_args(const gd_problem* p, const gd_particles* s, const double* m, const gd_interval* iv, double dt)
{
    PushArgs A{};
    A.P = to_dev(p);
    A.r = s->r;
    A.th = s->th;
    A.ph = s->ph;
    A.vr = s->vr;
    A.lth = s->lth;
    A.lph = s->lph;
    A.x = s->x;
    A.y = s->y;
    A.z = s->z;
    A.M = s->M;
    A.m = m;
    A.iv = iv;
    A.dt_host = dt;
    return A;
}

int launch_push(const gd_problem* p, const gd_particles* s, const gd_interval* iv, double dt, void* ws,
                const Layout& L, hipStream_t st)
{
    (void)ws;
    (void)L;
    const int64_t n = p->n;
    const int g = int((n + 255) / 256);
    prof_mark(GD_PROF_PUSH, 0, st);
    if (p->push == GD_PUSH_LOCAL) {
        hipLaunchKernelGGL(k_push_local, dim3(g), dim3(256), 0, st,
                           LocalPushArgs{n, s->z, s->vz, s->st_mid, s->M, iv, dt});
    } else if (p->push == GD_PUSH_GLOBAL) {
        hipLaunchKernelGGL(k_push_global, dim3(g), dim3(256), 0, st, push_args(p, s, s->m[s->cur], iv, dt));
    }
    prof_mark(GD_PROF_PUSH, 1, st);
    return 0;
}

// The push of every run that has one, over its own dt_exe, after sampling:
// the new masses are in m[cur ^ 1] of the interval's state.
void many_push(ManyBuilder& B, const std::vector<ManyRun>& R)
{
    const size_t nr = R.size();
    std::vector<LocalPushArgs> lo(nr);
    std::vector<PushArgs> gl(nr);
    std::vector<int64_t> nl(nr, 0), ng(nr, 0);
    bool any_l = false, any_g = false;
    for (size_t r = 0; r < nr; ++r) {
        const ManyRun& x = R[r];
        const gd_particles* s = &x.out;
        const int64_t nb = cdiv(x.p.n, 256);
        lo[r] = LocalPushArgs{x.p.n, s->z, s->vz, s->st_mid, s->M, x.iv, 0.0};
        gl[r] = push_args(&x.p, s, s->m[s->cur ^ 1], x.iv, 0.0);
        if (x.p.push == GD_PUSH_LOCAL) {
            nl[r] = nb;
            any_l = true;
        } else if (x.p.push == GD_PUSH_GLOBAL) {
            ng[r] = nb;
            any_g = true;
        }
    }
    if (any_l) B.add<PushLocal>(lo, nl);
    if (any_g) B.add<PushGlobal>(gl, ng);
}

}  // namespace gd
