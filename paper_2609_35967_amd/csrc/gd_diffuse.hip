// gd_diffuse.hip -- dust diffusion operator D (Sect. 2.4).
//
// One Euler--Maruyama step per call, one lane per particle.  In the local
// cylindrical basis the tensor is diag(D_R, D_Z, D_phi), D_a = nu/(Sc_a (1+St^2)),
// nu = alpha c_s H_g.  The drift terms are written with logarithmic
// derivatives, D_a (1/R + dln D/dR + chi dln rho_g/dR) and so on, where for the
// gas disk of Sect. 2.2 (x = R/R0, h^2 = h_g0^2 x^(q+1), w = 1 - R/r):
//   dln nu/dR    = (q + 3/2)/R                       (nu ~ R^(q+3/2), no Z dependence)
//   dln St/dR    = -p/R + W_R,   dln St/dZ = W_Z      (St ~ x^-p exp(w/h^2))
//   dln rho_g/dR = (p - (q+3)/2)/R - W_R,  dln rho_g/dZ = -W_Z
//   W_R = d(w/h^2)/dR = -Z^2/(r^3 h^2) - w (q+1)/(R h^2),  W_Z = R Z/(r^3 h^2)
//   dln D/d. = dln nu/d. - 2 St^2/(1+St^2) dln St/d.
// A vertically integrated disk evaluates everything at Z = 0 with Sigma_g
// (dln Sigma_g/dR = p/R) in place of rho_g.  The velocity is carried over in
// Cartesian form: (v_R, v_phi) rotate by the azimuthal step (plus pi when the
// step passes the axis) and (v_R, v_Z) are projected on the new (r, theta).
//
// Pure streaming: 60 bytes read (68 with the local Stokes number) and 72
// written per particle.  The powers of R/R0 share one logarithm, and only the
// normals of the directions stepped are formed.
#include "gd_common.hpp"
#include "gd_internal.hpp"
#include "gd_physics.hpp"

namespace gd {

constexpr uint32_t kDiffTag = 0x44494646u;

struct DiffArgs {
    DevProblem P;
    const uint32_t* id;
    double *r, *th, *ph, *vr, *lth, *lph, *x, *y, *z, *M;
    const double* m;
    double dt, chi, St_diff;
    double Sc[3];
    uint64_t seed;
    uint32_t step;
    int32_t vint, axisym;
};

// A standard normal pair from generator call w: sqrt(-2 ln u1) (cos, sin)(2 pi u2).
__device__ inline void diff_pair(uint64_t seed, uint32_t id, uint32_t step, uint32_t w, double& zc, double& zs)
{
    const double two53 = 1.0 / 9007199254740992.0;
    uint32_t ctr[4] = {id, step, kDiffTag, w};
    philox4x32_10(ctr, uint32_t(seed), uint32_t(seed >> 32));
    const uint64_t a = ((uint64_t(ctr[1]) << 32) | ctr[0]) >> 11;
    const uint64_t b = ((uint64_t(ctr[3]) << 32) | ctr[2]) >> 11;
    const double u1 = double(a + 1) * two53;
    const double u2 = double(b) * two53;
    const double rad = sqrt(-2.0 * log(u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    zc = rad * c;
    zs = rad * s;
}

__global__ __launch_bounds__(256) void k_diffuse(DiffArgs A)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= A.P.n) return;
    if (!(A.M[i] > 0.0)) return;
    const DevProblem& P = A.P;
    const double r0 = A.r[i], t0 = A.th[i], p0 = A.ph[i];
    double st0, ct0;
    sincos(t0, &st0, &ct0);
    const double R = r0 * st0, Z = r0 * ct0;
    const double invR = 1.0 / R;

    // gas at (R, Z) (midplane when vertically integrated): powers of R/R0
    // through one logarithm
    const double lx = log(R / P.R0);
    const double hg = P.h_g0 * exp(0.5 * (P.q + 1.0) * lx);
    const double hg2 = hg * hg;
    const double OmK = sqrt(P.GM / (R * R * R));
    const double nu = P.alpha * hg2 * (R * R) * OmK;
    double WR = 0.0, WZ = 0.0, w = 0.0;
    if (!A.vint) {
        const double r = sqrt(R * R + Z * Z);
        w = 1.0 - R / r;
        const double inv_r3h = 1.0 / (r * r * r * hg2);
        WR = -(Z * Z) * inv_r3h - w * (P.q + 1.0) * invR / hg2;
        WZ = R * Z * inv_r3h;
    }
    double St, lStR, lStZ;
    if (A.St_diff > 0.0) {
        St = A.St_diff;
        lStR = 0.0;
        lStZ = 0.0;
    } else {
        St = P.St0 / P.s0 * exp(-P.p * lx + w / hg2) * grain_size(P, A.m[i]);
        lStR = -P.p * invR + WR;
        lStZ = WZ;
    }
    const double St2 = St * St;
    const double G = 2.0 * St2 / (1.0 + St2);
    const double Dbase = nu / (1.0 + St2);
    const double lDR = (P.q + 1.5) * invR - G * lStR;
    const double lrR = A.vint ? P.p * invR : (P.p - 0.5 * (P.q + 3.0)) * invR - WR;

    double zR, zZ, zP = 0.0, unused;
    diff_pair(A.seed, A.id[i], A.step, 0, zR, zZ);
    const double dt = A.dt;
    const double DR = Dbase / A.Sc[0];
    const double dR = sqrt(2.0 * DR * dt) * zR + DR * (invR + lDR + A.chi * lrR) * dt;
    double dZ = 0.0, dP = 0.0, sa = 0.0, ca = 1.0;
    if (!A.vint) {
        const double DZ = Dbase / A.Sc[1];
        dZ = sqrt(2.0 * DZ * dt) * zZ + DZ * (-G * lStZ - A.chi * WZ) * dt;
    }
    if (!A.axisym) {
        diff_pair(A.seed, A.id[i], A.step, 1, zP, unused);
        const double DP = Dbase / A.Sc[2];
        dP = sqrt(2.0 * DP * dt) * zP * invR;
        sincos(dP, &sa, &ca);
    }

    // velocity in the cylindrical basis at the old position
    const double v_r = A.vr[i], v_t = A.lth[i] / r0;
    const double vR = v_r * st0 + v_t * ct0;
    const double vZ = v_r * ct0 - v_t * st0;
    const double vP = A.lph[i] * invR;
    double R1 = R + dR, P1 = p0 + dP;
    if (R1 < 0.0) {
        R1 = -R1;
        P1 = P1 + kPi;
        sa = -sa;
        ca = -ca;
    }
    const double vR1 = vR * ca + vP * sa;
    const double vP1 = vP * ca - vR * sa;
    const double Z1 = Z + dZ;
    const double r1 = sqrt(R1 * R1 + Z1 * Z1);
    const double inv_r1 = 1.0 / r1;
    const double st1 = R1 * inv_r1, ct1 = Z1 * inv_r1;
    double sp1, cp1;
    sincos(P1, &sp1, &cp1);
    A.r[i] = r1;
    A.th[i] = atan2(R1, Z1);
    A.ph[i] = P1;
    A.vr[i] = vR1 * st1 + vZ * ct1;
    A.lth[i] = r1 * (vR1 * ct1 - vZ * st1);
    A.lph[i] = R1 * vP1;
    A.x[i] = R1 * cp1;
    A.y[i] = R1 * sp1;
    A.z[i] = Z1;
    if (r1 < P.r_in || r1 > P.r_out) A.M[i] = 0.0;
}

int launch_diffuse(const gd_problem* p, const gd_particles* s, double dt, uint64_t seed, uint32_t step,
                   hipStream_t st)
{
    DiffArgs A{};
    A.P = to_dev(p);
    A.id = s->id;
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
    A.m = s->m[s->cur];
    A.dt = dt;
    A.chi = p->diffusion == GD_DIFFUSION_CONCENTRATION ? 1.0 : 0.0;
    A.St_diff = p->St_diff;
    for (int a = 0; a < 3; ++a) A.Sc[a] = p->Sc[a];
    A.seed = seed;
    A.step = step;
    A.vint = p->vint;
    A.axisym = p->axisym;
    const int g = int((p->n + 255) / 256);
    prof_mark(GD_PROF_DIFFUSE, 0, st);
    hipLaunchKernelGGL(k_diffuse, dim3(g), dim3(256), 0, st, A);
    prof_mark(GD_PROF_DIFFUSE, 1, st);
    return 0;
}

}  // namespace gd
