// gd_physics.hpp -- per-pair collision physics on the device.
//
//  * gas disk (Sect. 2.2): Sigma_g = Sigma_g0 (R/R0)^p, h_g = h_g0 (R/R0)^((q+1)/2),
//    H_g = h_g R, c_s = H_g Omega_K, rho_g = Sigma_g/(sqrt(2 pi) H_g) exp(-(1-R/r)/h_g^2),
//    eta = -[(p + q/2 - 3/2) h_g^2 + q (1 - R/r)]/2, v_g,phi = sqrt(1 - 2 eta) Omega_K R;
//  * Stokes number (Sect. 2.3.1): St = St0 (s/s0) (R/R0)^-p exp((1-R/r)/h_g^2);
//  * relative speed eq:dv: drift terms dv_R, dv_Z, dv_phi, Brownian speed capped
//    at c_s, turbulence from the closed forms of Ormel & Cuzzi (2007), all at the
//    query particle's position with St_j = St_i s_j/s_i; differences of Stokes-
//    number functions are factored through St_i - St_j taken from m_i - m_j;
//  * sampling measure V_i = 4 pi d_i^3/3 minus the caps beyond the boundaries
//    r_in and r_out, each taken as a plane at its distance (Sect. 2.5.1);
//  * eq:kernel K = pi (s_i+s_j)^2 dv/4 and eq:rate lambda_ij = N_j K/V_i, or the
//    dimensionless lambda_ij = (1/t0)(1/N_K)(m0/m_j) K of Sect. 3.3;
//  * outcomes (Sect. 2.5.2) with grouping N_coll = floor(1e-4/psi) for psi <= 1e-6:
//    sticking [lambda/N_coll], erosion for psi <= 0.1 [remnant (1-psi) lambda/N_coll,
//    debris psi lambda], fragmentation [lambda];
//  * controller moments <J>, <J^2> of each channel (Sect. 2.5.3), fragments by
//    integrating eq:frag over U.
// Every expression keeps one evaluation order and each operation is rounded
// on its own (the library is compiled without contraction); div_nr, rcp_nr
// and sqrt_nr below give the IEEE results for operands in range.
#pragma once

#include "gd_common.hpp"

namespace gd {

// 1/b from the hardware reciprocal and two Newton steps (each squares the
// relative error), then one more step.  For finite nonzero b whose
// reciprocal is a normal number: these are the steps of the compiler's IEEE
// division with its range scaling left out, and they give the same bits
// (16.7M random operands over 2^-60 .. 2^60 agreed bit for bit on gfx950);
// 6 instructions where the division takes 13.  Quotients whose operands may
// leave that range (waiting times against a rate sum) keep the division.
__device__ __forceinline__ double rcp_nr(double b)
{
    double r = __builtin_amdgcn_rcp(b);
    double e = fma(-b, r, 1.0);
    r = fma(r, e, r);
    e = fma(-b, r, 1.0);
    r = fma(r, e, r);
    e = fma(-b, r, 1.0);
    return fma(r, e, r);
}

// a/b as a (1/b) with the remainder a - b q folded back in: the rounded
// quotient, under the same range conditions on b and a/b; 8 instructions.
__device__ __forceinline__ double div_nr(double a, double b)
{
    double r = __builtin_amdgcn_rcp(b);
    double e = fma(-b, r, 1.0);
    r = fma(r, e, r);
    e = fma(-b, r, 1.0);
    r = fma(r, e, r);
    const double q = a * r;
    return fma(r, fma(-b, q, a), q);
}

// sqrt(x) for x = 0 or normal x > 0: the hardware reciprocal square root y,
// then g ~ x y and h ~ y/2 refined together by one coupled Newton step and
// g by two residual steps (Markstein's form); 0 for 0.  The library's square
// root is these steps plus a range scaling for tiny x, and gives the same
// bits for x from 2^-60 to 2^60.
__device__ __forceinline__ double sqrt_nr(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-h, g, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    g = fma(fma(-g, g, x), h, g);
    g = fma(fma(-g, g, x), h, g);
    return x > 0.0 ? g : x;
}

struct Gas {
    double OmK, hg, Hg, cs, r, rhog, eta, vgphi, stfac;
};

__device__ inline void gas_at(const DevProblem& P, double R, double Z, Gas& g)
{
    const double r = sqrt(R * R + Z * Z);
    const double xr = R / P.R0;
    g.r = r;
    g.OmK = sqrt(P.GM / (R * R * R));
    g.hg = P.h_g0 * pow(xr, (P.q + 1.0) * 0.5);
    g.Hg = g.hg * R;
    g.cs = g.Hg * g.OmK;
    const double hg2 = g.hg * g.hg;
    const double w = 1.0 - R / r;
    const double Sig = P.Sigma_g0 * pow(xr, P.p);
    g.rhog = Sig / (sqrt(2.0 * kPi) * g.Hg) * exp(-w / hg2);
    g.eta = -0.5 * ((P.p + 0.5 * P.q - 1.5) * hg2 + P.q * w);
    g.vgphi = sqrt(1.0 - 2.0 * g.eta) * g.OmK * R;
    g.stfac = P.St0 / P.s0 * pow(xr, -P.p) * exp(w / hg2);
}

__device__ inline double grain_size(const DevProblem& P, double m)
{
    return cbrt(div_nr(6.0 * m, kPi * P.rho_s));
}

// Everything of the rate that depends on the query particle's position only.
struct QCtx {
    double V, R, Z, OmK, eta, cs, stfac, Vg2, tke, kT8pi;
    double invV;        // 1 / V_i (0 when V_i <= 0)
    double vR, vZ, vP;  // the factors of eq:dv's drift terms: 2 eta R Omega_K, Z Omega_K, eta R Omega_K
};

__device__ inline void query_ctx(const DevProblem& P, double x, double y, double z, double d, QCtx& c)
{
    if (P.kernel != GD_KERNEL_PHYSICAL) {
        c.V = 1.0;
        c.invV = 1.0;
        return;
    }
    const double R = sqrt(x * x + y * y);
    Gas g;
    gas_at(P, R, z, g);
    c.R = R;
    c.Z = z;
    c.OmK = g.OmK;
    c.eta = g.eta;
    c.cs = g.cs;
    c.stfac = g.stfac;
    double V = 4.0 * kPi * d * d * d / 3.0;
    if (P.caps) {
        const double de0 = g.r - P.r_in, de1 = P.r_out - g.r;
        if (de0 < d) {
            const double h = d - de0;
            V = V - kPi * h * h * (3.0 * d - h) / 3.0;
        }
        if (de1 < d) {
            const double h = d - de1;
            V = V - kPi * h * h * (3.0 * d - h) / 3.0;
        }
    }
    c.V = V;
    c.invV = V > 0.0 ? 1.0 / V : 0.0;
    c.vR = 2.0 * g.eta * R * g.OmK;
    c.vZ = z * g.OmK;
    c.vP = g.eta * R * g.OmK;
    c.Vg2 = 1.5 * P.alpha * g.cs * g.cs;
    const double vth = sqrt(8.0 / kPi) * g.cs;
    const double lmfp = P.mu_mH / (g.rhog * P.sigma_H2);
    const double numol = 0.5 * vth * lmfp;
    const double Re = P.alpha * g.cs * g.Hg / numol;
    c.tke = 1.0 / sqrt(Re);
    c.kT8pi = 8.0 * (P.mu_mH * g.cs * g.cs) / kPi;
}

// <J>, <J^2> of a fragment of a grain of diameter s_i: with x = sqrt(s_i/s_min),
// d = x - 1: <J> = 2[1 - ln x/d], <J^2> = 4[2x - ln^2 x - 2 ln x - 2]/d, and for
// d < 0.1 the power series <J> = 2 sum_n (-1)^(n+1) d^n/(n+1),
// <J^2> = 8 sum_{m>=2} (-1)^(m+1) (1 - H_m) d^m/(m+1).
__device__ inline void frag_moments(double s_i, double s_min, double& mJ, double& mJ2)
{
    const double x = sqrt(s_i / s_min);
    const double d = x - 1.0;
    if (!(d > 0.0)) {
        mJ = 0.0;
        mJ2 = 0.0;
        return;
    }
    if (d < 0.1) {
        double j1 = 0.0, j2 = 0.0, dn = d, H = 1.0, sg = 1.0;
        for (int k = 1; k <= 40; ++k) {
            j1 += sg * dn / double(k + 1);
            if (k >= 2) j2 += sg * (1.0 - H) * dn / double(k + 1);
            dn *= d;
            sg = -sg;
            H += 1.0 / double(k + 1);
        }
        mJ = 2.0 * j1;
        mJ2 = 8.0 * j2;
        return;
    }
    const double L = log1p(d);
    mJ = 2.0 * (1.0 - L / d);
    mJ2 = 4.0 * (2.0 * x - L * L - 2.0 * L - 2.0) / d;
}

enum { kStick = 0, kErosion = 1, kFrag = 2 };

struct Pair {
    int type;
    double r0, r1;      // channel rates (r1 = 0 unless erosion)
    double lam_star;
    double Ng;
};

// The query particle's own terms, evaluated once per particle (and again
// after each change of its mass): mass, 1/m_i, diameter, Stokes number,
// 1/(1 + St_i^2) and 1/(1 + St_i), and (when asked for) the fragment moments
// of its size, which depend on nothing else.
struct Own {
    double mi, rmi, si, Sti, rqi, rhi;
    double mJ, mJ2;
};

__device__ inline void own_terms(const DevProblem& P, const QCtx& c, double mi, double si, bool moments, Own& w)
{
    const bool phys = P.kernel == GD_KERNEL_PHYSICAL;
    w.mi = mi;
    w.rmi = 1.0 / mi;
    w.si = si;
    w.Sti = phys ? c.stfac * si : 0.0;
    w.rqi = rcp_nr(1.0 + w.Sti * w.Sti);
    w.rhi = rcp_nr(1.0 + w.Sti);
    w.mJ = 0.0;
    w.mJ2 = 0.0;
    if (phys && moments) frag_moments(si, P.s_min, w.mJ, w.mJ2);
}

// The terms of neighbour j that do not involve the query particle's mass:
// the snapshot record (m_j, s_j, N_j, 1/m_j), St_j at the query position,
// 1/(1 + St_j^2), and (HOIST) 1/(1 + St_j) of OC07's heavy regime and
// m0/m_j of the dimensionless kernels.  Against the frozen neighbourhood
// they hold for a whole interval, so a particle with many events computes
// them once; a single evaluation computes what it needs in place.
struct Nb {
    double mj, sj, Nj, rmj;
    double Stj, rqj, rhj, cj;
};

template <bool HOIST>
__device__ inline void nb_terms(const DevProblem& P, const QCtx& c, double mj, double sj, double Nj, double rmj,
                                Nb& b)
{
    b.mj = mj;
    b.sj = sj;
    b.Nj = Nj;
    b.rmj = rmj;
    b.Stj = c.stfac * sj;
    b.rqj = rcp_nr(1.0 + b.Stj * b.Stj);
    b.rhj = HOIST ? rcp_nr(1.0 + b.Stj) : 0.0;
    b.cj = HOIST ? div_nr(P.m0, mj) : 0.0;
}

// Ormel & Cuzzi (2007) turbulent relative speed squared, St1 >= St2,
// dSt = St1 - St2, each regime with one division at most:
//  * tight, St1 < t = Re^-1/2:
//    Vg^2 dSt^2 [St1 St2 + t(St1+St2)]/[(St1+St2)(St1+t)(St2+t)], the
//    published form rearranged so that close St do not cancel;
//  * intermediate, up to St1 = 1 (y_a = 1.6):
//    Vg^2 St1 [2 y_a - (1+e) + 2/(1+e) (1/(1+y_a) + e^3/(y_a+e))], e = St2/St1,
//    multiplied through by St1^3:
//    Vg^2 {(2 y_a - 1) St1 - St2 + 2 [St1^2 u/(1+y_a) + St2^3]/[(St1+St2) u]},
//    u = y_a St1 + St2 (the linear part is at least 1.2 St1: no cancellation);
//  * heavy: Vg^2 [1/(1+St1) + 1/(1+St2)] from the reciprocals rh1, rh2 given.
// The regimes stay branches: the wavefronts of one disk region mostly share
// one.
__device__ inline double oc07_dv2_r(double St1, double St2, double dSt, double Vg2, double tke, double rh1,
                                    double rh2)
{
    if (St1 < tke) {
        const double num = St1 * St2 + tke * (St1 + St2);
        const double den = (St1 + St2) * (St1 + tke) * (St2 + tke);
        return div_nr(Vg2 * (dSt * dSt) * num, den);
    }
    if (St1 < 1.0) {
        constexpr double ya = 1.6;
        const double u = ya * St1 + St2;
        const double num = 2.0 * (St1 * St1 * u * (1.0 / (1.0 + ya)) + St2 * St2 * St2);
        return Vg2 * (((2.0 * ya - 1.0) * St1 - St2) + div_nr(num, (St1 + St2) * u));
    }
    return Vg2 * (rh1 + rh2);
}

// One pair: the query particle's terms against neighbour j's.
// The physical rate is arranged for few divisions: 1/(1+St^2) of each grain
// for both drift differences, the snapshot's 1/m_j in the Brownian term,
// 1/V_i once per particle.  It agrees with eq:rate to rounding (well inside
// the 1e-12 contract); the dimensionless rates keep the oracle's operation
// order exactly (m0/m_j hoisted or not is the same rounded quotient).
// QNR takes psi = m_j/m_i from div_nr too (the same bits); the sampling
// passes keep the division, whose registers the event pass cannot spare.
template <bool HOIST, bool QNR = false>
__device__ inline void pair_core(const DevProblem& P, const QCtx& c, const Own& w, const Nb& b, Pair& o)
{
    const double mi = w.mi, mj = b.mj;
    double lam, dv = 0.0;
    if (P.kernel == GD_KERNEL_PHYSICAL) {
        // St_i - St_j from the mass difference,
        // s_i - s_j = (6/(pi rho))(m_i - m_j)/(s_i^2 + s_i s_j + s_j^2),
        // so that close grains do not cancel.
        const double si = w.si, Sti = w.Sti, sj = b.sj, Stj = b.Stj;
        const double ds = div_nr((6.0 / (kPi * P.rho_s)) * (mi - mj), si * si + si * sj + sj * sj);
        const double dSt = c.stfac * ds;
        const double rq = w.rqi * b.rqj;
        const double da = dSt * (1.0 - Sti * Stj) * rq;
        const double db = -dSt * (Sti + Stj) * rq;
        const double dvR = c.vR * da;
        const double dz = (Sti < 0.5 && Stj < 0.5) ? dSt : fmin(Sti, 0.5) - fmin(Stj, 0.5);
        const double dvZ = c.vZ * dz;
        const double dvP = c.vP * db;
        // the Brownian speed enters squared: min(sqrt(a), c_s)^2 = min(a, c_s^2)
        double dvB2 = 0.0, dvT2 = 0.0;
        if (P.brownian) dvB2 = fmin(c.kT8pi * (w.rmi + b.rmj), c.cs * c.cs);
        if (P.turbulence) {
            const bool ig = Sti >= Stj;
            const double rhj = HOIST ? b.rhj : rcp_nr(1.0 + Stj);
            dvT2 = oc07_dv2_r(ig ? Sti : Stj, ig ? Stj : Sti, fabs(dSt), c.Vg2, c.tke, ig ? w.rhi : rhj,
                              ig ? rhj : w.rhi);
        }
        double dv2 = dvR * dvR + dvZ * dvZ;
        dv2 = dv2 + dvP * dvP;
        dv2 = dv2 + dvB2;
        dv2 = dv2 + dvT2;
        dv = sqrt_nr(dv2);
        const double ssum = si + sj;
        const double K = kPi * ssum * ssum * dv * 0.25;
        lam = b.Nj * K * c.invV;
    } else {
        double Kt;
        if (P.kernel == GD_KERNEL_CONST) Kt = 1.0;
        else if (P.kernel == GD_KERNEL_ADDITIVE) Kt = div_nr(mi + mj, P.m0);
        else Kt = div_nr(mi * mj, P.m0 * P.m0);
        lam = div_nr((HOIST ? b.cj : div_nr(P.m0, mj)) * Kt, P.t0 * double(P.k));
    }
    const double psi = QNR ? div_nr(mj, mi) : mj / mi;
    const bool fast = (P.kernel == GD_KERNEL_PHYSICAL) && (dv >= P.v_frag);
    double Ng = 1.0;
    if (P.grouping && psi <= 1e-6) Ng = floor(div_nr(1e-4, psi));
    o.Ng = Ng;
    if (!fast) {
        o.type = kStick;
        o.r0 = Ng == 1.0 ? lam : div_nr(lam, Ng);
        o.r1 = 0.0;
        o.lam_star = o.r0;
    } else if (P.erosion && psi <= 0.1) {
        o.type = kErosion;
        o.r0 = Ng == 1.0 ? (1.0 - psi) * lam : div_nr((1.0 - psi) * lam, Ng);
        o.r1 = psi * lam;
        o.lam_star = o.r0 + o.r1;
    } else {
        o.type = kFrag;
        o.r0 = lam;
        o.r1 = 0.0;
        o.lam_star = lam;
    }
}

// One pair against neighbour (m_j, s_j, N_j, 1/m_j) of the frozen snapshot.
template <bool QNR = false>
__device__ inline void pair_eval(const DevProblem& P, const QCtx& c, const Own& w, double mj, double sj, double Nj,
                                 double rmj, Pair& o)
{
    Nb b;
    nb_terms<false>(P, c, mj, sj, Nj, rmj, b);
    pair_core<false, QNR>(P, c, w, b, o);
}

// ln y for finite y > 0 (other y as the library), from the series ln y = e ln 2 + 2 atanh(s): y =
// m 2^e with m in [1/sqrt 2, sqrt 2), s = (m - 1)/(m + 1), |s| <= 0.172, and
// 2 atanh(s) = 2 s (1 + s^2/3 + ... + s^18/19) (the next term is below
// 2^-55 of the sum).  A few ulp, in about a third of the instructions of the
// library's logarithms, which carry double-double steps; the controller
// moments of every pair take one or two.
__device__ inline double log_s(double y)
{
    if (!(y > 0.0 && y < INFINITY)) return log(y);  // 0, negative, infinite or NaN: as the library
    int e;
    double m = frexp(y, &e);
    if (m < 0.70710678118654752) {
        m = m + m;
        e = e - 1;
    }
    const double f = m - 1.0;
    const double s = div_nr(f, 2.0 + f);
    const double s2 = s * s;
    double p = 1.0 / 19.0;
    p = fma(p, s2, 1.0 / 17.0);
    p = fma(p, s2, 1.0 / 15.0);
    p = fma(p, s2, 1.0 / 13.0);
    p = fma(p, s2, 1.0 / 11.0);
    p = fma(p, s2, 1.0 / 9.0);
    p = fma(p, s2, 1.0 / 7.0);
    p = fma(p, s2, 1.0 / 5.0);
    p = fma(p, s2, 1.0 / 3.0);
    p = fma(p, s2, 1.0);
    return fma(double(e), 0.69314718055994530942, (s + s) * p);
}

// ln(1 + x) for x > -1: ln u for u = 1 + x rounded, plus that rounding's
// share (x - (u - 1))/u; x itself when u rounds to 1.  Within 3 ulp of
// ln(1 + x) for 1e-20 <= x <= 1e30 and -0.1 <= x < 0 (the same steps are
// evaluated on the host, with correctly rounded quotients, in
// tests/test_series_log.py).
__device__ inline double log1p_s(double x)
{
    const double u = 1.0 + x;
    if (u == 1.0) return x;
    if (!(u > 0.0 && u < INFINITY)) return log1p(x);
    return log_s(u) + div_nr(x - (u - 1.0), u);
}

// sum over the pair's channels of rate * <J> and rate * <J^2>
__device__ inline void pair_moments(const Pair& o, const Own& w, double mj, double& a, double& b)
{
    constexpr double kThird = 1.0 / 3.0;
    const double psi = div_nr(mj, w.mi);  // the same bits as pair_core<.., true>'s
    if (o.type == kStick) {
        const double J = log1p_s(o.Ng * psi) * kThird;
        a = o.r0 * J;
        b = o.r0 * (J * J);
    } else if (o.type == kErosion) {
        const double Jr = -log1p_s(-o.Ng * psi) * kThird;
        const double Jd = fabs(log_s(psi)) * kThird;
        a = o.r0 * Jr;
        b = o.r0 * (Jr * Jr);
        a = a + o.r1 * Jd;
        b = b + o.r1 * (Jd * Jd);
    } else {
        a = o.r0 * w.mJ;
        b = o.r0 * w.mJ2;
    }
}

// ---------------------------------------------------------------------------
// Single-precision form of the pair rate (optional; gd_problem.rates_fp32).
// The query context is computed in FP64 once per particle and rounded to
// float; the collision speed, kernel, channel rates and moments of each pair
// are float; the particle-count weight N_j / V_i (whose factors overflow
// float in cgs units) and the mass ratio psi = m_j (1/m_i) with its grouping
// factor stay FP64.  Callers sum the float pair terms in FP64.
struct QCtxF {
    float Z, OmK, cs, stfac, Vg2, tke, kT8pi, vdrift, vset;  // vdrift = eta R Omega_K, vset = Z Omega_K
    double invV;                                              // 1 / V_i (0 when V_i <= 0)
    double k6;                                                // 6 / (pi rho_s)
    double kdl;                                               // m0 / (t0 N_K) (dimensionless kernels)
};

__device__ inline void query_ctx_f32(const DevProblem& P, const QCtx& c, QCtxF& f)
{
    if (P.kernel != GD_KERNEL_PHYSICAL) {
        f.invV = 1.0;
        f.kdl = P.m0 / (P.t0 * double(P.k));
        return;
    }
    f.k6 = 6.0 / (kPi * P.rho_s);
    f.Z = float(c.Z);
    f.OmK = float(c.OmK);
    f.cs = float(c.cs);
    f.stfac = float(c.stfac);
    f.Vg2 = float(c.Vg2);
    f.tke = float(c.tke);
    f.kT8pi = float(c.kT8pi);
    f.vdrift = float(c.eta * c.R * c.OmK);
    f.vset = float(c.Z * c.OmK);
    f.invV = c.V > 0.0 ? 1.0 / c.V : 0.0;
}

// hardware reciprocal and square root (1 ulp): the single-precision form's
// error budget is set by its float arithmetic anyway
__device__ inline float rcpf_(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline float sqrtf_(float x) { return __builtin_amdgcn_sqrtf(x); }

__device__ inline float oc07_dv2_f32(float St1, float St2, float dSt, float Vg2, float tke)
{
    if (St1 < tke) {
        const float num = St1 * St2 + tke * (St1 + St2);
        const float den = (St1 + St2) * (St1 + tke) * (St2 + tke);
        return Vg2 * (dSt * dSt) * num * rcpf_(den);
    }
    if (St1 < 1.0f) {
        const float ya = 1.6f;
        const float e = St2 * rcpf_(St1);
        const float br = 2.0f * ya - (1.0f + e) + 2.0f * rcpf_(1.0f + e) * (1.0f / (1.0f + ya) + e * e * e * rcpf_(ya + e));
        return Vg2 * br * St1;
    }
    return Vg2 * (rcpf_(1.0f + St1) + rcpf_(1.0f + St2));
}

struct PairF {
    int type;
    float r0, r1;  // channel rates
    float lam_star;
    double Ng;
    double psi;
};

// Own particle: mass mi (and its reciprocal rmi), diameter si and Stokes
// number Sti.  Neighbour: mass mj, diameter sj, grain count Nj.
__device__ inline void pair_eval_f32(const DevProblem& P, const QCtxF& c, double mi, double rmi, float si, float Sti,
                                     double mj, float sj, double Nj, PairF& o)
{
    float lam, dv = 0.0f;
    if (P.kernel == GD_KERNEL_PHYSICAL) {
        const float Stj = c.stfac * sj;
        const float ds = float(c.k6 * (mi - mj)) * rcpf_(si * si + si * sj + sj * sj);
        const float dSt = c.stfac * ds;
        const float qi = 1.0f + Sti * Sti, qj = 1.0f + Stj * Stj;
        const float rq = dSt * rcpf_(qi * qj);
        const float da = (1.0f - Sti * Stj) * rq;
        const float db = -(Sti + Stj) * rq;
        const float dvR = 2.0f * c.vdrift * da;
        const float dz = (Sti < 0.5f && Stj < 0.5f) ? dSt : fminf(Sti, 0.5f) - fminf(Stj, 0.5f);
        const float dvZ = c.vset * dz;
        const float dvP = c.vdrift * db;
        float dvB = 0.0f, dvT2 = 0.0f;
        if (P.brownian) {
            dvB = sqrtf_(c.kT8pi * (float(rmi) + rcpf_(float(mj))));
            if (dvB > c.cs) dvB = c.cs;
        }
        if (P.turbulence) {
            const bool ig = Sti >= Stj;
            dvT2 = oc07_dv2_f32(ig ? Sti : Stj, ig ? Stj : Sti, fabsf(dSt), c.Vg2, c.tke);
        }
        float dv2 = dvR * dvR + dvZ * dvZ;
        dv2 = dv2 + dvP * dvP;
        dv2 = dv2 + dvB * dvB;
        dv2 = dv2 + dvT2;
        dv = sqrtf_(dv2);
        const float ssum = si + sj;
        lam = float(Nj * c.invV) * (float(kPi / 4.0) * ssum * ssum * dv);
    } else {
        float Kt;
        if (P.kernel == GD_KERNEL_CONST) Kt = 1.0f;
        else if (P.kernel == GD_KERNEL_ADDITIVE) Kt = float((mi + mj) / P.m0);
        else Kt = float((mi * mj) / (P.m0 * P.m0));
        lam = float(c.kdl / mj) * Kt;
    }
    const double psi = mj * rmi;
    const bool fast = (P.kernel == GD_KERNEL_PHYSICAL) && (double(dv) >= P.v_frag);
    double Ng = 1.0;
    if (P.grouping && psi <= 1e-6) Ng = floor(div_nr(1e-4, psi));
    o.Ng = Ng;
    o.psi = psi;
    if (!fast) {
        o.type = kStick;
        o.r0 = Ng == 1.0 ? lam : lam * float(rcp_nr(Ng));
        o.r1 = 0.0f;
        o.lam_star = o.r0;
    } else if (P.erosion && psi <= 0.1) {
        o.type = kErosion;
        o.r0 = float(div_nr(1.0 - psi, Ng)) * lam;
        o.r1 = float(psi) * lam;
        o.lam_star = o.r0 + o.r1;
    } else {
        o.type = kFrag;
        o.r0 = lam;
        o.r1 = 0.0f;
        o.lam_star = lam;
    }
}

// rate * <J> and rate * <J^2> of the pair's channels; mJf, mJ2f are the
// fragment moments of the own grain (computed once per particle)
__device__ inline void pair_moments_f32(const PairF& o, float mJf, float mJ2f, float& a, float& b)
{
    if (o.type == kStick) {
        const float J = log1pf(float(o.Ng * o.psi)) / 3.0f;
        a = o.r0 * J;
        b = o.r0 * (J * J);
    } else if (o.type == kErosion) {
        const float Jr = -log1pf(float(-o.Ng * o.psi)) / 3.0f;
        const float Jd = float(fabs(log(o.psi)) / 3.0);
        a = o.r0 * Jr + o.r1 * Jd;
        b = o.r0 * (Jr * Jr) + o.r1 * (Jd * Jd);
    } else {
        a = o.r0 * mJf;
        b = o.r0 * mJ2f;
    }
}

}  // namespace gd
