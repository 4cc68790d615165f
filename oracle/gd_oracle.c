/*
 * gd_oracle.c -- plain, slow, FP64 CPU oracle for the representative-particle
 * collision hot path of "GameDev: GPU-accelerated model for dust evolution"
 * (Bi, arXiv 2609.35967).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no header, table or helper with the GPU
 * code: every formula below is written out again from the paper.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 * Every floating-point operation is rounded separately (no contraction).
 *
 * Contents and the passages they follow:
 *   orc_philox4x32_10   counter-based generator (Salmon et al. 2011)
 *   orc_uniforms        the four uniforms of one collision event
 *   orc_morton_keys     Morton order used by the neighbour search (Sect. 2.5.1)
 *   orc_knn             N_K nearest neighbours incl. self (Sect. 2.5.1)
 *   orc_frag_moments    <J>, <J^2> of the fragment draw (Sect. 2.5.3, eq:frag)
 *   orc_pair_channels   collision rate, outcome channels, grouping
 *                       (Sect. 2.5.1 eq:kernel/eq:rate, Sect. 2.5.2, App. A)
 *   orc_rates           lambda*_i, controller moments a_i, b_i (Sect. 2.5.3)
 *   orc_plan            controller bins, dt_fn,req, dyadic dt_fn,exe (Sect. 2.5.3)
 *   orc_mc              Gillespie sampling against the frozen neighbourhood
 *   orc_audit           post-interval audit of the safety factor C
 *   orc_push_local      drift-kick-drift vertical settling, local column
 *   orc_push_global     staggered semi-analytic push in spherical coords (Sect. 2.3.3)
 *   orc_diffuse         Euler--Maruyama dust diffusion step (Sect. 2.4)
 *   orc_transport_dt    the shared transport step from local constraints (Sect. 2.6)
 *   orc_fsum            exactly rounded sum (used for all reductions)
 *   orc_reshuffle       random relabelling of the cached neighbours before a
 *                       refresh (product-kernel test, Sect. 3.3)
 *
 * Readings of passages the paper leaves open are listed where they are used
 * and collected in the design notes of the repository.
 *
 * The physical pair rate (gas disk, Stokes numbers, every term of eq:dv
 * including the three Ormel & Cuzzi closed forms, the caps of V_i and the
 * outcome channels) is pinned by an independent 50-digit evaluation of the
 * printed formulas in each turbulence regime.  The gas disk is also pinned by
 * its vertical integral and hydrostatic balance, and eq:dv's composition by
 * the quadrature sum of its parts at points where all of them matter.
 * What no pin can fix is the reading of the turbulent term: the paper adopts
 * a six-branch form taken from another code without printing it; this file
 * uses the three published limiting forms (see oc07_dv2).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846
/* Relative margin below which a sampling decision counts as a near-tie
 * (1e-12 for the FP64 path; a comparison of a lower-precision form of the
 * rates sets a larger one). */
static double ORC_TIE = 1e-12;

/* ------------------------------------------------------------------------ */
/* Problem description (the oracle's own struct; mirrored by ctypes).        */
/* ------------------------------------------------------------------------ */
enum { ORC_CONST = 0, ORC_ADDITIVE = 1, ORC_PRODUCT = 2, ORC_PHYSICAL = 3 };

typedef struct {
    int32_t kernel;      /* ORC_CONST .. ORC_PHYSICAL */
    int32_t k;           /* N_K, neighbours including self */
    int32_t nbin_min;    /* minimum particles per merged controller bin */
    int32_t erosion;     /* 1: erosion channel on (Sect. 2.5.2) */
    int32_t grouping;    /* 1: grouping of small increments on */
    int32_t periodic[3]; /* minimum-image flags per axis */
    double L[3];         /* periods */
    double rmax;         /* maximum search scale (inf = none) */
    /* dimensionless kernels (Sect. 3.3) */
    double t0, m0;
    /* controller (Sect. 2.5.3) */
    double eps, dt_fn_max;
    /* grains and outcomes */
    double rho_s, s_min, v_frag;
    /* gas disk (Sect. 2.2) -- cgs or code units */
    double GM, Sigma_g0, R0, p, q, h_g0, alpha, mu_mH, sigma_H2;
    double s0, St0;      /* reference size and its midplane Stokes number at R0 */
    double r_in, r_out;  /* spherical domain bounds (caps, outflow) */
    int32_t drag;        /* 1: gas drag on in the global push */
    int32_t brownian;    /* 1: Brownian term in Delta v */
    int32_t turbulence;  /* 1: turbulent term in Delta v */
    int32_t caps;        /* 1: boundary caps subtracted from V_i */
    /* dust diffusion (Sect. 2.4) */
    int32_t diffusion;   /* 0 off, 1 concentration form (chi = 1), 2 density form (chi = 0) */
    int32_t vint;        /* 1: vertically integrated model (Sigma_g for rho_g, midplane St, no Z step) */
    int32_t axisym;      /* 1: axisymmetric model (no azimuthal step) */
    int32_t pad_;
    double Sc[3];        /* Schmidt numbers of the R, Z and phi directions */
    double St_diff;      /* > 0: spatially constant Stokes number in D (ring test, Sect. 3.2) */
} orc_problem;

/* ------------------------------------------------------------------------ */
/* Exactly rounded summation (Shewchuk partials, as in Python's math.fsum). */
/* A reduction of the method is the sum itself; the oracle returns that sum */
/* rounded once, so no summation order is implied.                          */
/* ------------------------------------------------------------------------ */
typedef struct { int n; double p[96]; } orc_xsum;

static void xsum_init(orc_xsum* s) { s->n = 0; }

static void xsum_add(orc_xsum* s, double x)
{
    int i = 0;
    for (int j = 0; j < s->n; j++) {
        double y = s->p[j];
        if (fabs(x) < fabs(y)) { double t = x; x = y; y = t; }
        double hi = x + y;
        double lo = y - (hi - x);
        if (lo != 0.0) s->p[i++] = lo;
        x = hi;
    }
    s->p[i++] = x;
    s->n = i;
}

static double xsum_value(const orc_xsum* s)
{
    int n = s->n;
    double hi = 0.0, lo = 0.0;
    if (n > 0) {
        hi = s->p[--n];
        while (n > 0) {
            double x = hi, y = s->p[--n];
            hi = x + y;
            double yr = hi - x;
            lo = y - yr;
            if (lo != 0.0) break;
        }
        if (n > 0 && ((lo < 0.0 && s->p[n - 1] < 0.0) || (lo > 0.0 && s->p[n - 1] > 0.0))) {
            double y = lo * 2.0;
            double x = hi + y;
            double yr = x - hi;
            if (y == yr) hi = x;
        }
    }
    return hi;
}

double orc_fsum(int64_t n, const double* v)
{
    orc_xsum s; xsum_init(&s);
    for (int64_t i = 0; i < n; i++) xsum_add(&s, v[i]);
    return xsum_value(&s);
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw 2011, "Parallel random numbers:*/
/* as easy as 1, 2, 3").  Ten rounds; each round multiplies words 0 and 2 by */
/* the two Philox multipliers, mixes the high halves with the other words    */
/* and the round key; the key advances by the two Weyl constants.            */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniforms of event e of particle `id` in interval `iv`.
 * Two generator calls per event, counters (id, iv, e, 0) and (id, iv, e, 1),
 * key = (low, high) words of the seed.  Each pair of 32-bit words gives a
 * 53-bit integer u = (hi:lo) >> 11.
 *   U_w = (u + 1) 2^-53 in (0, 1]   waiting time (Sect. 2.5.3, Gillespie draw)
 *   U_p =  u      2^-53 in [0, 1)   partner
 *   U_c                              channel within the pair
 *   U_f                              fragment size (eq:frag)
 * Every event consumes both calls whatever its outcome. */
void orc_uniforms(uint64_t seed, uint32_t id, uint32_t iv, uint32_t e, double u[4])
{
    const double two53 = 1.0 / 9007199254740992.0;
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t c[4] = { id, iv, e, 0u }, o[4];
    orc_philox4x32_10(c, key, o);
    uint64_t a = ((((uint64_t)o[1]) << 32) | o[0]) >> 11;
    uint64_t b = ((((uint64_t)o[3]) << 32) | o[2]) >> 11;
    u[0] = (double)(a + 1) * two53;
    u[1] = (double)b * two53;
    c[3] = 1u;
    orc_philox4x32_10(c, key, o);
    a = ((((uint64_t)o[1]) << 32) | o[0]) >> 11;
    b = ((((uint64_t)o[3]) << 32) | o[2]) >> 11;
    u[2] = (double)a * two53;
    u[3] = (double)b * two53;
}

/* ------------------------------------------------------------------------ */
/* Morton keys (Sect. 2.5.1: neighbour search on the Morton order).          */
/* 10 bits per axis inside the cube spanned by the active particles;        */
/* x takes bit 3b, y bit 3b+1, z bit 3b+2.  Inactive particles (M <= 0) get */
/* key 0xFFFFFFFF so that a stable sort puts them last.                     */
/* ------------------------------------------------------------------------ */
uint32_t orc_morton3_10(uint32_t qx, uint32_t qy, uint32_t qz)
{
    uint32_t key = 0;
    for (int b = 0; b < 10; b++) {
        key |= ((qx >> b) & 1u) << (3 * b);
        key |= ((qy >> b) & 1u) << (3 * b + 1);
        key |= ((qz >> b) & 1u) << (3 * b + 2);
    }
    return key;
}

void orc_morton_keys(int64_t n, const double* x, const double* y, const double* z,
                     const double* M, uint32_t* keys)
{
    double lo[3] = { INFINITY, INFINITY, INFINITY }, hi[3] = { -INFINITY, -INFINITY, -INFINITY };
    const double* c[3] = { x, y, z };
    for (int64_t i = 0; i < n; i++) {
        if (!(M[i] > 0.0)) continue;
        for (int d = 0; d < 3; d++) {
            if (c[d][i] < lo[d]) lo[d] = c[d][i];
            if (c[d][i] > hi[d]) hi[d] = c[d][i];
        }
    }
    double ext = 0.0;
    for (int d = 0; d < 3; d++) {
        double e = hi[d] - lo[d];
        if (e > ext) ext = e;
    }
    double inv = (ext > 0.0) ? 1024.0 / ext : 0.0;
    for (int64_t i = 0; i < n; i++) {
        if (!(M[i] > 0.0)) { keys[i] = 0xFFFFFFFFu; continue; }
        uint32_t q[3];
        for (int d = 0; d < 3; d++) {
            double t = (c[d][i] - lo[d]) * inv;
            uint32_t v = (uint32_t)t;
            q[d] = v > 1023u ? 1023u : v;
        }
        keys[i] = orc_morton3_10(q[0], q[1], q[2]);
    }
}

/* ------------------------------------------------------------------------ */
/* Squared separation, minimum image on periodic axes.  Each operation is   */
/* rounded separately: d2 = (dx*dx + dy*dy) + dz*dz.                         */
/* ------------------------------------------------------------------------ */
static double sep2(const orc_problem* P, double xi, double yi, double zi,
                   double xj, double yj, double zj)
{
    double d[3] = { xj - xi, yj - yi, zj - zi };
    for (int a = 0; a < 3; a++) {
        if (P->periodic[a]) {
            double h = 0.5 * P->L[a];
            if (d[a] > h) d[a] = d[a] - P->L[a];
            else if (d[a] < -h) d[a] = d[a] + P->L[a];
        }
    }
    double s = d[0] * d[0] + d[1] * d[1];
    return s + d[2] * d[2];
}

/* ------------------------------------------------------------------------ */
/* k nearest neighbours (Sect. 2.5.1).  Brute force over every active j.    */
/* The neighbourhood of i is i itself (slot 0, "the query particle at zero  */
/* distance") plus the k-1 nearest other active particles with              */
/* d2 <= rmax^2, nearest first by (d2, index).  The retained others are     */
/* written in ascending index order; d_i is the distance to the farthest    */
/* retained neighbour (0 when none).  Unused slots hold -1; inactive rows   */
/* have cnt = 0.                                                             */
/* ------------------------------------------------------------------------ */
void orc_knn(const orc_problem* P, int64_t n, const double* x, const double* y, const double* z,
             const double* M, int64_t nq, const int64_t* qidx,
             int32_t* nbr, int32_t* cnt, double* dmax)
{
    const int k = P->k;
    const double r2max = P->rmax * P->rmax;
#pragma omp parallel
    {
        double* bd = (double*)malloc(sizeof(double) * (size_t)k);
        int64_t* bj = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
#pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < nq; t++) {
            int64_t i = qidx ? qidx[t] : t;
            int32_t* row = nbr + t * (int64_t)k;
            for (int s = 0; s < k; s++) row[s] = -1;
            if (!(M[i] > 0.0)) { cnt[t] = 0; dmax[t] = 0.0; continue; }
            int have = 0; /* sorted list of the best `have` others, by (d2, j) */
            for (int64_t j = 0; j < n; j++) {
                if (j == i || !(M[j] > 0.0)) continue;
                double d2 = sep2(P, x[i], y[i], z[i], x[j], y[j], z[j]);
                if (!(d2 <= r2max)) continue;
                if (have == k - 1) {
                    double wd = bd[have - 1]; int64_t wj = bj[have - 1];
                    if (d2 > wd || (d2 == wd && j > wj)) continue;
                    have--;
                }
                int pos = have;
                while (pos > 0 && (bd[pos - 1] > d2 || (bd[pos - 1] == d2 && bj[pos - 1] > j))) {
                    bd[pos] = bd[pos - 1]; bj[pos] = bj[pos - 1]; pos--;
                }
                bd[pos] = d2; bj[pos] = j; have++;
            }
            cnt[t] = 1 + have;
            dmax[t] = have > 0 ? sqrt(bd[have - 1]) : 0.0;
            /* ascending index order for the others */
            for (int a = 1; a < have; a++) {
                int64_t v = bj[a]; int b = a;
                while (b > 0 && bj[b - 1] > v) { bj[b] = bj[b - 1]; b--; }
                bj[b] = v;
            }
            row[0] = (int32_t)i;
            for (int s = 0; s < have; s++) row[1 + s] = (int32_t)bj[s];
        }
        free(bd); free(bj);
    }
}

/* ------------------------------------------------------------------------ */
/* Fragment-size moments (Sect. 2.5.3, expectation of J over U in eq:frag). */
/* s' = [sqrt(s_min) + U (sqrt(s_i) - sqrt(s_min))]^2, J = |ln(s'/s_i)|.     */
/* With x = sqrt(s_i/s_min) and d = x - 1, integrating over U in [0, 1]:    */
/*   <J>   = 2 [1 - ln x/(x - 1)]                                           */
/*   <J^2> = 4 [2x - ln^2 x - 2 ln x - 2]/(x - 1)                           */
/* For d < 0.1 both are summed as power series in d to avoid cancellation: */
/*   <J>   = 2 sum_{n>=1} (-1)^(n+1) d^n/(n+1)                              */
/*   <J^2> = 8 sum_{m>=2} (-1)^(m+1) (1 - H_m) d^m/(m+1),  H_m harmonic no.  */
/* ------------------------------------------------------------------------ */
void orc_frag_moments(double s_i, double s_min, double* mJ, double* mJ2)
{
    double x = sqrt(s_i / s_min);
    double d = x - 1.0;
    if (!(d > 0.0)) { *mJ = 0.0; *mJ2 = 0.0; return; }
    if (d < 0.1) {
        double j1 = 0.0, j2 = 0.0, dn = d, H = 1.0, sgn = 1.0;
        for (int nn = 1; nn <= 40; nn++) {            /* d^n, (-1)^(n+1) */
            j1 += sgn * dn / (double)(nn + 1);
            if (nn >= 2) j2 += sgn * (1.0 - H) * dn / (double)(nn + 1);
            dn *= d;
            sgn = -sgn;
            H += 1.0 / (double)(nn + 1);
        }
        *mJ = 2.0 * j1;
        *mJ2 = 8.0 * j2;
        return;
    }
    double L = log1p(d);                              /* ln x */
    *mJ = 2.0 * (1.0 - L / d);
    *mJ2 = 4.0 * (2.0 * x - L * L - 2.0 * L - 2.0) / d;
}

/* ------------------------------------------------------------------------ */
/* Gas background at (R, Z) (Sect. 2.2) and the Stokes number (Sect. 2.3.1).*/
/* ------------------------------------------------------------------------ */
typedef struct { double OmK, hg, Hg, cs, r, rhog, eta, vgphi, stfac; } orc_gas;

static void gas_at(const orc_problem* P, double R, double Z, orc_gas* g)
{
    double r = sqrt(R * R + Z * Z);
    double xr = R / P->R0;
    g->r = r;
    g->OmK = sqrt(P->GM / (R * R * R));
    g->hg = P->h_g0 * pow(xr, (P->q + 1.0) * 0.5);
    g->Hg = g->hg * R;
    g->cs = g->Hg * g->OmK;
    double hg2 = g->hg * g->hg;
    double w = 1.0 - R / r;
    double Sig = P->Sigma_g0 * pow(xr, P->p);
    g->rhog = Sig / (sqrt(2.0 * ORC_PI) * g->Hg) * exp(-w / hg2);
    g->eta = -0.5 * ((P->p + 0.5 * P->q - 1.5) * hg2 + P->q * w);
    g->vgphi = sqrt(1.0 - 2.0 * g->eta) * g->OmK * R;
    /* St(R, Z, s) = St0 (s/s0) (R/R0)^-p exp((1 - R/r)/h_g^2); stfac = St/s */
    g->stfac = P->St0 / P->s0 * pow(xr, -P->p) * exp(w / hg2);
}

static double grain_size(const orc_problem* P, double m)
{
    return cbrt(6.0 * m / (ORC_PI * P->rho_s));   /* m = pi rho s^3 / 6, s = diameter */
}

/* Turbulent relative velocity squared, Ormel & Cuzzi (2007) closed forms:
 * tightly coupled (St1 < Re^-1/2), intermediate (Re^-1/2 <= St1 < 1) with
 * y_a = 1.6, heavy (St1 >= 1).  St1 >= St2, dSt = St1 - St2 >= 0.
 * Sect. 2.5.2 names a six-branch piecewise form of these expressions as
 * implemented in another code, which it does not print; the three published
 * limits used here are the reading, with hard switches at the thresholds
 * (equal grains jump from 0 to about 1.97 V_g^2 St at St = Re^-1/2).
 * The tightly coupled form
 *   Vg^2 (St1 - St2)/(St1 + St2) [St1^2/(St1 + t) - St2^2/(St2 + t)]
 * is evaluated as the algebraically equal
 *   Vg^2 dSt^2 [St1 St2 + t (St1 + St2)] / [(St1 + St2)(St1 + t)(St2 + t)],
 * which does not cancel when St1 and St2 are close. */
static double oc07_dv2(double St1, double St2, double dSt, double Vg2, double tke)
{
    if (St1 < tke) {
        double num = St1 * St2 + tke * (St1 + St2);
        double den = (St1 + St2) * (St1 + tke) * (St2 + tke);
        return Vg2 * (dSt * dSt) * num / den;
    }
    if (St1 < 1.0) {
        const double ya = 1.6;
        double e = St2 / St1;
        double br = 2.0 * ya - (1.0 + e) + 2.0 / (1.0 + e) * (1.0 / (1.0 + ya) + e * e * e / (ya + e));
        return Vg2 * br * St1;
    }
    return Vg2 * (1.0 / (1.0 + St1) + 1.0 / (1.0 + St2));
}

/* ------------------------------------------------------------------------ */
/* Per-query context: everything of the rate that depends on i only.       */
/* ------------------------------------------------------------------------ */
typedef struct {
    double V;           /* sampling measure V_i */
    orc_gas g;
    double R, Z;        /* cylindrical position of the query */
    double Vg2, tke, kT8pi;
} orc_qctx;

static void query_ctx(const orc_problem* P, double xi, double yi, double zi, double di, orc_qctx* c)
{
    memset(c, 0, sizeof(*c));
    if (P->kernel != ORC_PHYSICAL) { c->V = 1.0; return; }   /* V_i = 1 (Sect. 3.3) */
    double R = sqrt(xi * xi + yi * yi);
    gas_at(P, R, zi, &c->g);
    c->R = R;
    c->Z = zi;
    /* V_i = 4 pi d_i^3 / 3 (Sect. 2.5.1), minus the caps of the ball beyond
     * each spherical boundary closer than d_i, each boundary taken as a
     * plane at its distance delta: cap = pi h^2 (3 d - h)/3, h = d - delta. */
    double V = 4.0 * ORC_PI * di * di * di / 3.0;
    if (P->caps) {
        double r = c->g.r;
        double deltas[2] = { r - P->r_in, P->r_out - r };
        for (int b = 0; b < 2; b++) {
            double de = deltas[b];
            if (de < di) {
                double h = di - de;
                V = V - ORC_PI * h * h * (3.0 * di - h) / 3.0;
            }
        }
    }
    c->V = V;
    c->Vg2 = 1.5 * P->alpha * c->g.cs * c->g.cs;
    /* Re = alpha c_s H_g / nu_mol, nu_mol = v_th lambda_mfp / 2,
     * v_th = sqrt(8/pi) c_s, lambda_mfp = mu m_H / (rho_g sigma_H2). */
    double vth = sqrt(8.0 / ORC_PI) * c->g.cs;
    double lmfp = P->mu_mH / (c->g.rhog * P->sigma_H2);
    double numol = 0.5 * vth * lmfp;
    double Re = P->alpha * c->g.cs * c->g.Hg / numol;
    c->tke = 1.0 / sqrt(Re);
    c->kT8pi = 8.0 * (P->mu_mH * c->g.cs * c->g.cs) / ORC_PI;   /* 8 k_B T / pi */
}

/* ------------------------------------------------------------------------ */
/* One pair: the rate lambda_ij (eq:rate or its dimensionless form, Sect.  */
/* 3.3) and its outcome channels (Sect. 2.5.2).  Channel order:            */
/*   sticking:      [stick]                 rate lambda/Ng                   */
/*   erosion:       [remnant, debris]       (1-psi) lambda/Ng, psi lambda     */
/*   fragmentation: [fragment]              lambda                           */
/* Also <J> and <J^2> of each channel (Sect. 2.5.3).                        */
/* ------------------------------------------------------------------------ */
enum { OUT_STICK = 0, OUT_EROSION = 1, OUT_FRAG = 2 };

typedef struct {
    int type;            /* OUT_* */
    int nch;
    double rate[2];      /* channel rates lambda*_{ij,o} */
    double lam_star;     /* sum of channel rates */
    double J[2], J2[2];  /* <J>, <J^2> per channel */
    double Ng;
    double tie;          /* smallest relative margin of a threshold decision */
} orc_pair;

static void pair_eval(const orc_problem* P, const orc_qctx* c, double mi, double mj, double Mj,
                      int want_moments, orc_pair* o)
{
    double lam;
    double dv = 0.0;
    double tie = INFINITY;
    double si = 0.0, sj = 0.0;
    if (P->kernel == ORC_PHYSICAL) {
        si = grain_size(P, mi);
        sj = grain_size(P, mj);
        double Sti = c->g.stfac * si;
        double Stj = c->g.stfac * sj;          /* = St_i s_j/s_i at the query position */
        /* St_i - St_j from the mass difference: s_i - s_j = (6/(pi rho)) (m_i - m_j)/(s_i^2 + s_i s_j + s_j^2),
         * so nearly equal grains do not cancel */
        double ds = (6.0 / (ORC_PI * P->rho_s)) * (mi - mj) / (si * si + si * sj + sj * sj);
        double dSt = c->g.stfac * ds;
        double OR = c->g.OmK;
        double Rq = c->R;
        double qi = 1.0 + Sti * Sti, qj = 1.0 + Stj * Stj;
        /* St_i/(1+St_i^2) - St_j/(1+St_j^2) and 1/(1+St_i^2) - 1/(1+St_j^2), factored through dSt */
        double da = dSt * (1.0 - Sti * Stj) / (qi * qj);
        double db = -dSt * (Sti + Stj) / (qi * qj);
        double dvR = 2.0 * c->g.eta * Rq * OR * da;
        double zi = fmin(Sti, 0.5), zj = fmin(Stj, 0.5);
        double dz = (Sti < 0.5 && Stj < 0.5) ? dSt : zi - zj;
        double dvZ = c->Z * OR * dz;
        double dvP = c->g.eta * Rq * OR * db;
        double dvB = 0.0, dvT2 = 0.0;
        if (P->brownian) {
            dvB = sqrt(c->kT8pi * (1.0 / mi + 1.0 / mj));
            if (dvB > c->g.cs) dvB = c->g.cs;
        }
        if (P->turbulence) {
            double St1 = Sti >= Stj ? Sti : Stj, St2 = Sti >= Stj ? Stj : Sti;
            dvT2 = oc07_dv2(St1, St2, fabs(dSt), c->Vg2, c->tke);
        }
        double dv2 = dvR * dvR + dvZ * dvZ;
        dv2 = dv2 + dvP * dvP;
        dv2 = dv2 + dvB * dvB;
        dv2 = dv2 + dvT2;
        dv = sqrt(dv2);
        double Nj = Mj / mj;
        double ssum = si + sj;
        double K = ORC_PI * ssum * ssum * dv / 4.0;            /* eq:kernel */
        lam = Nj * K / c->V;                                   /* eq:rate */
        if (!(c->V > 0.0)) lam = 0.0;
    } else {
        /* lambda_ij = (1/t0) (1/N_K) (m0/m_j) K_ij (Sect. 3.3, App. A kernels) */
        double Kt;
        if (P->kernel == ORC_CONST) Kt = 1.0;
        else if (P->kernel == ORC_ADDITIVE) Kt = (mi + mj) / P->m0;
        else Kt = (mi * mj) / (P->m0 * P->m0);
        lam = ((P->m0 / mj) * Kt) / (P->t0 * (double)P->k);
    }
    double psi = mj / mi;
    int fast = (P->kernel == ORC_PHYSICAL) && (dv >= P->v_frag);
    if (P->kernel == ORC_PHYSICAL) {
        double mg = fabs(dv - P->v_frag) / P->v_frag;
        if (mg < tie) tie = mg;
    }
    double Ng = 1.0;
    if (P->grouping) {
        double mg = fabs(psi - 1e-6) / 1e-6;
        if (mg < tie) tie = mg;
        if (psi <= 1e-6) {
            double g = 1e-4 / psi;
            Ng = floor(g);
            double fr = g - Ng;
            double mg2 = fmin(fr, 1.0 - fr) / g;
            if (mg2 < tie) tie = mg2;
        }
    }
    o->Ng = Ng;
    if (!fast) {
        o->type = OUT_STICK; o->nch = 1;
        o->rate[0] = lam / Ng;
        o->lam_star = o->rate[0];
        if (want_moments) {
            double J = log1p(Ng * psi) / 3.0;
            o->J[0] = J; o->J2[0] = J * J;
        }
    } else {
        if (P->erosion) {
            double mg = fabs(psi - 0.1) / 0.1;
            if (mg < tie) tie = mg;
        }
        if (P->erosion && psi <= 0.1) {
            o->type = OUT_EROSION; o->nch = 2;
            o->rate[0] = (1.0 - psi) * lam / Ng;
            o->rate[1] = psi * lam;
            o->lam_star = o->rate[0] + o->rate[1];
            if (want_moments) {
                double Jr = -log1p(-Ng * psi) / 3.0;
                double Jd = fabs(log(psi)) / 3.0;
                o->J[0] = Jr; o->J2[0] = Jr * Jr;
                o->J[1] = Jd; o->J2[1] = Jd * Jd;
            }
        } else {
            o->type = OUT_FRAG; o->nch = 1;
            o->rate[0] = lam;
            o->lam_star = lam;
            if (want_moments) orc_frag_moments(si, P->s_min, &o->J[0], &o->J2[0]);
        }
    }
    o->tie = tie;
}

/* ------------------------------------------------------------------------ */
/* Rates over the frozen neighbourhood (Sect. 2.5.1, 2.5.3).                */
/* Neighbour properties m_j, M_j come from the snapshot taken at interval   */
/* start; the self slot uses the frozen copy of particle i too.  Slots with */
/* cnt <= 1 (no other neighbour) give zero rates.                           */
/* lambda*_i = sum over slots (in slot order) of lambda*_ij;                */
/* a_i = sum_j sum_o lambda*_o <J_o>, b_i = sum_j sum_o lambda*_o <J_o^2>.   */
/* ------------------------------------------------------------------------ */
void orc_rates(const orc_problem* P, int64_t n, int64_t nq, const int64_t* qidx,
               const int32_t* nbr, const int32_t* cnt,
               const double* dmax, const double* m_snap, const double* M,
               const double* x, const double* y, const double* z,
               double* lam_out, double* a_out, double* b_out, double* lam_pair_out)
{
    const int k = P->k;
    (void)n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < nq; t++) {
        const int64_t i = qidx ? qidx[t] : t;   /* query slot; outputs at row t */
        double* lam_pair = lam_pair_out ? lam_pair_out + t * k - i * k : NULL;
        double* lam_i = lam_out + t - i;
        double* a_i = a_out + t - i;
        double* b_i = b_out + t - i;
        if (lam_pair) for (int s = 0; s < k; s++) lam_pair[i * k + s] = 0.0;
        double li = 0.0;
        orc_xsum sa, sb; xsum_init(&sa); xsum_init(&sb);
        if (cnt[i] > 1) {
            orc_qctx c;
            query_ctx(P, x[i], y[i], z[i], dmax[i], &c);
            double mi = m_snap[i];
            for (int s = 0; s < cnt[i]; s++) {
                int32_t j = nbr[i * k + s];
                orc_pair o;
                pair_eval(P, &c, mi, m_snap[j], M[j], 1, &o);
                li = li + o.lam_star;
                if (lam_pair) lam_pair[i * k + s] = o.lam_star;
                for (int ch = 0; ch < o.nch; ch++) {
                    xsum_add(&sa, o.rate[ch] * o.J[ch]);
                    xsum_add(&sb, o.rate[ch] * o.J2[ch]);
                }
            }
        }
        lam_i[i] = li;
        a_i[i] = xsum_value(&sa);
        b_i[i] = xsum_value(&sb);
    }
}

/* ------------------------------------------------------------------------ */
/* Controller bins and the interval plan (Sect. 2.5.3).                     */
/* Bin of particle i: ilogb(m_i) clamped to [-64, 63] (factor-2 mass bins); */
/* adjacent non-empty bins are merged in ascending order until each holds   */
/* >= nbin_min particles; a short last group joins the one before it.       */
/* A_b = sum M a / sum M, B_b = sum M b / sum M.                            */
/* dt_req = min(dt_remain, dt_fn_max, min eps C/A_b, min (eps C)^2/B_b),    */
/* terms with a zero denominator omitted.  The collision step holds 2^30    */
/* ticks; the executed interval is the largest aligned dyadic fraction      */
/* dt_coll 2^-n (n <= 30) not above dt_req (halving the step).              */
/* ------------------------------------------------------------------------ */
#define ORC_NBIN 128
#define ORC_BIN_OFF 64
#define ORC_T (1LL << 30)

int32_t orc_bin_of(double m)
{
    int b = ilogb(m);
    if (b < -ORC_BIN_OFF) b = -ORC_BIN_OFF;
    if (b > ORC_NBIN - 1 - ORC_BIN_OFF) b = ORC_NBIN - 1 - ORC_BIN_OFF;
    return b + ORC_BIN_OFF;
}

/* group_of[raw bin] = merged group index or -1; returns number of groups */
static int merge_bins(const int64_t* count, int32_t nbin_min, int32_t* group_of)
{
    int ng = 0;
    int64_t acc = 0;
    int open = 0;
    for (int b = 0; b < ORC_NBIN; b++) {
        group_of[b] = -1;
        if (count[b] == 0) continue;
        if (!open) { open = 1; acc = 0; }
        group_of[b] = ng;
        acc += count[b];
        if (acc >= nbin_min) { ng++; open = 0; }
    }
    if (open) {
        if (ng > 0) {
            for (int b = 0; b < ORC_NBIN; b++) if (group_of[b] == ng) group_of[b] = ng - 1;
        } else {
            ng = 1;
        }
    }
    return ng;
}

/* out[0] = dt_req, out[1] = dt_exe, out[2] = relative margin of the dyadic
 * decision; exe_ticks[0] = ticks of the executed interval;
 * group_of[ORC_NBIN] = merge map; gM[ORC_NBIN] = sum M per group. */
void orc_plan(const orc_problem* P, int64_t n, const double* m_snap, const double* M,
              const double* a_i, const double* b_i, double dt_coll, int64_t ticks, double C,
              double* out, int64_t* exe_ticks, int32_t* group_of, double* gM)
{
    int64_t count[ORC_NBIN];
    memset(count, 0, sizeof(count));
    for (int64_t i = 0; i < n; i++) if (M[i] > 0.0) count[orc_bin_of(m_snap[i])]++;
    int ng = merge_bins(count, P->nbin_min, group_of);
    double A[ORC_NBIN], B[ORC_NBIN];
    for (int g = 0; g < ng; g++) {
        orc_xsum sm, sa, sb; xsum_init(&sm); xsum_init(&sa); xsum_init(&sb);
        for (int64_t i = 0; i < n; i++) {
            if (!(M[i] > 0.0)) continue;
            if (group_of[orc_bin_of(m_snap[i])] != g) continue;
            xsum_add(&sm, M[i]);
            xsum_add(&sa, M[i] * a_i[i]);
            xsum_add(&sb, M[i] * b_i[i]);
        }
        double SM = xsum_value(&sm);
        gM[g] = SM;
        A[g] = SM > 0.0 ? xsum_value(&sa) / SM : 0.0;
        B[g] = SM > 0.0 ? xsum_value(&sb) / SM : 0.0;
    }
    for (int g = ng; g < ORC_NBIN; g++) gM[g] = 0.0;
    double tick = ldexp(dt_coll, -30);
    double rem = (double)(ORC_T - ticks) * tick;
    double req = rem;
    if (P->dt_fn_max < req) req = P->dt_fn_max;
    double eC = P->eps * C;
    for (int g = 0; g < ng; g++) {
        if (A[g] > 0.0) { double t = eC / A[g]; if (t < req) req = t; }
        if (B[g] > 0.0) { double t = (eC * eC) / B[g]; if (t < req) req = t; }
    }
    int nh = 0;
    int64_t size = ORC_T;
    double margin = INFINITY;
    for (nh = 0; nh <= 30; nh++) {
        size = ORC_T >> nh;
        double len = (double)size * tick;
        if (len <= req && (ticks % size) == 0) break;
    }
    if (nh > 30) { nh = 30; size = 1; }
    /* margins of the two size comparisons that decided nh */
    {
        double len = (double)size * tick;
        double mg = fabs(len - req) / req;
        if (mg < margin) margin = mg;
        if (nh > 0) {
            double len2 = (double)(size * 2) * tick;
            double mg2 = fabs(len2 - req) / req;
            if (mg2 < margin) margin = mg2;
        }
    }
    out[0] = req;
    out[1] = (double)size * tick;
    out[2] = margin;
    exe_ticks[0] = size;
}

/* ------------------------------------------------------------------------ */
/* Monte Carlo sampling over one frozen-neighbour interval (Sect. 2.5.3).   */
/* Particle i evolves alone against its frozen neighbourhood:               */
/*   repeat: U = uniforms(id_i, interval, e);                               */
/*           dt_w = -ln(U_w)/lambda*_i; stop if lambda*_i = 0 or            */
/*           dt_w > dt_exe - t (an event happens iff dt_w <= remaining);     */
/*           t += dt_w; partner = first slot whose inclusive prefix of       */
/*           lambda*_ij exceeds U_p lambda*_i; channel = first channel whose */
/*           cumulative rate exceeds U_c lambda*_ij; apply the outcome;      */
/*           recompute every lambda*_ij from the new m_i; e += 1.            */
/* Outcomes (Sect. 2.5.2): stick m' = m + Ng m_j; erosion remnant           */
/* m' = m - Ng m_j, debris m' = m_j; fragment s' from eq:frag with U_f.     */
/* M_i is kept, so N_i' = M_i/m_i'.  No cap on the number of events.        */
/* near_tie[i] = 1 when any decision margin is <= 1e-12 (relative).        */
/* Event log (optional): per particle up to log_cap entries of              */
/* (slot, channel, outcome type).                                            */
/* ------------------------------------------------------------------------ */
void orc_mc(const orc_problem* P, int64_t n, int64_t nq, const int64_t* qidx,
            const uint32_t* id, const int32_t* nbr, const int32_t* cnt,
            const double* dmax, const double* m_snap, const double* M,
            const double* x, const double* y, const double* z,
            double dt_exe, uint64_t seed, uint32_t interval,
            double* m_res, int32_t* ev_res, uint8_t* tie_res,
            int32_t log_cap, int32_t* log_slot_res, int32_t* log_chan_res, int32_t* log_type_res)
{
    const int k = P->k;
    (void)n;
#pragma omp parallel
    {
        double* lam = (double*)malloc(sizeof(double) * (size_t)k);
        double* pre = (double*)malloc(sizeof(double) * (size_t)k);
        orc_pair* pr = (orc_pair*)malloc(sizeof(orc_pair) * (size_t)k);
#pragma omp for schedule(dynamic, 16)
        for (int64_t t_ = 0; t_ < nq; t_++) {
            const int64_t i = qidx ? qidx[t_] : t_;   /* query slot; outputs at row t_ */
            double* m_out = m_res + t_ - i;
            int32_t* n_events = ev_res + t_ - i;
            uint8_t* near_tie = tie_res + t_ - i;
            int32_t* log_slot = log_slot_res ? log_slot_res + (t_ - i) * (int64_t)log_cap : NULL;
            int32_t* log_chan = log_chan_res ? log_chan_res + (t_ - i) * (int64_t)log_cap : NULL;
            int32_t* log_type = log_type_res ? log_type_res + (t_ - i) * (int64_t)log_cap : NULL;
            double m = m_snap[i];
            int32_t e = 0;
            uint8_t tie = 0;
            if (cnt[i] > 1 && M[i] > 0.0) {
                orc_qctx c;
                query_ctx(P, x[i], y[i], z[i], dmax[i], &c);
                int nc = cnt[i];
                double t = 0.0;
                int recompute = 1;
                double li = 0.0;
                for (;;) {
                    if (recompute) {
                        li = 0.0;
                        for (int s = 0; s < nc; s++) {
                            int32_t j = nbr[i * k + s];
                            pair_eval(P, &c, m, m_snap[j], M[j], 0, &pr[s]);
                            if (pr[s].tie <= ORC_TIE) tie = 1;
                            lam[s] = pr[s].lam_star;
                            li = li + lam[s];
                            pre[s] = li;
                        }
                        recompute = 0;
                    }
                    if (!(li > 0.0)) break;
                    double u[4];
                    orc_uniforms(seed, id[i], interval, (uint32_t)e, u);
                    double dtw = -log(u[0]) / li;
                    double rem = dt_exe - t;
                    if (fabs(dtw - rem) <= ORC_TIE * dt_exe) tie = 1;
                    if (dtw > rem) break;
                    t = t + dtw;
                    double target = u[1] * li;
                    int s = 0;
                    while (s < nc - 1 && !(pre[s] > target)) s++;
                    for (int b = 0; b < nc - 1; b++)
                        if (fabs(pre[b] - target) <= ORC_TIE * li) tie = 1;
                    orc_pair* o = &pr[s];
                    int32_t j = nbr[i * k + s];
                    int ch = 0;
                    if (o->nch == 2) {
                        double tc = u[2] * o->lam_star;
                        ch = (o->rate[0] > tc) ? 0 : 1;
                        if (fabs(o->rate[0] - tc) <= ORC_TIE * o->lam_star) tie = 1;
                    }
                    double mj = m_snap[j];
                    double mnew = m;
                    if (o->type == OUT_STICK) {
                        mnew = m + o->Ng * mj;
                    } else if (o->type == OUT_EROSION) {
                        mnew = (ch == 0) ? m - o->Ng * mj : mj;
                    } else {
                        double si = grain_size(P, m);
                        double a = sqrt(P->s_min);
                        double w = a + u[3] * (sqrt(si) - a);
                        double sn = w * w;
                        mnew = ORC_PI * P->rho_s * sn * sn * sn / 6.0;
                    }
                    if (log_cap > 0 && e < log_cap) {
                        log_slot[i * (int64_t)log_cap + e] = s;
                        log_chan[i * (int64_t)log_cap + e] = ch;
                        log_type[i * (int64_t)log_cap + e] = o->type;
                    }
                    e++;
                    if (mnew != m) { m = mnew; recompute = 1; }
                }
            }
            m_out[i] = m;
            n_events[i] = e;
            near_tie[i] = tie;
        }
        free(lam); free(pre); free(pr);
    }
}

/* ------------------------------------------------------------------------ */
/* Post-interval audit of the safety factor C (Sect. 2.5.3; the rule is a   */
/* reading, the paper names only what the audits monitor): per merged bin   */
/* (membership by start-of-interval mass) the mass-weighted mean realised   */
/* |ln(s'/s)| = |ln(m'/m)|/3; if its maximum exceeds 2 eps C, C halves      */
/* (floor 0.25), else C grows by 1.25 (cap 1).                              */
/* out[0] = new C, out[1] = max realised, out[2] = relative margin.         */
/* ------------------------------------------------------------------------ */
void orc_audit(const orc_problem* P, int64_t n, const double* m_snap, const double* m_new,
               const double* M, const int32_t* group_of, const double* gM, double C, double* out)
{
    double worst = 0.0;
    for (int g = 0; g < ORC_NBIN; g++) {
        if (!(gM[g] > 0.0)) continue;
        orc_xsum s; xsum_init(&s);
        for (int64_t i = 0; i < n; i++) {
            if (!(M[i] > 0.0)) continue;
            if (group_of[orc_bin_of(m_snap[i])] != g) continue;
            xsum_add(&s, M[i] * (fabs(log(m_new[i] / m_snap[i])) / 3.0));
        }
        double r = xsum_value(&s) / gM[g];
        if (r > worst) worst = r;
    }
    double thr = 2.0 * P->eps * C;
    double Cn = (worst > thr) ? fmax(0.25, 0.5 * C) : fmin(1.0, 1.25 * C);
    out[0] = Cn;
    out[1] = worst;
    out[2] = fabs(worst - thr) / thr;
}

/* ------------------------------------------------------------------------ */
/* Local vertical column push (Sect. 2.3.3 in the local limit: Omega = H =  */
/* 1, gas at rest, gravity -z, St proportional to 1/rho_g = exp(z^2/2)).    */
/* Drift-kick-drift; the kick integrates drag exactly for the force held at */
/* the drifted position:                                                    */
/*   z* = z + v dt/2;  t_s = St_mid exp(z*^2/2);  E = exp(-dt/t_s),          */
/*   G = -expm1(-dt/t_s);  v' = v E + (-z*) t_s G;  z' = z* + v' dt/2.       */
/* ------------------------------------------------------------------------ */
void orc_push_local(int64_t n, double* z, double* vz, const double* st_mid, const double* M, double dt)
{
    double h = 0.5 * dt;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        if (!(M[i] > 0.0)) continue;
        double zs = z[i] + vz[i] * h;
        double ts = st_mid[i] * exp(0.5 * (zs * zs));
        double r = dt / ts;
        double E = exp(-r);
        double G = -expm1(-r);
        double v = vz[i] * E + (-zs) * ts * G;
        vz[i] = v;
        z[i] = zs + v * h;
    }
}

/* ------------------------------------------------------------------------ */
/* Global staggered semi-analytic push (Sect. 2.3.3).  y = (v_r, l_th, l_ph)*/
/* obeys dy/dt = -y/t_s + y_g/t_s + f with f_r = -GM/r^2 + l_th^2/r^3 +     */
/* l_ph^2/(r^3 sin^2 th), f_th = l_ph^2 cos th/(r^2 sin^3 th), f_ph = 0 and  */
/* y_g = (0, 0, v_g,phi R).  Step (a reading; the paper cites the method    */
/* without printing its steps): drift dt/2 at fixed y, kick dt with drag     */
/* integrated exactly for f held at the drifted position (its l-terms taken */
/* at a half-kick predictor), drift dt/2.  The drift at fixed y is exact:   */
/*   r(t) = r0 + v_r t,  u = t/(r0 r(t)),  th = th0 + l_th u,                */
/*   ph = ph0 + l_ph sin(l_th u)/(l_th sin th0 sin th).                     */
/* Particles leaving [r_in, r_out] become inactive (M = 0).                  */
/* ------------------------------------------------------------------------ */
static double sinc_(double a)
{
    if (fabs(a) < 1e-4) return 1.0 - a * a / 6.0;
    return sin(a) / a;
}

static void drift_fixed_y(double* r, double* th, double* ph, double vr, double lth, double lph, double tau)
{
    double r0 = *r, th0 = *th;
    double r1 = r0 + vr * tau;
    double u = tau / (r0 * r1);
    double a = lth * u;
    double th1 = th0 + a;
    double ph1 = *ph + lph * u * sinc_(a) / (sin(th0) * sin(th1));
    *r = r1; *th = th1; *ph = ph1;
}

static void forces(double GM, double r, double th, double lth, double lph, double* fr, double* fth)
{
    double st = sin(th), ct = cos(th);
    double r2 = r * r, r3 = r2 * r;
    *fr = -GM / r2 + lth * lth / r3 + lph * lph / (r3 * (st * st));
    *fth = lph * lph * ct / (r2 * (st * st * st));
}

void orc_push_global(const orc_problem* P, int64_t n, double* r, double* th, double* ph,
                     double* vr, double* lth, double* lph, const double* m, double* M,
                     double* x, double* y, double* z, double dt)
{
    double h = 0.5 * dt;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        if (!(M[i] > 0.0)) continue;
        double ri = r[i], ti = th[i], pi_ = ph[i];
        double y0 = vr[i], y1 = lth[i], y2 = lph[i];
        drift_fixed_y(&ri, &ti, &pi_, y0, y1, y2, h);
        double fr0, ft0;
        forces(P->GM, ri, ti, y1, y2, &fr0, &ft0);
        double n0, n1, n2;
        if (P->drag) {
            double R = ri * sin(ti), Z = ri * cos(ti);
            orc_gas g;
            gas_at(P, R, Z, &g);
            double s = grain_size(P, m[i]);
            double ts = g.stfac * s / g.OmK;
            double lg = g.vgphi * R;
            double rh = h / ts, rf = dt / ts;
            double Eh = exp(-rh), Gh = -expm1(-rh);
            double E = exp(-rf), G = -expm1(-rf);
            double p1 = y1 * Eh + (ft0 * ts) * Gh;
            double p2 = y2 * Eh + lg * Gh;
            double fr1, ft1;
            forces(P->GM, ri, ti, p1, p2, &fr1, &ft1);
            n0 = y0 * E + (fr1 * ts) * G;
            n1 = y1 * E + (ft1 * ts) * G;
            n2 = y2 * E + lg * G;
        } else {
            double p1 = y1 + ft0 * h;
            double p2 = y2;
            double fr1, ft1;
            forces(P->GM, ri, ti, p1, p2, &fr1, &ft1);
            n0 = y0 + fr1 * dt;
            n1 = y1 + ft1 * dt;
            n2 = y2;
        }
        drift_fixed_y(&ri, &ti, &pi_, n0, n1, n2, h);
        r[i] = ri; th[i] = ti; ph[i] = pi_;
        vr[i] = n0; lth[i] = n1; lph[i] = n2;
        double st = sin(ti);
        x[i] = ri * st * cos(pi_);
        y[i] = ri * st * sin(pi_);
        z[i] = ri * cos(ti);
        if (ri < P->r_in || ri > P->r_out) M[i] = 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* Dust diffusion (Sect. 2.4).  Diagonal tensor in the cylindrical basis,   */
/* D_a = nu / (Sc_a (1 + St^2)) with nu = alpha c_s H_g (Sect. 2.2), and    */
/* one Euler--Maruyama step per call:                                        */
/*   dR   = sqrt(2 D_R dt) z_R + (D_R/R + dD_R/dR + chi D_R dln rho_g/dR) dt */
/*   dZ   = sqrt(2 D_Z dt) z_Z + (dD_Z/dZ + chi D_Z dln rho_g/dZ) dt        */
/*   dphi = sqrt(2 D_phi dt) z_phi / R                                      */
/* (the azimuthal gradients vanish for the axisymmetric gas disk).  A       */
/* vertically integrated model takes Sigma_g for rho_g, the midplane Stokes */
/* number and no vertical step; an axisymmetric one no azimuthal step.      */
/* ------------------------------------------------------------------------ */
typedef struct {
    double D[3];        /* D_R, D_Z, D_phi */
    double dDR_dR;      /* dD_R/dR */
    double dDZ_dZ;      /* dD_Z/dZ */
    double dlnrho[2];   /* d ln rho_g / dR, d ln rho_g / dZ (Sigma_g when vint) */
    double lnrho;       /* ln rho_g (ln Sigma_g when vint), for the tests */
} orc_diffco;

/* Coefficients at cylindrical (R, Z) for a grain of diameter s.
 * With x = R/R0: h_g^2 = h_g0^2 x^(q+1), so nu = alpha h_g^2 R^2 Omega_K is
 * proportional to R^(q + 3/2) and independent of Z.  With w = 1 - R/r,
 * St = St0 (s/s0) x^-p exp(w/h_g^2) and rho_g = Sigma_g/(sqrt(2 pi) H_g) exp(-w/h_g^2):
 *   d(w/h^2)/dR = (-Z^2/r^3 - w (q+1)/R)/h^2,   d(w/h^2)/dZ = R Z/(r^3 h^2),
 *   dSt/dR = St (-p/R + d(w/h^2)/dR),           dSt/dZ = St d(w/h^2)/dZ,
 *   dln rho_g/dR = (p - (q+3)/2)/R - d(w/h^2)/dR,  dln rho_g/dZ = -d(w/h^2)/dZ,
 * and in a vertically integrated model ln Sigma_g has dR-derivative p/R.
 * D_a derivatives by the quotient rule on nu/(Sc (1 + St^2)). */
static void diff_coeffs(const orc_problem* P, double R, double Z, double s, orc_diffco* c)
{
    double Zg = P->vint ? 0.0 : Z;
    orc_gas g;
    gas_at(P, R, Zg, &g);
    double nu = P->alpha * g.cs * g.Hg;
    double dnu_dR = nu * (P->q + 1.5) / R;
    double hg2 = g.hg * g.hg;
    double r = g.r;
    double w = 1.0 - R / r;
    double gR = (-(Zg * Zg) / (r * r * r) - w * (P->q + 1.0) / R) / hg2;
    double gZ = R * Zg / (r * r * r * hg2);
    double St, dSt_dR, dSt_dZ;
    if (P->St_diff > 0.0) {
        St = P->St_diff;
        dSt_dR = 0.0;
        dSt_dZ = 0.0;
    } else {
        St = g.stfac * s;
        dSt_dR = St * (-P->p / R + gR);
        dSt_dZ = St * gZ;
    }
    double den = 1.0 + St * St;
    for (int a = 0; a < 3; a++) c->D[a] = nu / (P->Sc[a] * den);
    /* d/dx [nu/(Sc (1 + St^2))] = [nu' (1 + St^2) - nu 2 St St'] / (Sc (1 + St^2)^2) */
    c->dDR_dR = (dnu_dR * den - nu * 2.0 * St * dSt_dR) / (P->Sc[0] * den * den);
    c->dDZ_dZ = -(nu * 2.0 * St * dSt_dZ) / (P->Sc[1] * den * den);   /* nu is independent of Z */
    if (P->vint) {
        c->dlnrho[0] = P->p / R;
        c->dlnrho[1] = 0.0;
        c->lnrho = log(P->Sigma_g0 * pow(R / P->R0, P->p));
    } else {
        c->dlnrho[0] = (P->p - 0.5 * (P->q + 3.0)) / R - gR;
        c->dlnrho[1] = -gZ;
        c->lnrho = log(g.rhog);
    }
}

void orc_diff_coeffs(const orc_problem* P, double R, double Z, double s, double* out)
{
    orc_diffco c;
    diff_coeffs(P, R, Z, s, &c);
    out[0] = c.D[0]; out[1] = c.D[1]; out[2] = c.D[2];
    out[3] = c.dDR_dR; out[4] = c.dDZ_dZ;
    out[5] = c.dlnrho[0]; out[6] = c.dlnrho[1]; out[7] = c.lnrho;
}

/* Three standard normals of particle `id` in diffusion step `step`: two     */
/* generator calls with counters (id, step, 0x44494646, w), w = 0, 1, key =  */
/* the seed words; each call gives u1 = (a + 1) 2^-53 in (0, 1] and          */
/* u2 = b 2^-53 in [0, 1), and the Box--Muller transform (Box & Muller 1958) */
/* sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2).  z_R, z_Z are the first pair,  */
/* z_phi the cosine of the second.                                           */
void orc_diff_normals(uint64_t seed, uint32_t id, uint32_t step, double zeta[3])
{
    const double two53 = 1.0 / 9007199254740992.0;
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    double pair[4];
    for (uint32_t w = 0; w < 2; w++) {
        uint32_t c[4] = { id, step, 0x44494646u, w }, o[4];
        orc_philox4x32_10(c, key, o);
        uint64_t a = ((((uint64_t)o[1]) << 32) | o[0]) >> 11;
        uint64_t b = ((((uint64_t)o[3]) << 32) | o[2]) >> 11;
        double u1 = (double)(a + 1) * two53;
        double u2 = (double)b * two53;
        double rad = sqrt(-2.0 * log(u1));
        pair[2 * w] = rad * cos(2.0 * ORC_PI * u2);
        pair[2 * w + 1] = rad * sin(2.0 * ORC_PI * u2);
    }
    zeta[0] = pair[0];
    zeta[1] = pair[1];
    zeta[2] = pair[2];
}

/* One diffusion step of length dt on the spherical state.  The Cartesian    */
/* velocity is kept: it is formed at the old position and projected on the   */
/* spherical basis at the new one (v_r, l_theta = r v_theta,                 */
/* l_phi = R v_phi).  A radial step past the axis (R' < 0) is the same       */
/* Cartesian displacement: R' -> -R', phi' -> phi' + pi.  Particles leaving  */
/* r_in <= r <= r_out are deactivated (M = 0), as in the push.               */
void orc_diffuse(const orc_problem* P, int64_t n, const uint32_t* id, double* r, double* th, double* ph,
                 double* vr, double* lth, double* lph, const double* m, double* M,
                 double* x, double* y, double* z, double dt, uint64_t seed, uint32_t step)
{
    double chi = P->diffusion == 1 ? 1.0 : 0.0;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        if (!(M[i] > 0.0)) continue;
        double r0 = r[i], t0 = th[i], p0 = ph[i];
        double R = r0 * sin(t0), Z = r0 * cos(t0);
        double s = P->St_diff > 0.0 ? 0.0 : grain_size(P, m[i]);
        orc_diffco c;
        diff_coeffs(P, R, Z, s, &c);
        double zeta[3];
        orc_diff_normals(seed, id[i], step, zeta);
        double dR = sqrt(2.0 * c.D[0] * dt) * zeta[0]
                  + (c.D[0] / R + c.dDR_dR + chi * c.D[0] * c.dlnrho[0]) * dt;
        double dZ = 0.0, dphi = 0.0;
        if (!P->vint)
            dZ = sqrt(2.0 * c.D[1] * dt) * zeta[1] + (c.dDZ_dZ + chi * c.D[1] * c.dlnrho[1]) * dt;
        if (!P->axisym)
            dphi = sqrt(2.0 * c.D[2] * dt) * zeta[2] / R;
        /* Cartesian velocity at the old position */
        double st0 = sin(t0), ct0 = cos(t0), sp0 = sin(p0), cp0 = cos(p0);
        double v_r = vr[i], v_t = lth[i] / r0, v_p = lph[i] / R;
        double vx = v_r * st0 * cp0 + v_t * ct0 * cp0 - v_p * sp0;
        double vy = v_r * st0 * sp0 + v_t * ct0 * sp0 + v_p * cp0;
        double vz = v_r * ct0 - v_t * st0;
        /* new position */
        double R1 = R + dR, Z1 = Z + dZ, p1 = p0 + dphi;
        if (R1 < 0.0) { R1 = -R1; p1 = p1 + ORC_PI; }
        double r1 = sqrt(R1 * R1 + Z1 * Z1);
        double t1 = atan2(R1, Z1);
        double st1 = sin(t1), ct1 = cos(t1), sp1 = sin(p1), cp1 = cos(p1);
        /* projections on the new basis */
        double nvr = vx * st1 * cp1 + vy * st1 * sp1 + vz * ct1;
        double nvt = vx * ct1 * cp1 + vy * ct1 * sp1 - vz * st1;
        double nvp = -vx * sp1 + vy * cp1;
        r[i] = r1; th[i] = t1; ph[i] = p1;
        vr[i] = nvr; lth[i] = r1 * nvt; lph[i] = R1 * nvp;
        x[i] = R1 * cp1;
        y[i] = R1 * sp1;
        z[i] = Z1;
        if (r1 < P->r_in || r1 > P->r_out) M[i] = 0.0;
    }
}

/* The common transport step of Sect. 2.6: dt = min(dt_max, dt_out, min_i dt_i)
 * over the active particles.  The paper names the constraints of dt_i
 * (orbital motion, deterministic and diffusive displacement relative to the
 * local spacing) without their forms; the reading taken (R36):
 *   orbital        c_orb / Omega, Omega = sqrt(GM / R^3) at R = sqrt(x^2 + y^2)
 *                  for the global push, Omega = 1 for the local column;
 *   deterministic  c_adv d_i / u_i, d_i the particle's neighbourhood radius
 *                  (the local spacing of the particle representation) and
 *                  u_i its speed relative to the local circular orbit:
 *                  u^2 = v_r^2 + (l_theta / r)^2 + (l_phi / R - sqrt(GM / R))^2
 *                  (global), u = |v_z| (local column);
 *   diffusive      c_diff d_i^2 / D_i, D_i the largest diffusion coefficient
 *                  of the directions the diffusion step moves (R; Z unless
 *                  vertically integrated; phi unless axisymmetric).
 * A term is left out when it does not apply: no push, no orbital or
 * deterministic term; no diffusion, no diffusive term; d_i = 0 or u_i = 0.
 * push_kind: 0 none, 1 local column, 2 global. */
double orc_transport_dt(const orc_problem* P, int push_kind, int64_t n, const double* x, const double* y,
                        const double* r, const double* th, const double* vr, const double* lth,
                        const double* lph, const double* vz, const double* m, const double* M,
                        const double* d, double dt_max, double dt_out, double c_orb, double c_adv,
                        double c_diff)
{
    double dt = dt_max < dt_out ? dt_max : dt_out;
    for (int64_t i = 0; i < n; i++) {
        if (!(M[i] > 0.0)) continue;
        double di = d[i];
        double t = INFINITY;
        if (push_kind == 2) {
            double R = sqrt(x[i] * x[i] + y[i] * y[i]);
            double Om = sqrt(P->GM / (R * R * R));
            double to = c_orb / Om;
            if (to < t) t = to;
            double vt = lth[i] / r[i];
            double vp = lph[i] / R - sqrt(P->GM / R);
            double u = sqrt(vr[i] * vr[i] + vt * vt + vp * vp);
            if (di > 0.0 && u > 0.0) {
                double ta = c_adv * di / u;
                if (ta < t) t = ta;
            }
        } else if (push_kind == 1) {
            if (c_orb < t) t = c_orb;
            double u = fabs(vz[i]);
            if (di > 0.0 && u > 0.0) {
                double ta = c_adv * di / u;
                if (ta < t) t = ta;
            }
        }
        if (P->diffusion != 0 && di > 0.0) {
            double R = r[i] * sin(th[i]), Z = r[i] * cos(th[i]);
            double s = P->St_diff > 0.0 ? 0.0 : grain_size(P, m[i]);
            orc_diffco c;
            diff_coeffs(P, R, Z, s, &c);
            double D = c.D[0];
            if (!P->vint && c.D[1] > D) D = c.D[1];
            if (!P->axisym && c.D[2] > D) D = c.D[2];
            if (D > 0.0) {
                double tdf = c_diff * (di * di) / D;
                if (tdf < t) t = tdf;
            }
        }
        if (t < dt) dt = t;
    }
    return dt;
}

/* Diagnostics exposed for tests. */
void orc_pair_rate(const orc_problem* P, double xi, double yi, double zi, double di,
                   double mi, double mj, double Mj, double* out)
{
    orc_qctx c;
    query_ctx(P, xi, yi, zi, di, &c);
    orc_pair o;
    pair_eval(P, &c, mi, mj, Mj, 1, &o);
    out[0] = o.lam_star;
    out[1] = (double)o.type;
    out[2] = o.rate[0];
    out[3] = o.nch > 1 ? o.rate[1] : 0.0;
    out[4] = o.Ng;
    out[5] = c.V;
}

void orc_gas_at(const orc_problem* P, double R, double Z, double* out)
{
    orc_gas g;
    gas_at(P, R, Z, &g);
    out[0] = g.OmK; out[1] = g.hg; out[2] = g.Hg; out[3] = g.cs; out[4] = g.r;
    out[5] = g.rhog; out[6] = g.eta; out[7] = g.vgphi; out[8] = g.stfac;
}

double orc_oc07(double St1, double St2, double Vg2, double tke) { return oc07_dv2(St1, St2, St1 - St2, Vg2, tke); }

void orc_set_tie_margin(double eps) { ORC_TIE = eps > 0.0 ? eps : 1e-12; }

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int nt)
{
#ifdef _OPENMP
    if (nt > 0) omp_set_num_threads(nt);
#else
    (void)nt;
#endif
}

/* ------------------------------------------------------------------------ */
/* Neighbour reshuffling of the product-kernel test (Sect. 3.3): before every */
/* refresh the cached neighbour indices of all particles are permuted at     */
/* random, so that the frozen neighbourhoods sample a well-mixed population.  */
/* Reading: slot 0 (the particle itself) is kept; every other cached index j  */
/* becomes pi(j) for one random bijection pi of the N active slots drawn per  */
/* refresh.  pi: a balanced Feistel network (Luby and Rackoff 1988) of four   */
/* rounds on 2h bits, 4^h >= N, the round function being word 0 of Philox     */
/* with counter (right half, round, refresh, 0x52534831) and key = seed,      */
/* restricted to [0, N) by cycle walking (Black and Rogaway 2002): apply the  */
/* network until the value falls below N.                                     */
/* ------------------------------------------------------------------------ */
static uint32_t orc_feistel(uint32_t x, int h, uint64_t seed, uint32_t refresh)
{
    const uint32_t mask = (h >= 32) ? 0xFFFFFFFFu : ((1u << h) - 1u);
    uint32_t L = x >> h, R = x & mask;
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    for (uint32_t t = 0; t < 4; t++) {
        uint32_t c[4] = { R, t, refresh, 0x52534831u }, o[4];
        orc_philox4x32_10(c, key, o);
        uint32_t nL = R;
        uint32_t nR = L ^ (o[0] & mask);
        L = nL;
        R = nR;
    }
    return (L << h) | R;
}

int64_t orc_reshuffle_index(int64_t N, uint64_t seed, uint32_t refresh, int64_t j)
{
    if (N <= 1) return j;
    int bits = 0;
    while ((1LL << bits) < N) bits++;      /* 2^bits >= N */
    int h = (bits + 1) / 2;                /* 4^h >= N */
    uint32_t x = (uint32_t)j;
    do {
        x = orc_feistel(x, h, seed, refresh);
    } while ((int64_t)x >= N);
    return (int64_t)x;
}

void orc_reshuffle(int64_t n, int32_t k, int32_t* nbr, const int32_t* cnt, int64_t N, uint64_t seed,
                   uint32_t refresh)
{
    for (int64_t i = 0; i < n; i++) {
        for (int32_t s = 1; s < cnt[i] && s < k; s++) {
            int32_t* e = &nbr[i * k + s];
            if (*e >= 0 && *e < N) {
                /* the other that pi sends onto i itself takes pi(i) instead, so
                 * the row stays free of i (slot 0 holds it) and of repeats */
                int64_t v = orc_reshuffle_index(N, seed, refresh, *e);
                if (v == i) v = orc_reshuffle_index(N, seed, refresh, i);
                *e = (int32_t)v;
            }
        }
    }
}
