/*
 * gd.h -- C ABI of the MI355X (gfx950) library for the collision hot path of
 * the representative-particle dust model of Bi, "GameDev: GPU-accelerated
 * model for dust evolution" (arXiv 2609.35967).
 *
 * One frozen-neighbour interval of the method is the sequence
 *
 *     gd_build_neighbors -> gd_collision_rates -> gd_sample_collisions -> gd_push
 *
 * (Sect. 2.5.1 neighbourhoods, Sect. 2.5.3 rates/plan/sampling, Sect. 2.3.3
 * push).  All four enqueue work on one HIP stream and return at once.
 *
 * Conventions that hold for every call:
 *  - Ownership: every array pointer in gd_particles, gd_neighbors and
 *    gd_interval, and the workspace, is DEVICE memory owned by the caller.
 *    The library never allocates or frees device memory and keeps no pointer
 *    after a call returns.  Struct arguments themselves are read on the host
 *    during the call only.
 *  - Workspace: every call takes the caller's workspace of at least
 *    gd_workspace_size() bytes, 256-byte aligned; it carries state between the
 *    calls of one interval (Morton keys, tree, controller sums, status word),
 *    so one workspace serves one run at a time.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = default
 *    stream).  Calls on different streams with different workspaces and state
 *    are independent.
 *  - Return value: GD_OK, or a negative gd_status when the arguments are
 *    rejected on the host (nothing is enqueued then) or a HIP launch fails.
 *    Conditions found on the device are latched in the workspace status word
 *    and read with gd_status_read (the only call that synchronises).
 *  - gd_last_error() returns the calling thread's last host-side message.
 *  - Floating point: FP64 throughout.  Positions, separations and the
 *    dimensionless kernels use only +, -, *, / and sqrt, each rounded
 *    separately (no fused multiply-add), so they are reproducible bit for bit.
 */
#ifndef GD_H
#define GD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gd_status {
    GD_OK = 0,
    GD_E_INVALID_ARG = -1,   /* NULL or inconsistent argument */
    GD_E_WORKSPACE = -2,     /* workspace NULL, misaligned or too small */
    GD_E_HIP = -3,           /* a HIP runtime call or launch failed */
    GD_E_NONFINITE = -4,     /* device: non-finite mass or position met */
    GD_E_LOG_OVERFLOW = -5,  /* device: event log truncated (results valid) */
    GD_E_UNSUPPORTED = -6    /* option outside what this build supports */
} gd_status;

/* Device status-word bits (gd_status_read returns their OR). */
#define GD_DEV_NONFINITE 0x1      /* a non-finite input was met */
#define GD_DEV_LOG_OVERFLOW 0x2   /* a particle had more events than log_cap */
#define GD_DEV_KNN_FALLBACK 0x4   /* kNN used its slow exact tie path (info only) */
#define GD_DEV_TICK_FLOOR 0x8     /* dt_req fell below one tick; one tick executed */
#define GD_DEV_MASS_RANGE 0x10    /* a grain mass fell outside the 2^-64..2^64 bin range */
#define GD_DEV_INTERNAL 0x20      /* an internal consistency check failed (bad tree or neighbour index) */
#define GD_DEV_EVENT_CAP 0x40     /* a particle reached 2^24 events in one interval and stopped there */

typedef enum gd_kernel {
    GD_KERNEL_CONST = 0,     /* K = 1                 (App. A, constant kernel) */
    GD_KERNEL_ADDITIVE = 1,  /* K = (m_i + m_j)/m0    (App. A, linear kernel)   */
    GD_KERNEL_PRODUCT = 2,   /* K = m_i m_j / m0^2    (App. A, product kernel)  */
    GD_KERNEL_PHYSICAL = 3   /* K = pi (s_i+s_j)^2 dv/4 (eq:kernel), eq:rate      */
} gd_kernel;

typedef enum gd_push_kind {
    GD_PUSH_NONE = 0,
    GD_PUSH_LOCAL = 1,       /* vertical settling in a local column (Omega = H = 1) */
    GD_PUSH_GLOBAL = 2       /* spherical staggered semi-analytic push (Sect. 2.3.3) */
} gd_push_kind;

typedef enum gd_diffusion_form {
    GD_DIFFUSION_NONE = 0,
    GD_DIFFUSION_CONCENTRATION = 1,  /* acts on rho_d/rho_g (chi = 1, eq:diff_conc) */
    GD_DIFFUSION_DENSITY = 2         /* acts on rho_d (chi = 0, eq:diff_dens) */
} gd_diffusion_form;

/* Problem description (host struct, read during each call). */
typedef struct gd_problem {
    int64_t n;            /* length of every particle array */
    int32_t k;            /* N_K: neighbours per particle including itself, 2..256 */
    int32_t kernel;       /* gd_kernel */
    int32_t push;         /* gd_push_kind */
    int32_t nbin_min;     /* minimum particles per merged controller bin (0: max(2k, 64)) */
    int32_t erosion;      /* 1: erosion outcome for psi <= 0.1 (Sect. 2.5.2) */
    int32_t grouping;     /* 1: group small increments, N_coll = floor(1e-4/psi) */
    int32_t periodic[3];  /* 1: minimum-image separation on that axis */
    double L[3];          /* period of each periodic axis; positions in [0, L) */
    double rmax;          /* maximum search scale (INFINITY: none) */
    double t0, m0;        /* dimensionless kernels: unit time and mass (Sect. 3.3) */
    double eps;           /* tolerance epsilon of the interval controller */
    double dt_fn_max;     /* maximum frozen-neighbour interval */
    double rho_s;         /* grain internal density */
    double s_min;         /* minimum grain diameter of fragments (eq:frag) */
    double v_frag;        /* fragmentation speed: dv >= v_frag is fast (INFINITY: sticking only) */
    double GM;            /* gravitational parameter of the star */
    double Sigma_g0, R0, p, q, h_g0;  /* gas disk (Sect. 2.2) */
    double alpha;         /* turbulence parameter */
    double mu_mH;         /* mean molecular mass (k_B T = mu_mH c_s^2) */
    double sigma_H2;      /* molecular cross section (mean free path) */
    double s0, St0;       /* reference diameter and its Stokes number at R0, midplane */
    double r_in, r_out;   /* spherical domain (boundary caps, outflow) */
    int32_t drag;         /* global push: 1 = gas drag on */
    int32_t brownian;     /* 1: Brownian term in dv (eq:dv) */
    int32_t turbulence;   /* 1: turbulent term in dv (Ormel & Cuzzi 2007) */
    int32_t caps;         /* 1: subtract boundary caps from V_i */
    int32_t rates_fp32;   /* 0: FP64 pair rates (the reference form); 1: pair collision speeds,
                             kernels, channel rates and moments in FP32, summed in FP64 (the
                             context per particle, N_j/V_i, psi and grouping stay FP64) */
    /* dust diffusion (Sect. 2.4), read by gd_diffuse only */
    int32_t diffusion;    /* gd_diffusion_form */
    int32_t vint;         /* 1: vertically integrated disk: Sigma_g stands for rho_g, the
                             midplane Stokes number is used and there is no vertical step */
    int32_t axisym;       /* 1: axisymmetric model: no azimuthal step */
    int32_t pad_;
    double Sc[3];         /* Schmidt numbers of the R, Z and phi directions (> 0; INFINITY: none) */
    double St_diff;       /* > 0: this spatially constant Stokes number in D for every grain
                             (the ring test of Sect. 3.2); 0: the local Stokes number */
} gd_problem;

/* Particle state, structure of arrays, device pointers, length n.
 * id, x, y, z, M and m[0..1] are always required.  r..lph are required for
 * GD_PUSH_GLOBAL, vz and st_mid for GD_PUSH_LOCAL; set unused ones to NULL.
 * M_i <= 0 marks an inactive particle (no neighbours, no events, not pushed).
 * m[cur] is the grain mass of the current interval; m[cur ^ 1] receives the
 * masses after sampling. */
typedef struct gd_particles {
    uint32_t* id;                   /* identity (keys the random streams) */
    double *x, *y, *z;              /* Cartesian positions */
    double *r, *th, *ph;            /* spherical position (global push) */
    double *vr, *lth, *lph;         /* y = (v_r, l_theta, l_phi) (global push) */
    double *vz, *st_mid;            /* local column: v_z and midplane Stokes number */
    double* M;                      /* particle mass M_i = N_i m_i */
    double* m[2];                   /* grain mass, double buffer */
    int32_t cur;                    /* which m buffer is current (0 or 1) */
} gd_particles;

/* Neighbourhoods (Sect. 2.5.1), device pointers, indices are slots of the
 * Morton-ordered state written by gd_build_neighbors. */
typedef struct gd_neighbors {
    int32_t* nbr;       /* [n * k]: row i = i itself, then the retained others in
                           ascending slot order, then -1 padding */
    int32_t* cnt;       /* [n]: 1 + number of retained others (0: inactive) */
    double* dmax;       /* [n]: distance to the farthest retained neighbour (d_i) */
    int32_t* n_active;  /* [1]: active particles; they occupy slots 0..n_active-1 */
} gd_neighbors;

/* Interval state, one struct in DEVICE memory (initialise with
 * gd_interval_init).  The collision step dt_coll holds 2^30 ticks. */
typedef struct gd_interval {
    double dt_coll;       /* collision time step split into intervals */
    double dt_req;        /* requested interval (written by gd_collision_rates) */
    double dt_exe;        /* executed interval (written by gd_collision_rates) */
    double C;             /* adaptive safety factor, 0.25..1 */
    double time;          /* simulated time advanced by executed intervals */
    int64_t ticks;        /* ticks elapsed in the current collision step */
    int64_t exe_ticks;    /* ticks of the planned interval */
    int64_t n_intervals;  /* intervals completed */
    int64_t n_events;     /* collision events in the last sampled interval */
    double audit_worst;   /* largest realised mean |ln(s'/s)| of the last audit */
    int32_t n_groups;     /* merged controller bins of the last plan */
    int32_t pad;
} gd_interval;

/* Bytes of workspace needed for problem p (writes *bytes). */
int32_t gd_workspace_size(const gd_problem* p, size_t* bytes);

/* Prepare a fresh workspace for problem p: clear its device status word and
 * header.  Call once after allocating the workspace (its contents are
 * otherwise undefined); enqueued on `stream`. */
int32_t gd_workspace_init(const gd_problem* p, void* ws, size_t ws_bytes, void* stream);

/* Set *iv (device) to dt_coll, C = 1, zero ticks/time/counters. */
int32_t gd_interval_init(gd_interval* iv, double dt_coll, void* stream);

/* Neighbourhoods (Sect. 2.5.1).  Sorts the active particles of `in` into
 * Morton order (10 bits per axis in the cube spanned by the active particles;
 * stable; inactive last) and writes the permuted copy of EVERY non-NULL array
 * of `in` (and m[in->cur]) into `out` (which must not alias `in`; out->cur is
 * set equal to in->cur).  Then, on the Morton-ordered state, for each active
 * slot i: nbr row = i, then the k-1 nearest other active particles with
 * d^2 <= rmax^2, nearest first by (d^2, slot), written in ascending slot order;
 * d^2 = (dx*dx + dy*dy) + dz*dz with minimum image on periodic axes
 * (d > L/2: d - L; d < -L/2: d + L).  Exact: no approximation in the search.
 * On entry nb->dmax is read as a per-slot search hint in the order of `in`
 * (in a stepping loop it holds the previous call's distances, and `in` is that
 * call's output); any content is allowed and the result never depends on it. */
int32_t gd_build_neighbors(const gd_problem* p, const gd_particles* in, gd_particles* out,
                           const gd_neighbors* nb, void* ws, size_t ws_bytes, void* stream);

/* Rates over the frozen neighbourhood and the interval plan (Sect. 2.5.1-2.5.3).
 * Snapshot = m[st->cur].  Per active particle: lambda*_i (the slot-order sum of
 * the pairs' effective rates) into lam_i [n]; optional per-pair lambda*_ij into
 * lam_pair [n*k] and controller moments a_i, b_i into ab [2n] (a then b).  Then
 * bins of ilogb(m), merged to >= nbin_min particles, A_b, B_b, dt_req and the
 * dyadic executed interval are written into *iv on the device.  The workspace
 * keeps a packed copy of the snapshot (m, grain size, N) for the sampling
 * call that follows. */
int32_t gd_collision_rates(const gd_problem* p, const gd_particles* st, const gd_neighbors* nb,
                           gd_interval* iv, double* lam_i, double* lam_pair, double* ab,
                           void* ws, size_t ws_bytes, void* stream);

/* Monte Carlo sampling over the planned interval (Sect. 2.5.3).  Must follow
 * gd_collision_rates of the same interval on the same workspace: reads the
 * frozen neighbours from the snapshot copy it left there, m[st->cur] (own
 * start state) and lam_i; writes m[st->cur ^ 1] and, if non-NULL, the event count
 * per particle into n_events [n] and a per-particle event log into log
 * [n * log_cap] (entry = slot | channel << 16 | outcome << 24; -1 unused).
 * Random numbers: Philox4x32-10, key = seed, counters (id, interval_index,
 * event, 0 / 1).  Afterwards the safety factor C is audited and the ticks and
 * time advance by the executed interval.  The caller then flips st->cur
 * (the broadcast).  interval_index must be < 2^32, or GD_INTERVAL_ON_DEVICE:
 * the kernels then take iv->n_intervals (the intervals completed, read on the
 * device) as the index, so that a call recorded once in a HIP graph draws
 * fresh numbers on every replay. */
#define GD_INTERVAL_ON_DEVICE UINT64_MAX

/* Neighbour reshuffling of the product-kernel test (Sect. 3.3): before a
 * refresh of the frozen neighbourhoods, the cached neighbour indices of all
 * particles are permuted at random so that they sample a well-mixed
 * population.  Every entry nbr[i*k + s] with 1 <= s < cnt[i] and an index in
 * [0, N), N = *nb->n_active (read on the device), becomes pi(index); slot 0
 * (the particle itself), cnt, dmax and the rest of each row are kept.  pi is
 * one random bijection of [0, N) per (seed, refresh): a four-round balanced
 * Feistel network on two h-bit halves (4^h >= N) with round function word 0
 * of Philox4x32-10, counter (right half, round, refresh, 0x52534831), key =
 * seed, restricted to [0, N) by cycle walking.  The one other of row i
 * that pi sends onto i itself becomes pi(i) instead, so rows stay free of i
 * and of repeats.  In place on the caller's stream.  pi is tabulated in the
 * workspace (the part the neighbour build uses for its sort keys), so the
 * call may sit anywhere outside gd_build_neighbors. */
int32_t gd_reshuffle_neighbors(const gd_problem* p, const gd_neighbors* nb, uint64_t seed, uint32_t refresh,
                               void* ws, size_t ws_bytes, void* stream);

/* Neighbour reshuffling without allocation, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation.  The same operation and the same result as
 * gd_reshuffle_neighbors, with no workspace: pi's table is kept in a fixed
 * device array of GD_RESHUFFLE_STATIC_MAX int32 entries (16 MiB) that the
 * library holds on every GPU it runs on until the process ends.  p->n must be
 * at most GD_RESHUFFLE_STATIC_MAX (GD_E_INVALID_ARG otherwise, before any
 * device work).  The first call on a device, with that device current,
 * resolves the array's address there (GD_E_HIP if that fails).  No call
 * allocates or frees memory.  All calls on one GPU share its array, so calls
 * that overlap on one GPU (other streams, other host threads) race and must
 * be serialised by the caller; each call rewrites the entries it reads, so
 * no clearing is needed between calls.  In place on the caller's stream. */
#define GD_RESHUFFLE_STATIC_MAX (1 << 22)
int32_t gd_reshuffle_neighbors_static(const gd_problem* p, const gd_neighbors* nb, uint64_t seed, uint32_t refresh,
                                      void* stream);

/* Sampling over many independent runs (boxes) at once.  gd_sample_collisions
 * is, in order: the per-lane pass (each particle's first events; a particle
 * with more is recorded in the workspace at that event boundary), the pass
 * that runs the rest of every recorded particle with one wavefront each, and
 * the audit.  The three calls below make the same passes with the second
 * one shared by many runs, so that the recorded particles of every run are
 * sampled in one launch.  Results are those of gd_sample_collisions, bit for
 * bit.
 *
 * The table is device memory owned by the caller, gd_sample_table_size(nslot)
 * bytes (1 <= nslot <= 4096).  Per interval, for each run r in [0, nslot):
 * gd_sample_collisions_deferred(..., table, table_bytes, slot = r, stream_r),
 * which takes gd_sample_collisions' arguments and writes the run's sampling
 * arguments into slot r; then, on one stream ordered after all of them,
 * gd_sample_table_run(table, table_bytes, nslot, k, rates_fp32, stream), where
 * every run's k is at most the k passed here (the launch is shaped for the
 * class of that k: <= 32, <= 64, <= 128 or <= 256) and the same
 * rates_fp32 (a run that differs is skipped and raises GD_DEV_INTERNAL); then
 * gd_sample_audit for each run, after which the caller flips st->cur.  Every
 * slot below nslot must have been written in the same interval: a slot left
 * from an earlier interval would be sampled again.  Calls that overlap on one
 * table race. */
int32_t gd_sample_table_size(int32_t nslot, size_t* bytes);
int32_t gd_sample_collisions_deferred(const gd_problem* p, const gd_particles* st, const gd_neighbors* nb,
                                      gd_interval* iv, const double* lam_i, uint64_t seed,
                                      uint64_t interval_index, int32_t* n_events, int32_t* log,
                                      int32_t log_cap, void* ws, size_t ws_bytes, void* table,
                                      size_t table_bytes, int32_t slot, void* stream);
int32_t gd_sample_table_run(void* table, size_t table_bytes, int32_t nslot, int32_t k, int32_t rates_fp32,
                            void* stream);
int32_t gd_sample_audit(const gd_problem* p, const gd_particles* st, gd_interval* iv, void* ws,
                        size_t ws_bytes, void* stream);
int32_t gd_sample_collisions(const gd_problem* p, const gd_particles* st, const gd_neighbors* nb,
                             gd_interval* iv, const double* lam_i, uint64_t seed,
                             uint64_t interval_index, int32_t* n_events, int32_t* log,
                             int32_t log_cap, void* ws, size_t ws_bytes, void* stream);

/* The common transport step of Sect. 2.6: dt = min(dt_max, dt_out, min_i dt_i)
 * over the active particles.  The paper names dt_i's constraints (orbital
 * motion, deterministic and diffusive displacement against the local
 * spacing) without their forms; the reading taken, with d_i = nb->dmax[i]
 * the particle's neighbourhood radius from the last search:
 *   orbital        c_orb / Omega_K(R) for GD_PUSH_GLOBAL (R = sqrt(x^2 + y^2)),
 *                  c_orb for GD_PUSH_LOCAL (Omega = 1);
 *   deterministic  c_adv d_i / u_i, u_i the speed relative to the local
 *                  circular orbit (v_r, l_th / r, l_ph / R - sqrt(GM / R)), or
 *                  |v_z| in the local column;
 *   diffusive      c_diff d_i^2 / D_i when diffusion is on, D_i the largest
 *                  coefficient nu / (Sc (1 + St^2)) of the directions stepped.
 * A term that does not apply (no push, no diffusion, d_i = 0, u_i = 0) is left
 * out.  The result goes to *dt (one device double).  With iv non-NULL the
 * interval state takes dt_coll = dt / 2 for the step's two collision
 * operators; that is valid only at a collision-step boundary (iv->ticks ==
 * 0), and elsewhere iv is left alone and GD_DEV_INTERNAL is raised.  Uses
 * the workspace's reduction scratch.  Errors: GD_E_INVALID_ARG for NULL
 * arguments, arrays a term needs, or limits that are not positive. */
typedef struct gd_step_limits {
    double dt_max;  /* prescribed maximum step */
    double dt_out;  /* time left to the next output (INFINITY: none) */
    double c_orb, c_adv, c_diff;
} gd_step_limits;

int32_t gd_transport_dt(const gd_problem* p, const gd_particles* st, const gd_neighbors* nb,
                        const gd_step_limits* lim, gd_interval* iv, double* dt, void* ws, size_t ws_bytes,
                        void* stream);

/* Many independent runs stepped as one (Sect. 2.5: the interval of each run
 * is the one gd_build_neighbors, gd_collision_rates, gd_sample_collisions and
 * gd_push make; Sect. 4.3.1: many small independent domains on one device).
 * Every stage of the interval -- bounding box, Morton keys and radix sort,
 * permutation, search tree, neighbour search, snapshot and rates, bin sums and
 * plan, sampling (the per-lane pass, then one pass over the deferred
 * particles of all runs), audit, push -- is one launch over all runs: the
 * runs' blocks follow one another in one grid, and a block finds its run and
 * that run's arguments through tables the library keeps in device memory.
 * A run's results are those of its own calls, bit for bit, except that the
 * bin sums of the plan and the audit are split over a number of blocks that
 * depends on the run's size (their double-double totals round the same in
 * all but contrived cases).
 *
 * gd_run describes one run: its problem, its two state buffers (a holds the
 * current state, b receives the first interval's permutation; the buffers
 * then alternate, so that after an even number of intervals the state is in
 * a again with the same cur), its neighbour arrays, interval state (set up by
 * gd_interval_init), lam_i (n doubles), optional n_events (n int32) and a
 * workspace of gd_workspace_size bytes (initialised).  Sampling draws with
 * the interval index on the device (GD_INTERVAL_ON_DEVICE).  All runs need
 * the same rates_fp32, and k at most 256; runs with push enabled are pushed
 * over their own dt_exe.  Everything is caller-owned and must stay allocated
 * until gd_many_destroy; the library owns only its tables
 * (gd_many_create allocates them with hipMalloc on the current device).
 *
 * gd_many_tuning holds launch shapes only; no choice changes a result:
 *   knn_tile      1: the shared-candidate-tile search first (k <= 33), 0: the
 *                 per-lane search for every query;
 *   fallback_div  wavefronts of the tile search's fallback pass: n / fallback_div per run;
 *   event_div     workgroups of the per-lane sampling pass: n / event_div per run (<= 512);
 *   red_div       workgroups of each bin sum: n / red_div per run (<= 256);
 *   heavy_blocks  workgroups (4 wavefronts each) of the pass over the deferred particles.
 * Zero fields take the defaults (1, 256, 512, 2048, 768).
 *
 * gd_many_interval enqueues one interval of every run on `stream`; the host
 * keeps the parity of the buffers and flips it at each call (two calls can
 * be recorded into a graph and replayed).  gd_many_parity returns it: 0 when
 * each run's state is in a.  Errors: GD_E_INVALID_ARG for a NULL or
 * inconsistent description (message names the run), GD_E_HIP for a failed
 * allocation or launch. */
typedef struct gd_run {
    const gd_problem* p;
    gd_particles* a;
    gd_particles* b;
    const gd_neighbors* nb;
    gd_interval* iv;
    double* lam_i;
    int32_t* n_events;
    void* ws;
    size_t ws_bytes;
    uint64_t seed;
} gd_run;

typedef struct gd_many_tuning {
    int32_t knn_tile;
    int32_t fallback_div;
    int32_t event_div;
    int32_t red_div;
    int32_t heavy_blocks;
} gd_many_tuning;

typedef struct gd_many gd_many;

#define GD_MANY_MAX_RUNS 4096
int32_t gd_many_create(const gd_run* runs, int32_t nrun, const gd_many_tuning* tune, gd_many** out);
int32_t gd_many_interval(gd_many* m, void* stream);
int32_t gd_many_parity(const gd_many* m, int32_t* parity);
int32_t gd_many_destroy(gd_many* m);

/* Push (Sect. 2.3.3) of every active particle over iv->dt_exe (iv non-NULL,
 * read on the device) or over dt (iv NULL).  GD_PUSH_LOCAL: z, vz by
 * drift-kick-drift with exact drag for the force at the drifted position,
 * t_s = st_mid exp(z^2/2).  GD_PUSH_GLOBAL: spherical state and Cartesian
 * x, y, z; the grain size comes from m[st->cur]; particles leaving
 * [r_in, r_out] get M = 0 (inactive). */
int32_t gd_push(const gd_problem* p, const gd_particles* st, const gd_interval* iv, double dt,
                void* ws, size_t ws_bytes, void* stream);

/* Spatial groups (Sect. 2.5.3).  A group is a contiguous range of
 * Morton-ordered active slots; each keeps its own gd_interval (safety factor
 * C, ticks), so that groups run frozen-neighbour intervals of different
 * lengths within one collision step.  During a collision step m[cur] holds the
 * broadcast masses and m[cur ^ 1] each group's masses at the end of its
 * current interval; cur is not flipped.
 *
 * gd_group_interactions: mask[g] (DEVICE, n_groups uint64 rows) gets bit h set
 * when a retained neighbour of a particle of group g lies in group h, or one of
 * h in g (h != g).  group_lo (HOST, n_groups + 1 ascending slots, group_lo[0]
 * = 0, group_lo[n_groups] <= n) gives the ranges; 1 <= n_groups <= 64.
 * Reads the lists written by gd_build_neighbors. */
int32_t gd_group_interactions(const gd_problem* p, const gd_neighbors* nb, const int32_t* group_lo, int32_t n_groups,
                              uint64_t* mask, void* stream);

/* gd_collision_rates for the slots [lo, hi) of group `group` (of n_groups):
 * with snapshot != 0 the snapshot of the neighbourhood of every particle is
 * first refreshed from m[cur] (groups planned at the same instant share it;
 * pass 1 for the first of them); lambda*_i and the controller moments are
 * computed for the group's slots only; the plan uses the group's controller
 * bins and its interval state iv.  The executed interval is then held within
 * 1/16 and 16 times the scheduled interval sched[h] of every group h set in
 * rows[group] (rows from gd_group_interactions; sched: DEVICE int64[n_groups]
 * of ticks, 0 = nothing scheduled), the lower limit taking precedence where
 * the two conflict (a scheduled interval is kept; the refinement waits), then
 * halved until it starts on a multiple of itself and ends within the
 * collision step, and written to iv and to sched[group].  The caller sets
 * sched[h] = 0 when group h's interval ends. */
int32_t gd_collision_rates_group(const gd_problem* p, const gd_particles* st, const gd_neighbors* nb,
                                 gd_interval* iv, double* lambda_i, int64_t lo, int64_t hi, int32_t group,
                                 int32_t n_groups, const uint64_t* rows, int64_t* sched, int32_t snapshot, void* ws,
                                 size_t ws_bytes, void* stream);

/* gd_sample_collisions for the slots [lo, hi) of one group over iv->dt_exe,
 * against the snapshot of the preceding gd_collision_rates_group call, writing
 * m[cur ^ 1][lo, hi) (and n_events[lo, hi) if non-NULL), then the audit of
 * the group's C.  interval_index (< 2^32) keys the random numbers as in
 * gd_sample_collisions; a run numbers its group intervals so that no particle
 * meets an index twice.  cur is not flipped. */
int32_t gd_sample_collisions_group(const gd_problem* p, const gd_particles* st, const gd_neighbors* nb,
                                   gd_interval* iv, const double* lambda_i, uint64_t seed, uint64_t interval_index,
                                   int64_t lo, int64_t hi, int32_t* n_events, void* ws, size_t ws_bytes,
                                   void* stream);

/* Broadcast of group `group` at the end of its interval: m[cur][lo, hi) =
 * m[cur ^ 1][lo, hi), and sched[group] = 0 when sched (DEVICE, as in
 * gd_collision_rates_group) is non-NULL. */
int32_t gd_publish_group(const gd_problem* p, const gd_particles* st, int64_t lo, int64_t hi, int64_t* sched,
                         int32_t group, void* stream);

/* The collision step of the spatial groups with its scheduler on the device
 * (Sect. 2.5.3; the same schedule, results and random numbers as the
 * gd_*_group calls driven instant by instant).  Each instant is one fixed
 * sequence of launches over all groups, every stage predicated on flags a
 * device kernel sets: the groups whose interval ends publish their masses
 * (m[cur ^ 1] -> m[cur] over their slots), the snapshot of every particle
 * is refreshed in snap_ws when some group starts, the starting groups plan,
 * are clamped in ascending order by the ratio-16 rule (each interval takes
 * the next number in planning order, which keys its draws), and sample and
 * audit their intervals.  After the step's 2^30 ticks later instants do
 * nothing, so the caller queues several and reads one flag.
 *
 * gd_group_sched_create: the groups are group_lo[g] .. group_lo[g+1] of the
 * active slots (host array, G + 1 entries, 1 <= G <= 64, strictly
 * increasing from 0); ivs points at G consecutive interval states; rows (G
 * words, from gd_group_interactions) and sched (G int64) are device arrays;
 * ws holds G workspaces of ws_bytes each (gd_workspace_size of the whole
 * problem), snap_ws the workspace whose snapshot every group reads.  The
 * state's cur selects the broadcast masses.  Everything stays caller-owned;
 * the library allocates its tables and a small scheduler state
 * (hipMalloc).  gd_group_sched_begin starts a collision step whose first
 * interval takes number first_interval; gd_group_sched_instants queues
 * `count` instants; gd_group_sched_read synchronises the stream and returns
 * whether the step is done, the next interval number, and up to log_cap
 * (group, start tick, ticks) records of the step's intervals (n_log = -1
 * when more than 2^14 were dropped).  Errors: GD_E_INVALID_ARG,
 * GD_E_WORKSPACE, GD_E_HIP. */
typedef struct gd_group_sched gd_group_sched;
int32_t gd_group_sched_create(const gd_problem* p, const gd_particles* st, const gd_neighbors* nb,
                              const int32_t* group_lo, int32_t G, gd_interval* ivs, const uint64_t* rows,
                              int64_t* sched, double* lam_i, int32_t* n_events, void* const* ws,
                              size_t ws_bytes, void* snap_ws, uint64_t seed, gd_group_sched** out);
int32_t gd_group_sched_begin(gd_group_sched* g, int64_t first_interval, void* stream);
int32_t gd_group_sched_instants(gd_group_sched* g, int32_t count, void* stream);
int32_t gd_group_sched_read(gd_group_sched* g, void* stream, int32_t* done, int64_t* next_interval,
                            int32_t* n_log, int64_t* log, int32_t log_cap);
int32_t gd_group_sched_destroy(gd_group_sched* g);

/* Dust diffusion operator D (Sect. 2.4), one Euler--Maruyama step of length
 * dt >= 0 on every active particle of st (M_i > 0), in place.
 * D_a = nu/(Sc_a (1 + St^2)) in each cylindrical direction a = R, Z, phi with
 * nu = alpha c_s H_g of the gas disk (Sect. 2.2) and St the grain's local
 * Stokes number at (R, Z) (midplane when p->vint; p->St_diff when > 0):
 *   dR   = sqrt(2 D_R dt) z_R + (D_R/R + dD_R/dR + chi D_R dln rho_g/dR) dt
 *   dZ   = sqrt(2 D_Z dt) z_Z + (dD_Z/dZ + chi D_Z dln rho_g/dZ) dt     (none if vint)
 *   dphi = sqrt(2 D_phi dt) z_phi / R                                  (none if axisym)
 * with chi = 1 for GD_DIFFUSION_CONCENTRATION and 0 for GD_DIFFUSION_DENSITY
 * (the azimuthal gradients of the axisymmetric gas vanish).  The z are
 * standard normals by the Box--Muller transform of two Philox4x32-10 calls,
 * key = seed, counters (id, step, 0x44494646, w) for w = 0, 1: each call gives
 * u1 = ((hi:lo of words 1:0) >> 11 + 1) 2^-53 and u2 = (words 3:2 >> 11) 2^-53,
 * sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2); z_R, z_Z are the first pair and
 * z_phi the cosine of the second.  A step with R + dR < 0 passes the axis:
 * R' = -(R + dR), phi' += pi.  The Cartesian velocity is kept: v_r, l_theta,
 * l_phi are recomputed in the basis at the new position; r, th, ph, x, y, z
 * are rewritten, and a particle leaving r_in <= r <= r_out gets M = 0.
 * Requires id, x, y, z, M, r, th, ph, vr, lth, lph (and m[cur] unless
 * St_diff > 0), GM, R0, h_g0, alpha > 0, and Sc_a > 0 for each direction
 * stepped.  p->diffusion == GD_DIFFUSION_NONE enqueues nothing.  Needs no
 * workspace and no synchronisation; the paper's cadence calls it twice per
 * transport step with dt = Delta t / 2 (Sect. 2.6). */
int32_t gd_diffuse(const gd_problem* p, const gd_particles* st, double dt, uint64_t seed, uint32_t step,
                   void* stream);

/* Kernels that gd_profile_events can bracket. */
typedef enum gd_prof_kernel {
    GD_PROF_SORT = 0,       /* bounding box, Morton keys, radix sort, permutation */
    GD_PROF_TREE = 1,       /* search-tree boxes */
    GD_PROF_KNN_QUERY = 2,  /* neighbour query */
    GD_PROF_RATES = 3,      /* snapshot, pair rates, controller bins, plan */
    GD_PROF_MC = 4,         /* sampling kernel */
    GD_PROF_AUDIT = 5,      /* audit reduction */
    GD_PROF_PUSH = 6,       /* push */
    GD_PROF_DIFFUSE = 7,    /* diffusion step */
    GD_PROF_COUNT = 8
} gd_prof_kernel;

/* Diagnostics for measurement: from now on, record the HIP events `before`
 * and `after` (hipEvent_t passed as void*, created by the caller) on the
 * launch stream immediately before and after the kernels named by `which`
 * at every call.  NULL, NULL stops recording.  Process-wide setting; the
 * events stay owned by the caller. */
int32_t gd_profile_events(int32_t which, void* before, void* after);

/* A stream restricted to a subset of the current device's compute units
 * (hipExtStreamCreateWithCUMask), default priority: bit i of mask[i / 32]
 * selects CU i; words beyond the device's CU count are ignored.  For callers
 * that keep latency-bound launches apart from large ones (the serving tiers:
 * a small run's launches then never wait for CU slots behind a large run's
 * workgroups).  GD_E_INVALID_ARG for a NULL or empty mask, GD_E_HIP when the
 * runtime refuses it.  gd_stream_destroy releases it. */
int32_t gd_stream_create_cu_mask(const uint32_t* mask, int32_t mask_words, void** stream);
int32_t gd_stream_destroy(void* stream);

/* Copy the device status word of the workspace to *out (bits GD_DEV_*), then
 * clear it.  Synchronises `stream`. */
int32_t gd_status_read(void* ws, void* stream, int32_t* out);

/* Last host-side error message of the calling thread ("" if none). */
const char* gd_last_error(void);

/* Library version string. */
const char* gd_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GD_H */
