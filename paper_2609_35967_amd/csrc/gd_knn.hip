// gd_knn.hip -- N_K nearest neighbours of every active particle (Sect. 2.5.1),
// exact, on a shallow spatial hierarchy over the Morton order.
//
// Tree: implicit and 8-ary.  Level 0 holds the boxes of buckets of 4
// consecutive Morton slots; node i of level l holds the union of children
// 8i..8i+7 of level l-1; the root's children are the (<= 8) boxes of the top
// level.  No pointers: children and parents are index arithmetic, and the
// 8 child boxes of a node are contiguous (192 bytes in single precision,
// rounded outward), so one step of a walk issues its loads together.  A
// million particles give 6 levels.
//
// Query: one lane per particle, stackless depth-first walk that keeps, per
// level, the 8-bit mask of children still to visit (all levels in one 64-bit
// register).  Exact selection of the k-1 nearest others:
//   1. trial radius from the density of the smallest ancestor holding >= k
//      slots (its box also bounds the k-th distance);
//   2. pass A: count candidates inside the radius into 32 bins of d^2 (grow the
//      radius until k-1 others are inside);
//   3. the bin holding the (k-1)-th other splits candidates into "sure" (lower
//      bins) and "boundary"; an over-full boundary bin is re-binned (nested,
//      still monotone bins) until it holds <= 16 candidates;
//   4. pass B: walk again inside the tightened radius, append sure slots to the
//      output row, keep boundary slots, rank them by (d^2, slot);
//   5. sort the retained others by slot in registers.
// Per-lane scratch lives in LDS columns (no synchronisation).  d^2 is
// (dx*dx + dy*dy) + dz*dz, each operation rounded on its own; every bin
// function is monotone in d^2, so the result is exactly the k-1 smallest
// (d^2, slot).
#include "gd_common.hpp"
#include "gd_internal.hpp"

namespace gd {

constexpr int kNB = 64;   // bins of the per-lane distance histograms
constexpr int kC1 = 16;   // largest boundary bin ranked in registers
constexpr int kDMax = 3;  // levels of the nested bin chain
constexpr int kQBlock = 256;

// ---------------------------------------------------------------------------
// Tree build
struct TreeLevels {
    int32_t levels;
    int64_t off[kMaxTreeLevels];
    int64_t cap[kMaxTreeLevels];  // padded capacity of each level
};

// level 0: box of every bucket of kBucket active slots (empty beyond)
__global__ __launch_bounds__(256) void k_bucket_boxes(const double4* __restrict__ pos, const WsHeader* __restrict__ h,
                                                      FBox* __restrict__ box0, int64_t cap0)
{
    const int na = h->n_active;
    const int64_t b = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (b >= cap0) return;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int t = 0; t < kBucket; ++t) {
        const int64_t j = b * kBucket + t;
        if (j < na) {
            const double4 p = pos[j];
            lo[0] = fmin(lo[0], p.x);
            hi[0] = fmax(hi[0], p.x);
            lo[1] = fmin(lo[1], p.y);
            hi[1] = fmax(hi[1], p.y);
            lo[2] = fmin(lo[2], p.z);
            hi[2] = fmax(hi[2], p.z);
        }
    }
    FBox x;
    for (int a = 0; a < 3; ++a) {
        x.lo[a] = __double2float_rd(lo[a]);
        x.hi[a] = __double2float_ru(hi[a]);
    }
    box0[b] = x;
}

// level l >= 1: union of the 8 children (empty children are empty boxes)
__global__ __launch_bounds__(256) void k_level_boxes(const FBox* __restrict__ child, FBox* __restrict__ cur, int64_t cap)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= cap) return;
    FBox x;
    for (int a = 0; a < 3; ++a) {
        x.lo[a] = INFINITY;
        x.hi[a] = -INFINITY;
    }
    for (int c = 0; c < kFan; ++c) {
        const FBox y = child[i * kFan + c];
        for (int a = 0; a < 3; ++a) {
            x.lo[a] = fminf(x.lo[a], y.lo[a]);
            x.hi[a] = fmaxf(x.hi[a], y.hi[a]);
        }
    }
    cur[i] = x;
}

// ---------------------------------------------------------------------------
// Query
struct KnnArgs {
    int32_t* stats;
    const double4* pos;
    const FBox* boxes;
    TreeLevels T;
    const WsHeader* h;
    int64_t n;
    int32_t k;
    double rmax2;
    int32_t per[3];
    double L[3], hL[3];
    double tol;  // absolute slack of box distances on periodic axes
    int32_t* nbr;
    int32_t* cnt;
    double* dmax;
    void* ws;
};

template <bool PER>
__device__ inline double sep2(const KnnArgs& A, const double q[3], const double4 p)
{
    double dx = p.x - q[0], dy = p.y - q[1], dz = p.z - q[2];
    if (PER) {
        if (A.per[0]) { if (dx > A.hL[0]) dx = dx - A.L[0]; else if (dx < -A.hL[0]) dx = dx + A.L[0]; }
        if (A.per[1]) { if (dy > A.hL[1]) dy = dy - A.L[1]; else if (dy < -A.hL[1]) dy = dy + A.L[1]; }
        if (A.per[2]) { if (dz > A.hL[2]) dz = dz - A.L[2]; else if (dz < -A.hL[2]) dz = dz + A.L[2]; }
    }
    const double s = dx * dx + dy * dy;
    return s + dz * dz;
}

__device__ inline double gap(double x, double lo, double hi)
{
    return x < lo ? lo - x : (x > hi ? x - hi : 0.0);
}

// Squared distance from q to a box, minimum image on periodic axes.  On open
// axes lo <= p exactly and rounding is monotone, so the result never exceeds
// the rounded d^2 of a point in the box; periodic images are covered by the
// absolute slack of the walk.
template <bool PER>
__device__ inline double box2(const KnnArgs& A, const double q[3], const FBox& b)
{
    double g[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double lo = b.lo[a], hi = b.hi[a];
        double v = gap(q[a], lo, hi);
        if (PER && A.per[a]) v = fmin(v, fmin(gap(q[a] + A.L[a], lo, hi), gap(q[a] - A.L[a], lo, hi)));
        g[a] = v;
    }
    const double s = g[0] * g[0] + g[1] * g[1];
    return s + g[2] * g[2];
}

// mask of the children of node `idx` at `level` (>= 1) whose box may hold a
// point within R2 of q
template <bool PER>
__device__ inline uint32_t child_mask(const KnnArgs& A, int level, int64_t idx, const double q[3], double R2)
{
    double R2box = R2 * (1.0 + 1e-12);
    if (PER) {
        const double rb = sqrt(R2) * (1.0 + 1e-12) + A.tol;
        R2box = rb * rb;
    }
    const FBox* ch = A.boxes + A.T.off[level - 1] + idx * kFan;
    FBox b[kFan];
#pragma unroll
    for (int c = 0; c < kFan; ++c) b[c] = ch[c];
    uint32_t m = 0;
#pragma unroll
    for (int c = 0; c < kFan; ++c) m |= (box2<PER>(A, q, b[c]) <= R2box ? 1u : 0u) << c;
    return m;
}

// Visit every active slot j with d^2(q, j) <= R2 (j == q included; the
// visitor filters).  The walk starts at the level-1 ancestor of q's bucket
// and climbs one ancestor at a time, expanding the ancestor's other children
// depth first, so the space near q is seen first.  The visitor may shrink R2
// (never grow it); pruning uses the current value.  Returns the walk steps.
template <bool PER, class F>
__device__ inline int walk(const KnnArgs& A, int na, int q, const double qp[3], double& R2, F&& f)
{
    const int top = A.T.levels;  // the root sits one level above the stored ones
    int climb = 1, level = 1;
    int64_t idx = (q / kBucket) >> 3;
    uint64_t masks = child_mask<PER>(A, 1, idx, qp, R2);
    int steps = 1;
    for (;;) {
        const int sh = 8 * (level - 1);
        const uint32_t m = uint32_t(masks >> sh) & 0xFFu;
        if (m == 0) {
            if (level < climb) {
                ++level;
                idx >>= 3;
                continue;
            }
            if (climb == top) break;
            // the ancestor at `climb` is done: expand its parent's other children
            const int from = int(idx & 7);
            ++climb;
            level = climb;
            idx >>= 3;
            masks |= uint64_t(child_mask<PER>(A, level, idx, qp, R2) & ~(1u << from)) << (8 * (level - 1));
            ++steps;
            continue;
        }
        const int c = __ffs(m) - 1;
        masks &= ~(uint64_t(1) << (sh + c));
        const int64_t child = idx * kFan + c;
        ++steps;
        if (level == 1) {
            // a bucket: its particles are candidates
            double4 p[kBucket];
#pragma unroll
            for (int t = 0; t < kBucket; ++t) {
                const int64_t j = child * kBucket + t;
                if (j < na) p[t] = A.pos[j];
            }
#pragma unroll
            for (int t = 0; t < kBucket; ++t) {
                const int64_t j = child * kBucket + t;
                if (j < na) {
                    const double d2 = sep2<PER>(A, qp, p[t]);
                    if (d2 <= R2) f(int(j), d2);
                }
            }
            continue;
        }
        --level;
        idx = child;
        masks |= uint64_t(child_mask<PER>(A, level, idx, qp, R2)) << (8 * (level - 1));
    }
    return steps;
}

// First-level bins: logarithmic in x = d^2 / R2init, 8 per octave over 8
// octaves, read off the bits of the double (monotone for x >= 0); bin 0 takes
// everything below 2^-8 (x * 2^(1/8)), the last bin everything from 2^(-1/8).
constexpr int kLogShift = 49;
constexpr int64_t kLogBase = int64_t(1023) * 8 - kNB;

__device__ inline int log_bin(double x)
{
    const int64_t b = (int64_t(__double_as_longlong(x)) >> kLogShift) - kLogBase;
    return b < 0 ? 0 : (b > kNB - 1 ? kNB - 1 : int(b));
}

// lower edge of log bin b (1 <= b <= kNB); log_bin(x) < b exactly when x < edge
__device__ inline double log_edge(int b)
{
    return __longlong_as_double((long long)((int64_t(b) + kLogBase) << kLogShift));
}

__device__ inline int bin_at(double x, double lo, double s)
{
    const double t = (x - lo) * s;
    if (!(t < double(kNB))) return kNB - 1;
    if (!(t > 0.0)) return 0;
    return int(t);
}

// Nested bin chain over x = d^2 * s: level 0 is log_bin, levels >= 1 are
// linear bins bin_at(x, lo_l, s_l); b_l is the boundary bin of level l and
// depth the levels in use.  Scalar fields (no dynamic indexing).
struct Chain {
    int depth;
    double s;  // 1 / R2init
    double lo1, lo2;
    double s1, s2;
    int b0, b1, b2;
    __device__ double lo(int l) const { return l == 1 ? lo1 : lo2; }
    __device__ double sc(int l) const { return l == 1 ? s1 : s2; }
    __device__ int b(int l) const { return l == 0 ? b0 : l == 1 ? b1 : b2; }
    __device__ void set_level(int l, double lo_, double s_)
    {
        if (l == 1) { lo1 = lo_; s1 = s_; }
        else { lo2 = lo_; s2 = s_; }
    }
    __device__ void set_b(int l, int v)
    {
        if (l == 0) b0 = v;
        else if (l == 1) b1 = v;
        else b2 = v;
    }
};

enum { kSure = 0, kBoundary = 1, kReject = 2 };

__device__ inline int classify(const Chain& c, double d2)
{
    const double x = d2 * c.s;
    int b = log_bin(x);
    if (b < c.b0) return kSure;
    if (b > c.b0) return kReject;
    for (int l = 1; l < c.depth; ++l) {
        b = bin_at(x, c.lo(l), c.sc(l));
        if (b < c.b(l)) return kSure;
        if (b > c.b(l)) return kReject;
    }
    return kBoundary;
}

// Per-lane 16-bit bin counters in LDS: bin b of lane t is half (b & 1) of
// word (b >> 1) * kQBlock + t (a private column, free of bank conflicts).
__device__ inline void hist_clear(uint32_t* lds, int tid)
{
    for (int w = 0; w < kNB / 2; ++w) lds[w * kQBlock + tid] = 0;
}

__device__ inline int hist_get(const uint32_t* lds, int tid, int b)
{
    return int((lds[(b >> 1) * kQBlock + tid] >> (16 * (b & 1))) & 0xFFFFu);
}

// returns false (and counts nothing) once the counter is saturated
__device__ inline bool hist_inc(uint32_t* lds, int tid, int b)
{
    uint32_t* w = lds + (b >> 1) * kQBlock + tid;
    const uint32_t v = *w;
    if (((v >> (16 * (b & 1))) & 0xFFFFu) == 0xFFFFu) return false;
    *w = v + (1u << (16 * (b & 1)));
    return true;
}

template <int N>
__device__ inline void bitonic_sort(int32_t (&v)[N])
{
#pragma unroll
    for (int size = 2; size <= N; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int j = i ^ stride;
                if (j > i) {
                    const int32_t a = v[i], b = v[j];
                    const bool up = (i & size) == 0;
                    v[i] = up ? min(a, b) : max(a, b);
                    v[j] = up ? max(a, b) : min(a, b);
                }
            }
        }
    }
}

template <bool PER, int KP2>
__global__ __launch_bounds__(kQBlock) void k_knn_query(KnnArgs A)
{
    // per-lane bin counters, later the boundary list (kC1 slots)
    __shared__ uint32_t s_lds[(kNB / 2) * kQBlock];
    static_assert(kC1 <= kNB / 2, "boundary list must fit the counter words");
    const int tid = threadIdx.x;
    const int64_t q64 = blockIdx.x * int64_t(kQBlock) + tid;
    if (q64 >= A.n) return;
    const int q = int(q64);
    const int na = A.h->n_active;
    const int k = A.k;
    const int need = k - 1;
    int32_t* row = A.nbr + int64_t(q) * k;
    if (q >= na || na == 1) {
        const bool act = q < na;
        row[0] = act ? q : -1;
        for (int s = 1; s < k; ++s) row[s] = -1;
        A.cnt[q] = act ? 1 : 0;
        A.dmax[q] = 0.0;
        return;
    }
    const double4 q4 = A.pos[q];
    const double qp[3] = {q4.x, q4.y, q4.z};

    // 1. upper bound of the (k-1)-th distance: the smallest, over three windows
    //    of k consecutive slots holding q (ending at, centred on, starting at
    //    q), of the largest d^2 in the window; with fewer than k slots, all.
    double R2init;
    {
        const int span = na < k ? na : k;
        const int fmaxs = na - span;
        int f0 = q - span + 1, f1 = q - span / 2 + 1, f2 = q;
        f0 = f0 < 0 ? 0 : (f0 > fmaxs ? fmaxs : f0);
        f1 = f1 < 0 ? 0 : (f1 > fmaxs ? fmaxs : f1);
        f2 = f2 < 0 ? 0 : (f2 > fmaxs ? fmaxs : f2);
        double w0 = 0.0, w1 = 0.0, w2 = 0.0;
        for (int j = f0; j < f2 + span; ++j) {
            const double d2 = sep2<PER>(A, qp, A.pos[j]);
            if (j < f0 + span) w0 = fmax(w0, d2);
            if (j >= f1 && j < f1 + span) w1 = fmax(w1, d2);
            if (j >= f2) w2 = fmax(w2, d2);
        }
        R2init = fmin(w0, fmin(w1, w2));
    }
    if (!(R2init < INFINITY)) {  // non-finite positions
        set_status(A.ws, GD_DEV_NONFINITE);
        row[0] = q;
        for (int s = 1; s < k; ++s) row[s] = -1;
        A.cnt[q] = 1;
        A.dmax[q] = 0.0;
        return;
    }
    const double R2cap = fmin(R2init, A.rmax2);
    Chain c{};
    c.s = R2init > 0.0 ? 1.0 / R2init : 0.0;
    if (!(c.s < INFINITY)) c.s = 0.0;

    // 2. pass A: count others into the log bins, cutting the radius down to
    //    the upper edge of the bin that completes k-1 others
    hist_clear(s_lds, tid);
    double R2 = R2cap;
    int bcut = kNB - 1, cle = 0, candA = 0;
    bool sat = false;
    const double sA = c.s;
    const int visA = walk<PER>(A, na, q, qp, R2, [&](int j, double d2) {
        if (j == q) return;
        const int b = log_bin(d2 * sA);
        if (b > bcut) return;
        ++candA;
        if (!hist_inc(s_lds, tid, b)) {
            sat = true;
            return;
        }
        ++cle;
        bool cut = false;
        while (bcut > 0 && cle - hist_get(s_lds, tid, bcut) >= need) {
            cle -= hist_get(s_lds, tid, bcut);
            --bcut;
            cut = true;
        }
        if (cut) R2 = fmin(R2cap, (log_edge(bcut + 1) / sA) * (1.0 + 1e-12));
    });

    // 3. the boundary bin; refine it with nested linear bins while over-full
    int c0 = 0, hb = 0, refines = 0;
    bool fallback = sat;
    if (sat) {
        c.depth = 0;  // every candidate inside R2 is a boundary candidate
        c.b0 = -1;
    } else if (cle < need) {
        c.depth = 1;
        c.b0 = kNB;  // fewer than k-1 others within the cap: keep them all
        c0 = cle;
    } else {
        c.depth = 1;
        c.b0 = bcut;
        hb = hist_get(s_lds, tid, bcut);
        c0 = cle - hb;
        double loD = bcut == 0 ? 0.0 : log_edge(bcut);
        double sD = double(kNB) / (log_edge(bcut + 1) - loD);
        while (hb > kC1) {
            const int D = c.depth;
            if (D >= kDMax || !(c.s > 0.0) || !(sD < 1e300) || !(sD > 0.0) || loD + 1.0 / sD == loD) {
                fallback = true;
                break;
            }
            c.set_level(D, loD, sD);
            ++refines;
            hist_clear(s_lds, tid);
            bool sat2 = false;
            walk<PER>(A, na, q, qp, R2, [&](int j, double d2) {
                if (j != q && classify(c, d2) == kBoundary)
                    sat2 |= !hist_inc(s_lds, tid, bin_at(d2 * c.s, loD, sD));
            });
            if (sat2) {
                fallback = true;
                break;
            }
            const int needD = need - c0;
            int cum = 0, bs = kNB - 1, hv = 0;
            for (int b = 0; b < kNB; ++b) {
                hv = hist_get(s_lds, tid, b);
                if (cum + hv >= needD) {
                    bs = b;
                    break;
                }
                cum += hv;
            }
            c.set_b(D, bs);
            c.depth = D + 1;
            c0 += cum;
            hb = hv;
            loD = loD + double(bs) / sD;
            sD = sD * double(kNB);
        }
    }

    // 4. pass B inside the final radius: sure slots go to the row, boundary
    //    slots to the LDS list (the counters are no longer needed)
    int nsel = 0, nb = 0;
    double maxd2 = 0.0;
    int32_t* s_bnd = reinterpret_cast<int32_t*>(s_lds);
    const int visB = walk<PER>(A, na, q, qp, R2, [&](int j, double d2) {
        if (j == q) return;
        const int cl = sat ? kBoundary : classify(c, d2);
        if (cl == kSure) {
            if (nsel < need) row[1 + nsel] = j;
            ++nsel;
            maxd2 = fmax(maxd2, d2);
        } else if (cl == kBoundary) {
            if (nb < kC1) s_bnd[nb * kQBlock + tid] = j;
            ++nb;
        }
    });
#ifdef GD_KNN_STATS
    A.stats[q * 8 + 0] = refines;
    A.stats[q * 8 + 1] = visA;
    A.stats[q * 8 + 2] = candA;
    A.stats[q * 8 + 3] = visB;
    A.stats[q * 8 + 4] = c.depth;
    A.stats[q * 8 + 5] = fallback;
    A.stats[q * 8 + 6] = hb;
#else
    (void)visA;
    (void)visB;
    (void)candA;
    (void)refines;
#endif
    if (nsel != c0) set_status(A.ws, GD_DEV_INTERNAL);
    const int nsel_w = nsel < need ? nsel : need;
    const int needb = need - nsel_w < nb ? need - nsel_w : nb;
    if (!fallback) {
        double bd[kC1];
        int32_t bj[kC1];
#pragma unroll
        for (int e = 0; e < kC1; ++e) {
            if (e < nb) {
                const int j = s_bnd[e * kQBlock + tid];
                bj[e] = j;
                bd[e] = sep2<PER>(A, qp, A.pos[j]);
            } else {
                bj[e] = INT32_MAX;
                bd[e] = INFINITY;
            }
        }
#pragma unroll
        for (int e = 0; e < kC1; ++e) {
            int rank = 0;
#pragma unroll
            for (int f = 0; f < kC1; ++f) rank += (bd[f] < bd[e]) || (bd[f] == bd[e] && bj[f] < bj[e]);
            if (e < nb && rank < needb) {
                row[1 + nsel_w + rank] = bj[e];
                maxd2 = fmax(maxd2, bd[e]);
            }
        }
    } else {
        // exact selection among the boundary candidates (rare): repeated minimum
        set_status(A.ws, GD_DEV_KNN_FALLBACK);
        double lastd = -1.0;
        int lastj = -1;
        for (int t = 0; t < needb; ++t) {
            double bestd = INFINITY;
            int bestj = INT32_MAX;
            walk<PER>(A, na, q, qp, R2, [&](int j, double d2) {
                if (j == q || (!sat && classify(c, d2) != kBoundary)) return;
                const bool after = (d2 > lastd) || (d2 == lastd && j > lastj);
                const bool better = (d2 < bestd) || (d2 == bestd && j < bestj);
                if (after && better) {
                    bestd = d2;
                    bestj = j;
                }
            });
            row[1 + nsel_w + t] = bestj;
            maxd2 = fmax(maxd2, bestd);
            lastd = bestd;
            lastj = bestj;
        }
    }
    const int ntot = nsel_w + needb;

    // 5. retained others in ascending slot order
    int32_t v[KP2];
#pragma unroll
    for (int e = 0; e < KP2; ++e) v[e] = (e < ntot) ? row[1 + e] : INT32_MAX;
    bitonic_sort<KP2>(v);
    row[0] = q;
#pragma unroll
    for (int e = 0; e < KP2; ++e)
        if (e < k - 1) row[1 + e] = (e < ntot) ? v[e] : -1;
    A.cnt[q] = 1 + ntot;
    A.dmax[q] = ntot > 0 ? sqrt(maxd2) : 0.0;
}

// ---------------------------------------------------------------------------
int launch_knn(const gd_problem* p, const gd_neighbors* nb, void* ws, const Layout& L, hipStream_t st)
{
    const int64_t n = p->n;
    const WsHeader* h = at<WsHeader>(ws, L.hdr);
    FBox* boxes = at<FBox>(ws, L.boxes);
    const double4* pos = at<double4>(ws, L.pos4);
    TreeLevels T{};
    T.levels = L.levels;
    for (int l = 0; l < L.levels; ++l) {
        T.off[l] = L.lvl_off[l];
        T.cap[l] = (L.lvl_cnt[l] + kFan - 1) / kFan * kFan;
    }
    prof_mark(GD_PROF_TREE, 0, st);
    hipLaunchKernelGGL(k_bucket_boxes, dim3(unsigned((T.cap[0] + 255) / 256)), dim3(256), 0, st, pos, h,
                       boxes + T.off[0], T.cap[0]);
    for (int l = 1; l < L.levels; ++l)
        hipLaunchKernelGGL(k_level_boxes, dim3(unsigned((T.cap[l] + 255) / 256)), dim3(256), 0, st,
                           boxes + T.off[l - 1], boxes + T.off[l], T.cap[l]);
    prof_mark(GD_PROF_TREE, 1, st);
    KnnArgs A{};
#ifdef GD_KNN_STATS
    A.stats = at<int32_t>(ws, L.stats);
    launch_fill_i32(A.stats, 8 * n, 0, st);
#endif
    A.pos = pos;
    A.boxes = boxes;
    A.T = T;
    A.h = h;
    A.n = n;
    A.k = p->k;
    A.rmax2 = p->rmax * p->rmax;
    bool per = false;
    double maxL = 0.0;
    for (int a = 0; a < 3; ++a) {
        A.per[a] = p->periodic[a] ? 1 : 0;
        A.L[a] = p->L[a];
        A.hL[a] = 0.5 * p->L[a];
        per = per || A.per[a];
        if (A.per[a]) maxL = std::max(maxL, std::fabs(p->L[a]));
    }
    A.tol = 1e-15 * maxL;
    A.nbr = nb->nbr;
    A.cnt = nb->cnt;
    A.dmax = nb->dmax;
    A.ws = ws;
    const dim3 grid(unsigned((n + kQBlock - 1) / kQBlock));
    prof_mark(GD_PROF_KNN_QUERY, 0, st);
    if (p->k <= 33) {
        if (per) hipLaunchKernelGGL((k_knn_query<true, 32>), grid, dim3(kQBlock), 0, st, A);
        else hipLaunchKernelGGL((k_knn_query<false, 32>), grid, dim3(kQBlock), 0, st, A);
    } else {
        if (per) hipLaunchKernelGGL((k_knn_query<true, 64>), grid, dim3(kQBlock), 0, st, A);
        else hipLaunchKernelGGL((k_knn_query<false, 64>), grid, dim3(kQBlock), 0, st, A);
    }
    prof_mark(GD_PROF_KNN_QUERY, 1, st);
    return 0;
}

}  // namespace gd
