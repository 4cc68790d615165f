// gd_knn.hip -- N_K nearest neighbours of every active particle (Sect. 2.5.1),
// exact, on a shallow spatial hierarchy over the Morton order.
//
// Tree: implicit and 8-ary.  Level 0 holds the boxes of buckets of 4
// consecutive Morton slots; node i of level l holds the union of children
// 8i..8i+7 of level l-1; the root's children are the (<= 8) boxes of the top
// level.  No pointers: children and parents are index arithmetic, and the
// 8 child boxes of a node are contiguous (192 bytes), so one step of a walk
// issues its loads together.  A million particles give 6 levels.  Boxes are
// single precision, rounded outward and widened by a margin that absorbs the
// rounding of the single-precision box tests, so a box is never pruned while
// it holds a point within the search radius.
//
// Query: one lane per particle, stackless walk that keeps, per level, the
// 8-bit mask of children still to visit (all levels in one 64-bit register).
// It starts at the level-1 ancestor of the query's bucket and climbs one
// ancestor at a time, so the space near the query is seen first.  Each
// iteration expands one node and scans one bucket of a short queue of
// level-1 bucket masks, with the loads of both issued together and no
// branch around either (see walk()).  Exact selection of the k-1 nearest
// others:
//   1. upper bound R2init of the (k-1)-th d^2: the smallest, over three
//      windows of k consecutive slots holding the query, of the window's
//      largest d^2;
//   2. pass A: count others into per-lane bins, logarithmic in d^2 over the
//      pass's first radius (the particle's distance from the previous search
//      when one is given, else R2init); whenever the bins below some bin
//      already hold k-1 others, cut the radius to that bin's upper edge (the
//      walk prunes with the cut radius).  Every counted other is also kept,
//      with its bin, in a per-lane list (entries above the cut are dropped
//      when it fills);
//   3. the bin holding the (k-1)-th other splits the list into "sure" (lower
//      bins) and "boundary" entries; the boundary ones are ranked by
//      (d^2, slot);
//   4. only a lane whose list overflowed walks again (pass B) inside the final
//      radius, after re-binning an over-full boundary bin with nested linear
//      bins;
//   5. the retained others are sorted by slot in registers and the row is
//      written once.
// Per-lane bins and lists live in LDS columns (no synchronisation).  d^2 is
// (dx*dx + dy*dy) + dz*dz, each operation rounded on its own; every bin
// function is monotone in d^2, so the result is exactly the k-1 smallest
// (d^2, slot).
#include "gd_common.hpp"
#include "gd_internal.hpp"
#include "gd_knn.hpp"

#include <algorithm>

namespace gd {

constexpr int kDMax = 3;  // levels of the nested bin chain
constexpr int kRescales = 4;  // restarts of pass A on a finer distance scale
constexpr int kQBlock = 128;
constexpr bool kTileSearch = true;  // shared candidate tiles before the per-lane search (k <= 33)
constexpr int kFallbackBlocks = 8192;  // one-wavefront workgroups that take the handed-back queries (about one each)
constexpr int kQueue = 4;  // level-1 bucket masks a walk keeps queued
static_assert(kQueue >= 1 && kQueue <= 4, "the queue keeps its masks in the bytes of one word");

// ---------------------------------------------------------------------------
// Tree build
// level 0: widened box of every bucket of kBucket active slots (empty beyond)
struct BucketArgs {
    const double4* pos;
    const WsHeader* h;
    FBox* box0;
    int64_t cap0;
    Periodicity P;
};

struct BucketBoxes {
    using Args = BucketArgs;
    static constexpr int kThreads = 256;
    static __device__ __forceinline__ void body(const Args& A, Blk B);
};

__global__ __launch_bounds__(256) void k_bucket_boxes(BucketArgs A)
{
    BucketBoxes::body(A, Blk{int64_t(blockIdx.x), int64_t(gridDim.x)});
}

// the widened box of bucket b (< cap0): empty when it holds no active slot
__device__ inline FBox bucket_box(const BucketArgs& A, int64_t b)
{
    const double4* __restrict__ pos = A.pos;
    const WsHeader* __restrict__ h = A.h;
    const Periodicity P = A.P;
    const int na = h->n_active;
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
        const double del = box_margin(h, P, a);
        x.lo[a] = __double2float_rd(lo[a] - del);
        x.hi[a] = __double2float_ru(hi[a] + del);
    }
    return x;
}

__device__ __forceinline__ void BucketBoxes::body(const Args& A, Blk B)
{
    const int64_t b = B.id * int64_t(blockDim.x) + threadIdx.x;
    if (b < A.cap0) A.box0[b] = bucket_box(A, b);
}

__device__ inline FBox empty_box()
{
    FBox x;
    for (int a = 0; a < 3; ++a) {
        x.lo[a] = INFINITY;
        x.hi[a] = -INFINITY;
    }
    return x;
}

__device__ inline void box_union(FBox& x, const FBox& y)
{
    for (int a = 0; a < 3; ++a) {
        x.lo[a] = fminf(x.lo[a], y.lo[a]);
        x.hi[a] = fmaxf(x.hi[a], y.hi[a]);
    }
}

// level l >= 1: union of the 8 children; children past the stored capacity
// of level l-1 (the padding of the levels above) are empty
struct LevelArgs {
    const FBox* child;
    int64_t child_cap;
    FBox* cur;
    int64_t cap;
};

struct LevelBoxes {
    using Args = LevelArgs;
    static constexpr int kThreads = 256;
    static __device__ __forceinline__ void body(const Args& A, Blk B);
};

__global__ __launch_bounds__(256) void k_level_boxes(LevelArgs A)
{
    LevelBoxes::body(A, Blk{int64_t(blockIdx.x), int64_t(gridDim.x)});
}

__device__ __forceinline__ void LevelBoxes::body(const Args& A, Blk B)
{
    const FBox* __restrict__ child = A.child;
    const int64_t child_cap = A.child_cap, cap = A.cap;
    FBox* __restrict__ cur = A.cur;
    const int64_t i = B.id * int64_t(blockDim.x) + threadIdx.x;
    if (i >= cap) return;
    FBox x;
    for (int a = 0; a < 3; ++a) {
        x.lo[a] = INFINITY;
        x.hi[a] = -INFINITY;
    }
    for (int c = 0; c < kFan; ++c) {
        if (i * kFan + c >= child_cap) break;
        const FBox y = child[i * kFan + c];
        for (int a = 0; a < 3; ++a) {
            x.lo[a] = fminf(x.lo[a], y.lo[a]);
            x.hi[a] = fmaxf(x.hi[a], y.hi[a]);
        }
    }
    cur[i] = x;
}

// Levels 0, 1 and (box2 set) 2 in one pass: the 256 buckets of a block are
// the children of its 32 level-1 nodes, and these of its 4 level-2 nodes,
// so the unions above the buckets are taken in LDS.  Children past a
// level's capacity enter as empty boxes, which leave a union unchanged: the
// boxes are those of the level-by-level passes.  The grid covers cap1 (it is
// at most a multiple of 32 above cap0 / 8); the host passes box2 only when
// 4 nodes per block cover cap2.  Block 0 also clears the query's counters
// (zq: the per-die queue, kXcd entries; zf: the two fallback list lengths).
struct TreeLowArgs {
    BucketArgs b;
    FBox* box1;
    int64_t cap1;
    FBox* box2;
    int64_t cap2;
    int32_t* zq;
    int32_t* zf;
};

__global__ __launch_bounds__(256) void k_tree_low(TreeLowArgs A)
{
    __shared__ FBox s0[256];
    __shared__ FBox s1[32];
    const int t = threadIdx.x;
    if (blockIdx.x == 0) {
        if (t < kXcd) A.zq[t] = 0;
        if (t < 2) A.zf[t] = 0;
    }
    const int64_t b = int64_t(blockIdx.x) * 256 + t;
    FBox x = empty_box();
    if (b < A.b.cap0) {
        x = bucket_box(A.b, b);
        A.b.box0[b] = x;
    }
    s0[t] = x;
    __syncthreads();
    if (t < 32) {
        FBox u = empty_box();
        for (int c = 0; c < kFan; ++c) box_union(u, s0[t * kFan + c]);
        const int64_t i1 = int64_t(blockIdx.x) * 32 + t;
        if (i1 < A.cap1) A.box1[i1] = u;
        else u = empty_box();
        s1[t] = u;
    }
    if (!A.box2) return;  // the same for every thread of the grid
    __syncthreads();
    if (t < 4) {
        FBox u = empty_box();
        for (int c = 0; c < kFan; ++c) box_union(u, s1[t * kFan + c]);
        const int64_t i2 = int64_t(blockIdx.x) * 4 + t;
        if (i2 < A.cap2) A.box2[i2] = u;
    }
}

// The levels l0 .. levels-1 (each of at most kTailCap nodes) in one
// workgroup, a level at a time: level l0 from the boxes of level l0-1 in
// memory, the ones above from the previous level kept in LDS.
constexpr int kTailCap = 1024;

struct TreeTailArgs {
    FBox* boxes;
    TreeLevels T;
    int32_t l0;
};

__global__ __launch_bounds__(256) void k_tree_tail(TreeTailArgs A)
{
    __shared__ FBox s[2][kTailCap];
    const int t = threadIdx.x;
    for (int l = A.l0; l < A.T.levels; ++l) {
        const FBox* __restrict__ child = A.boxes + A.T.off[l - 1];
        const int64_t ccap = A.T.cap[l - 1], cap = A.T.cap[l];
        FBox* __restrict__ cur = A.boxes + A.T.off[l];
        const FBox* prev = s[(l - A.l0 + 1) & 1];
        FBox* next = s[(l - A.l0) & 1];
        for (int64_t i = t; i < cap; i += 256) {
            FBox x = empty_box();
            for (int c = 0; c < kFan; ++c) {
                const int64_t j = i * kFan + c;
                if (j < ccap) box_union(x, l == A.l0 ? child[j] : prev[j]);
            }
            cur[i] = x;
            next[i] = x;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Query
// Visit every active slot j with d^2(q, j) <= R2 (j == q included; the
// visitor filters), a bucket at a time: f(j0, d2[kBucket], mask) gets the
// bucket's first slot, the d^2 of its slots and the mask of those within R2.
// A visitor that sets R2 negative ends the walk.
// Nearest region first: the level-1 ancestor of q's bucket, then the other
// children of each further ancestor, depth first.  The visitor may lower R2;
// pruning uses the current value.  Two units advance in every iteration:
// the traversal expands one node (a level-1 node yields the mask of its
// buckets to visit, queued in one of kQueue slots), and the scan visits one
// bucket of the oldest queued mask.  Both read their operands at the top of
// the iteration (one wait for the 8 child boxes and the 4 positions), and
// both run in every lane: a lane with no node to expand re-reads a stored
// node (the walk's current one) and drops the mask, a lane with no bucket
// queued reads its own bucket and visits nothing.  The lanes of a
// wavefront, whose iterations run both paths anyway, so share iterations
// without branching around them.  Returns the iterations.
template <bool PER, class F>
__device__ inline int walk(const KnnArgs& A, int na, int q, const double qp[3], const QF& qf, double& R2, F&& f)
{
    const int top = A.T.levels;  // the root sits one level above the stored ones
    int climb = 1, level = 1;
    int idx = (q / kBucket) >> 3;  // (level, idx) is a stored node (or the root) in every state
    uint32_t excl = 0;
    uint64_t masks = 0;  // children still to expand, 8 bits per level >= 2
    bool pend = true;    // node (level, idx) is to be expanded
    // queue of the bucket masks of expanded level-1 nodes: slot s is byte s
    // of qm, for node qb[s]; nq slots in use
    uint32_t qm = 0;
    int qb0 = 0, qb1 = 0, qb2 = 0, qb3 = 0, nq = 0;
    float R2f = r2f(R2);
    int steps = 0;
    for (;;) {
        if (!(R2 >= 0.0)) break;  // the visitor ended the walk
        ++steps;
        const bool ex = pend && (level > 1 || nq < kQueue);
        const bool sc = nq > 0;
        // operands of both units
        const FBox* ch = A.boxes + (level_off(A.T, level - 1) + idx * kFan);
        FBox bx[kFan];
#pragma unroll
        for (int c = 0; c < kFan; ++c) bx[c] = ch[c];
        const int j0 = (sc ? qb0 * kFan + __ffs(qm) - 1 : q / kBucket) * kBucket;
        // the whole bucket (the position buffer is padded to a multiple of 8
        // slots); slots past the active ones are masked out below
        double px[kBucket], py[kBucket], pz[kBucket];
#pragma unroll
        for (int t = 0; t < kBucket; ++t) {
            const double* pj = reinterpret_cast<const double*>(A.pos + j0 + t);
            const double2 xy = *reinterpret_cast<const double2*>(pj);
            px[t] = xy.x;
            py[t] = xy.y;
            pz[t] = pj[2];
        }
        // traversal unit
        const uint32_t m = child_mask<PER>(A, bx, qf, R2f) & live_children(na, level, idx) & ~excl;
        if (ex) {
            excl = 0;
            pend = false;
            if (level > 1) {
                masks |= uint64_t(m) << (8 * (level - 1));
            } else if (m != 0) {
                qm |= m << (8 * nq);
                qb0 = nq == 0 ? idx : qb0;
                qb1 = nq == 1 ? idx : qb1;
                qb2 = nq == 2 ? idx : qb2;
                qb3 = nq == 3 ? idx : qb3;
                ++nq;
            }
            // next node to expand: the first child still to visit at the
            // lowest level >= max(level, 2) (masks are empty above climb),
            // else the other children of the next ancestor
            const int lo = level > 1 ? level : 2;
            const uint64_t up = masks >> (8 * (lo - 1));
            if (up != 0) {
                const int bit = int(__builtin_ctzll(up));
                const int lv = lo + (bit >> 3);  // level of the node whose child is taken
                const int c = bit & 7;
                masks &= ~(uint64_t(1) << (8 * (lv - 1) + c));
                idx = ((idx >> (3 * (lv - level))) << 3) + c;
                level = lv - 1;
                pend = true;
            } else if (climb < top) {
                const int ia = idx >> (3 * (climb - level));  // the ancestor at level climb
                excl = 1u << (ia & 7);
                ++climb;
                level = climb;
                idx = ia >> 3;
                pend = true;
            } else {
                idx >>= 3 * (climb - level);  // exhausted: rest on the root
                level = climb;
            }
        }
        // scan unit: its particles within R2 go to the visitor together
        double d2[kBucket];
        uint32_t vm = 0;
#pragma unroll
        for (int t = 0; t < kBucket; ++t) {
            d2[t] = sep2<PER>(A, qp, px[t], py[t], pz[t]);
            vm |= (d2[t] <= R2 ? 1u : 0u) << t;
        }
        // only the bucket's active slots, and only a bucket from the queue
        const int live = na - j0;
        vm &= !sc ? 0u : (live >= kBucket ? 0xFu : (1u << (live > 0 ? live : 0)) - 1u);
        // the scanned bucket leaves the queue (a slot whose mask empties, too)
        const uint32_t qn = qm & (qm - 1);
        const bool shift = sc && (qn & 0xFFu) == 0;
        qm = !sc ? qm : (shift ? qn >> 8 : qn);
        qb0 = shift ? qb1 : qb0;
        qb1 = shift ? qb2 : qb1;
        qb2 = shift ? qb3 : qb2;
        nq -= shift ? 1 : 0;
        if (vm) f(j0, d2, vm);
        R2f = r2f(R2);
        if (!pend && nq == 0) break;
    }
    return steps;
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
// A lane counts fewer than 2^16 - 1 candidates in all, so no counter wraps.
__device__ inline void hist_clear(uint32_t* lds, int tid)
{
    for (int w = 0; w < kNB / 2; ++w) lds[w * kQBlock + tid] = 0;
}

__device__ inline int hist_get(const uint32_t* lds, int tid, int b)
{
    return int((lds[(b >> 1) * kQBlock + tid] >> (16 * (b & 1))) & 0xFFFFu);
}

// an LDS add whose result is not read (no wait on the lane's path)
__device__ inline void hist_inc(uint32_t* lds, int tid, int b)
{
    atomicAdd(lds + (b >> 1) * kQBlock + tid, 1u << (16 * (b & 1)));
}

// candidates a lane counts before its 16-bit counters are distrusted (a
// bucket may add kBucket past the check)
constexpr int kCandMax = 0xFFFF - 2 * kBucket;

// LDS words per lane: the bin counters (kNB / 2 words, later the boundary
// list) and the candidate list (later the retained others).  The list holds
// the k-1 nearest plus a boundary bin of up to 16, with slack enough that a
// walk rarely has to drop the entries above its cut (measured faster than a
// tighter list at higher occupancy).
template <int KP2>
struct QueryLds {
    static constexpr int kList = KP2 > 32 ? 80 : 64;
    static constexpr int kWords = kNB / 2 + kList;
};
constexpr uint32_t kSlotMask = (1u << 26) - 1;  // list word: bin << 26 | slot
static_assert(QueryLds<32>::kList % 8 == 0 && QueryLds<64>::kList % 8 == 0, "the list is read 8 words at a time");
static_assert(kC1 <= kNB / 2, "the boundary list reuses the counter words");
static_assert(kNB <= 32, "list words keep the bin in 5 bits");

template <bool PER, int KP2>
struct KnnQuery {
    using Args = KnnArgs;
    static constexpr int kThreads = kQBlock;
    static __device__ __forceinline__ void body(const Args& A, Blk B);
};

template <bool PER, int KP2>
__global__ __launch_bounds__(kQBlock) void k_knn_query(KnnArgs A)
{
    KnnQuery<PER, KP2>::body(A, Blk{int64_t(blockIdx.x), int64_t(gridDim.x)});
}

template <bool PER, int KP2>
__device__ __forceinline__ void KnnQuery<PER, KP2>::body(const Args& A, Blk B)
{
    using QL = QueryLds<KP2>;
    __shared__ uint32_t s_lds[QL::kWords * kQBlock];
    const int tid = threadIdx.x;
    int64_t q64;
    if (A.list) {  // the queries of a list (those the tile search handed back)
        const int64_t idx = (B.id * (kQBlock / kWave) + tid / kWave) * kWave + (tid & (kWave - 1));
        q64 = idx < *A.list_n ? A.list[idx] : A.n;
    } else {
        const int32_t item = xcd_take(A.xq, int32_t(B.n * (kQBlock / kWave)));
        q64 = item < 0 ? A.n : int64_t(item) * kWave + (tid & (kWave - 1));
    }
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

    if (!(fabs(qp[0]) < INFINITY && fabs(qp[1]) < INFINITY && fabs(qp[2]) < INFINITY)) {
        set_status(A.ws, GD_DEV_NONFINITE);  // non-finite position: self only
        row[0] = q;
        for (int s = 1; s < k; ++s) row[s] = -1;
        A.cnt[q] = 1;
        A.dmax[q] = 0.0;
        return;
    }

    // 1. upper bound of the (k-1)-th d^2 from three windows of k slots holding
    //    q (ending at, centred on, starting at q); with fewer than k slots, all.
    //    Needed only when there is no usable hint, or the hint falls short.
    double R2init = INFINITY;
    int wlo = 0, whi = 0;  // the slots of the three windows (none yet)
    auto window_bound = [&]() {
        const int span = na < k ? na : k;
        const int fmaxs = na - span;
        int f0 = q - span + 1, f1 = q - span / 2 + 1, f2 = q;
        f0 = f0 < 0 ? 0 : (f0 > fmaxs ? fmaxs : f0);
        f1 = f1 < 0 ? 0 : (f1 > fmaxs ? fmaxs : f1);
        f2 = f2 < 0 ? 0 : (f2 > fmaxs ? fmaxs : f2);
        wlo = f0;
        whi = f2 + span;
        double w0 = 0.0, w1 = 0.0, w2 = 0.0;
        for (int j = wlo; j < whi; ++j) {
            const double d2 = sep2_slot<PER>(A, qp, j);
            if (j < f0 + span) w0 = fmax(w0, d2);
            if (j >= f1 && j < f1 + span) w1 = fmax(w1, d2);
            if (j >= f2) w2 = fmax(w2, d2);
        }
        R2init = fmin(w0, fmin(w1, w2));
    };
    QF qf;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        qf.c[a] = float(qp[a]);
        qf.p[a] = PER ? float(qp[a] + A.L[a]) : 0.0f;
        qf.m[a] = PER ? float(qp[a] - A.L[a]) : 0.0f;
    }
    Chain c{};

    // 2. pass A: count others into the log bins; once the bins below the cut
    //    bin hold k-1 others, lower the cut and the radius with it.  The
    //    window slots go first (their d^2 are cheap to recompute), then the
    //    walk, which skips them.  The particle's neighbour distance from the
    //    previous search, widened by kHintSlack, sets the first radius: only
    //    others inside it are counted, and if fewer than k-1 turn up the pass
    //    runs again on the guaranteed bound.  If bin 0 alone comes to hold
    //    k-1 others, the scale was too coarse (the window bound far above
    //    the (k-1)-th distance): bin 0's upper edge, 2^(-31/8) of the scale,
    //    is a new bound and the pass starts again on it (at most kRescales
    //    times).
    double R2hint = INFINITY;
    {
        const double hv = A.hint[q] * kHintSlack;
        if (hv > 0.0 && hv < INFINITY) {
            // a radius beyond the diagonal of the active set's box is no hint
            const FBox* tb = A.boxes + A.T.off[A.T.levels - 1];
            double e2 = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                float lo = INFINITY, hi = -INFINITY;
#pragma unroll
                for (int c = 0; c < kFan; ++c) {
                    lo = fminf(lo, tb[c].lo[a]);
                    hi = fmaxf(hi, tb[c].hi[a]);
                }
                const double ext = double(hi) - double(lo);
                e2 += ext * ext;
            }
            if (hv * hv <= e2) R2hint = hv * hv;
        }
    }
    bool use_hint = R2hint < INFINITY;
    if (!use_hint) window_bound();
    double R2cap, R2;
    int bcut, cle, hcut, candA, visA = 0, rescales = 0;
    bool sat;
    uint32_t* s_list = s_lds + (kNB / 2) * kQBlock;  // entry e of lane tid at s_list[e * kQBlock + tid]
    constexpr int cap = QL::kList;
    int len;
    bool ovf;
    for (;;) {
        R2cap = fmin(R2init, A.rmax2);
        const double R2s = use_hint ? fmin(R2cap, R2hint) : R2cap;  // first radius and bin scale
        c.s = R2s > 0.0 ? 1.0 / R2s : 0.0;
        if (!(c.s < INFINITY)) c.s = 0.0;
        const double sA = c.s;
        hist_clear(s_lds, tid);
        R2 = R2s;
        bcut = kNB - 1;
        cle = hcut = candA = len = 0;
        sat = ovf = false;
        bool deep = false;
        // lower the cut while the bins below it already hold k-1 others
        auto cut = [&]() {
            if (bcut > 0 && cle - hcut >= need) {
                do {
                    cle -= hcut;
                    --bcut;
                    hcut = hist_get(s_lds, tid, bcut);
                } while (bcut > 0 && cle - hcut >= need);
                // every x with log_bin(x) <= bcut has d^2 below this radius
                // (the radius never grows: boxes already pruned stay pruned)
                if (sA > 0.0) R2 = fmin(R2, (log_edge(bcut + 1) * R2s) * (1.0 + 1e-12));
            }
            if (bcut == 0 && hcut >= need && sA > 0.0 && rescales < kRescales) {
                deep = true;
                R2 = -1.0;  // ends the walk
            }
        };
        // count one other and record it (with its bin) in the list; a full
        // list drops the entries above the cut, and a list still full after
        // that is given up (the lane then walks again for its neighbours)
        auto take = [&](int j, int b) {
            hist_inc(s_lds, tid, b);
            ++cle;
            ++candA;
            hcut += (b == bcut) ? 1 : 0;
            if (ovf) return;
            if (len == cap) {
                int kept = 0;
                for (int e = 0; e < cap; ++e) {
                    const uint32_t w = s_list[e * kQBlock + tid];
                    if (int(w >> 26) <= bcut) s_list[(kept++) * kQBlock + tid] = w;
                }
                len = kept;
                if (len == cap) {
                    ovf = true;
                    return;
                }
            }
            s_list[(len++) * kQBlock + tid] = (uint32_t(b) << 26) | uint32_t(j);
        };
        // take for the slots of one bucket in mask tm, without a branch per
        // slot: the list keeps room for a whole bucket (a list that cannot,
        // after dropping the entries above the cut, is given up), and the
        // counter add of a slot not taken adds 0
        auto take_bucket = [&](int j0, const int (&b)[kBucket], uint32_t tm) {
            if (!ovf && len > cap - kBucket) {
                int kept = 0;
                for (int e = 0; e < len; ++e) {
                    const uint32_t w = s_list[e * kQBlock + tid];
                    if (int(w >> 26) <= bcut) s_list[(kept++) * kQBlock + tid] = w;
                }
                len = kept;
                ovf = len > cap - kBucket;
            }
#pragma unroll
            for (int t = 0; t < kBucket; ++t) {
                const bool tk = (tm >> t) & 1u;
                atomicAdd(s_lds + (b[t] >> 1) * kQBlock + tid, tk ? 1u << (16 * (b[t] & 1)) : 0u);
                cle += tk ? 1 : 0;
                hcut += (tk && b[t] == bcut) ? 1 : 0;
                s_list[(ovf ? 0 : len) * kQBlock + tid] = (uint32_t(b[t]) << 26) | uint32_t(j0 + t);
                len += (tk && !ovf) ? 1 : 0;
            }
            candA += __builtin_popcount(tm);
        };
        for (int j = wlo; j < whi && !deep; ++j) {
            if (j == q) continue;
            const double d2 = sep2_slot<PER>(A, qp, j);
            if (!(d2 <= R2)) continue;
            const int b = log_bin(d2 * sA);
            if (b > bcut) continue;
            take(j, b);
            cut();
        }
        if (!deep)
            visA += walk<PER>(A, na, q, qp, qf, R2, [&](int j0, const double (&d2)[kBucket], uint32_t vm) {
                if (sat || deep) return;
                int b[kBucket];
                uint32_t tm = 0;
#pragma unroll
                for (int t = 0; t < kBucket; ++t) {
                    const int j = j0 + t;
                    b[t] = log_bin(d2[t] * sA);
                    // bitwise, not short-circuit: no branch per slot
                    const uint32_t ok = ((vm >> t) & 1u) & uint32_t(j != q) & (uint32_t(j < wlo) | uint32_t(j >= whi)) &
                                        uint32_t(b[t] <= bcut);
                    tm |= ok << t;
                }
                if (!tm) return;
                take_bucket(j0, b, tm);
                if (candA > kCandMax) {
                    sat = true;
                    return;
                }
                cut();
            });
        if (!deep && use_hint && cle < need && R2hint < R2cap) {
            use_hint = false;  // the hint was too small: count again on the bound
            window_bound();
            continue;
        }
        if (!deep) break;
        // bin 0 holds k-1 others: x < log_edge(1), so d^2 < log_edge(1) R2s
        R2init = (log_edge(1) * R2s) * (1.0 + 1e-12);
        ++rescales;
    }

    // 3. sure and boundary others.  From the list when it kept every counted
    //    other (the usual case); otherwise (sat / overflow) by refining an
    //    over-full boundary bin with nested linear bins and walking again.
    //    Either way the retained others end in list words [0, ntot).
    int32_t* s_bnd = reinterpret_cast<int32_t*>(s_lds);  // the counters are no longer needed
    bool from_list = !sat && !ovf;
    const bool keep = cle < need;  // fewer than k-1 others within the cap: keep them all
    int c0 = 0, hb = 0, refines = 0, visB = 0, visR = 0, nsel = 0, nb = 0, ntot = 0;
    double maxd2 = 0.0;
    bool fallback = sat;
    const int b0 = keep ? kNB : bcut;
    if (from_list) {
        // one pass over the list, read 8 words at a time: sure entries (below
        // the boundary bin) move to the front as slots, boundary entries'
        // slots go to the boundary words.  A write never passes the read.
        for (int e0 = 0; e0 < len; e0 += 8) {
            uint32_t wv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) wv[u] = e0 + u < cap ? s_list[(e0 + u) * kQBlock + tid] : 0u;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const bool live = e0 + u < len;
                const int bn = int((wv[u] >> 26) & 31u);
                const int j = int(wv[u] & kSlotMask);
                const bool sure = live && bn < b0;
                s_list[ntot * kQBlock + tid] = uint32_t(j);  // kept only if sure
                ntot += sure ? 1 : 0;
                if (keep && sure) maxd2 = fmax(maxd2, sep2_slot<PER>(A, qp, j));
                if (live && bn == b0) {
                    if (nb < kC1) s_bnd[nb * kQBlock + tid] = j;
                    ++nb;
                }
            }
        }
        // more boundary entries than the registers rank: give the list up
        // (the lane refines the boundary bin and walks again)
        if (nb > kC1) from_list = false;
    }
    if (from_list) {
        c0 = keep ? cle : cle - hcut;
        hb = keep ? 0 : hcut;
        if (ntot != c0) set_status(A.ws, GD_DEV_INTERNAL);
        const int needb = need - c0 < nb ? need - c0 : nb;
        // rank the boundary slots by (d^2, slot) in registers; the chosen
        // ones follow the sure ones
        double bd[kC1];
        int32_t bj[kC1];
#pragma unroll
        for (int e = 0; e < kC1; ++e) {
            bj[e] = e < nb ? s_bnd[e * kQBlock + tid] : INT32_MAX;
            bd[e] = e < nb ? sep2_slot<PER>(A, qp, bj[e]) : INFINITY;
        }
#pragma unroll
        for (int e = 0; e < kC1; ++e) {
            int rank = 0;
#pragma unroll
            for (int f = 0; f < kC1; ++f) rank += (bd[f] < bd[e]) || (bd[f] == bd[e] && bj[f] < bj[e]);
            if (e < nb && rank < needb) {
                s_list[(ntot++) * kQBlock + tid] = uint32_t(bj[e]);
                maxd2 = fmax(maxd2, bd[e]);
            }
        }
        nsel = c0;
        if (ntot != c0 + needb) set_status(A.ws, GD_DEV_INTERNAL);
    } else {
        nb = ntot = 0;  // (a list given up in the pass above)
        maxd2 = 0.0;
        if (sat) {
            c.depth = 0;  // every candidate inside R2 is a boundary candidate
        } else if (keep) {
            c.depth = 1;
            c.b0 = kNB;
            c0 = cle;
        } else {
            c.depth = 1;
            c.b0 = bcut;
            hb = hcut;
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
                visR += walk<PER>(A, na, q, qp, qf, R2, [&](int j0, const double (&d2)[kBucket], uint32_t vm) {
#pragma unroll
                    for (int t = 0; t < kBucket; ++t)
                        if (((vm >> t) & 1u) && j0 + t != q && classify(c, d2[t]) == kBoundary)
                            hist_inc(s_lds, tid, bin_at(d2[t] * c.s, loD, sD));
                });
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
        // 4. pass B inside the final radius: sure slots to the list words,
        //    boundary slots to the boundary words
        visB = walk<PER>(A, na, q, qp, qf, R2, [&](int j0, const double (&d2)[kBucket], uint32_t vm) {
#pragma unroll
            for (int t = 0; t < kBucket; ++t) {
                const int j = j0 + t;
                if (!((vm >> t) & 1u) || j == q) continue;
                const int cl = sat ? kBoundary : classify(c, d2[t]);
                if (cl == kSure) {
                    if (nsel < need) s_list[nsel * kQBlock + tid] = uint32_t(j);
                    ++nsel;
                    maxd2 = fmax(maxd2, d2[t]);
                } else if (cl == kBoundary) {
                    if (nb < kC1) s_bnd[nb * kQBlock + tid] = j;
                    ++nb;
                }
            }
        });
        if (nsel != c0) set_status(A.ws, GD_DEV_INTERNAL);
        const int nsel_w = nsel < need ? nsel : need;
        const int needb = need - nsel_w < nb ? need - nsel_w : nb;
        if (nb > kC1) fallback = true;
        if (!fallback) {
            double bd[kC1];
            int32_t bj[kC1];
#pragma unroll
            for (int e = 0; e < kC1; ++e) {
                if (e < nb) {
                    const int j = s_bnd[e * kQBlock + tid];
                    bj[e] = j;
                    bd[e] = sep2_slot<PER>(A, qp, j);
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
                    s_list[(nsel_w + rank) * kQBlock + tid] = uint32_t(bj[e]);
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
                visR += walk<PER>(A, na, q, qp, qf, R2, [&](int j0, const double (&d2)[kBucket], uint32_t vm) {
                    for (int t2 = 0; t2 < kBucket; ++t2) {
                        const int j = j0 + t2;
                        if (!((vm >> t2) & 1u) || j == q || (!sat && classify(c, d2[t2]) != kBoundary)) continue;
                        const bool after = (d2[t2] > lastd) || (d2[t2] == lastd && j > lastj);
                        const bool better = (d2[t2] < bestd) || (d2[t2] == bestd && j < bestj);
                        if (after && better) {
                            bestd = d2[t2];
                            bestj = j;
                        }
                    }
                });
                s_list[(nsel_w + t) * kQBlock + tid] = uint32_t(bestj);
                maxd2 = fmax(maxd2, bestd);
                lastd = bestd;
                lastj = bestj;
            }
        }
        ntot = nsel_w + needb;
    }
#ifdef GD_KNN_STATS
    A.stats[q * 8 + 0] = refines + 16 * rescales + (ovf ? 1024 : 0);
    A.stats[q * 8 + 1] = visA;
    A.stats[q * 8 + 2] = candA;
    A.stats[q * 8 + 3] = visB;
    A.stats[q * 8 + 4] = c.depth;
    A.stats[q * 8 + 5] = fallback;
    A.stats[q * 8 + 6] = hb;
    A.stats[q * 8 + 7] = visA + visB + visR;
#else
    (void)visA;
    (void)visB;
    (void)visR;
    (void)refines;
    (void)hb;
#endif

    // 5. retained others in ascending slot order; the row is written once
    int32_t v[KP2];
#pragma unroll
    for (int e = 0; e < KP2; ++e) v[e] = (e < ntot) ? int32_t(s_list[e * kQBlock + tid]) : INT32_MAX;
    bitonic_sort<KP2>(v);
    if (k == KP2 && A.row_vec) {  // 16-byte aligned rows: vector stores
#pragma unroll
        for (int c4 = 0; c4 < KP2 / 4; ++c4) {
            int32_t o[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int e = 4 * c4 + t;  // row element; others start at element 1
                o[t] = e == 0 ? q : ((e - 1 < ntot) ? v[e - 1] : -1);
            }
            reinterpret_cast<int4*>(row)[c4] = make_int4(o[0], o[1], o[2], o[3]);
        }
    } else {
        row[0] = q;
#pragma unroll
        for (int e = 0; e < KP2; ++e)
            if (e < k - 1) row[1 + e] = (e < ntot) ? v[e] : -1;
    }
    A.cnt[q] = 1 + ntot;
    A.dmax[q] = ntot > 0 ? sqrt(maxd2) : 0.0;
}

// ---------------------------------------------------------------------------
struct CopyNaArgs {
    const WsHeader* h;
    int32_t* out;
};

struct CopyNa {
    using Args = CopyNaArgs;
    static constexpr int kThreads = 64;
    static __device__ __forceinline__ void body(const Args& A, Blk)
    {
        if (threadIdx.x == 0) *A.out = A.h->n_active;
    }
};

struct KnnSetup {
    TreeLevels T;
    Periodicity P;
    bool per;
    BucketArgs bucket;
    LevelArgs level[kMaxTreeLevels];
    KnnArgs A;
};

static KnnSetup knn_setup(const gd_problem* p, const gd_neighbors* nb, void* ws, const Layout& L)
{
    KnnSetup S{};
    const int64_t n = p->n;
    const WsHeader* h = at<WsHeader>(ws, L.hdr);
    FBox* boxes = at<FBox>(ws, L.boxes);
    const double4* pos = at<double4>(ws, L.pos4);
    TreeLevels& T = S.T;
    T.levels = L.levels;
    for (int l = 0; l < L.levels; ++l) {
        T.off[l] = L.lvl_off[l];
        T.cap[l] = (L.lvl_cnt[l] + kFan - 1) / kFan * kFan;
    }
    T.off1 = int32_t(L.off1);
    T.stride1 = int32_t(L.stride1);
    S.per = false;
    for (int a = 0; a < 3; ++a) {
        S.P.per[a] = p->periodic[a] ? 1 : 0;
        S.P.L[a] = p->L[a];
        S.per = S.per || S.P.per[a];
    }
    S.bucket = BucketArgs{pos, h, boxes + T.off[0], T.cap[0], S.P};
    for (int l = 1; l < L.levels; ++l)
        S.level[l] = LevelArgs{boxes + T.off[l - 1], T.cap[l - 1], boxes + T.off[l], T.cap[l]};
    KnnArgs& A = S.A;
    A.pos = pos;
    A.boxes = boxes;
    A.T = T;
    A.h = h;
    A.n = n;
    A.k = p->k;
    A.rmax2 = p->rmax * p->rmax;
    for (int a = 0; a < 3; ++a) {
        A.per[a] = S.P.per[a];
        A.L[a] = p->L[a];
        A.hL[a] = 0.5 * p->L[a];
    }
    A.nbr = nb->nbr;
    A.row_vec = (reinterpret_cast<uintptr_t>(nb->nbr) & 15) == 0 ? 1 : 0;
    A.cnt = nb->cnt;
    A.dmax = nb->dmax;
    A.hint = at<double>(ws, L.hint);
    A.ws = ws;
    A.xq = at<WsHeader>(ws, L.hdr)->xq[kQueueKnn];
    return S;
}

int launch_knn(const gd_problem* p, const gd_neighbors* nb, void* ws, const Layout& L, hipStream_t st)
{
    const int64_t n = p->n;
    KnnSetup S = knn_setup(p, nb, ws, L);
    const TreeLevels& T = S.T;
    const bool per = S.per;
    prof_mark(GD_PROF_TREE, 0, st);
    // buckets and level 1 (and 2) in one pass, the wide levels above one
    // pass each, the small top levels in one workgroup
    const int64_t g0 = (T.cap[0] + 255) / 256;
    WsHeader* hw = at<WsHeader>(ws, L.hdr);
    int built = 0;
    if (L.levels == 1) {
        hipLaunchKernelGGL(k_bucket_boxes, dim3(unsigned(g0)), dim3(256), 0, st, S.bucket);
    } else {
        const bool two = L.levels > 2 && g0 * 4 >= T.cap[2];
        const TreeLowArgs TL{S.bucket, S.level[1].cur, T.cap[1], two ? S.level[2].cur : nullptr, two ? T.cap[2] : 0,
                             S.A.xq, hw->knn_fb_n};
        hipLaunchKernelGGL(k_tree_low, dim3(unsigned(g0)), dim3(256), 0, st, TL);
        built = two ? 2 : 1;
    }
    int l = built + 1;
    for (; l < L.levels && T.cap[l] > kTailCap; ++l)
        hipLaunchKernelGGL(k_level_boxes, dim3(unsigned((T.cap[l] + 255) / 256)), dim3(256), 0, st, S.level[l]);
    if (l < L.levels) {
        const TreeTailArgs TT{at<FBox>(ws, L.boxes), T, int32_t(l)};
        hipLaunchKernelGGL(k_tree_tail, dim3(1), dim3(256), 0, st, TT);
    }
    prof_mark(GD_PROF_TREE, 1, st);
    KnnArgs& A = S.A;
#ifdef GD_KNN_STATS
    A.stats = at<int32_t>(ws, L.stats);
    launch_fill_i32(A.stats, 8 * n, 0, st);
#endif
    prof_mark(GD_PROF_KNN_QUERY, 0, st);
    if (p->k > 64) {  // one wavefront per query: the per-lane search's lists hold at most 64
        launch_knn_wave(A, per, nullptr, nullptr, n, st);
        prof_mark(GD_PROF_KNN_QUERY, 1, st);
        return 0;
    }
    const dim3 grid(unsigned((n + kQBlock - 1) / kQBlock));
    const bool cleared = L.levels > 1;  // the tree's first pass cleared the counters
    if (!cleared) launch_fill_i32(A.xq, kXcd, 0, st);
    if (p->k <= 33 && kTileSearch) {
        // shared candidate tiles first; the queries they cannot complete go
        // through the per-lane search
        int32_t* fb0 = at<int32_t>(ws, L.keys1);  // keys1 and vals1 (n entries each): free after the sort
        int32_t* fb1 = at<int32_t>(ws, L.vals1);
        if (!cleared) launch_fill_i32(hw->knn_fb_n, 2, 0, st);
        launch_knn_tile(A, per, fb0, fb1, hw->knn_fb_n, st);
        // handed-back queries with a previous distance (usually well under 1%:
        // sparse regions with many candidates) take a wavefront each
        launch_knn_wave(A, per, fb1, hw->knn_fb_n + 1, kFallbackBlocks, st);
        // those without one (the first search of a run) take the per-lane search
        A.list = fb0;
        A.list_n = hw->knn_fb_n;
    }
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

// The search of every run as stages of one interval: the bucket boxes, each
// tree level over the runs that have it, then the queries: k > 64 one
// wavefront per query; k <= 33 (with tiles) the tile search, its fallback
// wavefronts and the per-lane search of the first list; otherwise the
// per-lane search over every query.  Runs are grouped by periodicity and
// k class, a launch per group and stage.
void many_knn(ManyBuilder& B, const std::vector<ManyRun>& R)
{
    const size_t nr = R.size();
    std::vector<KnnSetup> S(nr);
    int maxl = 0;
    for (size_t r = 0; r < nr; ++r) {
        S[r] = knn_setup(&R[r].p, &R[r].nb, R[r].ws, R[r].L);
        maxl = std::max(maxl, R[r].L.levels);
    }
    std::vector<int64_t> nb(nr);
    {
        std::vector<BucketArgs> tab(nr);
        for (size_t r = 0; r < nr; ++r) {
            tab[r] = S[r].bucket;
            nb[r] = cdiv(S[r].T.cap[0], 256);
        }
        B.add<BucketBoxes>(tab, nb);
    }
    for (int l = 1; l < maxl; ++l) {
        std::vector<LevelArgs> tab(nr);
        for (size_t r = 0; r < nr; ++r) {
            const bool has = l < R[r].L.levels;
            tab[r] = has ? S[r].level[l] : LevelArgs{};
            nb[r] = has ? cdiv(S[r].T.cap[l], 256) : 0;
        }
        B.add<LevelBoxes>(tab, nb);
    }
    // query groups: (periodic, class) with class 0: k <= 33, 1: 34..64, 2: > 64
    for (int per = 0; per < 2; ++per) {
        for (int cls = 0; cls < 3; ++cls) {
            std::vector<int64_t> mine(nr, 0);
            bool any = false;
            for (size_t r = 0; r < nr; ++r) {
                const int k = R[r].p.k;
                const int c = k <= 33 ? 0 : (k <= 64 ? 1 : 2);
                mine[r] = (int(S[r].per) == per && c == cls) ? 1 : 0;
                any = any || mine[r];
            }
            if (!any) continue;
            if (cls == 2) {
                std::vector<WaveArgs> tab(nr);
                for (size_t r = 0; r < nr; ++r) {
                    tab[r] = WaveArgs{S[r].A, nullptr, nullptr};
                    nb[r] = mine[r] ? R[r].p.n : 0;
                }
                many_add_wave(B, tab, nb, per);
                continue;
            }
            const bool tile = cls == 0 && B.tune.knn_tile;
            std::vector<ClearArgs> clr(nr);
            for (size_t r = 0; r < nr; ++r) {
                WsHeader* hw = at<WsHeader>(R[r].ws, R[r].L.hdr);
                clr[r] = ClearArgs{S[r].A.xq, kXcd, tile ? hw->knn_fb_n : nullptr, 2};
                nb[r] = mine[r];
            }
            B.add<ClearCounters>(clr, nb);
            std::vector<KnnArgs> qa(nr);
            for (size_t r = 0; r < nr; ++r) qa[r] = S[r].A;
            if (tile) {
                std::vector<TileArgs> tt(nr);
                std::vector<WaveArgs> wt(nr);
                std::vector<int64_t> fnb(nr);
                for (size_t r = 0; r < nr; ++r) {
                    WsHeader* hw = at<WsHeader>(R[r].ws, R[r].L.hdr);
                    int32_t* fb0 = at<int32_t>(R[r].ws, R[r].L.keys1);
                    int32_t* fb1 = at<int32_t>(R[r].ws, R[r].L.vals1);
                    tt[r] = TileArgs{S[r].A, fb0, fb1, hw->knn_fb_n};
                    wt[r] = WaveArgs{S[r].A, fb1, hw->knn_fb_n + 1};
                    qa[r].list = fb0;
                    qa[r].list_n = hw->knn_fb_n;
                    nb[r] = mine[r] ? cdiv(R[r].p.n, kWave) : 0;
                    fnb[r] = mine[r] ? std::max<int64_t>(1, cdiv(R[r].p.n, B.tune.fallback_div)) : 0;
                }
                many_add_tile(B, tt, nb, per);
                many_add_wave(B, wt, fnb, per);
            }
            for (size_t r = 0; r < nr; ++r) nb[r] = mine[r] ? cdiv(R[r].p.n, kQBlock) : 0;
            if (cls == 0) {
                if (per) B.add<KnnQuery<true, 32>>(qa, nb);
                else B.add<KnnQuery<false, 32>>(qa, nb);
            } else {
                if (per) B.add<KnnQuery<true, 64>>(qa, nb);
                else B.add<KnnQuery<false, 64>>(qa, nb);
            }
        }
    }
    // the active counts, for the runs that ask for them
    std::vector<CopyNaArgs> na(nr);
    for (size_t r = 0; r < nr; ++r) {
        na[r] = CopyNaArgs{S[r].A.h, R[r].nb.n_active};
        nb[r] = R[r].nb.n_active ? 1 : 0;
    }
    B.add<CopyNa>(na, nb);
}

}  // namespace gd
