// gd_knn.hip -- N_K nearest neighbours of every active particle (Sect. 2.5.1),
// exact, on a linear bounding-volume hierarchy over the Morton order.
//
// Tree: the binary radix tree of Karras (2012, "Maximizing parallelism in the
// construction of BVHs, octrees, and k-d trees") over the sorted 30-bit keys
// (ties broken by slot), boxes filled bottom-up.  Each internal node covers a
// contiguous slot range; subtrees of <= kLeafB slots are scanned directly.
// Stackless depth-first traversal: every node stores its "rope", the next
// node after its subtree; the rope of a subtree ending at slot l is the right
// child of the node that splits at l.
//
// Query (one lane per particle; all per-lane scratch in LDS columns, so no
// barriers):
//   1. descend by slot to the deepest ancestor holding >= k particles; its box
//      bounds the k-th distance from above and gives a density estimate;
//   2. pass A: count candidates inside a trial radius into 32 bins of d^2
//      (grow the radius until k-1 others are inside);
//   3. the bin holding the (k-1)-th other splits the candidates into "sure"
//      (lower bins) and "boundary"; an over-full boundary bin is re-binned
//      (nested bins) until it holds <= kC1 candidates;
//   4. pass B: walk again inside the tightened radius, append sure slots to the
//      output row and keep boundary slots; rank the boundary by (d^2, slot);
//   5. sort the retained others by slot in registers.
// Every bin function is monotone in d^2, so the selection is exactly the k-1
// smallest (d^2, slot); d^2 is computed as (dx*dx + dy*dy) + dz*dz, unfused.
#include "gd_common.hpp"
#include "gd_internal.hpp"

namespace gd {

constexpr int32_t kEnd = INT32_MIN;
constexpr int kLeafB = 8;
constexpr int kNB = 32;
constexpr int kC1 = 16;
constexpr int kDMax = 4;
constexpr int kQBlock = 256;

// ---------------------------------------------------------------------------
// Tree build
__device__ inline int delta(const uint32_t* __restrict__ keys, int na, int i, int64_t j)
{
    if (j < 0 || j >= na) return -1;
    const uint32_t a = keys[i], b = keys[j];
    if (a == b) return 32 + __clz(uint32_t(i) ^ uint32_t(j));
    return __clz(a ^ b);
}

__global__ __launch_bounds__(256) void k_lbvh_internal(const uint32_t* __restrict__ keys,
                                                       const WsHeader* __restrict__ h, Node* __restrict__ nodes,
                                                       int32_t* __restrict__ parent, int32_t* __restrict__ rc,
                                                       int64_t n)
{
    const int na = h->n_active;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= na - 1) return;
    const int d = (delta(keys, na, i, i + 1) - delta(keys, na, i, i - 1)) >= 0 ? 1 : -1;
    const int dmin = delta(keys, na, i, i - d);
    int64_t lmax = 2;
    while (delta(keys, na, i, i + lmax * d) > dmin) lmax <<= 1;
    int64_t l = 0;
    for (int64_t t = lmax >> 1; t >= 1; t >>= 1)
        if (delta(keys, na, i, i + (l + t) * d) > dmin) l += t;
    const int j = int(i + l * d);
    const int dnode = delta(keys, na, i, j);
    int64_t s = 0;
    for (int64_t div = 2;; div <<= 1) {
        const int64_t t = (l + div - 1) / div;
        if (delta(keys, na, i, i + (s + t) * d) > dnode) s += t;
        if (t <= 1) break;
    }
    const int gamma = int(i + s * d + (d < 0 ? d : 0));
    const int first = i < j ? i : j, last = i < j ? j : i;
    nodes[i].first = first;
    nodes[i].last = last;
    nodes[i].split = gamma;
    const int left = (first == gamma) ? ~gamma : gamma;
    const int right = (last == gamma + 1) ? ~(gamma + 1) : gamma + 1;
    if (left >= 0) parent[left] = i; else parent[n + gamma] = i;
    if (right >= 0) parent[right] = i; else parent[n + gamma + 1] = i;
    rc[gamma] = right;
    if (i == 0) parent[0] = -1;
}

__global__ __launch_bounds__(256) void k_lbvh_boxes(const double4* __restrict__ pos, const WsHeader* __restrict__ h,
                                                    Node* nodes, const int32_t* __restrict__ parent,
                                                    int32_t* flags, const int32_t* __restrict__ rc, int64_t n)
{
    const int na = h->n_active;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= na || na < 2) return;
    int p = parent[n + j];
    volatile Node* vn = nodes;
    while (p >= 0) {
        __threadfence();
        if (atomicAdd(&flags[p], 1) == 0) return;
        __threadfence();
        const int first = vn[p].first, last = vn[p].last, sp = vn[p].split;
        double lo[3], hi[3];
        const int ch[2] = {(sp == first) ? ~sp : sp, (sp + 1 == last) ? ~(sp + 1) : sp + 1};
        for (int c = 0; c < 2; ++c) {
            double clo[3], chi[3];
            if (ch[c] < 0) {
                const double4 q = pos[~ch[c]];
                clo[0] = chi[0] = q.x;
                clo[1] = chi[1] = q.y;
                clo[2] = chi[2] = q.z;
            } else {
                for (int a = 0; a < 3; ++a) {
                    clo[a] = vn[ch[c]].lo[a];
                    chi[a] = vn[ch[c]].hi[a];
                }
            }
            for (int a = 0; a < 3; ++a) {
                lo[a] = c ? fmin(lo[a], clo[a]) : clo[a];
                hi[a] = c ? fmax(hi[a], chi[a]) : chi[a];
            }
        }
        for (int a = 0; a < 3; ++a) {
            vn[p].lo[a] = lo[a];
            vn[p].hi[a] = hi[a];
        }
        vn[p].rope = (last == na - 1) ? kEnd : rc[last];
        p = parent[p];
    }
}

// ---------------------------------------------------------------------------
// Query
struct KnnArgs {
    const double4* pos;
    const Node* nodes;
    const int32_t* rc;
    const WsHeader* h;
    int64_t n;
    int32_t k;
    double rmax2;
    int32_t per[3];
    double L[3], hL[3];
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

template <bool PER>
__device__ inline double box2(const KnnArgs& A, const double q[3], const Node& nd)
{
    double g[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double v = gap(q[a], nd.lo[a], nd.hi[a]);
        if (PER && A.per[a]) v = fmin(v, fmin(gap(q[a] + A.L[a], nd.lo[a], nd.hi[a]), gap(q[a] - A.L[a], nd.lo[a], nd.hi[a])));
        g[a] = v;
    }
    const double s = g[0] * g[0] + g[1] * g[1];
    return s + g[2] * g[2];
}

// Visit every active slot j != q with d^2(q, j) <= R2; f(j, d2).
template <bool PER, class F>
__device__ inline void traverse(const KnnArgs& A, int na, int q, const double qp[3], double R2, F&& f)
{
    const double R2box = R2 * (1.0 + 1e-12);
    int node = 0;
    // a well-formed tree visits each of its 2 na - 1 nodes at most once
    for (int64_t steps = 0; node != kEnd; ++steps) {
        if (steps > 2 * int64_t(na) + 8) {
            set_status(A.ws, GD_DEV_INTERNAL);
            break;
        }
        if (node < 0) {
            const int j = ~node;
            if (j != q) {
                const double d2 = sep2<PER>(A, qp, A.pos[j]);
                if (d2 <= R2) f(j, d2);
            }
            node = (j == na - 1) ? kEnd : A.rc[j];
            continue;
        }
        const Node nd = A.nodes[node];
        if (box2<PER>(A, qp, nd) > R2box) {
            node = nd.rope;
            continue;
        }
        if (nd.last - nd.first < kLeafB) {
            for (int j = nd.first; j <= nd.last; ++j) {
                if (j == q) continue;
                const double d2 = sep2<PER>(A, qp, A.pos[j]);
                if (d2 <= R2) f(j, d2);
            }
            node = nd.rope;
            continue;
        }
        node = (nd.split == nd.first) ? ~nd.split : nd.split;
    }
}

__device__ inline int bin_at(double d2, double lo, double s)
{
    const double t = (d2 - lo) * s;
    if (!(t < double(kNB))) return kNB - 1;
    if (!(t > 0.0)) return 0;
    return int(t);
}

struct Chain {
    int depth;
    double lo[kDMax + 1];
    double s[kDMax + 1];
    int bstar[kDMax];
};

enum { kSure = 0, kBoundary = 1, kReject = 2 };

__device__ inline int classify(const Chain& c, double d2)
{
#pragma unroll
    for (int l = 0; l < kDMax; ++l) {
        if (l < c.depth) {
            const int b = bin_at(d2, c.lo[l], c.s[l]);
            if (b < c.bstar[l]) return kSure;
            if (b > c.bstar[l]) return kReject;
        }
    }
    return kBoundary;
}

__device__ inline int chain_bin(const Chain& c, double d2)
{
    double lo = c.lo[0], s = c.s[0];
#pragma unroll
    for (int l = 1; l <= kDMax; ++l)
        if (l == c.depth) { lo = c.lo[l]; s = c.s[l]; }
    return bin_at(d2, lo, s);
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
    __shared__ uint32_t s_hist[kNB * kQBlock];
    __shared__ int32_t s_bnd[kC1 * kQBlock];
    const int tid = threadIdx.x;
    const int64_t q64 = blockIdx.x * int64_t(kQBlock) + tid;
    if (q64 >= A.n) return;
    const int q = int(q64);
    const int na = A.h->n_active;
    const int k = A.k;
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

    // 1. descent to the deepest ancestor of q holding >= k slots
    int first = 0, last = na - 1;
    Node nd = A.nodes[0];
    for (;;) {
        const int sp = nd.split;
        int cf, cl, cref;
        if (q <= sp) { cf = first; cl = sp; cref = (sp == first) ? ~sp : sp; }
        else { cf = sp + 1; cl = last; cref = (sp + 1 == last) ? ~(sp + 1) : sp + 1; }
        if (cref < 0 || cl - cf + 1 < k) break;
        first = cf;
        last = cl;
        nd = A.nodes[cref];
    }
    double ub[3], vol = 1.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double m = fmax(qp[a] - nd.lo[a], nd.hi[a] - qp[a]);
        if (PER && A.per[a]) m = fmin(m, A.hL[a]);
        ub[a] = m;
        vol *= (nd.hi[a] - nd.lo[a]);
    }
    double R2ub = (ub[0] * ub[0] + ub[1] * ub[1]) + ub[2] * ub[2];
    R2ub = R2ub * (1.0 + 1e-12);
    const int size = last - first + 1;
    double R2 = R2ub;
    if (vol > 0.0) {
        const double r = cbrt(3.0 * double(k) * vol / (4.0 * kPi * double(size))) * 1.3;
        R2 = fmin(R2, r * r);
    }
    const double R2cap = fmin(R2ub, A.rmax2);
    R2 = fmin(R2, R2cap);
    const int need = k - 1;

    // 2. pass A at depth 0, growing the radius until k-1 others are inside
    Chain c;
    c.depth = 0;
    int total = 0;
    for (int it = 0;; ++it) {
        if (it > 64 || !(R2 >= 0.0)) {  // non-finite positions: give up on this particle
            set_status(A.ws, GD_DEV_NONFINITE);
            break;
        }
        for (int b = 0; b < kNB; ++b) s_hist[b * kQBlock + tid] = 0;
        total = 0;
        c.lo[0] = 0.0;
        c.s[0] = R2 > 0.0 ? double(kNB) / R2 : 0.0;
        const double s0 = c.s[0];
        traverse<PER>(A, na, q, qp, R2, [&](int j, double d2) {
            ++total;
            s_hist[bin_at(d2, 0.0, s0) * kQBlock + tid] += 1u;
        });
        if (total >= need || R2 >= R2cap) break;
        if (R2 > 0.0) {
            const double g = fmax(4.0, 2.0 * pow((need + 1.0) / (total + 1.0), 2.0 / 3.0));
            R2 = fmin(R2cap, R2 * g);
        } else {
            R2 = R2cap;
        }
    }

    // 3. locate the (k-1)-th other; refine an over-full boundary bin
    int c0 = 0, c1 = 0;
    bool fallback = false;
    if (total < need) {
        c.depth = 1;
        c.bstar[0] = kNB;   // every candidate inside R2 is kept
        c0 = total;
        c1 = 0;
    } else {
        for (;;) {
            const int D = c.depth;
            const int needD = need - c0;
            int cum = 0, bs = kNB - 1, hb = 0;
            for (int b = 0; b < kNB; ++b) {
                const int hv = int(s_hist[b * kQBlock + tid]);
                if (cum + hv >= needD) { bs = b; hb = hv; break; }
                cum += hv;
            }
#pragma unroll
            for (int l = 0; l < kDMax; ++l)
                if (l == D) c.bstar[l] = bs;
            c.depth = D + 1;
            c0 += cum;
            c1 = hb;
            if (c1 <= kC1) break;
            // next level splits bin bs of this level into kNB sub-bins
            double loD = c.lo[0], sD = c.s[0];
#pragma unroll
            for (int l = 1; l < kDMax; ++l)
                if (l == D) { loD = c.lo[l]; sD = c.s[l]; }
            const double lo2 = loD + double(bs) / sD;
            const double s2 = sD * double(kNB);
            if (c.depth >= kDMax || !(s2 < 1e300) || lo2 + 1.0 / s2 == lo2) {
                fallback = true;
                break;
            }
#pragma unroll
            for (int l = 1; l <= kDMax; ++l)
                if (l == c.depth) { c.lo[l] = lo2; c.s[l] = s2; }
            for (int b = 0; b < kNB; ++b) s_hist[b * kQBlock + tid] = 0;
            traverse<PER>(A, na, q, qp, R2, [&](int j, double d2) {
                if (classify(c, d2) == kBoundary) s_hist[chain_bin(c, d2) * kQBlock + tid] += 1u;
            });
        }
    }

    // 4. pass B inside the tightened radius
    double R2B = R2;
    if (c.bstar[0] < kNB && c.s[0] > 0.0) R2B = fmin(R2, (double(c.bstar[0] + 1) / c.s[0]) * (1.0 + 1e-12));
    int nsel = 0, nb = 0;
    double maxd2 = 0.0;
    traverse<PER>(A, na, q, qp, R2B, [&](int j, double d2) {
        const int cl = classify(c, d2);
        if (cl == kSure) {
            if (nsel < need) row[1 + nsel] = j;
            ++nsel;
            maxd2 = fmax(maxd2, d2);
        } else if (cl == kBoundary) {
            if (nb < kC1) s_bnd[nb * kQBlock + tid] = j;
            ++nb;
        }
    });
    if (nsel != c0) set_status(A.ws, GD_DEV_INTERNAL);
    const int needb = need - nsel < nb ? need - nsel : nb;
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
                row[1 + nsel + rank] = bj[e];
                maxd2 = fmax(maxd2, bd[e]);
            }
        }
    } else {
        set_status(A.ws, GD_DEV_KNN_FALLBACK);
        double lastd = -1.0;
        int lastj = -1;
        for (int t = 0; t < needb; ++t) {
            double bestd = INFINITY;
            int bestj = INT32_MAX;
            traverse<PER>(A, na, q, qp, R2B, [&](int j, double d2) {
                if (classify(c, d2) != kBoundary) return;
                const bool after = (d2 > lastd) || (d2 == lastd && j > lastj);
                const bool better = (d2 < bestd) || (d2 == bestd && j < bestj);
                if (after && better) { bestd = d2; bestj = j; }
            });
            row[1 + nsel + t] = bestj;
            maxd2 = fmax(maxd2, bestd);
            lastd = bestd;
            lastj = bestj;
        }
    }
    const int ntot = nsel + needb;

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
int launch_lbvh_knn(const gd_problem* p, const gd_neighbors* nb, void* ws, const Layout& L, hipStream_t st)
{
    const int64_t n = p->n;
    const WsHeader* h = at<WsHeader>(ws, L.hdr);
    const uint32_t* keys = at<uint32_t>(ws, L.keys0);
    Node* nodes = at<Node>(ws, L.nodes);
    int32_t* parent = at<int32_t>(ws, L.parent);
    int32_t* flags = at<int32_t>(ws, L.flags);
    int32_t* rc = at<int32_t>(ws, L.rc);
    const double4* pos = at<double4>(ws, L.pos4);
    const int nb_ = int((n + 255) / 256);
    prof_mark(GD_PROF_TREE, 0, st);
    launch_fill_i32(flags, n, 0, st);
    hipLaunchKernelGGL(k_lbvh_internal, dim3(nb_), dim3(256), 0, st, keys, h, nodes, parent, rc, n);
    hipLaunchKernelGGL(k_lbvh_boxes, dim3(nb_), dim3(256), 0, st, pos, h, nodes, parent, flags, rc, n);
    prof_mark(GD_PROF_TREE, 1, st);
    KnnArgs A{};
    A.pos = pos;
    A.nodes = nodes;
    A.rc = rc;
    A.h = h;
    A.n = n;
    A.k = p->k;
    A.rmax2 = p->rmax * p->rmax;
    bool per = false;
    for (int a = 0; a < 3; ++a) {
        A.per[a] = p->periodic[a] ? 1 : 0;
        A.L[a] = p->L[a];
        A.hL[a] = 0.5 * p->L[a];
        per = per || A.per[a];
    }
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
