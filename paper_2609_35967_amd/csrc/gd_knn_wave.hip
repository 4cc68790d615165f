// gd_knn_wave.hip -- the N_K nearest neighbours of one query per wavefront
// (Sect. 2.5.1), exact, for any k up to kMaxK.  It serves neighbourhoods too
// large for the per-lane search's registers and LDS lists, and the queries
// that search hands back.
//
// Per query (one 64-lane wavefront):
//   1. the search radius: the particle's distance from the previous search
//      widened by kHintSlack when that is usable, else the smallest, over
//      three windows of k consecutive Morton slots holding the query, of the
//      window's largest d^2 (each window holds k-1 others, so that is an upper
//      bound of the (k-1)-th d^2), capped by the maximum search scale;
//   2. a depth-first traversal of the box tree, eight nodes at a time: each
//      lane tests one child box against the query's sphere (the conservative
//      single-precision test of gd_knn.hpp); passing internal children go on
//      an LDS stack, passing buckets to a bucket buffer;
//   3. the buffered buckets' slots are evaluated four per lane: every other
//      at or below the cut (d^2, slot) <= (R2, J) joins an LDS list of
//      (d^2, slot) pairs, compacted across the wavefront.  When the list
//      would overflow, it is sorted and cut to its k-1 smallest pairs, and the
//      cut moves to the last of them (so equal distances beyond it are
//      decided by slot, and the radius only shrinks, which keeps the pruning
//      of step 2 exact);
//   4. if the previous distance held fewer than k-1 others, the query runs
//      again on the window bound;
//   5. the list is sorted by (d^2, slot), its first min(n, k-1) pairs are
//      sorted by slot and written as the row.
// d^2 is (dx*dx + dy*dy) + dz*dz with every operation rounded on its own, and
// non-negative doubles order as their bit patterns, so the selection is the
// k-1 smallest (d^2, slot) exactly.
#include "gd_common.hpp"
#include "gd_internal.hpp"
#include "gd_knn.hpp"

namespace gd {

constexpr int kWList = 512;    // (d^2, slot) pairs a query keeps; >= (kMaxK - 1) + 4 * kWave
constexpr int kWStack = 1024;  // traversal stack: at most 64 children per level wait on it
constexpr int kWBuf = 128;     // buckets waiting for evaluation: flushed from 64 on
static_assert(kWList >= (kMaxK - 1) + 4 * kWave, "a flush after a cut must fit the list");
static_assert(kWStack >= kMaxTreeLevels * kWave, "the stack holds one expansion per level");

struct WaveLds {
    uint64_t key[kWList];   // d^2 as its bit pattern
    int32_t slot[kWList];
    int32_t stack[kWStack];  // node: level << 27 | index
    int32_t buf[kWBuf];      // bucket indices
};

__device__ inline bool pair_less(uint64_t ka, int32_t sa, uint64_t kb, int32_t sb)
{
    return ka < kb || (ka == kb && sa < sb);
}

// Ascending bitonic sort of (key, slot) pairs [0, size) in LDS, size a power
// of two in [64, kWList]; one wavefront.
__device__ inline void wave_sort_pairs(uint64_t* key, int32_t* slot, int size, int lane)
{
    for (int len = 2; len <= size; len <<= 1) {
        for (int stride = len >> 1; stride > 0; stride >>= 1) {
            for (int i = lane; i < size; i += kWave) {
                const int j = i ^ stride;
                if (j > i) {
                    const uint64_t ki = key[i], kj = key[j];
                    const int32_t si = slot[i], sj = slot[j];
                    const bool up = (i & len) == 0;
                    const bool swap = up ? pair_less(kj, sj, ki, si) : pair_less(ki, si, kj, sj);
                    if (swap) {
                        key[i] = kj;
                        key[j] = ki;
                        slot[i] = sj;
                        slot[j] = si;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Ascending bitonic sort of int32 [0, size) in LDS, size a power of two.
__device__ inline void wave_sort_i32(int32_t* v, int size, int lane)
{
    for (int len = 2; len <= size; len <<= 1) {
        for (int stride = len >> 1; stride > 0; stride >>= 1) {
            for (int i = lane; i < size; i += kWave) {
                const int j = i ^ stride;
                if (j > i) {
                    const int32_t a = v[i], b = v[j];
                    const bool up = (i & len) == 0;
                    if (up ? (b < a) : (a < b)) {
                        v[i] = b;
                        v[j] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
}

__device__ inline int pow2_at_least(int n, int lo)
{
    int s = lo;
    while (s < n) s <<= 1;
    return s;
}

__device__ inline uint64_t d2_key(double d2) { return uint64_t(__double_as_longlong(d2)); }

template <bool PER>
__device__ void knn_wave_query(const KnnArgs& A, int q, WaveLds& L, int lane)
{
    const int na = A.h->n_active;
    const int k = A.k;
    const int need = k - 1;
    int32_t* row = A.nbr + int64_t(q) * k;
    if (q >= na || na == 1) {
        const bool act = q < na;
        for (int s = lane; s < k; s += kWave) row[s] = s == 0 ? (act ? q : -1) : -1;
        if (lane == 0) {
            A.cnt[q] = act ? 1 : 0;
            A.dmax[q] = 0.0;
        }
        return;
    }
    const double4 q4 = A.pos[q];
    const double qp[3] = {q4.x, q4.y, q4.z};
    if (!(fabs(qp[0]) < INFINITY && fabs(qp[1]) < INFINITY && fabs(qp[2]) < INFINITY)) {
        if (lane == 0) set_status(A.ws, GD_DEV_NONFINITE);  // non-finite position: self only
        for (int s = lane; s < k; s += kWave) row[s] = s == 0 ? q : -1;
        if (lane == 0) {
            A.cnt[q] = 1;
            A.dmax[q] = 0.0;
        }
        return;
    }
    QF qf;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        qf.c[a] = float(qp[a]);
        qf.p[a] = PER ? float(qp[a] + A.L[a]) : 0.0f;
        qf.m[a] = PER ? float(qp[a] - A.L[a]) : 0.0f;
    }

    // 1. the previous distance as the first radius, when usable: positive,
    //    finite and within the diagonal of the active set's box
    double R2hint = INFINITY;
    {
        const double hv = A.hint[q] * kHintSlack;
        if (hv > 0.0 && hv < INFINITY) {
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
    // the window bound (computed only when needed)
    auto window_bound = [&]() {
        const int span = na < k ? na : k;
        const int fmaxs = na - span;
        int f[3] = {q - span + 1, q - span / 2 + 1, q};
        double w[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            f[t] = f[t] < 0 ? 0 : (f[t] > fmaxs ? fmaxs : f[t]);
            for (int j = f[t] + lane; j < f[t] + span; j += kWave) w[t] = fmax(w[t], sep2_slot<PER>(A, qp, j));
            w[t] = wave_max_d(w[t]);
        }
        return fmin(w[0], fmin(w[1], w[2]));
    };

    bool use_hint = R2hint < INFINITY;
    double R2cap = use_hint ? A.rmax2 : fmin(window_bound(), A.rmax2);
    int n = 0;
    double R2 = 0.0;
    int32_t Jc = INT32_MAX;
    const int top = A.T.levels - 1;  // the root's children: the boxes of the top stored level
    for (;;) {
        R2 = use_hint ? fmin(R2hint, R2cap) : R2cap;
        Jc = INT32_MAX;
        n = 0;
        float R2f = r2f(R2);
        int sp = 0, nbuf = 0;
        // cut the list to its k-1 smallest pairs; the cut moves to the last
        auto cut_list = [&]() {
            const int size = pow2_at_least(n, kWave);
            for (int e = n + lane; e < size; e += kWave) {
                L.key[e] = ~uint64_t(0);
                L.slot[e] = INT32_MAX;
            }
            __syncthreads();
            wave_sort_pairs(L.key, L.slot, size, lane);
            const int keep = need < n ? need : n;
            if (keep > 0) {
                R2 = __longlong_as_double((long long)L.key[keep - 1]);
                Jc = L.slot[keep - 1];
                R2f = r2f(R2);
            }
            n = keep;
            __syncthreads();
        };
        // evaluate the buffered buckets, 64 at a time, four slots per lane
        auto flush = [&]() {
            for (int b0 = 0; b0 < nbuf; b0 += kWave) {
                const int nb = nbuf - b0 < kWave ? nbuf - b0 : kWave;
                double d2[4];
                int32_t jj[4];
                bool acc[4];
                int total = 0;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int p = lane + kWave * t;
                    const int b = p >> 2;
                    const int j = b < nb ? L.buf[b0 + b] * kBucket + (p & 3) : -1;
                    jj[t] = j;
                    const bool ok = j >= 0 && j < na && j != q;
                    d2[t] = ok ? sep2_slot<PER>(A, qp, j) : INFINITY;
                    acc[t] = ok && (d2[t] < R2 || (d2[t] == R2 && j <= Jc));
                    total += __popcll(__ballot(acc[t]));
                }
                if (n + total > kWList) {
                    cut_list();
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        acc[t] = acc[t] && (d2[t] < R2 || (d2[t] == R2 && jj[t] <= Jc));
                }
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const uint64_t bal = __ballot(acc[t]);
                    if (acc[t]) {
                        const int at = n + int(__popcll(bal & ((uint64_t(1) << lane) - 1)));
                        L.key[at] = d2_key(d2[t]);
                        L.slot[at] = jj[t];
                    }
                    n += int(__popcll(bal));
                }
            }
            nbuf = 0;
            __syncthreads();
        };
        // the root's children
        {
            const int lv = top;
            const bool valid = lane < kFan && (uint32_t(lane) < uint32_t(A.T.cap[top])) &&
                               ((live_children(na, top + 1, 0) >> lane) & 1u);
            bool pass = false;
            if (valid) pass = box2f<PER>(A, qf, A.boxes[level_off(A.T, lv) + lane]) <= R2f;
            const uint64_t bal = __ballot(pass);
            if (pass) {
                const int at = int(__popcll(bal & ((uint64_t(1) << lane) - 1)));
                if (lv == 0) L.buf[at] = lane;
                else L.stack[at] = (lv << 27) | lane;
            }
            if (lv == 0) nbuf = int(__popcll(bal));
            else sp = int(__popcll(bal));
            __syncthreads();
        }
        while (sp > 0) {
            const int nt = sp < kFan ? sp : kFan;
            const int src = sp - nt;
            const int my = lane >> 3, c = lane & 7;
            const int32_t node = my < nt ? L.stack[src + my] : 0;
            __syncthreads();
            sp = src;
            const int lv = node >> 27, idx = node & ((1 << 27) - 1);
            bool pass = false;
            bool leaf = false;
            if (my < nt && ((live_children(na, lv, idx) >> c) & 1u)) {
                const FBox bx = A.boxes[level_off(A.T, lv - 1) + idx * kFan + c];
                pass = box2f<PER>(A, qf, bx) <= R2f;
                leaf = lv == 1;
            }
            const uint64_t bin = __ballot(pass && !leaf), bleaf = __ballot(pass && leaf);
            const uint64_t below = (uint64_t(1) << lane) - 1;
            if (pass && !leaf) L.stack[sp + int(__popcll(bin & below))] = ((lv - 1) << 27) | (idx * kFan + c);
            if (pass && leaf) L.buf[nbuf + int(__popcll(bleaf & below))] = idx * kFan + c;
            sp += int(__popcll(bin));
            nbuf += int(__popcll(bleaf));
            __syncthreads();
            if (nbuf >= kWave) flush();
        }
        flush();
        if (use_hint && n < need && R2hint < R2cap) {
            use_hint = false;  // the previous distance held too few others: again on the bound
            R2cap = fmin(window_bound(), A.rmax2);
            continue;
        }
        break;
    }
    // 5. the k-1 smallest pairs (all of them when fewer are within the cap),
    //    then their slots in ascending order
    const int size = pow2_at_least(n, kWave);
    for (int e = n + lane; e < size; e += kWave) {
        L.key[e] = ~uint64_t(0);
        L.slot[e] = INT32_MAX;
    }
    __syncthreads();
    wave_sort_pairs(L.key, L.slot, size, lane);
    const int m = need < n ? need : n;
    const double maxd2 = m > 0 ? __longlong_as_double((long long)L.key[m - 1]) : 0.0;
    const int size2 = pow2_at_least(m, kWave);
    for (int e = m + lane; e < size2; e += kWave) L.slot[e] = INT32_MAX;
    __syncthreads();
    wave_sort_i32(L.slot, size2, lane);
    for (int s = lane; s < k; s += kWave) row[s] = s == 0 ? q : (s - 1 < m ? L.slot[s - 1] : -1);
    if (lane == 0) {
        A.cnt[q] = 1 + m;
        A.dmax[q] = m > 0 ? sqrt(maxd2) : 0.0;
    }
    __syncthreads();
}

// One query per 64-thread workgroup: every slot [0, n), or the slots of
// `list` [0, *count) when a list is given.
template <bool PER>
struct KnnWave {
    using Args = WaveArgs;
    static constexpr int kThreads = kWave;
    static __device__ __forceinline__ void body(const Args& W, Blk B)
    {
        __shared__ WaveLds L;
        const int lane = threadIdx.x;
        if (W.list) {
            const int32_t nl = *W.count;
            for (int64_t t = B.id; t < nl; t += B.n) knn_wave_query<PER>(W.A, W.list[t], L, lane);
        } else {
            const int64_t q = B.id;
            if (q < W.A.n) knn_wave_query<PER>(W.A, int(q), L, lane);
        }
    }
};

template <bool PER>
__global__ __launch_bounds__(kWave) void k_knn_wave(WaveArgs W)
{
    KnnWave<PER>::body(W, Blk{W.list ? int64_t(blockIdx.x) : xcd_block(), int64_t(gridDim.x)});
}

void launch_knn_wave(const KnnArgs& A, bool per, const int32_t* list, const int32_t* count, int64_t nblocks,
                     hipStream_t st)
{
    const dim3 grid(unsigned(nblocks > 0 ? nblocks : 1));
    const WaveArgs W{A, list, count};
    if (per) hipLaunchKernelGGL(k_knn_wave<true>, grid, dim3(kWave), 0, st, W);
    else hipLaunchKernelGGL(k_knn_wave<false>, grid, dim3(kWave), 0, st, W);
}

void many_add_wave(ManyBuilder& B, const std::vector<WaveArgs>& tab, const std::vector<int64_t>& nb, bool per)
{
    if (per) B.add<KnnWave<true>>(tab, nb);
    else B.add<KnnWave<false>>(tab, nb);
}

}  // namespace gd
