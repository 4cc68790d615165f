// gd_knn_tile.hip -- the N_K nearest neighbours (N_K <= 33) of the 64
// Morton-consecutive queries of a wavefront from shared candidate lists
// (Sect. 2.5.1), exact.
//
// The per-lane search of gd_knn.hip walks the tree once per query; most of
// its instructions go to box tests and walk bookkeeping, not to distances.
// Here the wavefront's queries share the walk:
//   1. each lane's radius is its particle's distance from the previous search
//      widened by kHintSlack (a lane without a usable one is handed back, see
//      6); eight groups of eight Morton-consecutive lanes each bound their
//      spheres by one box, rounded outward to single precision;
//   2. the box tree is traversed breadth first, eight nodes (64 child boxes)
//      at a time, testing each child against the boxes of the groups its
//      parent met; the buckets reached come out as (bucket, group) pairs;
//   3. each pair's bucket is tested against the spheres of its group's eight
//      lanes (the conservative single-precision test of gd_knn.hpp); a bucket
//      one of them may reach joins that group's bucket list, and the lanes
//      whose sphere may reach it mark its place in their own bit masks;
//   4. every lane takes the buckets of its mask in turn, loads their four
//      positions and evaluates the exact d^2 to each (the next bucket's loads
//      in flight meanwhile).  Others within the radius are counted into the
//      lane's logarithmic bins and recorded, with their bin, in its LDS list
//      (a full list drops the entries above the bin that already completes
//      k-1);
//   5. the bin holding the (k-1)-th other splits the list into sure entries
//      and a boundary bin ranked by (d^2, slot); the row is written once, in
//      slot order;
//   6. lanes without a usable previous distance, whose radius held fewer
//      than k-1 others, whose list or group list overflowed, or whose
//      boundary bin is over-full, go to a list that the per-lane search then
//      completes.  The result never depends on which lanes go there.
// d^2 is (dx*dx + dy*dy) + dz*dz with every operation rounded on its own, and
// every bin function is monotone in d^2, so each row is the k-1 smallest
// (d^2, slot) exactly.
#include "gd_common.hpp"
#include "gd_internal.hpp"
#include "gd_knn.hpp"

namespace gd {

constexpr int kTG = 8;               // lanes (queries) per group
constexpr int kNGrp = kWave / kTG;   // groups per wavefront
constexpr int kTList = 64;           // candidate list entries per lane
constexpr int kFront = 512;          // traversal frontier (nodes of one level)
constexpr int kPairs = 512;          // (bucket, group) pairs awaiting their sphere tests
constexpr int kGList = 128;          // buckets per group after the sphere tests
constexpr int kMaskW = kGList / 32;  // words of a lane's bucket mask
static_assert(kGList * kBucket <= 2048, "a list entry keeps the bucket's place and slot in 11 bits");

template <bool PER>
struct TileLds {
    union {
        // traversal and sphere tests
        struct {
            uint32_t front[2][kFront];  // node | group mask << 24
            uint32_t pairs[kPairs];     // bucket | group << 24
            uint8_t gm[kNGrp][kGList];  // per place in a group's list: its lanes whose sphere may reach it
            float4 sc[kWave];           // query (single precision) and its threshold (negative: none)
            float4 sp[PER ? kWave : 1]; // its +L and -L images on periodic axes
            float4 sm[PER ? kWave : 1];
        } t;
        // distances: per-lane candidate lists (bin << 11 | place in the
        // group's list * 4 + slot in the bucket); at the end the boundary
        // entries wait at the tail
        struct {
            uint16_t list[kTList][kWave];
        } d;
    } u;
    uint32_t glist[kNGrp][kGList];
    float gbox[kNGrp][6];            // group boxes: lo[3], hi[3]
};

// 32 per-lane 8-bit bin counters in 8 registers
struct Hist8 {
    uint32_t w[kNB / 4];
    __device__ void clear()
    {
#pragma unroll
        for (int i = 0; i < kNB / 4; ++i) w[i] = 0;
    }
    __device__ void add(int b)
    {
#pragma unroll
        for (int i = 0; i < kNB / 4; ++i) w[i] += (b >> 2) == i ? (1u << (8 * (b & 3))) : 0u;
    }
    __device__ int get(int b) const { return int((w[b >> 2] >> (8 * (b & 3))) & 0xFFu); }
};

__device__ inline bool span_meets(float lo, float hi, float blo, float bhi) { return (blo <= hi) & (lo <= bhi); }

// does box b meet group box g (with its periodic images)?
template <bool PER>
__device__ inline bool group_meets(const KnnArgs& A, const float (&g)[6], const FBox& b)
{
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        bool m = span_meets(g[a], g[3 + a], b.lo[a], b.hi[a]);
        if (PER && A.per[a]) {
            const double L = A.L[a];
            m = m | span_meets(__double2float_rd(double(g[a]) + L), __double2float_ru(double(g[3 + a]) + L), b.lo[a],
                               b.hi[a]);
            m = m | span_meets(__double2float_rd(double(g[a]) - L), __double2float_ru(double(g[3 + a]) - L), b.lo[a],
                               b.hi[a]);
        }
        ok = ok & m;
    }
    return ok;
}

template <bool PER>
struct KnnTile {
    using Args = TileArgs;
    static constexpr int kThreads = kWave;
    static __device__ __forceinline__ void body(const Args& TA, Blk B);
};

template <bool PER>
__global__ __launch_bounds__(kWave) void k_knn_tile(TileArgs TA)
{
    KnnTile<PER>::body(TA, Blk{int64_t(blockIdx.x), int64_t(gridDim.x)});
}

// (the grid holds exactly the run's items, one wavefront each; the item of a
// block is fixed by the die it runs on, so that the Morton-near particles a
// die's wavefronts gather stay in its L2.  A queue of atomic counters per die
// balanced the dies dynamically but cost more than it gained: ~30 us per
// launch on the 1M disk)
template <bool PER>
__device__ __forceinline__ void KnnTile<PER>::body(const Args& TA, Blk B)
{
    const KnnArgs& A = TA.A;
    int32_t* __restrict__ fb0 = TA.fb0;
    int32_t* __restrict__ fb1 = TA.fb1;
    int32_t* __restrict__ fb_n = TA.fb_n;
    __shared__ TileLds<PER> L;
    const int lane = threadIdx.x;
    const int64_t item = xcd_item(B.id, B.n);
    if (item * kWave >= A.n) return;
    const int64_t q64 = int64_t(item) * kWave + lane;
    const int q = int(q64);
    const int na = A.h->n_active;
    const int k = A.k;
    const int need = k - 1;
    const bool inq = q64 < A.n;
    const bool act = inq && q < na;
    int32_t* row = A.nbr + (inq ? int64_t(q) * k : 0);
    if (inq && !act) {  // an inactive slot
        for (int s = 0; s < k; ++s) row[s] = -1;
        A.cnt[q] = 0;
        A.dmax[q] = 0.0;
    }
    double qp[3] = {0.0, 0.0, 0.0};
    bool ok = false, fb = false;
    if (act) {
        const double4 q4 = A.pos[q];
        qp[0] = q4.x;
        qp[1] = q4.y;
        qp[2] = q4.z;
        if (!(fabs(qp[0]) < INFINITY && fabs(qp[1]) < INFINITY && fabs(qp[2]) < INFINITY)) {
            set_status(A.ws, GD_DEV_NONFINITE);  // non-finite position: self only
            row[0] = q;
            for (int s = 1; s < k; ++s) row[s] = -1;
            A.cnt[q] = 1;
            A.dmax[q] = 0.0;
        } else {
            fb = true;  // unless the tiles complete it
            ok = na > k;
        }
    }
    // 1. radius from the previous distance: positive, finite, within the
    //    diagonal of the active set's box and below the maximum search scale
    double R2 = 0.0;
    if (ok) {
        const double hv = A.hint[q] * kHintSlack;
        ok = hv > 0.0 && hv < INFINITY;
        if (ok) {
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
            R2 = hv * hv;
            ok = R2 <= e2 && R2 < A.rmax2;
        }
    }
    const bool tried = ok;  // searched with a usable previous distance
    QF qf;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        qf.c[a] = float(qp[a]);
        qf.p[a] = PER ? float(qp[a] + A.L[a]) : 0.0f;
        qf.m[a] = PER ? float(qp[a] - A.L[a]) : 0.0f;
    }
    L.u.t.sc[lane] = make_float4(qf.c[0], qf.c[1], qf.c[2], ok ? r2f(R2) : -1.0f);
    if (PER) {
        L.u.t.sp[lane] = make_float4(qf.p[0], qf.p[1], qf.p[2], 0.0f);
        L.u.t.sm[lane] = make_float4(qf.m[0], qf.m[1], qf.m[2], 0.0f);
    }
    reinterpret_cast<uint4*>(&L.u.t.gm[0][0])[lane] = make_uint4(0u, 0u, 0u, 0u);
    static_assert(sizeof(L.u.t.gm) == kWave * sizeof(uint4), "one 16-byte store per lane clears the lane masks");
    // the group boxes: each sphere's box, widened far beyond the rounding of
    // q +- R in double and rounded outward to single precision
    {
        const double Rw = ok ? sqrt(R2) * (1.0 + 0x1p-30) : 0.0;
        float g[6];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double mg = (fabs(qp[a]) + Rw) * 0x1p-40;
            g[a] = ok ? __double2float_rd(qp[a] - Rw - mg) : INFINITY;
            g[3 + a] = ok ? __double2float_ru(qp[a] + Rw + mg) : -INFINITY;
        }
#pragma unroll
        for (int o = 1; o < kTG; o <<= 1) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                g[a] = fminf(g[a], __shfl_xor(g[a], o, kWave));
                g[3 + a] = fmaxf(g[3 + a], __shfl_xor(g[3 + a], o, kWave));
            }
        }
        if ((lane & (kTG - 1)) == 0) {
#pragma unroll
            for (int a = 0; a < 6; ++a) L.gbox[lane / kTG][a] = g[a];
        }
    }
    const uint64_t okmask = __ballot(ok);
    uint32_t gall = 0;  // groups with at least one searching lane
#pragma unroll
    for (int g = 0; g < kNGrp; ++g) gall |= ((okmask >> (kTG * g)) & 0xFFu) ? (1u << g) : 0u;
    __syncthreads();

    bool wave_ok = gall != 0;
    int npairs = 0;  // pairs waiting (uniform over the wavefront)
#ifdef GD_KNN_STATS
    const long long tc1 = clock64();
    long long tcull = 0;
#endif
    // 3. sphere tests of the pending pairs, 64 at a time: a bucket joins its
    //    group's list if the sphere of one of the group's searching lanes may
    //    reach it, with the mask of those lanes
    int gn[kNGrp];  // buckets listed per group (uniform over the wavefront)
#pragma unroll
    for (int g = 0; g < kNGrp; ++g) gn[g] = 0;
    auto cull = [&]() {
#ifdef GD_KNN_STATS
        const long long t0 = clock64();
#endif
        __syncthreads();  // the pairs written by every lane
        // the next 64 pairs' boxes are in flight while these are tested
        uint32_t en = 0;
        FBox bn{};
        if (lane < npairs) {
            en = L.u.t.pairs[lane];
            bn = A.boxes[en & 0xFFFFFFu];
        }
        for (int p0 = 0; p0 < npairs; p0 += kWave) {
            const bool valid = p0 + lane < npairs;
            const uint32_t e = en;
            const FBox bx = bn;
            if (p0 + kWave + lane < npairs) {
                en = L.u.t.pairs[p0 + kWave + lane];
                bn = A.boxes[en & 0xFFFFFFu];
            }
            const int g = int(e >> 24);
            uint32_t hit = 0;
            if (valid) {
#pragma unroll
                for (int t = 0; t < kTG; ++t) {
                    const float4 sq = L.u.t.sc[g * kTG + t];
                    QF f;
                    f.c[0] = sq.x;
                    f.c[1] = sq.y;
                    f.c[2] = sq.z;
                    if (PER) {
                        const float4 sp = L.u.t.sp[g * kTG + t], sm = L.u.t.sm[g * kTG + t];
                        f.p[0] = sp.x;
                        f.p[1] = sp.y;
                        f.p[2] = sp.z;
                        f.m[0] = sm.x;
                        f.m[1] = sm.y;
                        f.m[2] = sm.z;
                    }
                    // (a lane without a search has a negative threshold, below any box2f)
                    hit |= uint32_t(box2f<PER>(A, f, bx) <= sq.w) << t;
                }
            }
            // places in the groups' lists: per group, after the lanes below
            int at = 0;
#pragma unroll
            for (int gq = 0; gq < kNGrp; ++gq) {
                const bool mine = hit != 0 && g == gq;
                const uint64_t bal = __ballot(mine);
                if (mine) at = gn[gq] + int(__popcll(bal & ((uint64_t(1) << lane) - 1)));
                gn[gq] += int(__popcll(bal));
            }
            if (hit && at < kGList) {
                L.glist[g][at] = e & 0xFFFFFFu;
                L.u.t.gm[g][at] = uint8_t(hit);
            }
        }
        __syncthreads();
        npairs = 0;
#ifdef GD_KNN_STATS
        tcull += clock64() - t0;
#endif
    };
    // 2. breadth-first traversal: frontier nodes of level lv (their boxes met
    //    the groups of their mask); their children are tested 32 nodes at a
    //    time (four per lane, loads issued together).  The virtual root (level
    //    top + 1) has the top level as children.  Buckets come out as
    //    (bucket, group) pairs, whose sphere tests run whenever enough wait.
    if (wave_ok) {
        int lv = A.T.levels;  // the root
        int cur = 0, nf = 1;
        if (lane == 0) L.u.t.front[0][0] = gall << 24;
        __syncthreads();
        constexpr int kU = 4;
        while (lv >= 1 && wave_ok) {
            int nn = 0;  // next frontier written
            for (int f0 = 0; f0 < nf && wave_ok; f0 += kU * kFan) {
                FBox bx[kU];
                uint32_t pm[kU];
                int child[kU];
                // the four frontier entries and then the four child boxes are
                // read unconditionally (a lane past the frontier or at a dead
                // child reads entry 0 and box 0 and drops them), so that each
                // group of reads is in flight together
                uint32_t fe[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int fi = f0 + u * kFan + (lane >> 3);
                    fe[u] = L.u.t.front[cur][fi < nf ? fi : 0];
                }
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int fi = f0 + u * kFan + (lane >> 3), c = lane & 7;
                    const int idx = int(fe[u] & 0xFFFFFFu);
                    const bool live = fi < nf && ((live_children(na, lv, idx) >> c) & 1u);
                    pm[u] = live ? fe[u] >> 24 : 0u;
                    child[u] = live ? idx * kFan + c : 0;
                }
#pragma unroll
                for (int u = 0; u < kU; ++u) bx[u] = A.boxes[level_off(A.T, lv - 1) + child[u]];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    uint32_t cm = 0;
                    if (pm[u]) {
#pragma unroll
                        for (int g = 0; g < kNGrp; ++g) {
                            float gb[6];
#pragma unroll
                            for (int a = 0; a < 6; ++a) gb[a] = L.gbox[g][a];
                            cm |= (((pm[u] >> g) & 1u) & uint32_t(group_meets<PER>(A, gb, bx[u]))) << g;
                        }
                    }
                    if (lv > 1) {
                        const uint64_t bal = __ballot(cm != 0);
                        const int at = nn + int(__popcll(bal & ((uint64_t(1) << lane) - 1)));
                        const int tot = int(__popcll(bal));
                        if (nn + tot > kFront) {
                            wave_ok = false;
                            break;
                        }
                        if (cm) L.u.t.front[cur ^ 1][at] = uint32_t(child[u]) | (cm << 24);
                        nn += tot;
                    } else {
                        // this lane's pairs go after those of the lanes below
                        // it: prefix and total of the counts (<= 8) from one
                        // ballot per bit
                        const int cnt = __popc(cm);
                        int below = 0, tot = 0;
#pragma unroll
                        for (int bit = 0; bit < 4; ++bit) {
                            const uint64_t bal = __ballot((cnt >> bit) & 1);
                            below += int(__popcll(bal & ((uint64_t(1) << lane) - 1))) << bit;
                            tot += int(__popcll(bal)) << bit;
                        }
                        if (npairs + tot > kPairs) cull();  // room for these
                        if (npairs + tot > kPairs) {
                            wave_ok = false;
                            break;
                        }
                        int w = npairs + below;
                        for (uint32_t m = cm; m; m &= m - 1)
                            L.u.t.pairs[w++] = uint32_t(child[u]) | (uint32_t(__ffs(m) - 1) << 24);
                        npairs += tot;
                    }
                }
            }
            __syncthreads();
            if (lv > 1) {
                cur ^= 1;
                nf = nn;
            }
            --lv;
            if (nf == 0 && lv >= 1) break;
        }
        if (wave_ok) cull();
    }
    __syncthreads();
#ifdef GD_KNN_STATS
    const long long tc2 = clock64();
#endif

    // 4. distances: every lane takes the buckets of its own mask in turn
    const int gg = lane / kTG;
    int gcnt = 0;
#pragma unroll
    for (int g = 0; g < kNGrp; ++g) gcnt = g == gg ? gn[g] : gcnt;
    if (!wave_ok) gcnt = 0;
    if (gcnt > kGList) ok = false;  // the group's list overflowed
    ok = ok && wave_ok;
    // this lane's bit of each place of its group's list, four places per
    // word read: bit t of bytes 0..3 gathered into bits 0..3 by one product
    // (the partial products land on distinct bits, so nothing carries)
    uint32_t mw[kMaskW];
    {
        const int t = lane & (kTG - 1);
        const uint4* gw = reinterpret_cast<const uint4*>(&L.u.t.gm[gg][0]);
#pragma unroll
        for (int w = 0; w < kMaskW; ++w) mw[w] = 0u;
#pragma unroll
        for (int c = 0; c < kGList / 16; ++c) {
            const uint4 v4 = gw[c];
            const uint32_t v[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t bits = (v[i] >> t) & 0x01010101u;
                const uint32_t nib = ((bits * 0x00204081u) >> 21) & 0xFu;
                const int place = 16 * c + 4 * i;  // of byte 0
                mw[place >> 5] |= nib << (place & 31);
            }
        }
        if (!ok) {
#pragma unroll
            for (int w = 0; w < kMaskW; ++w) mw[w] = 0u;
        }
    }
#ifdef GD_KNN_STATS
    int gmax = 0;
#pragma unroll
    for (int g = 0; g < kNGrp; ++g) gmax = max(gmax, wave_ok ? min(gn[g], kGList) : 0);
#endif
    const double R2s = R2;                                  // bin scale: the first radius
    const double sA = ok && R2s > 0.0 ? 1.0 / R2s : 0.0;
    double R2cut = ok ? R2 : -1.0;
    int bcut = kNB - 1, len = 0;
    bool ovf = false, cut = false;
    __syncthreads();  // the traversal's data are dead: the lists take their place
#ifdef GD_KNN_STATS
    const long long tc3 = clock64();
#endif
    auto entry_bin = [](uint32_t wv) { return int(wv >> 11); };
    Hist8 hist;
    auto hist_from_list = [&]() {
        hist.clear();
        for (int e = 0; e < len; ++e) hist.add(entry_bin(L.u.d.list[e][lane]));
    };
    // a list without room for a bucket: the bin completing k-1 others bounds
    // what stays and what may still come
    auto cut_list = [&]() {
        hist_from_list();
        int cum = 0, bc = kNB - 1;
        for (int b = 0; b < kNB; ++b) {
            cum += hist.get(b);
            if (cum >= need) {
                bc = b;
                break;
            }
        }
        if (cum >= need) cut = true;  // at least k-1 others are counted
        if (bc < bcut) {
            bcut = bc;
            R2cut = fmin(R2cut, (log_edge(bcut + 1) * R2s) * (1.0 + 1e-12));
        }
        int kept = 0;
        for (int e = 0; e < len; ++e) {
            const uint16_t wv = L.u.d.list[e][lane];
            if (entry_bin(wv) <= bcut) L.u.d.list[kept++][lane] = wv;
        }
        len = kept;
        ovf = len > kTList - kBucket;
    };
    // the lowest marked place (cleared from the mask), or -1
    auto take_place = [&]() {
        int at = -1;
#pragma unroll
        for (int w = kMaskW - 1; w >= 0; --w)
            if (mw[w]) at = w * 32 + __ffs(mw[w]) - 1;
#pragma unroll
        for (int w = 0; w < kMaskW; ++w)
            if (w == (at >> 5)) mw[w] &= mw[w] - 1u;
        return at;
    };
    // the four positions of the bucket at place `at`; its first slot, or na
    // without a bucket (slots from na on are not evaluated)
    struct Bk {
        double x[kBucket], y[kBucket], z[kBucket];
        int j0;
    };
    auto fetch = [&](int at) {
        Bk r;
        r.j0 = at >= 0 ? int(L.glist[gg][at]) * kBucket : na;
#pragma unroll
        for (int s = 0; s < kBucket; ++s) {
            const double* pj = reinterpret_cast<const double*>(A.pos + (r.j0 + s < na ? r.j0 + s : 0));
            const double2 xy = *reinterpret_cast<const double2*>(pj);
            r.x[s] = xy.x;
            r.y[s] = xy.y;
            r.z[s] = pj[2];
        }
        return r;
    };
    auto eval = [&](const Bk& c, int at) {
        if (len > kTList - kBucket && !ovf) cut_list();  // room for a whole bucket
#pragma unroll
        for (int s = 0; s < kBucket; ++s) {
            const double d2 = sep2<PER>(A, qp, c.x[s], c.y[s], c.z[s]);
            const int j = c.j0 + s;
            if (j < na && d2 <= R2cut && j != q && !ovf) {
                const int b = log_bin(d2 * sA);
                if (b <= bcut) L.u.d.list[len++][lane] = uint16_t((b << 11) | (at * kBucket + s));
            }
        }
    };
    // two buckets in turn, each one's loads in flight while the other is
    // evaluated (the two register sets fixed, not indexed)
#ifdef GD_KNN_STATS
    int iters = 0;
#endif
    int at0 = take_place(), at1 = -1;
    Bk bk0 = fetch(at0), bk1;
    for (;;) {
        if (!__ballot(at0 >= 0)) break;
        at1 = take_place();
        bk1 = fetch(at1);
        eval(bk0, at0);
        if (!__ballot(at1 >= 0)) break;
        at0 = take_place();
        bk0 = fetch(at0);
        eval(bk1, at1);
#ifdef GD_KNN_STATS
        iters += 2;
#endif
    }
#ifdef GD_KNN_STATS
    const long long tc4 = clock64();
#endif
    auto slot_of = [&](uint32_t wv) {
        const int pos = int(wv & 0x7FFu);
        return int(L.glist[gg][pos >> 2]) * kBucket + (pos & (kBucket - 1));
    };

    // 5. sure and boundary entries from the list
    ok = ok && !ovf && (cut || len >= need);
    int b0 = 0, c0 = 0, hb = 0;
    if (ok) {
        hist_from_list();
        int cum = 0;
        bool found = false;
#pragma unroll
        for (int b = 0; b < kNB; ++b) {
            const int h = hist.get(b);
            if (!found && cum + h >= need) {
                b0 = b;
                hb = h;
                found = true;
            }
            if (!found) cum += h;
        }
        c0 = cum;
        ok = hb <= kC1;
    }
    // the ranking below runs over the wavefront's largest boundary bin only
    int nbw = ok ? hb : 0;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) nbw = max(nbw, __shfl_xor(nbw, o, kWave));
    int ntot = 0, nb = 0;
    double maxd2 = 0.0;
    // boundary entry e waits at list place kTList - 1 - e: fewer than k - 1
    // sure entries and at most kC1 boundary ones leave room for them there
    // once the entries beyond the boundary bin are gone
    static_assert(32 + 2 * kC1 <= kTList, "the boundary entries fit the list's tail");
    auto bnd = [&](int e) -> uint16_t& { return L.u.d.list[kTList - 1 - e][lane]; };
    if (ok) {
        if (len + hb > kTList) {  // first the entries beyond the boundary bin go
            int kept = 0;
            for (int e = 0; e < len; ++e) {
                const uint16_t wv = L.u.d.list[e][lane];
                if (entry_bin(wv) <= b0) L.u.d.list[kept++][lane] = wv;
            }
            len = kept;
        }
        // sure entries move to the front of the list, boundary entries to the tail
        for (int e = 0; e < len; ++e) {
            const uint16_t wv = L.u.d.list[e][lane];
            const int bn = entry_bin(wv);
            if (bn < b0) L.u.d.list[ntot++][lane] = wv;
            else if (bn == b0) bnd(nb++) = wv;
        }
        if (ntot != c0 || nb != hb) set_status(A.ws, GD_DEV_INTERNAL);
        // boundary entries ranked by (d^2, slot); the chosen ones follow
        const int needb = need - c0 < nb ? need - c0 : nb;
        double bd[kC1];
        int32_t bj[kC1];
        uint16_t bw[kC1];
#pragma unroll
        for (int e = 0; e < kC1; ++e) {
            bw[e] = e < nb ? bnd(e) : uint16_t(0);
            bj[e] = e < nb ? slot_of(bw[e]) : INT32_MAX;
            bd[e] = e < nb ? sep2_slot<PER>(A, qp, bj[e]) : INFINITY;
        }
#pragma unroll
        for (int e = 0; e < kC1; ++e) {
            if (e < nbw) {  // uniform
                int rank = 0;
#pragma unroll
                for (int f = 0; f < kC1; ++f)
                    if (f < nbw) rank += (bd[f] < bd[e]) | ((bd[f] == bd[e]) & (bj[f] < bj[e]));
                if (e < nb && rank < needb) {
                    L.u.d.list[ntot + rank][lane] = bw[e];
                    maxd2 = fmax(maxd2, bd[e]);
                }
            }
        }
        ntot += needb;
        if (ntot != need) set_status(A.ws, GD_DEV_INTERNAL);
    }
    // the row in slot order
    int32_t v[32];
#pragma unroll
    for (int e = 0; e < 32; ++e) v[e] = (ok && e < ntot) ? int32_t(slot_of(L.u.d.list[e][lane])) : INT32_MAX;
    bitonic_sort<32>(v);
    if (ok) {
        if (k == 32 && A.row_vec) {
#pragma unroll
            for (int c4 = 0; c4 < 8; ++c4) {
                int32_t o[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int e = 4 * c4 + t;
                    o[t] = e == 0 ? q : ((e - 1 < ntot) ? v[e - 1] : -1);
                }
                reinterpret_cast<int4*>(row)[c4] = make_int4(o[0], o[1], o[2], o[3]);
            }
        } else {
            row[0] = q;
#pragma unroll
            for (int e = 0; e < 32; ++e)
                if (e < k - 1) row[1 + e] = (e < ntot) ? v[e] : -1;
        }
        A.cnt[q] = 1 + ntot;
        A.dmax[q] = ntot > 0 ? sqrt(maxd2) : 0.0;
    }
#ifdef GD_KNN_STATS
    if (lane == 0) {  // per wavefront: cycles of traversal, sphere tests, distances, finish; largest group list, buckets per lane (the largest)
        int32_t* w = A.stats + int64_t(item) * 8;
        w[0] = int32_t(tc2 - tc1 - tcull);
        w[1] = int32_t(tcull);
        w[2] = int32_t(tc4 - tc3);
        w[3] = int32_t(clock64() - tc4);
        w[4] = gmax;
        w[5] = iters;
        w[6] = wave_ok ? 1 : 0;
    }
#endif
    // 6. the rest: lanes that had no usable previous distance to the per-lane
    //    search (list 0), the others (sparse regions, many candidates) to the
    //    wavefront-per-query search (list 1)
    fb = fb && !ok;
#pragma unroll
    for (int l = 0; l < 2; ++l) {
        const bool mine = fb && (l == 0 ? !tried : tried);
        const uint64_t fbm = __ballot(mine);
        int32_t base = 0;
        if (lane == 0 && fbm) base = atomicAdd(fb_n + l, int32_t(__popcll(fbm)));
        base = __builtin_amdgcn_readfirstlane(base);
        if (mine) (l == 0 ? fb0 : fb1)[base + int(__popcll(fbm & ((uint64_t(1) << lane) - 1)))] = q;
    }
}

// fb0 and fb1 receive the handed-back queries (n entries each): those with no
// usable previous distance, and the rest; fb_n[0], fb_n[1] count them
void launch_knn_tile(const KnnArgs& A, bool per, int32_t* fb0, int32_t* fb1, int32_t* fb_n, hipStream_t st)
{
    const dim3 grid(unsigned((A.n + kWave - 1) / kWave));
    const TileArgs TA{A, fb0, fb1, fb_n};
    if (per) hipLaunchKernelGGL(k_knn_tile<true>, grid, dim3(kWave), 0, st, TA);
    else hipLaunchKernelGGL(k_knn_tile<false>, grid, dim3(kWave), 0, st, TA);
}

void many_add_tile(ManyBuilder& B, const std::vector<TileArgs>& tab, const std::vector<int64_t>& nb, bool per)
{
    if (per) B.add<KnnTile<true>>(tab, nb);
    else B.add<KnnTile<false>>(tab, nb);
}

}  // namespace gd
