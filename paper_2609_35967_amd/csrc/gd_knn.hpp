// gd_knn.hpp -- definitions shared by the neighbour-search kernels: the
// implicit 8-ary box tree over Morton-ordered buckets, the query arguments,
// the exact squared distance (minimum image on periodic axes) and the
// conservative single-precision box tests.
#pragma once

#include "gd_common.hpp"

namespace gd {

constexpr double kHintSlack = 1.08;  // first radius: previous neighbour distance times this
constexpr int kNB = 32;   // bins of the per-lane distance histograms
constexpr int kC1 = 16;   // largest boundary bin ranked in registers

// ---------------------------------------------------------------------------
// Tree
struct TreeLevels {
    int32_t levels;
    int64_t off[kMaxTreeLevels];
    int64_t cap[kMaxTreeLevels];  // padded capacity of each level
    int32_t off1, stride1;        // off[l] = off1 + (l - 1) stride1 for l >= 1
};

// first box of level l (arithmetic, no table lookup on the walk's path)
__device__ inline int32_t level_off(const TreeLevels& T, int l)
{
    return l == 0 ? 0 : T.off1 + (l - 1) * T.stride1;
}

struct Periodicity {
    int32_t per[3];
    double L[3];
};

// Margin of the single-precision box tests on axis a: 2^-21 (M + L), M the
// largest coordinate magnitude of the active set, L the period on periodic
// axes (whose images q +- L are tested).  Rounding q or q +- L to float and
// the float subtraction move a gap by less than 3 * 2^-24 (M + L).
__device__ inline double box_margin(const WsHeader* h, const Periodicity& P, int a)
{
    double M = fmax(fabs(h->lo[a]), fabs(h->hi[a]));
    if (P.per[a]) M += fabs(P.L[a]);
    return M * 0x1p-21;
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
    int32_t* nbr;
    int32_t* cnt;
    double* dmax;
    int32_t row_vec;  // nbr is 16-byte aligned
    int32_t* xq;      // per-die work queue counters
    const double* hint;  // previous neighbour distance per slot (search hint only)
    void* ws;
    const int32_t* list;    // when set: the queries are list[0 .. *list_n)
    const int32_t* list_n;
};

// the tile search's arguments: the search's, and its two lists of handed-back
// queries with their counts
struct TileArgs {
    KnnArgs A;
    int32_t* fb0;
    int32_t* fb1;
    int32_t* fb_n;
};

// the wavefront-per-query search's: the queries list[0 .. *count), or every
// slot when list is null
struct WaveArgs {
    KnnArgs A;
    const int32_t* list;
    const int32_t* count;
};

template <bool PER>
__device__ inline double sep2(const KnnArgs& A, const double q[3], double px, double py, double pz)
{
    double dx = px - q[0], dy = py - q[1], dz = pz - q[2];
    if (PER) {
        if (A.per[0]) { if (dx > A.hL[0]) dx = dx - A.L[0]; else if (dx < -A.hL[0]) dx = dx + A.L[0]; }
        if (A.per[1]) { if (dy > A.hL[1]) dy = dy - A.L[1]; else if (dy < -A.hL[1]) dy = dy + A.L[1]; }
        if (A.per[2]) { if (dz > A.hL[2]) dz = dz - A.L[2]; else if (dz < -A.hL[2]) dz = dz + A.L[2]; }
    }
    const double s = dx * dx + dy * dy;
    return s + dz * dz;
}

template <bool PER>
__device__ inline double sep2_slot(const KnnArgs& A, const double q[3], int j)
{
    const double* pj = reinterpret_cast<const double*>(A.pos + j);
    const double2 xy = *reinterpret_cast<const double2*>(pj);
    return sep2<PER>(A, q, xy.x, xy.y, pj[2]);
}

// the query point in single precision, with its periodic images
struct QF {
    float c[3], p[3], m[3];
};

__device__ inline float gapf(float x, float lo, float hi)
{
    return fmaxf(fmaxf(lo - x, x - hi), 0.0f);
}

// Lower bound of the squared distance from q to a (widened) box, minimum
// image on periodic axes; its own float rounding (one product, two fused
// multiply-adds, each term rounded at most three times) is covered by r2f.
template <bool PER>
__device__ inline float box2f(const KnnArgs& A, const QF& f, const FBox& b)
{
    float g[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float v = gapf(f.c[a], b.lo[a], b.hi[a]);
        if (PER && A.per[a]) v = fminf(v, fminf(gapf(f.p[a], b.lo[a], b.hi[a]), gapf(f.m[a], b.lo[a], b.hi[a])));
        g[a] = v;
    }
    return fmaf(g[2], g[2], fmaf(g[1], g[1], g[0] * g[0]));
}

// Single-precision threshold of the box tests for radius R2: at least
// R2 (1 + 2^-19), above the three roundings of box2f's sum of squares.
__device__ inline float r2f(double R2)
{
    return float(R2 * (1.0 + 0x1p-19)) * (1.0f + 0x1p-22f);
}

// mask of the children of a node (boxes b[0..7], already loaded) whose box
// may hold a point within the radius
template <bool PER>
__device__ inline uint32_t child_mask(const KnnArgs& A, const FBox (&b)[kFan], const QF& f, float R2f)
{
    uint32_t m = 0;
#pragma unroll
    for (int c = 0; c < kFan; ++c) m |= (box2f<PER>(A, f, b[c]) <= R2f ? 1u : 0u) << c;
    return m;
}

// mask of the children of node `idx` at `level` (>= 1) that hold active
// slots: child c covers the 4 8^(level-1) slots from (8 idx + c) 4 8^(level-1)
// on, and the active slots are [0, na).  Children without any (the padding
// of a level among them) are never entered, so a walk only reads children
// of stored nodes.
__device__ inline uint32_t live_children(int na, int level, int idx)
{
    const int sh = 2 + 3 * (level - 1);  // log2 of the slots per child
    const int64_t left = int64_t(na) - (int64_t(idx) << (sh + 3));
    const int64_t nv = (left + (int64_t(1) << sh) - 1) >> sh;
    return nv >= kFan ? 0xFFu : (nv <= 0 ? 0u : (1u << int(nv)) - 1u);
}

// First-level bins: logarithmic in x = d^2 / (the pass's first radius), 8 per
// octave over the kNB / 8 octaves below 1, read off the bits of the double
// (monotone for x >= 0); bin 0 also takes everything below, the last bin
// everything from 2^(-1/8).
constexpr int kLogShift = 49;
constexpr int64_t kLogBase = int64_t(1023) * 8 - kNB;

__device__ inline int log_bin(double x)
{
    // the 64-bit pattern shifted right by kLogShift is the high word shifted
    // right by kLogShift - 32 (both arithmetic)
    const int b = (__double2hiint(x) >> (kLogShift - 32)) - int(kLogBase);
    return min(max(b, 0), kNB - 1);
}

// lower edge of log bin b (1 <= b <= kNB); log_bin(x) < b exactly when x < edge
__device__ inline double log_edge(int b)
{
    return __longlong_as_double((long long)((int64_t(b) + kLogBase) << kLogShift));
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

// one wavefront per query (gd_knn_wave.hip): every slot, or those of `list`
// [0, *count) when a list is given
void launch_knn_wave(const KnnArgs& A, bool per, const int32_t* list, const int32_t* count, int64_t nblocks,
                     hipStream_t st);
// 64 Morton-consecutive queries per wavefront from shared candidate tiles
// (gd_knn_tile.hip), k <= 33; the queries it cannot complete go to fb0 (no
// usable previous distance) or fb1 (the rest)
void launch_knn_tile(const KnnArgs& A, bool per, int32_t* fb0, int32_t* fb1, int32_t* fb_n, hipStream_t st);
// the same two searches as stages of a many-run interval
void many_add_tile(ManyBuilder& B, const std::vector<TileArgs>& tab, const std::vector<int64_t>& nb, bool per);
void many_add_wave(ManyBuilder& B, const std::vector<WaveArgs>& tab, const std::vector<int64_t>& nb, bool per);

}  // namespace gd
