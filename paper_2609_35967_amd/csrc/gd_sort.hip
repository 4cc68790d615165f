// gd_sort.hip -- Morton order of the active particles (Sect. 2.5.1: the
// neighbour search runs on an adaptive spatial hierarchy over the Morton
// order).  Bounding box reduction, 30-bit keys, stable LSD radix sort of
// (key, slot) pairs with 8-bit digits, and the gather of every state array
// into the sorted order.  All kernels are bandwidth-bound streaming passes:
// coalesced loads of the SoA arrays, one 4-byte key and value per particle.
#include "gd_common.hpp"
#include "gd_internal.hpp"

#include <algorithm>
#include <type_traits>

namespace gd {

// ---------------------------------------------------------------------------
// Bounding box and active count: per-block partials, then one block combines.
struct BboxArgs {
    const double *x, *y, *z, *M;
    int64_t n;
    double* red;
};

struct BboxPartial {
    using Args = BboxArgs;
    static constexpr int kThreads = 256;
    static __device__ __forceinline__ void body(const Args& A, Blk B);
};

__device__ __forceinline__ void BboxPartial::body(const Args& A, Blk B)
{
    const double *x = A.x, *y = A.y, *z = A.z, *M = A.M;
    const int64_t n = A.n;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double cnt = 0.0;
    // the four arrays are read for every slot (an inactive one is then left
    // out), so that the unrolled iterations' loads are in flight together
#pragma unroll 4
    for (int64_t i = B.id * int64_t(blockDim.x) + threadIdx.x; i < n; i += B.n * blockDim.x) {
        const bool act = M[i] > 0.0;
        const double c[3] = {x[i], y[i], z[i]};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            lo[d] = act ? fmin(lo[d], c[d]) : lo[d];
            hi[d] = act ? fmax(hi[d], c[d]) : hi[d];
        }
        cnt += act ? 1.0 : 0.0;
    }
    __shared__ double s[4][7];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double v[7] = {lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], cnt};
#pragma unroll
    for (int d = 0; d < 3; ++d) v[d] = wave_min_d(v[d]);
#pragma unroll
    for (int d = 3; d < 6; ++d) v[d] = wave_max_d(v[d]);
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v[6] += shfl_xor_d(v[6], m);
    if (lane == 0)
        for (int d = 0; d < 7; ++d) s[w][d] = v[d];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int ww = 1; ww < int(blockDim.x >> 6); ++ww) {
            for (int d = 0; d < 3; ++d) s[0][d] = fmin(s[0][d], s[ww][d]);
            for (int d = 3; d < 6; ++d) s[0][d] = fmax(s[0][d], s[ww][d]);
            s[0][6] += s[ww][6];
        }
        for (int d = 0; d < 7; ++d) A.red[B.id * 8 + d] = s[0][d];
    }
}

__global__ __launch_bounds__(256) void k_bbox_partial(BboxArgs A)
{
    BboxPartial::body(A, Blk{int64_t(blockIdx.x), int64_t(gridDim.x)});
}

// one wavefront combines the per-block partials
struct BboxFinalArgs {
    const double* red;
    int nblk;
    WsHeader* h;
};

struct BboxFinal {
    using Args = BboxFinalArgs;
    static constexpr int kThreads = 64;
    static __device__ __forceinline__ void body(const Args& A, Blk B);
};

__device__ __forceinline__ void BboxFinal::body(const Args& A, Blk)
{
    const double* red = A.red;
    const int nblk = A.nblk;
    WsHeader* h = A.h;
    const int lane = threadIdx.x;
    double v[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0};
    for (int b = lane; b < nblk; b += 64) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            v[d] = fmin(v[d], red[b * 8 + d]);
            v[3 + d] = fmax(v[3 + d], red[b * 8 + 3 + d]);
        }
        v[6] += red[b * 8 + 6];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        v[d] = wave_min_d(v[d]);
        v[3 + d] = wave_max_d(v[3 + d]);
    }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v[6] += shfl_xor_d(v[6], m);
    if (lane != 0) return;
    double ext = 0.0;
    for (int d = 0; d < 3; ++d) {
        const double e = v[3 + d] - v[d];
        if (e > ext) ext = e;
        h->lo[d] = v[d];
        h->hi[d] = v[3 + d];
    }
    h->inv = ext > 0.0 ? 1024.0 / ext : 0.0;
    h->n_active = int32_t(v[6]);
}

__global__ __launch_bounds__(64) void k_bbox_final(BboxFinalArgs A)
{
    BboxFinal::body(A, Blk{0, 1});
}

// ---------------------------------------------------------------------------
// Morton key: 10 bits per axis, x in bit 3b, y in 3b+1, z in 3b+2.
__device__ inline uint32_t spread3(uint32_t v)
{
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ inline uint32_t quant(double c, double lo, double inv)
{
    const double t = (c - lo) * inv;
    const uint32_t q = uint32_t(t);
    return q > 1023u ? 1023u : q;
}

struct MortonArgs {
    const double *x, *y, *z, *M;
    int64_t n;
    const WsHeader* h;
    uint32_t* keys;
    uint32_t* vals;
};

struct Morton {
    using Args = MortonArgs;
    static constexpr int kThreads = 256;
    static __device__ __forceinline__ void body(const Args& A, Blk B)
    {
        const int64_t i = B.id * int64_t(blockDim.x) + threadIdx.x;
        if (i >= A.n) return;
        uint32_t key = 0xFFFFFFFFu;
        if (A.M[i] > 0.0) {
            const WsHeader* h = A.h;
            const double inv = h->inv;
            key = spread3(quant(A.x[i], h->lo[0], inv)) | (spread3(quant(A.y[i], h->lo[1], inv)) << 1) |
                  (spread3(quant(A.z[i], h->lo[2], inv)) << 2);
        }
        A.keys[i] = key;
        A.vals[i] = uint32_t(i);
    }
};

__global__ __launch_bounds__(256) void k_morton(MortonArgs A)
{
    Morton::body(A, Blk{int64_t(blockIdx.x), int64_t(gridDim.x)});
}

// ---------------------------------------------------------------------------
// LSD radix sort, 8-bit digits.  Block b owns keys [b*4096, (b+1)*4096).
// hist is digit-major: hist[d * nblk + b]; each digit's row is exclusive-
// scanned in place by its own block, and the scatter adds the exclusive scan
// of the digit totals.
struct RadixArgs {
    const uint32_t *kin, *vin;
    uint32_t *kout, *vout;
    int64_t n;
    int shift;
    uint32_t* hist;
    int nblk;
    uint32_t* tot;
};

struct RadixHist {
    using Args = RadixArgs;
    static constexpr int kThreads = 256;
    static __device__ __forceinline__ void body(const Args& A, Blk B)
    {
        __shared__ uint32_t h[256];
        h[threadIdx.x] = 0;
        __syncthreads();
        const int64_t base = B.id * kSortTile;
        const int shift = A.shift;
        // the tile's keys are loaded first, all in flight together
        constexpr int R = kSortTile / 256;
        uint32_t kr[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t i = base + r * 256 + threadIdx.x;
            kr[r] = i < A.n ? A.kin[i] : 0u;
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (base + r * 256 + threadIdx.x < A.n) atomicAdd(&h[(kr[r] >> shift) & 0xFFu], 1u);
        __syncthreads();
        A.hist[int64_t(threadIdx.x) * A.nblk + B.id] = h[threadIdx.x];
    }
};

__global__ __launch_bounds__(256) void k_radix_hist(RadixArgs A)
{
    RadixHist::body(A, Blk{int64_t(blockIdx.x), int64_t(gridDim.x)});
}

// Exclusive scan of 256 values held one per thread of a 256-thread block;
// returns this thread's prefix, and the total in *total.
__device__ inline uint32_t block_scan_excl_256(uint32_t v, uint32_t* s_w, uint32_t* total)
{
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    uint32_t before = 0;
    for (int ww = 0; ww < w; ++ww) before += s_w[ww];
    *total = s_w[0] + s_w[1] + s_w[2] + s_w[3];
    __syncthreads();
    return before + x - v;
}

// Row d of the digit-major histogram (the counts of digit d in every block)
// becomes its exclusive prefix; the row total goes to tot[d].
struct ScanRows {
    using Args = RadixArgs;
    static constexpr int kThreads = 256;
    static __device__ __forceinline__ void body(const Args& A, Blk B)
    {
        __shared__ uint32_t s_w[4];
        const int nblk = A.nblk;
        uint32_t* row = A.hist + B.id * nblk;
        uint32_t carry = 0;
        for (int c = 0; c < nblk; c += 256) {
            const int i = c + int(threadIdx.x);
            const uint32_t v = i < nblk ? row[i] : 0u;
            uint32_t chunk;
            const uint32_t pre = block_scan_excl_256(v, s_w, &chunk);
            if (i < nblk) row[i] = carry + pre;
            carry += chunk;
        }
        if (threadIdx.x == 0) A.tot[B.id] = carry;
    }
};

__global__ __launch_bounds__(256) void k_scan_rows(RadixArgs A)
{
    ScanRows::body(A, Blk{int64_t(blockIdx.x), int64_t(gridDim.x)});
}

struct RadixScatter {
    using Args = RadixArgs;
    static constexpr int kThreads = 256;
    static __device__ __forceinline__ void body(const Args& A, Blk B);
};

__device__ __forceinline__ void RadixScatter::body(const Args& A, Blk B)
{
    const uint32_t* __restrict__ kin = A.kin;
    const uint32_t* __restrict__ vin = A.vin;
    uint32_t* __restrict__ kout = A.kout;
    uint32_t* __restrict__ vout = A.vout;
    const int64_t n = A.n;
    const int shift = A.shift;
    const uint32_t* __restrict__ hist = A.hist;
    const int nblk = A.nblk;
    const uint32_t* __restrict__ tot = A.tot;
    __shared__ uint32_t goff[256];   // global offset of each digit for this block
    __shared__ uint32_t run[256];    // items of each digit placed in earlier rounds
    __shared__ uint32_t wcnt[4][256];
    __shared__ uint32_t s_w[4];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint32_t all;
    const uint32_t below = block_scan_excl_256(tot[t], s_w, &all);  // keys of smaller digits
    goff[t] = below + hist[int64_t(t) * nblk + B.id];
    run[t] = 0;
    const int64_t base = B.id * kSortTile;
    const uint64_t lt = (uint64_t(1) << lane) - 1;
    // the tile's keys and values are loaded first, all in flight together;
    // the rounds then take them from registers
    constexpr int R = kSortTile / 256;
    uint32_t kr[R], vr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = base + r * 256 + t;
        kr[r] = i < n ? kin[i] : 0u;
        vr[r] = i < n ? vin[i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        for (int ww = 0; ww < 4; ++ww) wcnt[ww][t] = 0;
        __syncthreads();
        const int64_t i = base + r * 256 + t;
        const bool valid = i < n;
        const uint32_t key = kr[r], val = vr[r];
        const uint32_t dig = valid ? (key >> shift) & 0xFFu : 0u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool set = (dig >> bit) & 1u;
            const uint64_t bs = __ballot(set);
            peers &= set ? bs : ~bs;
        }
        const uint32_t rank = __popcll(peers & lt);
        if (valid && rank == 0) wcnt[w][dig] = __popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t off = goff[dig] + run[dig];
            for (int ww = 0; ww < w; ++ww) off += wcnt[ww][dig];
            kout[off + rank] = key;
            vout[off + rank] = val;
        }
        __syncthreads();
        run[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_radix_scatter(RadixArgs A)
{
    RadixScatter::body(A, Blk{int64_t(blockIdx.x), int64_t(gridDim.x)});
}

// ---------------------------------------------------------------------------
// Gather of every state array into Morton order, plus the packed positions.
struct Permute {
    using Args = PermuteArgs;
    static constexpr int kThreads = 256;
    static __device__ __forceinline__ void body(const Args& A, Blk B);
};

__global__ __launch_bounds__(256) void k_permute(PermuteArgs A)
{
    Permute::body(A, Blk{int64_t(blockIdx.x), int64_t(gridDim.x)});
}

__device__ __forceinline__ void Permute::body(const Args& A, Blk B)
{
    const int64_t i = B.id * int64_t(blockDim.x) + threadIdx.x;
    if (i >= A.n) return;
    const uint32_t s = A.perm[i];
    // every gather is issued before any store (the array count is uniform),
    // so a lane keeps all of its loads in flight at once
    double v[16];
#pragma unroll
    for (int a = 0; a < 16; ++a) v[a] = a < A.nd ? A.src[a][s] : 0.0;
    const uint32_t id = A.id_src[s];
    const double hint = A.hint_src ? A.hint_src[s] : 0.0;
#pragma unroll
    for (int a = 0; a < 16; ++a)
        if (a < A.nd) A.dst[a][i] = v[a];
    A.id_dst[i] = id;
    A.pos4[i] = make_double4(v[0], v[1], v[2], 0.0);  // x, y, z are the first three arrays
    A.hint_dst[i] = hint;
}

__global__ void k_fill_i32(int32_t* __restrict__ a, int64_t n, int32_t v)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) a[i] = v;
}

// ---------------------------------------------------------------------------
// the sort's arguments for one run (state `in` into `out`); the radix passes
// alternate between (keys0, vals0) and (keys1, vals1)
struct SortArgs {
    BboxArgs bbox;
    BboxFinalArgs fin;
    MortonArgs morton;
    RadixArgs pass[4];
    PermuteArgs perm;
};

static SortArgs sort_args(const gd_problem* p, const gd_particles* in, gd_particles* out, const double* hint, void* ws,
                          const Layout& L, int nblk_bbox)
{
    const int64_t n = p->n;
    WsHeader* h = at<WsHeader>(ws, L.hdr);
    double* red = at<double>(ws, L.red);
    SortArgs S{};
    S.bbox = BboxArgs{in->x, in->y, in->z, in->M, n, red};
    S.fin = BboxFinalArgs{red, nblk_bbox, h};
    uint32_t* k0 = at<uint32_t>(ws, L.keys0);
    uint32_t* k1 = at<uint32_t>(ws, L.keys1);
    uint32_t* v0 = at<uint32_t>(ws, L.vals0);
    uint32_t* v1 = at<uint32_t>(ws, L.vals1);
    uint32_t* hist = at<uint32_t>(ws, L.hist);
    S.morton = MortonArgs{in->x, in->y, in->z, in->M, n, h, k0, v0};
    const int nsb = L.nsort_blocks;
    uint32_t* tot = hist + int64_t(256) * nsb;  // per-digit totals (the spare row of hist)
    for (int pass = 0; pass < 4; ++pass) {
        const bool odd = pass & 1;
        S.pass[pass] = RadixArgs{odd ? k1 : k0, odd ? v1 : v0, odd ? k0 : k1, odd ? v0 : v1, n, 8 * pass, hist, nsb, tot};
    }
    // sorted (key, slot) pairs are back in (k0, v0)
    PermuteArgs& A = S.perm;
    A.n = n;
    A.perm = v0;
    int nd = 0;
    auto add = [&](const double* s, double* d) {
        if (s) {
            A.src[nd] = s;
            A.dst[nd] = d;
            ++nd;
        }
    };
    add(in->x, out->x);
    add(in->y, out->y);
    add(in->z, out->z);
    add(in->M, out->M);
    add(in->m[in->cur], out->m[in->cur]);
    add(in->r, out->r);
    add(in->th, out->th);
    add(in->ph, out->ph);
    add(in->vr, out->vr);
    add(in->lth, out->lth);
    add(in->lph, out->lph);
    add(in->vz, out->vz);
    add(in->st_mid, out->st_mid);
    A.nd = nd;
    A.id_src = in->id;
    A.id_dst = out->id;
    A.pos4 = at<double4>(ws, L.pos4);
    A.hint_src = hint;
    A.hint_dst = at<double>(ws, L.hint);
    return S;
}

int launch_morton_sort(const gd_problem* p, const gd_particles* in, gd_particles* out, const double* hint, void* ws,
                       const Layout& L, hipStream_t st)
{
    const int64_t n = p->n;
    const SortArgs S = sort_args(p, in, out, hint, ws, L, kRedBlocks);
    prof_mark(GD_PROF_SORT, 0, st);
    hipLaunchKernelGGL(k_bbox_partial, dim3(kRedBlocks), dim3(256), 0, st, S.bbox);
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(64), 0, st, S.fin);
    const int nb = int((n + 255) / 256);
    hipLaunchKernelGGL(k_morton, dim3(nb), dim3(256), 0, st, S.morton);
    const int nsb = L.nsort_blocks;
    for (int pass = 0; pass < 4; ++pass) {
        hipLaunchKernelGGL(k_radix_hist, dim3(nsb), dim3(256), 0, st, S.pass[pass]);
        hipLaunchKernelGGL(k_scan_rows, dim3(256), dim3(256), 0, st, S.pass[pass]);
        hipLaunchKernelGGL(k_radix_scatter, dim3(nsb), dim3(256), 0, st, S.pass[pass]);
    }
    hipLaunchKernelGGL(k_permute, dim3(nb), dim3(256), 0, st, S.perm);
    prof_mark(GD_PROF_SORT, 1, st);
    out->cur = in->cur;
    return 0;
}

void many_sort(ManyBuilder& B, const std::vector<ManyRun>& R)
{
    const size_t nr = R.size();
    std::vector<SortArgs> S(nr);
    std::vector<int64_t> nbb(nr), one(nr, 1), nb(nr), nsb(nr), digits(nr, 256);
    for (size_t r = 0; r < nr; ++r) {
        const ManyRun& x = R[r];
        const int64_t n = x.p.n;
        nbb[r] = n > 0 ? std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, cdiv(n, B.tune.red_div))) : 0;
        gd_particles out = x.out;
        S[r] = sort_args(&x.p, &x.in, &out, x.nb.dmax, x.ws, x.L, int(nbb[r]));
        one[r] = n > 0 ? 1 : 0;
        nb[r] = cdiv(n, 256);
        nsb[r] = n > 0 ? x.L.nsort_blocks : 0;
        if (n == 0) digits[r] = 0;
    }
    auto pick = [&](auto f) {
        using A = std::remove_reference_t<decltype(f(S[0]))>;
        std::vector<A> v(nr);
        for (size_t r = 0; r < nr; ++r) v[r] = f(S[r]);
        return v;
    };
    B.add<BboxPartial>(pick([](SortArgs& a) -> BboxArgs& { return a.bbox; }), nbb);
    B.add<BboxFinal>(pick([](SortArgs& a) -> BboxFinalArgs& { return a.fin; }), one);
    B.add<Morton>(pick([](SortArgs& a) -> MortonArgs& { return a.morton; }), nb);
    for (int pass = 0; pass < 4; ++pass) {
        auto tab = pick([pass](SortArgs& a) -> RadixArgs& { return a.pass[pass]; });
        B.add<RadixHist>(tab, nsb);
        B.add<ScanRows>(tab, digits);
        B.add<RadixScatter>(tab, nsb);
    }
    B.add<Permute>(pick([](SortArgs& a) -> PermuteArgs& { return a.perm; }), nb);
}

void launch_fill_i32(int32_t* a, int64_t n, int32_t v, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_i32, dim3(int((n + 255) / 256)), dim3(256), 0, st, a, n, v);
}

}  // namespace gd
