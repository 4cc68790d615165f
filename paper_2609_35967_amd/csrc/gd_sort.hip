// gd_sort.hip -- Morton order of the active particles (Sect. 2.5.1: the
// neighbour search runs on an adaptive spatial hierarchy over the Morton
// order).  Bounding box reduction, 30-bit keys, stable LSD radix sort of
// (key, slot) pairs with 8-bit digits, and the gather of every state array
// into the sorted order.  All kernels are bandwidth-bound streaming passes:
// coalesced loads of the SoA arrays, one 4-byte key and value per particle.
#include "gd_common.hpp"
#include "gd_internal.hpp"

namespace gd {

// ---------------------------------------------------------------------------
// Bounding box and active count: per-block partials, then one block combines.
__global__ __launch_bounds__(256) void k_bbox_partial(const double* __restrict__ x, const double* __restrict__ y,
                                                      const double* __restrict__ z, const double* __restrict__ M,
                                                      int64_t n, double* __restrict__ red)
{
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double cnt = 0.0;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        if (!(M[i] > 0.0)) continue;
        const double c[3] = {x[i], y[i], z[i]};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            lo[d] = fmin(lo[d], c[d]);
            hi[d] = fmax(hi[d], c[d]);
        }
        cnt += 1.0;
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
        for (int d = 0; d < 7; ++d) red[blockIdx.x * 8 + d] = s[0][d];
    }
}

// one wavefront combines the per-block partials
__global__ __launch_bounds__(64) void k_bbox_final(const double* __restrict__ red, int nblk, WsHeader* __restrict__ h)
{
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

__global__ __launch_bounds__(256) void k_morton(const double* __restrict__ x, const double* __restrict__ y,
                                                const double* __restrict__ z, const double* __restrict__ M, int64_t n,
                                                const WsHeader* __restrict__ h, uint32_t* __restrict__ keys,
                                                uint32_t* __restrict__ vals)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    uint32_t key = 0xFFFFFFFFu;
    if (M[i] > 0.0) {
        const double inv = h->inv;
        key = spread3(quant(x[i], h->lo[0], inv)) | (spread3(quant(y[i], h->lo[1], inv)) << 1) |
              (spread3(quant(z[i], h->lo[2], inv)) << 2);
    }
    keys[i] = key;
    vals[i] = uint32_t(i);
}

// ---------------------------------------------------------------------------
// LSD radix sort, 8-bit digits.  Block b owns keys [b*4096, (b+1)*4096).
// hist is digit-major: hist[d * nblk + b]; each digit's row is exclusive-
// scanned in place by its own block, and the scatter adds the exclusive scan
// of the digit totals.
__global__ __launch_bounds__(256) void k_radix_hist(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                                    uint32_t* __restrict__ hist, int nblk)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = int64_t(blockIdx.x) * kSortTile;
    for (int r = 0; r < kSortTile / 256; ++r) {
        const int64_t i = base + r * 256 + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 0xFFu], 1u);
    }
    __syncthreads();
    hist[int64_t(threadIdx.x) * nblk + blockIdx.x] = h[threadIdx.x];
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
__global__ __launch_bounds__(256) void k_scan_rows(uint32_t* __restrict__ hist, int nblk, uint32_t* __restrict__ tot)
{
    __shared__ uint32_t s_w[4];
    uint32_t* row = hist + int64_t(blockIdx.x) * nblk;
    uint32_t carry = 0;
    for (int c = 0; c < nblk; c += 256) {
        const int i = c + int(threadIdx.x);
        const uint32_t v = i < nblk ? row[i] : 0u;
        uint32_t chunk;
        const uint32_t pre = block_scan_excl_256(v, s_w, &chunk);
        if (i < nblk) row[i] = carry + pre;
        carry += chunk;
    }
    if (threadIdx.x == 0) tot[blockIdx.x] = carry;
}

__global__ __launch_bounds__(256) void k_radix_scatter(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                       uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                       int64_t n, int shift, const uint32_t* __restrict__ hist, int nblk,
                                                       const uint32_t* __restrict__ tot)
{
    __shared__ uint32_t goff[256];   // global offset of each digit for this block
    __shared__ uint32_t run[256];    // items of each digit placed in earlier rounds
    __shared__ uint32_t wcnt[4][256];
    __shared__ uint32_t s_w[4];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint32_t all;
    const uint32_t below = block_scan_excl_256(tot[t], s_w, &all);  // keys of smaller digits
    goff[t] = below + hist[int64_t(t) * nblk + blockIdx.x];
    run[t] = 0;
    const int64_t base = int64_t(blockIdx.x) * kSortTile;
    const uint64_t lt = (uint64_t(1) << lane) - 1;
    for (int r = 0; r < kSortTile / 256; ++r) {
        for (int ww = 0; ww < 4; ++ww) wcnt[ww][t] = 0;
        __syncthreads();
        const int64_t i = base + r * 256 + t;
        const bool valid = i < n;
        uint32_t key = 0, val = 0, dig = 0;
        if (valid) {
            key = kin[i];
            val = vin[i];
            dig = (key >> shift) & 0xFFu;
        }
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

// ---------------------------------------------------------------------------
// Gather of every state array into Morton order, plus the packed positions.
__global__ __launch_bounds__(256) void k_permute(PermuteArgs A)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
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
int launch_morton_sort(const gd_problem* p, const gd_particles* in, gd_particles* out, const double* hint, void* ws,
                       const Layout& L, hipStream_t st)
{
    const int64_t n = p->n;
    WsHeader* h = at<WsHeader>(ws, L.hdr);
    double* red = at<double>(ws, L.red);
    prof_mark(GD_PROF_SORT, 0, st);
    hipLaunchKernelGGL(k_bbox_partial, dim3(kRedBlocks), dim3(256), 0, st, in->x, in->y, in->z, in->M, n, red);
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(64), 0, st, red, kRedBlocks, h);
    uint32_t* k0 = at<uint32_t>(ws, L.keys0);
    uint32_t* k1 = at<uint32_t>(ws, L.keys1);
    uint32_t* v0 = at<uint32_t>(ws, L.vals0);
    uint32_t* v1 = at<uint32_t>(ws, L.vals1);
    uint32_t* hist = at<uint32_t>(ws, L.hist);
    const int nb = int((n + 255) / 256);
    hipLaunchKernelGGL(k_morton, dim3(nb), dim3(256), 0, st, in->x, in->y, in->z, in->M, n, h, k0, v0);
    const int nsb = L.nsort_blocks;
    uint32_t* tot = hist + int64_t(256) * nsb;  // per-digit totals (the spare row of hist)
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 8 * pass;
        const uint32_t* ki = (pass & 1) ? k1 : k0;
        const uint32_t* vi = (pass & 1) ? v1 : v0;
        uint32_t* ko = (pass & 1) ? k0 : k1;
        uint32_t* vo = (pass & 1) ? v0 : v1;
        hipLaunchKernelGGL(k_radix_hist, dim3(nsb), dim3(256), 0, st, ki, n, shift, hist, nsb);
        hipLaunchKernelGGL(k_scan_rows, dim3(256), dim3(256), 0, st, hist, nsb, tot);
        hipLaunchKernelGGL(k_radix_scatter, dim3(nsb), dim3(256), 0, st, ki, vi, ko, vo, n, shift, hist, nsb, tot);
    }
    // sorted (key, slot) pairs are back in (k0, v0)
    PermuteArgs A{};
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
    hipLaunchKernelGGL(k_permute, dim3(nb), dim3(256), 0, st, A);
    prof_mark(GD_PROF_SORT, 1, st);
    out->cur = in->cur;
    return 0;
}

void launch_fill_i32(int32_t* a, int64_t n, int32_t v, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_i32, dim3(int((n + 255) / 256)), dim3(256), 0, st, a, n, v);
}

}  // namespace gd
