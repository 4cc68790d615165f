// gd_groups.hip -- spatial groups (Sect. 2.5.3): which groups interact
// through the neighbour lists, and the broadcast of a group's masses at the
// end of its interval.
//
// A group is a contiguous range of Morton-ordered slots, group_lo[g] ..
// group_lo[g+1].  sched[g] holds the ticks of group g's scheduled interval
// (0: none); the broadcast at the end of the interval clears it.  Groups g != h interact when a retained neighbour of a
// particle of one lies in the other; the relation is returned as one 64-bit
// row per group.
#include "gd_common.hpp"
#include "gd_internal.hpp"

namespace gd {

constexpr int kMaxGroups = 64;

__device__ inline int group_of_slot(const int32_t* lo, int G, int32_t s)
{
    int a = 0, b = G - 1;  // largest g with lo[g] <= s
    while (a < b) {
        const int mid = (a + b + 1) >> 1;
        if (lo[mid] <= s) a = mid;
        else b = mid - 1;
    }
    return a;
}

struct GroupBounds {
    int32_t lo[kMaxGroups + 1];
};

__global__ __launch_bounds__(256) void k_group_interactions(const int32_t* __restrict__ nbr,
                                                            const int32_t* __restrict__ cnt, int k,
                                                            GroupBounds B, int G,
                                                            unsigned long long* __restrict__ mask)
{
    __shared__ int32_t s_lo[kMaxGroups + 1];
    __shared__ unsigned long long s_mask[kMaxGroups];
    for (int t = threadIdx.x; t <= G; t += blockDim.x) s_lo[t] = B.lo[t];
    for (int t = threadIdx.x; t < G; t += blockDim.x) s_mask[t] = 0ull;
    __syncthreads();
    const int32_t n_act = s_lo[G];
    const int lane = threadIdx.x & 63;
    // a fixed grid strides over the particles, so that few blocks update the
    // global rows (updates of one word from many blocks serialise)
    for (int64_t base = blockIdx.x * int64_t(blockDim.x); base < n_act; base += int64_t(gridDim.x) * blockDim.x) {
        const int64_t i = base + threadIdx.x;
        const bool in = i < n_act;
        const int gi = in ? group_of_slot(s_lo, G, int32_t(i)) : -1;
        unsigned long long row = 0ull;
        if (in) {
            const int c = cnt[i];
            for (int t = 1; t < c; ++t) {
                const int32_t j = nbr[i * k + t];
                if (j < 0 || j >= n_act) continue;
                const int gj = group_of_slot(s_lo, G, j);
                if (gj != gi) row |= 1ull << gj;
            }
        }
        // the lanes of a wavefront nearly always share their group: OR their
        // rows across the wavefront and let one lane update the LDS row
        const int g0 = __shfl(gi, 0, 64);
        if (__all(gi == g0 || gi < 0)) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) row |= __shfl_xor(row, o, 64);
            if (lane == 0 && g0 >= 0 && row) atomicOr(&s_mask[g0], row);
        } else if (row) {
            atomicOr(&s_mask[gi], row);  // k_group_symmetric adds the reverse relation
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < G; t += blockDim.x)
        if (s_mask[t]) atomicOr(&mask[t], s_mask[t]);
}

// row g |= bit h for every h whose row holds g (the relation is symmetric)
__global__ void k_group_symmetric(unsigned long long* mask, int G)
{
    __shared__ unsigned long long s[kMaxGroups];
    const int g = threadIdx.x;
    if (g < G) s[g] = mask[g];
    __syncthreads();
    if (g >= G) return;
    unsigned long long row = s[g];
    for (int h = 0; h < G; ++h)
        if ((s[h] >> g) & 1ull) row |= 1ull << h;
    mask[g] = row;
}

// broadcast of a group's masses; its scheduled interval is over
__global__ __launch_bounds__(256) void k_copy_range(double* __restrict__ dst, const double* __restrict__ src,
                                                    int64_t n, int64_t* sched, int group)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) dst[i] = src[i];
    if (i == 0 && sched) sched[group] = 0;
}

int max_groups() { return kMaxGroups; }

int launch_group_interactions(const gd_problem* p, const gd_neighbors* nb, const int32_t* group_lo, int32_t G,
                              uint64_t* mask, hipStream_t st)
{
    launch_fill_i32(reinterpret_cast<int32_t*>(mask), 2 * int64_t(G), 0, st);
    GroupBounds B{};
    for (int g = 0; g <= G; ++g) B.lo[g] = group_lo[g];
    if (B.lo[G] <= 0) return 0;
    const int64_t want = (int64_t(B.lo[G]) + 255) / 256;
    const int grid = int(want < 1024 ? want : 1024);
    hipLaunchKernelGGL(k_group_interactions, dim3(grid), dim3(256), 0, st, nb->nbr, nb->cnt, p->k, B, G,
                       reinterpret_cast<unsigned long long*>(mask));
    hipLaunchKernelGGL(k_group_symmetric, dim3(1), dim3(kMaxGroups), 0, st, reinterpret_cast<unsigned long long*>(mask),
                       G);
    return 0;
}

int launch_publish_group(const gd_particles* s, int64_t lo, int64_t hi, int64_t* sched, int32_t group,
                         hipStream_t st)
{
    const int64_t n = hi - lo;
    const int64_t blocks = n > 0 ? (n + 255) / 256 : 1;
    hipLaunchKernelGGL(k_copy_range, dim3(int(blocks)), dim3(256), 0, st, s->m[s->cur] + lo, s->m[s->cur ^ 1] + lo,
                       n, sched, int(group));
    return 0;
}

}  // namespace gd
