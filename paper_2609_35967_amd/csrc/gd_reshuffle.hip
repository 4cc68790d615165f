// gd_reshuffle.hip -- random relabelling of the cached neighbours before a
// refresh, as the product-kernel test does (Sect. 3.3): the frozen
// neighbourhoods then sample a well-mixed population.
//
// Slot 0 (the particle itself) is kept.  Every other cached index j becomes
// pi(j), pi one random bijection of the N active slots per (seed, refresh):
// a balanced Feistel network (Luby and Rackoff) of four rounds on two h-bit
// halves, 4^h >= N, whose round function is word 0 of Philox4x32-10 with
// counter (right half, round, refresh, 0x52534831) and the seed as key,
// restricted to [0, N) by cycle walking (Black and Rogaway): the network is
// applied until the value falls below N.  A walk stays on the cycle of the
// network's permutation through j, so it ends within 4^h <= 4N steps.
// pi is evaluated once per slot into a table (the workspace's sort keys,
// free outside the neighbour build, or a fixed device array in the
// allocation-free form), then every cached entry is relabelled by one read
// of the table.  The one other that pi sends onto the row's own particle
// takes pi of that particle instead, so a row never holds itself twice.
#include <mutex>

#include "gd_common.hpp"
#include "gd_internal.hpp"

namespace gd {

__device__ inline uint32_t feistel4(uint32_t x, int h, uint32_t mask, uint32_t k0, uint32_t k1, uint32_t refresh)
{
    uint32_t L = x >> h, R = x & mask;
#pragma unroll
    for (uint32_t t = 0; t < 4; ++t) {
        uint32_t c[4] = {R, t, refresh, 0x52534831u};
        philox4x32_10(c, k0, k1);
        const uint32_t nR = L ^ (c[0] & mask);
        L = R;
        R = nR;
    }
    return (L << h) | R;
}

__device__ inline uint32_t pi_of(uint32_t j, int64_t N, uint64_t seed, uint32_t refresh)
{
    int bits = 0;
    while ((int64_t(1) << bits) < N) ++bits;
    const int h = (bits + 1) >> 1;
    const uint32_t mask = (1u << h) - 1u;
    const uint32_t k0 = uint32_t(seed), k1 = uint32_t(seed >> 32);
    const int64_t cap = int64_t(1) << (2 * h);  // the network's domain: a walk is shorter
    uint32_t x = j;
    for (int64_t step = 0; step < cap; ++step) {
        x = feistel4(x, h, mask, k0, k1, refresh);
        if (int64_t(x) < N) break;
    }
    return x;
}

// pi once per active slot: table[j] = pi(j), j < N
__global__ __launch_bounds__(256) void k_reshuffle_table(int32_t* __restrict__ table,
                                                         const int32_t* __restrict__ n_active, int64_t n,
                                                         uint64_t seed, uint32_t refresh)
{
    const int64_t j = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int64_t N = *n_active;
    if (j >= n || j >= N || N <= 1) return;
    table[j] = int32_t(pi_of(uint32_t(j), N, seed, refresh));
}

// one thread per (particle, slot); slots 1 .. cnt-1 of active rows are
// relabelled.  n * k < 2^31 (checked on the host), so 32-bit index arithmetic
// holds; KS > 0 is log2(k) for a power-of-two k, 0 for any other k.
template <int KS>
__global__ __launch_bounds__(256) void k_reshuffle_apply(int32_t* __restrict__ nbr, const int32_t* __restrict__ cnt,
                                                         const int32_t* __restrict__ n_active,
                                                         const int32_t* __restrict__ table, uint32_t total, uint32_t k)
{
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const uint32_t i = KS > 0 ? (e >> KS) : e / k;
    const uint32_t s = e - i * k;
    const int32_t N = *n_active;
    if (s == 0 || N <= 1 || int32_t(i) >= N || int32_t(s) >= cnt[i]) return;
    const int32_t j = nbr[e];
    if (j < 0 || j >= N) return;
    // pi is a bijection and the row's others exclude i, so exactly one other
    // can be sent onto i; it takes pi(i), which no other slot receives
    const int32_t v = table[j];
    nbr[e] = v == int32_t(i) ? table[i] : v;
}

// pi of every active slot into `table`, then every cached entry relabelled
static void launch_with_table(const gd_problem* p, const gd_neighbors* nb, uint64_t seed, uint32_t refresh,
                              int32_t* table, hipStream_t st)
{
    const int64_t total = p->n * int64_t(p->k);
    if (total <= 0) return;
    hipLaunchKernelGGL(k_reshuffle_table, dim3(unsigned((p->n + 255) / 256)), dim3(256), 0, st, table, nb->n_active,
                       p->n, seed, refresh);
    const dim3 grid(unsigned((total + 255) / 256));
    const uint32_t t32 = uint32_t(total), k = uint32_t(p->k);
    if (k == 32)
        hipLaunchKernelGGL(k_reshuffle_apply<5>, grid, dim3(256), 0, st, nb->nbr, nb->cnt, nb->n_active, table, t32, k);
    else if (k == 64)
        hipLaunchKernelGGL(k_reshuffle_apply<6>, grid, dim3(256), 0, st, nb->nbr, nb->cnt, nb->n_active, table, t32, k);
    else
        hipLaunchKernelGGL(k_reshuffle_apply<0>, grid, dim3(256), 0, st, nb->nbr, nb->cnt, nb->n_active, table, t32, k);
}

int launch_reshuffle(const gd_problem* p, const gd_neighbors* nb, uint64_t seed, uint32_t refresh, void* ws,
                     const Layout& L, hipStream_t st)
{
    launch_with_table(p, nb, seed, refresh, at<int32_t>(ws, L.keys0), st);
    return 0;
}

// ---------------------------------------------------------------------------
// The allocation-free form: pi's table lives in this fixed device array, one
// copy per GPU, held until the process ends.  In host code the name `scratch`
// is a host-side stand-in, not a device address; the array's address on a
// device is resolved once, with that device current, by hipGetSymbolAddress,
// and only that address is ever passed to kernels.  Calls on one GPU share
// the array: overlapping calls there race.  Each call writes entries 0 .. N-1
// before reading them, so nothing needs clearing between calls.
static __device__ __align__(256) int32_t scratch[GD_RESHUFFLE_STATIC_MAX];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int32_t* g_scratch[kMaxDevices] = {};
}  // namespace

hipError_t reshuffle_static_table(int32_t** table)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch[dev] = static_cast<int32_t*>(ptr);
    }
    *table = g_scratch[dev];
    return hipSuccess;
}

int launch_reshuffle_static(const gd_problem* p, const gd_neighbors* nb, uint64_t seed, uint32_t refresh,
                            int32_t* table, hipStream_t st)
{
    launch_with_table(p, nb, seed, refresh, table, st);
    return 0;
}

}  // namespace gd
