// Ensemble reduction: Eq. (2) weighted averages sum(w A) / sum(w) and
// Eq. (6) mean weight, over per-chain outputs in HBM.
//
// w = exp(log W - L) with L = max log W over live chains (taken by the growth
// kernel as an atomicMax of the bit pattern: log W >= 0 for live chains).
// Determinism: every sum is taken in a fixed order.  Each thread of a block
// sums its chains in index order, the block combines its 256 threads by a
// fixed tree, and the final kernel combines the block partials in block order
// by another fixed tree.  The R^2 histogram is summed in fixed point with
// integer atomics (exact and order-independent), see split_limbs.
#include "rsaw_device.hpp"
#include "rsaw_reduce.hpp"

#include <math.h>

namespace rsaw {

// Zero the max-log-W cell, the status word and the histogram accumulators.
__global__ void reduce_init(unsigned long long *lmax_bits, int32_t *status,
                            unsigned long long *hist_acc, int n_acc)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) {
        *lmax_bits = 0ull;
        *status = 0;
    }
    for (int q = t; q < n_acc; q += gridDim.x * blockDim.x) hist_acc[q] = 0ull;
}

constexpr int kRT = 256; // reduce block size (4 waves)

struct ThreadSums {
    double s[kNumSums];
    uint64_t alive, steps;
    unsigned __int128 ex[3];
};

__device__ __forceinline__ void add_into(ThreadSums &a, const ThreadSums &b)
{
#pragma unroll
    for (int q = 0; q < kNumSums; ++q) a.s[q] = a.s[q] + b.s[q];
    a.alive += b.alive;
    a.steps += b.steps;
    a.ex[0] += b.ex[0];
    a.ex[1] += b.ex[1];
    a.ex[2] += b.ex[2];
}

// Histogram weights are accumulated as fixed-point integers: w in [0, 1] is
// split into three 32-bit limbs (w = l0 2^-32 + l1 2^-64 + l2 2^-96 + t with
// 0 <= t < 2^-96; each step of the split is exact in binary64).  Integer
// sums do not depend on the order of the additions, so LDS and global
// atomics give bit-identical results run to run.  Each limb sum stays below
// 2^32 M < 2^64.
__device__ __forceinline__ void split_limbs(double w, uint64_t &l0, uint64_t &l1, uint64_t &l2)
{
    double t = w * 0x1p32;
    const double f0 = floor(t);
    t = (t - f0) * 0x1p32;
    const double f1 = floor(t);
    t = (t - f1) * 0x1p32;
    const double f2 = floor(t);
    l0 = (uint64_t)f0;
    l1 = (uint64_t)f1;
    l2 = (uint64_t)f2;
}

__device__ __forceinline__ void reduce_partials_body(const ReduceArgs &a, uint64_t bid)
{
    extern __shared__ unsigned char smem[];
    ThreadSums *ts = (ThreadSums *)smem;                                   // [kRT]
    unsigned long long *hacc = (unsigned long long *)(smem + sizeof(ThreadSums) * kRT); // [4][bins]
    const int tid = threadIdx.x;
    for (int q = tid; q < 4 * a.bins; q += kRT) hacc[q] = 0ull;
    __syncthreads();

    const double L = __longlong_as_double((long long)*a.lmax_bits);
    const double nsq1 = (double)(a.n_monomers - 1) * (double)(a.n_monomers - 1) + 1.0;
    const uint64_t begin = bid * a.chunk;
    uint64_t end = begin + a.chunk;
    if (end > a.n_chains) end = a.n_chains;

    ThreadSums my;
#pragma unroll
    for (int q = 0; q < kNumSums; ++q) my.s[q] = 0.0;
    my.alive = 0; my.steps = 0; my.ex[0] = 0; my.ex[1] = 0; my.ex[2] = 0;

    for (uint64_t q = begin + tid; q < end; q += kRT) {
        const double lw = a.log_w[q];
        my.steps += (uint64_t)a.n_grown[q] - 1u;
        if (!(lw > -__builtin_huge_val())) continue;
        const double w = exp(lw - L);
        const double A = a.r2[q];
        const double G = a.rg2[q];
        const double ww = w * w;
        my.alive += 1;
        my.s[0] = my.s[0] + w;
        my.s[1] = my.s[1] + ww;
        my.s[2] = my.s[2] + w * A;
        my.s[3] = my.s[3] + ww * A;
        my.s[4] = my.s[4] + ww * A * A;
        my.s[5] = my.s[5] + w * G;
        my.s[6] = my.s[6] + ww * G;
        my.s[7] = my.s[7] + ww * G * G;
        if (a.exact) {
            const unsigned __int128 W = a.w_exact[q];
            my.ex[0] += W;
            my.ex[1] += W * (unsigned __int128)(uint64_t)A;
            my.ex[2] += W * (unsigned __int128)(uint64_t)a.n2rg2[q];
        }
        if (a.bins > 0) {
            const double fb = floor((A * (double)a.bins) / nsq1);
            const int bin = fb < 0.0 ? 0 : (fb >= (double)a.bins ? a.bins - 1 : (int)fb);
            uint64_t l0, l1, l2;
            split_limbs(w, l0, l1, l2);
            atomicAdd(&hacc[bin], (unsigned long long)l0);
            atomicAdd(&hacc[a.bins + bin], (unsigned long long)l1);
            atomicAdd(&hacc[2 * a.bins + bin], (unsigned long long)l2);
            atomicAdd(&hacc[3 * a.bins + bin], 1ull);
        }
    }

    ts[tid] = my;
    __syncthreads();
    for (int stride = kRT / 2; stride > 0; stride >>= 1) {
        if (tid < stride) add_into(ts[tid], ts[tid + stride]);
        __syncthreads();
    }
    if (tid == 0) {
        BlockPartial &bp = a.partials[bid];
        for (int q = 0; q < kNumSums; ++q) bp.s[q] = ts[0].s[q];
        bp.alive = ts[0].alive;
        bp.steps = ts[0].steps;
        for (int q = 0; q < 3; ++q) {
            bp.ex[2 * q] = (uint64_t)ts[0].ex[q];
            bp.ex[2 * q + 1] = (uint64_t)(ts[0].ex[q] >> 64);
        }
    }
    for (int q = tid; q < 4 * a.bins; q += kRT) {
        const unsigned long long v = hacc[q];
        if (v) atomicAdd(&a.hist_acc[q], v);
    }
}

__global__ __launch_bounds__(kRT) void reduce_partials(ReduceArgs a)
{
    reduce_partials_body(a, blockIdx.x);
}

__device__ __forceinline__ void reduce_final_body(const ReduceArgs &a, uint32_t n_blocks, rsaw_summary *out,
                                                  double *hist_w, uint64_t *hist_n)
{
    __shared__ ThreadSums ts[kRT];
    const int tid = threadIdx.x;
    ThreadSums my;
#pragma unroll
    for (int q = 0; q < kNumSums; ++q) my.s[q] = 0.0;
    my.alive = 0; my.steps = 0; my.ex[0] = 0; my.ex[1] = 0; my.ex[2] = 0;
    for (uint32_t b = tid; b < n_blocks; b += kRT) {
        const BlockPartial &bp = a.partials[b];
        ThreadSums o;
        for (int q = 0; q < kNumSums; ++q) o.s[q] = bp.s[q];
        o.alive = bp.alive;
        o.steps = bp.steps;
        for (int q = 0; q < 3; ++q)
            o.ex[q] = ((unsigned __int128)bp.ex[2 * q + 1] << 64) | bp.ex[2 * q];
        add_into(my, o);
    }
    ts[tid] = my;
    __syncthreads();
    for (int stride = kRT / 2; stride > 0; stride >>= 1) {
        if (tid < stride) add_into(ts[tid], ts[tid + stride]);
        __syncthreads();
    }
    if (tid == 0) {
        const ThreadSums &t = ts[0];
        const double M = (double)a.n_chains;
        const double S0 = t.s[0], S2 = t.s[1];
        const bool any = t.alive > 0;
        const double nan = __builtin_nan("");
        out->n_chains = a.n_chains;
        out->n_alive = t.alive;
        out->log_w_max = any ? __longlong_as_double((long long)*a.lmax_bits) : -__builtin_huge_val();
        out->sum_w = t.s[0];
        out->sum_w2 = t.s[1];
        out->sum_w_r2 = t.s[2];
        out->sum_w2_r2 = t.s[3];
        out->sum_w2_r2sq = t.s[4];
        out->sum_w_rg2 = t.s[5];
        out->sum_w2_rg2 = t.s[6];
        out->sum_w2_rg2sq = t.s[7];
        out->log_c_est = any ? out->log_w_max + log(S0 / M) : -__builtin_huge_val();
        out->c_rel_err = (any && a.n_chains > 1) ? sqrt((M * S2 / (S0 * S0) - 1.0) / (M - 1.0)) : nan;
        const double mr = t.s[2] / S0, mg = t.s[5] / S0;
        out->r2_mean = any ? mr : nan;
        out->r2_err = any ? sqrt(fabs(t.s[4] - 2.0 * mr * t.s[3] + mr * mr * S2)) / S0 : nan;
        out->rg2_mean = any ? mg : nan;
        out->rg2_err = any ? sqrt(fabs(t.s[7] - 2.0 * mg * t.s[6] + mg * mg * S2)) / S0 : nan;
        out->ess = any ? S0 * S0 / S2 : 0.0;
        out->steps = (double)t.steps;
        uint64_t *ex[3] = {out->sum_w_exact, out->sum_w_r2_exact, out->sum_w_n2rg2_exact};
        for (int q = 0; q < 3; ++q) {
            ex[q][0] = (uint64_t)t.ex[q];
            ex[q][1] = (uint64_t)(t.ex[q] >> 64);
        }
        out->exact_valid = a.exact ? 1 : 0;
        out->status = *a.status;
    }
    for (int bi = tid; bi < a.bins; bi += kRT) {
        const unsigned long long *h = a.hist_acc;
        const double sw = (double)h[bi] * 0x1p-32 + (double)h[a.bins + bi] * 0x1p-64 +
                          (double)h[2 * a.bins + bi] * 0x1p-96;
        if (hist_w) hist_w[bi] = sw;
        if (hist_n) hist_n[bi] = h[3 * a.bins + bi];
    }
}

__global__ __launch_bounds__(kRT) void reduce_final(ReduceArgs a, uint32_t n_blocks, rsaw_summary *out,
                                                     double *hist_w, uint64_t *hist_n)
{
    reduce_final_body(a, n_blocks, out, hist_w, hist_n);
}

// Batched forms: one entry per ensemble.
__global__ void reduce_init_batch(const ReduceEntry *tab, int n, uint64_t base)
{
    const ReduceEntry &e = tab[base + blockIdx.x];
    if (threadIdx.x == 0) {
        *e.lmax = 0ull;
        *e.status = 0;
    }
    for (int q = threadIdx.x; q < 4 * e.r.bins; q += blockDim.x) e.r.hist_acc[q] = 0ull;
}

__global__ __launch_bounds__(kRT) void reduce_partials_batch(const ReduceEntry *tab, const uint64_t *block0, int n,
                                                              uint64_t base)
{
    const uint64_t bid = base + blockIdx.x;
    const int e = find_segment(block0, n, bid);
    reduce_partials_body(tab[e].r, bid - block0[e]);
}

__global__ __launch_bounds__(kRT) void reduce_final_batch(const ReduceEntry *tab, int n, uint64_t base)
{
    const ReduceEntry &e = tab[base + blockIdx.x];
    reduce_final_body(e.r, e.n_blocks, e.out, e.hist_w, e.hist_n);
}

size_t reduce_partials_shmem(int bins)
{
    return sizeof(ThreadSums) * kRT + (size_t)4 * bins * sizeof(unsigned long long);
}

hipError_t launch_reduce(const ReduceArgs &a, uint32_t n_blocks, rsaw_summary *out,
                         double *hist_w, uint64_t *hist_n, hipStream_t s)
{
    if (n_blocks > 0) {
        hipLaunchKernelGGL(reduce_partials, dim3(n_blocks), dim3(kRT), reduce_partials_shmem(a.bins), s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(reduce_final, dim3(1), dim3(kRT), 0, s, a, n_blocks, out, hist_w, hist_n);
    return hipGetLastError();
}

hipError_t launch_reduce_init(unsigned long long *lmax_bits, int32_t *status,
                              unsigned long long *hist_acc, int n_acc, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_init, dim3(4), dim3(256), 0, s, lmax_bits, status, hist_acc, n_acc);
    return hipGetLastError();
}

hipError_t launch_reduce_batch(const ReduceEntry *tab, const uint64_t *block0, int n, uint64_t total_blocks,
                               int max_bins, hipStream_t s, bool init_only)
{
    if (n <= 0) return hipSuccess;
    if (init_only)
        return launch_sliced((uint64_t)n, 256, [&](uint64_t b0, uint32_t nb) {
            hipLaunchKernelGGL(reduce_init_batch, dim3(nb), dim3(256), 0, s, tab, n, b0);
        });
    const size_t shmem = reduce_partials_shmem(max_bins);
    hipError_t e = launch_sliced(total_blocks, kRT, [&](uint64_t b0, uint32_t nb) {
        hipLaunchKernelGGL(reduce_partials_batch, dim3(nb), dim3(kRT), shmem, s, tab, block0, n, b0);
    });
    if (e != hipSuccess) return e;
    return launch_sliced((uint64_t)n, kRT, [&](uint64_t b0, uint32_t nb) {
        hipLaunchKernelGGL(reduce_final_batch, dim3(nb), dim3(kRT), 0, s, tab, n, b0);
    });
}

} // namespace rsaw
