// Ensemble reduction: Eq. (2) weighted averages sum(w A) / sum(w) and
// Eq. (6) mean weight, over per-chain outputs in HBM.
//
// w = exp(log W - L) with L = max log W over live chains (taken by the growth
// kernel as an atomicMax of the bit pattern: log W >= 0 for live chains).
// Determinism: every sum is taken in a fixed order.  Each thread of a block
// sums its chains in index order, the block combines its 256 threads by a
// fixed tree, and the final kernel combines the block partials in block order
// by another fixed tree.  The histogram is accumulated per wave in LDS, one
// lane at a time in lane order, and combined in wave order, then block order.
#include "rsaw_device.hpp"
#include "rsaw_reduce.hpp"

#include <math.h>

namespace rsaw {

__global__ void reduce_init(unsigned long long *lmax_bits, int32_t *status)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *lmax_bits = 0ull;
        *status = 0;
    }
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

__global__ __launch_bounds__(kRT) void reduce_partials(ReduceArgs a)
{
    extern __shared__ unsigned char smem[];
    ThreadSums *ts = (ThreadSums *)smem;                            // [kRT]
    double *hw = (double *)(smem + sizeof(ThreadSums) * kRT);      // [4][bins]
    uint64_t *hn = (uint64_t *)(hw + 4 * a.bins);                   // [4][bins]
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int q = tid; q < 4 * a.bins; q += kRT) { hw[q] = 0.0; hn[q] = 0; }
    __syncthreads();

    const double L = __longlong_as_double((long long)*a.lmax_bits);
    const double nsq1 = (double)(a.n_monomers - 1) * (double)(a.n_monomers - 1) + 1.0;
    const uint64_t begin = (uint64_t)blockIdx.x * a.chunk;
    uint64_t end = begin + a.chunk;
    if (end > a.n_chains) end = a.n_chains;

    ThreadSums my;
#pragma unroll
    for (int q = 0; q < kNumSums; ++q) my.s[q] = 0.0;
    my.alive = 0; my.steps = 0; my.ex[0] = 0; my.ex[1] = 0; my.ex[2] = 0;

    for (uint64_t base = begin; base < end; base += kRT) {
        const uint64_t q = base + tid;
        const bool ok = q < end;
        double w = 0.0, A = 0.0;
        bool live = false;
        if (ok) {
            const double lw = a.log_w[q];
            my.steps += (uint64_t)a.n_grown[q] - 1u;
            live = lw > -__builtin_huge_val();
            if (live) {
                w = exp(lw - L);
                A = a.r2[q];
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
            }
        }
        if (a.bins > 0) {
            int bin = 0;
            if (live) {
                const double fb = floor((A * (double)a.bins) / nsq1);
                bin = fb < 0.0 ? 0 : (fb >= (double)a.bins ? a.bins - 1 : (int)fb);
            }
            double *hwv = hw + wave * a.bins;
            uint64_t *hnv = hn + wave * a.bins;
            for (int l = 0; l < 64; ++l) {
                if (lane == l && live) {
                    hwv[bin] = hwv[bin] + w;
                    hnv[bin] = hnv[bin] + 1;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
    }

    ts[tid] = my;
    __syncthreads();
    for (int stride = kRT / 2; stride > 0; stride >>= 1) {
        if (tid < stride) add_into(ts[tid], ts[tid + stride]);
        __syncthreads();
    }
    if (tid == 0) {
        BlockPartial &bp = a.partials[blockIdx.x];
        for (int q = 0; q < kNumSums; ++q) bp.s[q] = ts[0].s[q];
        bp.alive = ts[0].alive;
        bp.steps = ts[0].steps;
        for (int q = 0; q < 3; ++q) {
            bp.ex[2 * q] = (uint64_t)ts[0].ex[q];
            bp.ex[2 * q + 1] = (uint64_t)(ts[0].ex[q] >> 64);
        }
    }
    for (int bi = tid; bi < a.bins; bi += kRT) {
        double sw = hw[bi];
        uint64_t sn = hn[bi];
        for (int w = 1; w < 4; ++w) {
            sw = sw + hw[w * a.bins + bi];
            sn += hn[w * a.bins + bi];
        }
        a.part_hist_w[(size_t)blockIdx.x * a.bins + bi] = sw;
        a.part_hist_n[(size_t)blockIdx.x * a.bins + bi] = sn;
    }
}

__global__ __launch_bounds__(kRT) void reduce_final(ReduceArgs a, uint32_t n_blocks,
                                                     rsaw_summary *out, double *hist_w,
                                                     uint64_t *hist_n)
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
        double sw = 0.0;
        uint64_t sn = 0;
        for (uint32_t b = 0; b < n_blocks; ++b) {
            sw = sw + a.part_hist_w[(size_t)b * a.bins + bi];
            sn += a.part_hist_n[(size_t)b * a.bins + bi];
        }
        if (hist_w) hist_w[bi] = sw;
        if (hist_n) hist_n[bi] = sn;
    }
}

size_t reduce_partials_shmem(int bins)
{
    return sizeof(ThreadSums) * kRT + (size_t)4 * bins * (sizeof(double) + sizeof(uint64_t));
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

hipError_t launch_reduce_init(unsigned long long *lmax_bits, int32_t *status, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_init, dim3(1), dim3(64), 0, s, lmax_bits, status);
    return hipGetLastError();
}

} // namespace rsaw
