// Hard-sphere chain growth in continuous space (Sec. 3.3.3, Algorithm 2;
// weight of Eq. 3).  Trial-parallel mapping: a group of G lanes (G = 8 or the
// next power of two >= k) serves one chain, lane t of the group owns trial t.
// Bead coordinates (binary64) live in LDS as [bead][chain of block][xyz], so
// the 8 chains of a wave read 8 consecutive 24-byte records per bead.
//
// Per step i:
//   1. lane t draws its Marsaglia direction (Philox slot t, first accepted
//      attempt) and forms the candidate tip + b e;
//   2. it tests the candidate against beads 0 .. i-2 of its chain:
//      ((dx dx + dy dy) + dz dz) < sigma^2 means overlap (no contraction);
//   3. a ballot over the group gives the free mask; m = popcount;
//   4. Lemire's pick (16-bit word from the 8-step selection block) chooses
//      the r-th free trial; its candidate is broadcast with a lane shuffle and
//      written to LDS as bead i by its owner;
//   5. lane m - 1 of the group counts the steps with m free trials, and
//      log W = sum_m n_m log m is formed once after the last step.
// The final observables (two-pass Rg^2, R^2) are computed by lane 0 of each
// group in bead order, exactly as the definitions read.
#include "rsaw_device.hpp"

namespace rsaw {

template <int G>
__global__ __launch_bounds__(256) void grow_real_tp(GrowArgs a)
{
    extern __shared__ double beads[]; // [N][cpb][3]
    __shared__ double logm[65];
    for (int t = threadIdx.x; t < 65; t += blockDim.x) logm[t] = a.logm[t];

    const int cpb = blockDim.x / G;
    const int t = threadIdx.x & (G - 1);
    const int chb = threadIdx.x / G;
    const int lane = threadIdx.x & 63;
    const int gbase = lane & ~(G - 1);
    const uint64_t gmask_bits = (G == 64) ? ~0ull : ((1ull << G) - 1ull);
    const uint64_t c = (uint64_t)blockIdx.x * cpb + chb;
    const bool valid = c < a.n_chains;
    const uint64_t g = a.chain_offset + c;
    const int N = a.n_monomers;
    const int k = a.k_trials;
    const bool has_trial = t < k;
    const double b = a.bond_length;
    const double sigma2 = a.sigma2;

    if (t == 0) {
        double *r0 = &beads[(size_t)chb * 3];
        r0[0] = 0.0; r0[1] = 0.0; r0[2] = 0.0;
    }
    __syncthreads();

    double tx = 0.0, ty = 0.0, tz = 0.0;
    bool alive = valid;
    int grown = 1;
    uint32_t n_mine = 0; // steps with m = t + 1 (lane t counts one value of m)
    bool rng_fail = false;
    Philox4 sel{0, 0, 0, 0};

    for (int i = 1; i < N; ++i) {
        // 1. Marsaglia direction of trial t: first attempt with 0 < s < 1
        double v1 = 0.0, v2 = 0.0, s = 0.5;
        bool done = !(alive && has_trial);
        uint32_t att = 0;
        while (!done) {
            const Philox4 q = draw(a.seed, g, (uint32_t)i, (uint32_t)t, att);
            const int64_t j1 = ((int64_t)(q.x0 >> 5) << 26) + (int64_t)(q.x1 >> 6);
            const int64_t j2 = ((int64_t)(q.x2 >> 5) << 26) + (int64_t)(q.x3 >> 6);
            const double u1 = (double)(j1 - (1ll << 52)) * 0x1p-52;
            const double u2 = (double)(j2 - (1ll << 52)) * 0x1p-52;
            const double ss = u1 * u1 + u2 * u2;
            if (ss < 1.0 && ss != 0.0) {
                v1 = u1; v2 = u2; s = ss;
                done = true;
            } else if (++att == kMaxAttempt) {
                rng_fail = true;
                done = true;
            }
        }
        const double qf = 2.0 * sqrt(1.0 - s);
        const double ex = v1 * qf, ey = v2 * qf, ez = 1.0 - 2.0 * s;
        const double cx = tx + b * ex, cy = ty + b * ey, cz = tz + b * ez;

        // 2. overlap test against beads 0 .. i-2 of this chain
        bool fr = alive && has_trial;
        for (int j = 0; j <= i - 2; ++j) {
            const double *r = &beads[((size_t)j * cpb + chb) * 3];
            const double dx = cx - r[0], dy = cy - r[1], dz = cz - r[2];
            double d2 = dx * dx + dy * dy;
            d2 = d2 + dz * dz;
            fr = fr && !(d2 < sigma2);
        }

        // 3. free mask of the group and m
        const uint64_t bal = __ballot(fr);
        const uint64_t gm = (bal >> gbase) & gmask_bits;
        const uint32_t m = (uint32_t)__popcll(gm);

        // 4. uniform pick among the free trials (16-bit Lemire word)
        if (i == 1 || (i & 7) == 0) sel = draw(a.seed, g, (uint32_t)(i >> 3), kSlotSelect, 0);
        const uint32_t x = half_word(sel, (uint32_t)(i & 7));
        const uint32_t p = x * m;
        uint32_t r = p >> 16;
        if (__builtin_expect(alive && (p & 0xFFFFu) < m, 0))
            r = lemire_redraw16(a.seed, g, (uint32_t)i, m, x, &rng_fail);
        const uint64_t below = (t == 0) ? 0ull : (gm & ((1ull << t) - 1ull));
        const bool chosen = fr && ((uint32_t)__popcll(below) == r);
        const uint64_t cb = __ballot(chosen);
        const uint64_t gcb = (cb >> gbase) & gmask_bits;
        const int src = gbase + (gcb ? (__ffsll((long long)gcb) - 1) : 0);
        const double nx = __shfl(cx, src, 64);
        const double ny = __shfl(cy, src, 64);
        const double nz = __shfl(cz, src, 64);

        if (alive && m == 0) {
            alive = false;
            grown = i;
        }
        if (alive) {
            if (chosen) {
                double *ri = &beads[((size_t)i * cpb + chb) * 3];
                ri[0] = nx; ri[1] = ny; ri[2] = nz;
            }
            tx = nx; ty = ny; tz = nz;
            n_mine += (m == (uint32_t)t + 1u) ? 1u : 0u;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (alive) grown = N;

    // log W = sum over m = 1..k, ascending, of n_m log m (Eq. 3 grouped by
    // value); n_m is held by lane m - 1 of the group
    double lw = 0.0;
    for (int mm = 1; mm <= k; ++mm) {
        const uint32_t nm = __shfl(n_mine, gbase + mm - 1, 64);
        lw = lw + (double)nm * logm[mm];
    }
    if (!alive) lw = -__builtin_huge_val();

    // observables, lane 0 of the group, in bead order
    if (t == 0 && valid) {
        double sx = 0.0, sy = 0.0, sz = 0.0;
        for (int j = 0; j < grown; ++j) {
            const double *r = &beads[((size_t)j * cpb + chb) * 3];
            sx = sx + r[0]; sy = sy + r[1]; sz = sz + r[2];
        }
        const double gd = (double)grown;
        const double cmx = sx / gd, cmy = sy / gd, cmz = sz / gd;
        double acc = 0.0;
        for (int j = 0; j < grown; ++j) {
            const double *r = &beads[((size_t)j * cpb + chb) * 3];
            const double dx = r[0] - cmx, dy = r[1] - cmy, dz = r[2] - cmz;
            double q = dx * dx + dy * dy;
            q = q + dz * dz;
            acc = acc + q;
        }
        const double *re = &beads[((size_t)(grown - 1) * cpb + chb) * 3];
        const double ex = re[0], ey = re[1], ez = re[2];
        double r2 = ex * ex + ey * ey;
        r2 = r2 + ez * ez;
        if (a.log_w) a.log_w[c] = lw;
        if (a.r_end) {
            double *o = (double *)a.r_end;
            o[c] = ex; o[a.n_chains + c] = ey; o[2 * a.n_chains + c] = ez;
        }
        if (a.r2) a.r2[c] = r2;
        if (a.rg2) a.rg2[c] = acc / gd;
        if (a.n_grown) a.n_grown[c] = (uint16_t)grown;
    }
    if (rng_fail) atomicExch(a.status, 6);
    const uint64_t bits = (alive && t == 0) ? (uint64_t)__double_as_longlong(lw) : 0ull;
    const uint64_t wmax = wave_max_u64(bits);
    if (lane == 0 && wmax != 0) atomicMax(a.log_w_max_bits, (unsigned long long)wmax);
}

template <int G>
static hipError_t launch_g(const GrowArgs &a, hipStream_t s)
{
    // 256-thread blocks when the bead store fits in 64 KiB, else one wave.
    const size_t per_chain = (size_t)a.n_monomers * 3 * sizeof(double);
    int threads = 256;
    if ((size_t)(threads / G) * per_chain > 65536) threads = 64;
    const int cpb = threads / G;
    const uint64_t blocks = (a.n_chains + cpb - 1) / cpb;
    const size_t shmem = (size_t)cpb * per_chain;
    hipLaunchKernelGGL((grow_real_tp<G>), dim3((uint32_t)blocks), dim3(threads), shmem, s, a);
    return hipGetLastError();
}

// Largest bead count supported by the LDS-resident kernel.
int real_max_monomers() { return 256; }

hipError_t launch_grow_real(const GrowArgs &a, hipStream_t s)
{
    const int k = a.k_trials;
    if (k <= 8) return launch_g<8>(a, s);
    if (k <= 16) return launch_g<16>(a, s);
    if (k <= 32) return launch_g<32>(a, s);
    return launch_g<64>(a, s);
}

} // namespace rsaw
