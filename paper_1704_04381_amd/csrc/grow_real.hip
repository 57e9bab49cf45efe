// Hard-sphere chain growth in continuous space (Sec. 3.3.3, Algorithm 2;
// weight of Eq. 3).  Trial-parallel mapping: a group of G lanes (G = 8 or the
// next power of two >= k) serves one chain, lane t of the group owns trial t.
// Bead coordinates (binary64) live in LDS as (x, y, z) triples laid out
// [bead][chain of block] with an XOR swizzle of the chain index (see
// plane_row).
//
// Per step i:
//   1. lane t obtains the Marsaglia direction of trial t (Philox slot t, the
//      first accepted attempt) and forms the candidate c_t = tip + b e.
//      Each trial lane keeps a short queue of the accepted pairs of its own
//      trial for the coming steps, drawn ahead in rounds in which every lane
//      with room tries its next attempt; a step only waits for a new round
//      when some lane's queue is empty.  (With one chain per wave and
//      G >= 4 k, the spare lanes instead try later attempts of the same
//      step at once, see `spread`.);
//   2. culling: beads i-2 and i-3 are always tested; the G lanes of the
//      chain split beads 0 .. i-4 (lane t takes every G-th bead) and flag
//      those whose squared tip distance is below (b + sigma)^2 (1 + 2^-30);
//      every other bead is farther than sigma from every candidate (see
//      below), so it cannot overlap;
//   3. each lane tests its candidate against beads i-2, i-3 and the flagged
//      beads: ((dx dx + dy dy) + dz dz) < sigma^2 means overlap (no
//      contraction).  The flag offsets are merged over the wave so that the
//      loop is uniform; re-testing a culled bead is harmless;
//   4. a ballot over the group gives the free mask; m = popcount;
//   5. Lemire's pick (16-bit word from the 8-step selection block) chooses
//      the r-th free trial; its candidate is broadcast with a lane shuffle and
//      written to LDS as bead i by its owner;
//   6. lane m - 1 of the group counts the steps with m free trials, and
//      log W = sum_m n_m log m is formed once after the last step.
//
// Culling is exact, not an approximation.  With u = 2^-53, a bead is
// dropped only when its computed squared tip distance D~^2 (three
// differences, squares and two additions of non-negative terms) is at least
// T = (b + sigma)^2 (1 + e), e = 2^-30.  Then:
//   - the exact tip distance is D >= sqrt(T) (1 + u)^-2.5;
//   - the computed direction has |e| <= 1 + 5u, so the computed candidate
//     lies within b (1 + 9u) + u |tip| of the tip;
//   - the candidate's exact distance to the bead is d >= D - b (1 + 9u) - u |tip|,
//     and its computed d~^2 >= d^2 (1 - u)^5, which is >= sigma^2 whenever
//     d >= sigma (1 - u)^-2.5.
// Putting these together, 0.49 e (b + sigma) >= 11.5 u (b + sigma) + u |tip|
// suffices, and with |tip| <= (N - 1) b that holds for N <= 4 10^6: a culled
// bead would also have passed the full test.
#include "rsaw_device.hpp"

namespace rsaw {

// Uniform on [-1, 1) from the 53-bit integer j = (a >> 5) 2^26 + (b >> 6):
// (j - 2^52) 2^-52, built from bits rather than converted.  With m the low
// 52 bits of j, d = 1 + m 2^-52 is a double of exponent 0, and the result is
// d - 1 when bit 52 of j (bit 31 of a) is set, else d - 2; both
// subtractions are exact (Sterbenz), so the value is the same double.
__device__ __forceinline__ double uniform53(uint32_t a, uint32_t b)
{
    const uint32_t lo = __builtin_amdgcn_alignbit(a >> 5, b, 6); // m bits 0..31
    const uint32_t h = a >> 11;
    const uint32_t hi = (h & 0xFFFFFu) | 0x3FF00000u;           // m bits 32..51, exponent 0
    const uint32_t chi = 0x40000000u - (h & 0x100000u);         // 2.0, or 1.0 for bit 52
    return __hiloint2double((int)hi, (int)lo) - __hiloint2double((int)chi, 0);
}

// OR of the G-bit groups of a wave-wide ballot: bit q is set when lane q of
// any group of G lanes had its predicate set.
template <int G>
__device__ __forceinline__ uint64_t fold_groups(uint64_t v)
{
#pragma unroll
    for (int sh = 32; sh >= G; sh >>= 1) v |= v >> sh;
    return G == 64 ? v : (v & ((1ull << G) - 1ull));
}

// Orders LDS accesses of the lanes of one wave.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One Marsaglia attempt from a Philox block: the two 53-bit uniforms on
// [-1, 1) (always set) and whether the pair lies strictly inside the unit
// disc, off its centre.
__device__ __forceinline__ bool marsaglia_pair(const Philox4 q, double &u1, double &u2)
{
    u1 = uniform53(q.x0, q.x1);
    u2 = uniform53(q.x2, q.x3);
    const double ss = u1 * u1 + u2 * u2;
    return ss < 1.0 && ss != 0.0;
}

// Row length (in elements) of the bead array for cpb chains per block.
// Bead j of chain c is element j row + (c ^ ((j H) mod cpb)), H = 32 / G,
// an (x, y, z) triple of 24 bytes.  A wave reads binary64 words half a wave
// at a time over 64 four-byte banks; the culling pass has lane t of chain c
// read bead b0 + t (b0 a multiple of G), and with cpb = 32 (G = 8, 256
// threads) the 32 (t, c) pairs of a half wave then fall on distinct
// elements modulo 32, whose 24-byte strides cover distinct bank pairs, as
// do the other accesses, where all chains of a wave read the same bead
// index.  Smaller cpb leaves at most 2-way conflicts (4-way for G = 32 in
// 256-thread blocks).  G = 64 (one chain per wave) uses an odd row and no
// swizzle instead.
__host__ __device__ inline int plane_row(int cpb, int G) { return G == 64 ? (cpb | 1) : cpb; }

// Bead e of an (x, y, z) triple array.  LDS serves 8-byte reads over 32
// banks of 8 bytes, 32 lanes per pass; the swizzle of plane_row puts the
// lanes of a pass on distinct banks for each 8-byte read, but a 16-byte read
// of the x, y pair (which the compiler would otherwise merge the first two
// into) spans two banks per lane and meets 2-way conflicts.  The empty asm
// statements keep the three reads apart.
template <bool HBM>
__device__ __forceinline__ void load_bead(const double *P, int e, double &x, double &y, double &z)
{
    if constexpr (HBM) {
        const double *q = P + 3 * e;
        x = q[0]; y = q[1]; z = q[2];
    } else {
        typedef const double __attribute__((address_space(3))) *lds_ptr;
        lds_ptr q = (lds_ptr)(P + 3 * e);
        x = q[0];
        asm volatile("" : "+v"(q));
        y = q[1];
        asm volatile("" : "+v"(q));
        z = q[2];
    }
}

// Accepted Marsaglia pairs a trial lane keeps ahead of the current step.
constexpr int kQueue = 4;

// Orders the bead accesses of the lanes of one wave: beads in LDS need the
// wavefront scope, beads in global memory (one wave per block) the
// workgroup scope, which waits for the stores before later loads.
template <bool HBM>
__device__ __forceinline__ void plane_sync()
{
    if constexpr (HBM) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    } else {
        wave_sync();
    }
}

// HBM: the beads of chain `bid` live in global memory, in the region of
// resident block `slot` (one 64-lane chain per block, row 1, no swizzle).
template <int G, bool HBM>
__device__ __forceinline__ void grow_real_body(const GrowArgs &a, uint64_t bid, uint32_t slot = 0)
{
    extern __shared__ double lds[]; // [N][row] (x, y, z) bead triples, swizzled

    const int cpb = blockDim.x / G;
    // wave-uniform: bead offsets of uniform bead indices stay scalar
    const int row = __builtin_amdgcn_readfirstlane(plane_row(cpb, G));
    const int swz_mul = G == 64 ? 0 : 32 / G;
    const int swz_mask = cpb - 1;
    const int N = a.n_monomers;
    double *P = HBM ? a.bead_slots + (size_t)slot * 3 * N : lds;
    const int t = threadIdx.x & (G - 1);
    const int chb = threadIdx.x / G;
    const int lane = threadIdx.x & 63;
    const int gbase = lane & ~(G - 1);
    // element of bead j of this chain
    const auto at = [&](int j) { return j * row + (chb ^ ((j * swz_mul) & swz_mask)); };
    // bead b0 + t for b0 a multiple of G: (b0 H) mod cpb = 0 (32 divides b0 H
    // and cpb <= 32), so its element is b0 row + at(t); elements past the
    // last one are clamped to it (their results are discarded)
    const int at_lane = at(t);
    const int last_el = N * row - 1;
    const uint64_t gmask_bits = (G == 64) ? ~0ull : ((1ull << G) - 1ull);
    const uint64_t c = bid * cpb + chb;
    const bool valid = c < a.n_chains;
    const uint64_t g = a.chain_offset + c;
    const int k = a.k_trials;
    const bool has_trial = t < k;
    // Round 1 of the Marsaglia draws spreads attempts 0 .. reps-1 of the k
    // trials over the G lanes of the chain: lane t tries attempt t / k of
    // trial t mod k (G >= k).  Used when reps >= 4, where a second round is
    // rarely needed (measured 1.08-1.36x faster for k = 8, 256 <= N <= 1536);
    // otherwise each trial lane draws its own trial ahead through its queue.
    const int reps = G / k;
    bool spread = false;
    if constexpr (G >= 32) spread = reps >= 4;
    const uint32_t r1_trial = (uint32_t)(t % k), r1_att = (uint32_t)(t / k);
    const bool r1_lane = t < reps * k;
    uint64_t r1_pattern = 0; // bits 0, k, 2k, ...: the lanes of one trial
    for (int q = 0; q < reps; ++q) r1_pattern |= 1ull << (q * k);
    // a double from lane src of the wave
    const auto pull_from = [](int src, double v) {
        const int64_t bits = __double_as_longlong(v);
        const int lo = __builtin_amdgcn_ds_bpermute(src * 4, (int)(uint32_t)bits);
        const int hi = __builtin_amdgcn_ds_bpermute(src * 4, (int)(uint32_t)(bits >> 32));
        return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
    };
    const double b = a.bond_length;
    const double sigma2 = a.sigma2;
    const double cull2 = a.cull2;

    if (t == 0) {
        const int o = 3 * at(0);
        P[o] = 0.0; P[o + 1] = 0.0; P[o + 2] = 0.0;
    }
    if constexpr (HBM) plane_sync<true>();
    __syncthreads();

    double tx = 0.0, ty = 0.0, tz = 0.0;
    bool alive = false;
    int grown = 1;
    uint32_t n_mine = 0; // steps with m = t + 1 (lane t counts one value of m)
    bool rng_fail = false;
    Philox4 sel{0, 0, 0, 0};
    // this lane's queue: q1[0..lvl), q2[0..lvl) hold the accepted pairs of
    // trial t for steps i, i + 1, ...; the next draw is step nstep, attempt natt
    double q1[kQueue], q2[kQueue];
#pragma unroll
    for (int q = 0; q < kQueue; ++q) { q1[q] = 0.0; q2[q] = 0.0; }
    int lvl = 0;
    uint32_t nstep = 1, natt = 0;
    // the attempt that ends the chain: the first complete one, or the last
    // allowed one (one attempt without restarts); bead 0 stays at the origin
    bool res_alive = false;
    double res_lw = -__builtin_huge_val();
    bool pending = valid;

    for (uint32_t rd = 0; rd < a.max_rounds; ++rd) {
        if (pending) {
            tx = 0.0; ty = 0.0; tz = 0.0;
            n_mine = 0;
            lvl = 0; nstep = 1; natt = 0;
        }
        alive = pending;
        grown = 1;
        const uint32_t hi = rd << 16; // attempt in the high half of the step word
        // One production round of the trial queues: each lane with room
        // tries its next attempt; an accepted pair joins the queue and the
        // lane moves on to the next step (a lane reaching the attempt cap
        // queues its last pair and reports the failure).  Every step runs one
        // round while its first bead reads are in flight, and more at its end
        // until every lane that grows a trial at the next step holds its pair.
        const auto round = [&]() {
            const bool room = alive && has_trial && lvl < kQueue && nstep < (uint32_t)N;
            double u1, u2;
            const bool ok = marsaglia_pair(draw(a.seed, g, nstep | hi, (uint32_t)t, natt), u1, u2);
            const bool capped = !ok && natt + 1u == kMaxAttempt;
            const bool put = room && (ok || capped);
            rng_fail = rng_fail || (room && capped);
#pragma unroll
            for (int q = 0; q < kQueue; ++q) {
                const bool here = put && lvl == q;
                q1[q] = here ? u1 : q1[q];
                q2[q] = here ? u2 : q2[q];
            }
            lvl += put ? 1 : 0;
            nstep += put ? 1u : 0u;
            natt = put ? 0u : natt + (room ? 1u : 0u);
        };
        // a lane starves when its queue is empty and the step it needs next
        // (nstep, when the queue is empty) exists; a starving lane always has
        // room, so every round moves it on (an acceptance, or its attempt cap)
        const auto starving = [&]() { return alive && has_trial && lvl == 0 && nstep < (uint32_t)N; };
        if (!spread)
            while (__ballot(starving()) != 0) round();

        for (int i = 1; i < N; ++i) {
            // 1. Marsaglia direction of trial t: the first accepted attempt.
            double v1 = 0.0, v2 = 0.0, s = 0.5;
            const bool need = alive && has_trial;
            if (!spread) {
                v1 = q1[0]; v2 = q2[0];
#pragma unroll
                for (int q = 0; q + 1 < kQueue; ++q) { q1[q] = q1[q + 1]; q2[q] = q2[q + 1]; }
                if (need) --lvl;
                s = v1 * v1 + v2 * v2;
            } else {
                // Round 1: the chain's G lanes try attempts 0 .. reps-1 of its
                // k trials (lane u: trial u mod k, attempt u / k) and each
                // trial takes its smallest accepted one.  Round 2 (when a
                // trial failed all of them): the 64 lanes of the wave serve
                // the failed trials, lane l taking the failed trial of rank
                // q = l mod nF at attempt reps + l / nF; each failed trial then
                // takes its first accepting helper in lane order, which is its
                // smallest accepted attempt.  Values move through the
                // cross-lane permute network (no LDS storage).  A trial whose
                // helpers all rejected continues alone after its last helped
                // attempt.
                double w1 = 0.0, w2 = 0.0;
                const bool wok = marsaglia_pair(draw(a.seed, g, (uint32_t)i | hi, r1_trial, r1_att), w1, w2) &
                                 r1_lane;
                const uint64_t B = (__ballot(wok) >> gbase) & gmask_bits;
                const uint64_t cand = has_trial ? ((B >> t) & r1_pattern) : 0ull;
                const int src = cand ? gbase + t + __builtin_ctzll(cand) : lane;
                v1 = pull_from(src, w1);
                v2 = pull_from(src, w2);
                bool acc = cand != 0;
                uint32_t att = (uint32_t)reps; // the next attempt of a trial still failing
                const uint64_t F = __ballot(need && !acc);
                if (F != 0) {
                    const uint32_t nF = (uint32_t)__popcll(F);
                    const bool failing = need && !acc;
                    const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(F >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)F, 0u));
                    // lane q < nF learns the lane of the failed trial of rank q
                    const int owner_of_q = __builtin_amdgcn_ds_permute((int)((failing ? rank : 63u) * 4u), lane);
                    // l / nF and l mod nF (l < 64: the float quotient is never
                    // within rounding of an integer boundary)
                    const uint32_t jh = (uint32_t)(((float)lane + 0.5f) * __builtin_amdgcn_rcpf((float)nF));
                    const uint32_t q = (uint32_t)lane - jh * nF;
                    const int owner = __builtin_amdgcn_ds_bpermute((int)(q * 4u), owner_of_q);
                    const uint64_t og = a.chain_offset + bid * cpb +
                                        (uint64_t)(((threadIdx.x & ~63) + (owner & ~(G - 1))) / G);
                    double h1 = 0.0, h2 = 0.0;
                    const bool hok = marsaglia_pair(draw(a.seed, og, (uint32_t)i | hi,
                                                         (uint32_t)(owner & (G - 1)), att + jh),
                                                    h1, h2);
                    const uint64_t H = __ballot(hok);
                    // helpers of rank r are lanes r, r + nF, r + 2 nF, ...
                    uint64_t pattern = 0;
                    for (uint32_t l = 0; l < 64u; l += nF) pattern |= 1ull << l;
                    const uint64_t mine = failing ? (H & (pattern << rank)) : 0ull;
                    const int hsrc = mine ? __builtin_ctzll(mine) : lane;
                    const double n1 = pull_from(hsrc, h1), n2 = pull_from(hsrc, h2);
                    if (failing) {
                        if (mine) {
                            v1 = n1; v2 = n2;
                            acc = true;
                        } else {
                            att = att + (64u - rank + nF - 1u) / nF;
                        }
                    }
                }
                // round 3 (rare): the remaining trials continue alone
                bool done = !need || acc;
                while (!done) {
                    double u1, u2;
                    if (marsaglia_pair(draw(a.seed, g, (uint32_t)i | hi, (uint32_t)t, att), u1, u2)) {
                        v1 = u1; v2 = u2;
                        done = true;
                    } else if (++att == kMaxAttempt) {
                        rng_fail = true;
                        done = true;
                    }
                }
                s = v1 * v1 + v2 * v2;
            }
            const double qf = 2.0 * sqrt_unit(1.0 - s); // 1 - s in [2^-53, 1)
            const double ex = v1 * qf, ey = v2 * qf, ez = 1.0 - 2.0 * s;
            const double cx = tx + b * ex, cy = ty + b * ey, cz = tz + b * ez;

            // 2-3. exact test of this lane's candidate: beads i-2 and i-3 (within
            // 2b of the tip) directly, beads 0 .. i-4 after the culling pass
            bool blocked = false; // bitwise accumulation keeps the tests branch-free
            const auto test_el = [&](int e) {
                double x, y, z;
                load_bead<HBM>(P, e, x, y, z);
                const double dx = cx - x, dy = cy - y, dz = cz - z;
                double d2 = dx * dx + dy * dy;
                d2 = d2 + dz * dz;
                blocked = blocked | (d2 < sigma2);
            };
            const auto is_near_el = [&](int e) {
                double x, y, z;
                load_bead<HBM>(P, e, x, y, z);
                const double dx = x - tx, dy = y - ty, dz = z - tz;
                double d2 = dx * dx + dy * dy;
                d2 = d2 + dz * dz;
                return !(d2 >= cull2);
            };
            {
                // beads i-2 and i-3 (masked before step 2 and 3): reads, one
                // production round while they are in flight, tests
                double x2, y2, z2, x3, y3, z3;
                load_bead<HBM>(P, at(i >= 2 ? i - 2 : 0), x2, y2, z2);
                load_bead<HBM>(P, at(i >= 3 ? i - 3 : 0), x3, y3, z3);
                if (!spread) {
                    round();
                    // keeps the round here, ahead of the tests that wait for the reads
                    asm volatile("" ::"v"(lvl), "v"(natt));
                }
                const auto overlaps = [&](double x, double y, double z) {
                    const double dx = cx - x, dy = cy - y, dz = cz - z;
                    double d2 = dx * dx + dy * dy;
                    d2 = d2 + dz * dz;
                    return d2 < sigma2;
                };
                const bool o2 = overlaps(x2, y2, z2), o3 = overlaps(x3, y3, z3);
                blocked = (i >= 2 && o2) || (i >= 3 && o3);
            }
            const int nb = __builtin_amdgcn_readfirstlane(i - 3);
            // Culling passes of two blocks of G beads, lane t taking beads
            // b0 + t and b0 + G + t; the offsets flagged by any chain of the
            // wave are re-tested exactly by every chain (a culled bead cannot
            // overlap, so testing it again changes nothing), two at a time so
            // that their reads are in flight together.  (Four blocks per pass
            // measured 4 % slower at N = 64, k = 8.)
            constexpr int PB = 2;
            const auto retest = [&](uint64_t u, int base) {
                while (u) {
                    const int qa = __builtin_ctzll(u);
                    u &= u - 1;
                    if (u) {
                        const int qb = __builtin_ctzll(u);
                        u &= u - 1;
                        double xa, ya, za, xb, yb, zb;
                        load_bead<HBM>(P, at(base + qa), xa, ya, za);
                        load_bead<HBM>(P, at(base + qb), xb, yb, zb);
                        const auto hit = [&](double x, double y, double z) {
                            const double dx = cx - x, dy = cy - y, dz = cz - z;
                            double d2 = dx * dx + dy * dy;
                            d2 = d2 + dz * dz;
                            return d2 < sigma2;
                        };
                        const bool ha = hit(xa, ya, za), hb = hit(xb, yb, zb);
                        blocked = blocked || ha || hb;
                    } else {
                        test_el(at(base + qa));
                    }
                }
            };
            for (int b0 = 0; b0 < nb; b0 += PB * G) {
                bool nearv[PB];
#pragma unroll
                for (int pb = 0; pb < PB; ++pb) {
                    const int e = min((b0 + pb * G) * row + at_lane, last_el);
                    nearv[pb] = alive & (b0 + pb * G + t < nb) & is_near_el(e);
                }
                if constexpr (PB * G <= 64) {
                    uint64_t u = 0;
#pragma unroll
                    for (int pb = 0; pb < PB; ++pb) u |= fold_groups<G>(__ballot(nearv[pb])) << (pb * G);
                    retest(u, b0);
                } else {
#pragma unroll
                    for (int pb = 0; pb < PB; ++pb) retest(fold_groups<G>(__ballot(nearv[pb])), b0 + pb * G);
                }
            }

            const bool fr = alive & has_trial & !blocked;

            // 4. free mask of the group and m
            const uint64_t bal = __ballot(fr);
            const uint64_t gm = (bal >> gbase) & gmask_bits;
            const uint32_t m = (uint32_t)__popcll(gm);

            // 5. uniform pick among the free trials (16-bit Lemire word)
            if (i == 1 || (i & 7) == 0) sel = draw(a.seed, g, (uint32_t)(i >> 3) | hi, kSlotSelect, 0);
            const uint32_t x = half_word(sel, (uint32_t)(i & 7));
            const uint32_t p = x * m;
            uint32_t r = p >> 16;
            if (__builtin_expect(alive && (p & 0xFFFFu) < m, 0)) {
                r = lemire_redraw16(a.seed, g, (uint32_t)i | hi, m, x);
                if (r == kPickFailed) {
                    rng_fail = true;
                    r = 0;
                }
            }
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
                    const int o = 3 * at(i);
                    P[o] = nx; P[o + 1] = ny; P[o + 2] = nz;
                }
                tx = nx; ty = ny; tz = nz;
                n_mine += (m == (uint32_t)t + 1u) ? 1u : 0u;
            }
            if (!spread)
                while (__ballot(starving()) != 0) round();
            plane_sync<HBM>();
            // long chains: once every chain of the wave has ended (most hard-sphere
            // chains beyond a few hundred beads meet a dead end), the wave leaves
            // the step loop instead of running the remaining steps on dead
            // chains (N = 1000, 2 10^4 chains: 22.9 -> 7.6 ms; N = 3000:
            // 45.9 -> 6.7 ms); at N <= 256 the test costs more than it saves
            if (N > 256 && __ballot(alive) == 0) break;
        }
        if (alive) grown = N;
        const bool ends = pending && (alive || rd + 1 >= a.max_rounds);

        // log W = sum over m = 1..k, ascending, of n_m log m (Eq. 3 grouped by
        // value); n_m is held by lane m - 1 of the group
        double lw = 0.0;
        for (int mm = 1; mm <= k; ++mm) {
            const uint32_t nm = __shfl(n_mine, gbase + mm - 1, 64);
            lw = lw + (double)nm * a.logm[mm];
        }
        if (!alive) lw = -__builtin_huge_val();

        // observables, lane 0 of the group, in bead order
        if (ends && t == 0 && valid) {
            double sx = 0.0, sy = 0.0, sz = 0.0;
            for (int j = 0; j < grown; ++j) {
                const int o = 3 * at(j);
                sx = sx + P[o]; sy = sy + P[o + 1]; sz = sz + P[o + 2];
            }
            const double gd = (double)grown;
            const double cmx = sx / gd, cmy = sy / gd, cmz = sz / gd;
            double acc = 0.0;
            for (int j = 0; j < grown; ++j) {
                const int o = 3 * at(j);
                const double dx = P[o] - cmx, dy = P[o + 1] - cmy, dz = P[o + 2] - cmz;
                double q = dx * dx + dy * dy;
                q = q + dz * dz;
                acc = acc + q;
            }
            const int oe = 3 * at(grown - 1);
            const double ex = P[oe], ey = P[oe + 1], ez = P[oe + 2];
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
        if (ends) {
            res_alive = alive;
            res_lw = lw;
            pending = false;
        }
        if (__ballot(pending) == 0) break;
    }
    if (rng_fail) atomicExch(a.status, 6);
    const uint64_t bits = (res_alive && t == 0) ? (uint64_t)__double_as_longlong(res_lw) : 0ull;
    const uint64_t wmax = wave_max_u64(bits);
    if (lane == 0 && wmax != 0) atomicMax(a.log_w_max_bits, (unsigned long long)wmax);
}

template <int G>
__global__ __launch_bounds__(256) void grow_real_tp(GrowArgs a, uint64_t base)
{
    grow_real_body<G, false>(a, base + blockIdx.x);
}

// Batched launch: block b serves the ensemble whose block range holds b.
template <int G>
__global__ __launch_bounds__(256) void grow_real_tp_batch(const GrowEntry *tab, const uint64_t *block0, int n,
                                                          uint64_t base)
{
    const uint64_t bid = base + blockIdx.x;
    const int e = find_segment(block0, n, bid);
    grow_real_body<G, false>(tab[e].a, bid - block0[e]);
}

// Chains beyond the LDS limit: a persistent grid of one-wave blocks, block s
// growing chains s, s + grid, s + 2 grid, ... in its own HBM plane region.
__global__ __launch_bounds__(64) void grow_real_hbm(GrowArgs a)
{
    for (uint64_t bid = blockIdx.x; bid < a.n_chains; bid += gridDim.x)
        grow_real_body<64, true>(a, bid, blockIdx.x);
}

// Largest bead count of the LDS-resident kernel, and of the HBM one.  LDS
// planes fit up to N = 6826, but beyond N ~ 1500 they leave fewer than 4
// waves per CU, and the HBM planes (8 waves per CU, cached in L2) are faster:
// measured on MI355X, k = 8, per launch: N = 1024 LDS 15.7 ms / HBM 20.3 ms,
// N = 2048 30.8 / 28.4, N = 4096 121.7 / 53.2, N = 6144 126.2 / 78.0.
constexpr int kRealLdsMax = 1536;
int real_max_monomers() { return 16384; }

// Resident blocks (and HBM plane regions) of the HBM kernel for M chains.
uint32_t real_hbm_slots(int n_monomers, uint64_t n_chains)
{
    if (n_monomers <= kRealLdsMax) return 0;
    return (uint32_t)(n_chains < 2048 ? n_chains : 2048);
}

// Shape of the LDS kernel for N beads, G lanes per chain (8..64, G >= k: one
// trial per lane) and `threads` per block (64 or 256; G = 64 only in
// one-wave blocks).  hipErrorInvalidValue when the combination is not legal
// or the block's planes and logarithm table exceed the CU's 160 KiB.
static hipError_t real_shape(int N, int k, int G, int threads, GrowVariant *v)
{
    if (G != 8 && G != 16 && G != 32 && G != 64) return hipErrorInvalidValue;
    if (G < k) return hipErrorInvalidValue;
    if (threads != 64 && (threads != 256 || G == 64)) return hipErrorInvalidValue;
    const size_t planes = (size_t)3 * N * plane_row(threads / G, G) * sizeof(double);
    if (planes > 163840) return hipErrorInvalidValue;
    v->family = 2;
    v->p0 = G;
    v->p1 = 0;
    v->p2 = 0;
    v->threads = threads;
    v->cpb = threads / G;
    v->shmem = planes;
    v->H = 0;
    v->S = 0;
    return hipSuccess;
}

// Built-in rule.  Lanes per chain: at least the next power of two >= k (one
// trial per lane), and enough that the chains whose planes fit in a CU's LDS
// still fill about 8 waves (G >= 0.075 N); the extra lanes share the culling
// pass.  256-thread blocks when the bead planes fit in half a CU's LDS, else
// one wave per block (up to the whole 160 KiB).  G = 64 always runs one-wave
// blocks: four one-chain waves sharing a block's padded planes were measured
// 1.2-2.3x slower for 432 <= N <= 672 (k = 8) than four one-wave blocks.  A
// legal mapping of the tuning table replaces the rule.
hipError_t real_variant(const GrowArgs &a, GrowVariant *v)
{
    const int N = a.n_monomers;
    if (N > kRealLdsMax) {
        // HBM planes, launched on its own (p1 = 1)
        v->family = 2;
        v->p0 = 64;
        v->p1 = 1;
        v->p2 = 0;
        v->threads = 64;
        v->cpb = 1;
        v->shmem = 0;
        v->H = 0;
        v->S = 0;
        return hipSuccess;
    }
    int tl = 0, tt = 0;
    if (tuned_mapping(1 /* hard spheres */, N, a.k_trials, &tl, &tt) &&
        real_shape(N, a.k_trials, tl, tt, v) == hipSuccess)
        return hipSuccess;
    int need = a.k_trials;
    const int occ = (3 * N + 39) / 40; // ceil(0.075 N)
    if (occ > need) need = occ;
    const int G = need <= 8 ? 8 : (need <= 16 ? 16 : (need <= 32 ? 32 : 64));
    // k = 8 or 16 with 2k lanes in 256-thread blocks whose planes leave
    // fewer than 3 blocks per CU: 4k lanes in one-wave blocks are faster
    // (the extra lanes also carry the round-1 Marsaglia attempts); measured
    // on MI355X: k = 8, 144 <= N <= 208, 1.18-1.22x; k = 16, 320 <= N <= 416,
    // 1.13-1.20x.
    const int k = a.k_trials;
    GrowVariant wide, at256;
    if ((k == 8 || k == 16) && G == 2 * k && real_shape(N, k, G, 256, &at256) == hipSuccess &&
        at256.shmem > 163840 / 3 && real_shape(N, k, 4 * k, 64, &wide) == hipSuccess) {
        *v = wide;
        return hipSuccess;
    }
    GrowVariant half_cu;
    if (G != 64 && real_shape(N, a.k_trials, G, 256, &half_cu) == hipSuccess && half_cu.shmem <= 81920) {
        *v = half_cu;
        return hipSuccess;
    }
    return real_shape(N, a.k_trials, G, 64, v);
}

template <int G>
static hipError_t launch_g(const GrowArgs &a, const GrowVariant &v, const GrowEntry *tab,
                           const uint64_t *block0, int n, uint64_t blocks, size_t shmem, hipStream_t s)
{
    const void *fn = tab ? (const void *)grow_real_tp_batch<G> : (const void *)grow_real_tp<G>;
    if (shmem > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess) return e;
    }
    return launch_sliced(blocks, v.threads, [&](uint64_t b0, uint32_t nb) {
        if (tab)
            hipLaunchKernelGGL((grow_real_tp_batch<G>), dim3(nb), dim3(v.threads), shmem, s, tab, block0, n, b0);
        else
            hipLaunchKernelGGL((grow_real_tp<G>), dim3(nb), dim3(v.threads), shmem, s, a, b0);
    });
}

static hipError_t dispatch_real(const GrowArgs &a, const GrowVariant &v, const GrowEntry *tab,
                                const uint64_t *block0, int n, uint64_t blocks, size_t shmem, hipStream_t s)
{
    switch (v.p0) {
    case 8: return launch_g<8>(a, v, tab, block0, n, blocks, shmem, s);
    case 16: return launch_g<16>(a, v, tab, block0, n, blocks, shmem, s);
    case 32: return launch_g<32>(a, v, tab, block0, n, blocks, shmem, s);
    default: return launch_g<64>(a, v, tab, block0, n, blocks, shmem, s);
    }
}

hipError_t launch_grow_real(const GrowArgs &a, hipStream_t s)
{
    GrowVariant v;
    hipError_t e = real_variant(a, &v);
    if (e != hipSuccess) return e;
    if (v.p1) {
        if (!a.bead_slots || a.n_slots == 0) return hipErrorInvalidValue;
        hipLaunchKernelGGL(grow_real_hbm, dim3(a.n_slots), dim3(64), 0, s, a);
        return hipGetLastError();
    }
    const uint64_t blocks = (a.n_chains + v.cpb - 1) / v.cpb;
    return dispatch_real(a, v, nullptr, nullptr, 0, blocks, v.shmem, s);
}

hipError_t launch_real_batch(const GrowVariant &v, const GrowEntry *tab, const uint64_t *block0, int n,
                             uint64_t blocks, size_t shmem, hipStream_t s)
{
    return dispatch_real(GrowArgs{}, v, tab, block0, n, blocks, shmem, s);
}

} // namespace rsaw
