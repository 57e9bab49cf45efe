// Lattice chain growth on the simple cubic lattice (Sec. 3.3.2, Algorithm 1;
// weight of Eq. 3), one chain per lane, chain state in VGPRs.
//
// Monomer word (one 32-bit VGPR per monomer, fully unrolled over NMAX):
//   byte 0 : Q = x + 2y + 3z  (mod 256)
//   byte 1 : x + 128,  byte 2 : y + 128,  byte 3 : z + 128
// Coordinates of an N <= 64 chain stay in [-63, 63], so bytes 1..3 never
// wrap and never become zero.
//
// Pair test of step i (tip t = monomer i-1), for each earlier monomer j of the
// parity that can touch the tip's neighbours (j = i-2, i-4, ...; the cubic
// lattice is bipartite, so the other parity never neighbours the tip):
//   L    = v_msad_u8(r_j, t & ~0xFF)   L1 distance; byte 0 is masked because
//                                      the reference byte is zero
//   bit  = sat(2 - L)                  1 iff r_j is a neighbour of t
//   code = (Q_j - Q_t + 3) mod 32      = 0..6 without 3: -z, -y, -x, +x, +y, +z
//   occ |= bit << code                 v_lshl_or_b32
// Four VALU operations per pair, no memory access.  The six neighbour codes
// are also the candidates' canonical order, so free = ~occ & 0x77 is already
// the ordered candidate mask and the pick is one LDS table lookup.
//
// log W = sum over m of n_m log m (Eq. 3 grouped by value): the counts of
// m = 2..5 are kept as 6-bit fields of one register (2 operations per step)
// and the sum is formed once after the last step.
//
// Measured on MI355X (10^7 chains, N = 64): splitting the occupied mask over
// two accumulators shortens the per-step dependency chain and gains ~10%;
// capping the kernel at 4 waves per SIMD (spilling) loses ~10%.
#include "lattice_common.hpp"

#include <type_traits>

namespace rsaw {

// Compile-time loop: f(integral_constant<int, I>) for I = B .. E-1, so that
// every index into the register-resident chain is a constant.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

constexpr uint32_t kOrigin = 0x80808000u; // origin, Q = 0

template <int NMAX, bool EXACT, typename CT>
__device__ __forceinline__ void grow_lattice_reg_body(const GrowArgs &a, uint64_t bid)
{
    __shared__ uint32_t lut[kLutSize];
    __shared__ double logm[8];
    for (int t = threadIdx.x; t < kLutSize; t += blockDim.x) lut[t] = lattice_move((uint32_t)t);
    if (threadIdx.x < 8) logm[threadIdx.x] = a.logm[threadIdx.x];
    __syncthreads();

    const uint64_t c = bid * blockDim.x + threadIdx.x;
    const bool valid = c < a.n_chains;
    const uint64_t g = a.chain_offset + c;
    const int N = a.n_monomers;

    uint32_t pos[NMAX];
    static_for<0, NMAX>([&](auto J) { pos[J.value] = kOrigin; });
    uint32_t tip = kOrigin;
    bool alive = false;
    int grown = 1;
    uint32_t cntp = 0;
    uint64_t wx = 1;
    bool rng_fail = false;
    Philox4 blk{0, 0, 0, 0};
    // outputs of the attempt that ends the chain: the first complete one, or
    // the last allowed one (one attempt without restarts)
    double res_lw = -__builtin_huge_val();
    uint64_t res_wx = 0;
    int64_t res_nn = 0;
    int32_t res_ex = 0, res_ey = 0, res_ez = 0;
    int res_grown = 1;
    bool res_alive = false;
    bool pending = valid;

    for (uint32_t rd = 0; rd < a.max_rounds; ++rd) {
        if (rd > 0) {
            static_for<0, NMAX>([&](auto J) { pos[J.value] = pending ? kOrigin : pos[J.value]; });
            tip = pending ? kOrigin : tip;
            cntp = pending ? 0u : cntp;
            wx = pending ? 1ull : wx;
        }
        alive = pending;
        grown = 1;
        const uint32_t hi = rd << 16; // attempt in the high half of the step word

        static_for<1, NMAX>([&](auto I) {
            constexpr int i = I.value;
            if (i >= N) return;
            // occupied-neighbour mask from the same-parity monomers, accumulated
            // in two independent registers to halve the dependency chain
            const uint32_t tref = tip & 0xFFFFFF00u;
            const uint32_t tq = tip - 3u;
            uint32_t occ = 0, occ2 = 0;
            static_for<0, i / 2>([&](auto Q) {
                constexpr int j = i - 2 - 2 * Q.value;
                const uint32_t L = __builtin_amdgcn_msad_u8(pos[j], tref, 0u);
                const uint32_t bit = __builtin_elementwise_sub_sat(2u, L);
                if constexpr (Q.value & 1) occ2 = (bit << ((pos[j] - tq) & 31u)) | occ2;
                else occ = (bit << ((pos[j] - tq) & 31u)) | occ;
            });
            occ |= occ2;
            const uint32_t freem = ~occ & 0x77u;
            const uint32_t m = __builtin_popcount(freem);

            // 16-bit selection word: half i mod 8 of one Philox block per 8 steps
            if constexpr (i == 1 || (i & 7) == 0)
                blk = draw(a.seed, g, (uint32_t)(i >> 3) | hi, kSlotSelect, 0);
            constexpr int h = i & 7;
            const uint32_t wd = (h >> 1) == 0 ? blk.x0 : ((h >> 1) == 1 ? blk.x1 : ((h >> 1) == 2 ? blk.x2 : blk.x3));
            const uint32_t x = (h & 1) ? (wd >> 16) : (wd & 0xFFFFu);
            const uint32_t p = x * m;
            uint32_t r = p >> 16;
            if (__builtin_expect(alive && (p & 0xFFFFu) < m, 0)) {
                r = lemire_redraw16(a.seed, g, (uint32_t)i | hi, m, x);
                if (r == kPickFailed) {
                    rng_fail = true;
                    r = 0;
                }
            }

            const bool step_ok = alive && m != 0;
            const uint32_t mv = lut[(freem << 3) | (r & 7u)];
            const uint32_t nxt = ((tip & 0xFFFFFF00u) + (mv & 0xFFFFFF00u)) | ((tip + mv) & 0xFFu);
            if (alive && m == 0) {
                alive = false;
                grown = i;
            }
            tip = step_ok ? nxt : tip;
            pos[i] = tip;
            if (step_ok) {
                // n_m field at bit 6 (m - 2) mod 32: m = 2..5 at 0, 6, 12, 18, m = 1
                // at 26 (unused); step 1 always has m = 6 and is not counted
                if constexpr (i >= 2) cntp += 1u << ((6u * m + 20u) & 31u);
                if (EXACT) wx = wx * (uint64_t)m;
            }
        });
        if (alive) grown = N;
        const bool ends = pending && (alive || rd + 1 >= a.max_rounds);
        if (ends) {
            // log W = sum over m = 1..6, ascending, of n_m log m (one rounding
            // each); n_1 log 1 = 0 and m_1 = 6 always
            double lw = 0.0;
            if (N >= 2) {
                lw = lw + (double)(cntp & 63u) * logm[2];
                lw = lw + (double)((cntp >> 6) & 63u) * logm[3];
                lw = lw + (double)((cntp >> 12) & 63u) * logm[4];
                lw = lw + (double)((cntp >> 18) & 63u) * logm[5];
                lw = lw + logm[6];
            }
            // observables over the g placed monomers, from the biased coordinate bytes
            uint32_t sx = 0, sy = 0, sz = 0, s2 = 0;
            static_for<0, NMAX>([&](auto J) {
                constexpr int j = J.value;
                const uint32_t w = j < grown ? (pos[j] & 0xFFFFFF00u) : 0u;
                sx = __builtin_amdgcn_udot4(w, 0x00000100u, sx, false);
                sy = __builtin_amdgcn_udot4(w, 0x00010000u, sy, false);
                sz = __builtin_amdgcn_udot4(w, 0x01000000u, sz, false);
                s2 = __builtin_amdgcn_udot4(w, w, s2, false);
            });
            const int64_t gg = grown;
            const int64_t Sx = (int64_t)sx - 128 * gg, Sy = (int64_t)sy - 128 * gg, Sz = (int64_t)sz - 128 * gg;
            const int64_t S2 = (int64_t)s2 - 256 * ((int64_t)sx + (int64_t)sy + (int64_t)sz) + 3 * 16384 * gg;
            res_nn = gg * S2 - (Sx * Sx + Sy * Sy + Sz * Sz);
            res_ex = (int32_t)((tip >> 8) & 0xFFu) - 128;
            res_ey = (int32_t)((tip >> 16) & 0xFFu) - 128;
            res_ez = (int32_t)(tip >> 24) - 128;
            res_lw = alive ? lw : -__builtin_huge_val();
            res_wx = alive ? wx : 0ull;
            res_grown = grown;
            res_alive = alive;
            pending = false;
        }
        if (__ballot(pending) == 0) break;
    }

    if (valid) {
        if (a.log_w) a.log_w[c] = res_lw;
        if (EXACT && a.w_exact) a.w_exact[c] = res_wx;
        if (a.r_end) {
            CT *re = (CT *)a.r_end;
            re[c] = (CT)res_ex;
            re[a.n_chains + c] = (CT)res_ey;
            re[2 * a.n_chains + c] = (CT)res_ez;
        }
        if (a.r2) a.r2[c] = (double)(res_ex * res_ex + res_ey * res_ey + res_ez * res_ez);
        if (a.n2rg2) a.n2rg2[c] = res_nn;
        if (a.rg2) a.rg2[c] = (double)res_nn / ((double)res_grown * (double)res_grown);
        if (a.n_grown) a.n_grown[c] = (uint16_t)res_grown;
    }
    if (rng_fail) atomicExch(a.status, 6);
    const uint64_t bits = res_alive ? (uint64_t)__double_as_longlong(res_lw) : 0ull;
    const uint64_t wmax = wave_max_u64(bits);
    if ((threadIdx.x & 63) == 0 && wmax != 0) atomicMax(a.log_w_max_bits, (unsigned long long)wmax);
}

template <int NMAX, bool EXACT, typename CT>
__global__ __launch_bounds__(256) void grow_lattice_reg(GrowArgs a, uint64_t base)
{
    grow_lattice_reg_body<NMAX, EXACT, CT>(a, base + blockIdx.x);
}

// Batched launch: block b serves the ensemble whose block range holds b.
template <int NMAX, bool EXACT, typename CT>
__global__ __launch_bounds__(256) void grow_lattice_reg_batch(const GrowEntry *tab, const uint64_t *block0, int n,
                                                              uint64_t base)
{
    const uint64_t bid = base + blockIdx.x;
    const int e = find_segment(block0, n, bid);
    grow_lattice_reg_body<NMAX, EXACT, CT>(tab[e].a, bid - block0[e]);
}

template <int NMAX, bool EXACT, typename CT>
static hipError_t launch(const GrowArgs &a, hipStream_t s)
{
    const uint64_t blocks = (a.n_chains + 255) / 256;
    return launch_sliced(blocks, 256, [&](uint64_t b0, uint32_t nb) {
        hipLaunchKernelGGL((grow_lattice_reg<NMAX, EXACT, CT>), dim3(nb), dim3(256), 0, s, a, b0);
    });
}

// Dispatch on the N bucket, exact-weight flag and output coordinate type.
hipError_t launch_grow_lattice_lds(const GrowArgs &a, bool i16, hipStream_t s);

hipError_t launch_grow_lattice(const GrowArgs &a, bool exact, bool i16, hipStream_t s)
{
    const int N = a.n_monomers;
    if (!exact && N > 64) return launch_grow_lattice_lds(a, i16, s);
    if (exact) {
        // RSAW_EXACT_W is limited to N <= 28 by the caller
        if (N <= 16) return i16 ? launch<16, true, int16_t>(a, s) : launch<16, true, int32_t>(a, s);
        return i16 ? launch<32, true, int16_t>(a, s) : launch<32, true, int32_t>(a, s);
    }
    if (N <= 16) return i16 ? launch<16, false, int16_t>(a, s) : launch<16, false, int32_t>(a, s);
    if (N <= 32) return i16 ? launch<32, false, int16_t>(a, s) : launch<32, false, int32_t>(a, s);
    return i16 ? launch<64, false, int16_t>(a, s) : launch<64, false, int32_t>(a, s);
}

// Variant of the register kernel for one ensemble (N <= 64, or exact weights).
void lattice_reg_variant(const GrowArgs &a, bool exact, bool i16, GrowVariant *v)
{
    const int N = a.n_monomers;
    v->family = 0;
    v->p0 = exact ? (N <= 16 ? 16 : 32) : (N <= 16 ? 16 : (N <= 32 ? 32 : 64));
    v->p1 = exact ? 1 : 0;
    v->p2 = i16 ? 1 : 0;
    v->threads = 256;
    v->cpb = 256;
    v->shmem = 0;
    v->H = 0;
    v->S = 0;
}

template <int NMAX, bool EXACT, typename CT>
static hipError_t launch_batch(const GrowEntry *tab, const uint64_t *block0, int n, uint64_t blocks,
                               hipStream_t s)
{
    return launch_sliced(blocks, 256, [&](uint64_t b0, uint32_t nb) {
        hipLaunchKernelGGL((grow_lattice_reg_batch<NMAX, EXACT, CT>), dim3(nb), dim3(256), 0, s, tab, block0, n,
                           b0);
    });
}

hipError_t launch_lattice_reg_batch(const GrowVariant &v, const GrowEntry *tab, const uint64_t *block0,
                                    int n, uint64_t blocks, hipStream_t s)
{
    const bool i16 = v.p2 != 0;
    if (v.p1) {
        if (v.p0 == 16) return i16 ? launch_batch<16, true, int16_t>(tab, block0, n, blocks, s)
                                   : launch_batch<16, true, int32_t>(tab, block0, n, blocks, s);
        return i16 ? launch_batch<32, true, int16_t>(tab, block0, n, blocks, s)
                   : launch_batch<32, true, int32_t>(tab, block0, n, blocks, s);
    }
    if (v.p0 == 16) return i16 ? launch_batch<16, false, int16_t>(tab, block0, n, blocks, s)
                               : launch_batch<16, false, int32_t>(tab, block0, n, blocks, s);
    if (v.p0 == 32) return i16 ? launch_batch<32, false, int16_t>(tab, block0, n, blocks, s)
                               : launch_batch<32, false, int32_t>(tab, block0, n, blocks, s);
    return i16 ? launch_batch<64, false, int16_t>(tab, block0, n, blocks, s)
               : launch_batch<64, false, int32_t>(tab, block0, n, blocks, s);
}

} // namespace rsaw
