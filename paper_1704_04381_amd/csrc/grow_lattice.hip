// Lattice chain growth on the simple cubic lattice (Sec. 3.3.2, Algorithm 1;
// weight of Eq. 3), one chain per lane, chain state in VGPRs.
//
// Monomer word (one 32-bit VGPR per monomer, fully unrolled over NMAX):
//   byte 0 : 128 + (Q mod 32), Q = x + 2y + 3z; bit 7 is a guard so that a
//            move (dQ in -3..3) never borrows from or carries into byte 1
//   byte 1 : x + 128,  byte 2 : y + 128,  byte 3 : z + 128
// Coordinates of an N <= 64 chain stay in [-63, 63], so bytes 1..3 never
// wrap and never become zero.
//
// Pair test of step i (tip t = monomer i-1), for each earlier monomer j of the
// parity that can touch the tip's neighbours (the cubic lattice is bipartite;
// j = i-2 is the bonded predecessor, whose direction is known, so the tests
// run over j = i-4, i-6, ...):
//   L    = v_msad_u8(r_j, t & ~0xFF)   L1 distance; byte 0 is masked because
//                                      the reference byte is zero
//   bit  = sat(2 - L)                  1 iff r_j is a neighbour of t
//   code = (Q_j - Q_t + 5) mod 32      = 2 + {0,1,2,4,5,6}: -z, -y, -x, +x, +y, +z
//   occ |= bit << code                 v_lshl_or_b32
// Four VALU operations per pair, no memory access.  The neighbour codes are
// the candidates' canonical order, so free = ~occ & (0x77 << 2) is the
// ordered candidate mask, and the move to the r-th free candidate is entry
// 5 mask + r of a 2.4 KiB LDS table (the odd stride spreads the common
// masks, one or two neighbours occupied, over the LDS banks).  That table read
// is the only memory access of a step.
//
// log W = sum over m of n_m log m (Eq. 3 grouped by value): the counts of
// m = 2..5 are kept as 6-bit fields of one register (2 operations per step),
// m_1 = 6 always, and the sum is formed once after the last step.
//
// A dead end needs no branch: the alive mask becomes 0, so every later step
// sees m = 0 and the tip stays put; log W is set to -inf at the end.
#include "rsaw_device.hpp"

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

constexpr uint32_t kOrigin = 0x80808080u;
constexpr uint32_t kCand = 0x77u << 2; // candidate bits 2..8 (bit 5 never set)
constexpr int kLutStride = 5;           // LUT entry of (mask, r) is 5 mask + r

// LUT[5 mask + r]: the move to the r-th free candidate of the 7-bit mask, as
// the signed 32-bit increment of the monomer word (coordinate byte +-1 and dQ
// in byte 0).  Entry 0 (no free candidate) is the null move.  Entries whose
// r exceeds the mask's popcount overlap the next mask and are never read.
__device__ __forceinline__ uint32_t lattice_move(uint32_t mask, uint32_t r)
{
    uint32_t seen = 0;
    for (uint32_t c = 0; c < 7; ++c) {
        if (c == 3 || !((mask >> c) & 1u)) continue;
        if (seen == r) {
            const int dq = (int)c - 3;
            const int axis = dq < 0 ? -dq : dq; // 1 = x, 2 = y, 3 = z
            const int32_t dcoord = (dq < 0 ? -1 : 1) * (int32_t)(1u << (8 * axis));
            return (uint32_t)(dcoord + dq);
        }
        ++seen;
    }
    return 0;
}

constexpr int kLutSize = kLutStride * 0x77 + 6; // largest mask, r <= 5

// (w & 0xFFFFFF9F) | 0x80: renormalise byte 0 to 128 + (Q mod 32).  Written as
// one opaque VALU instruction so that the compiler keeps a single register
// per monomer instead of also tracking the unnormalised sum (which only the
// byte-masked L1 distance could use).
__device__ __forceinline__ uint32_t renorm(uint32_t w)
{
    uint32_t out;
    asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(out) : "v"(w), "s"(0xFFFFFF9Fu), "v"(0x80u));
    return out;
}

template <int NMAX, bool EXACT, typename CT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void grow_lattice_reg(GrowArgs a)
{
    __shared__ uint32_t lut[kLutSize];
    __shared__ double logm[8];
    // entry 5 mask + r for every valid (mask, r < popcount(mask)); these never
    // overlap, since r <= 4 except for the full mask 0x77 (the entry past it,
    // mask 0x78, has bit 3 set and is never indexed)
    for (uint32_t t = threadIdx.x; t < 120u * 6u; t += blockDim.x) {
        const uint32_t mask = t / 6u, r = t % 6u;
        const uint32_t pc = __builtin_popcount(mask);
        if (!(mask & 8u) && r < (pc ? pc : 1u)) lut[kLutStride * mask + r] = lattice_move(mask, r);
    }
    if (threadIdx.x < 8) logm[threadIdx.x] = a.logm[threadIdx.x];
    __syncthreads();

    const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = c < a.n_chains;
    const uint64_t g = a.chain_offset + c;
    const int N = a.n_monomers;

    uint32_t pos[NMAX]; // slots >= N are never read
    pos[0] = kOrigin;
    uint32_t amask = valid ? kCand : 0u; // kCand while alive, 0 after a dead end
    uint32_t cnt = 0;                    // sum of amask over steps = kCand * (placed - 1)
    uint32_t cntp = 0;                   // n_2..n_5 at bits 0, 6, 12, 18 (n_1 at 26)
    uint64_t wx = 1;
    bool rng_fail = false;
    Philox4 blk{0, 0, 0, 0};

    static_for<1, NMAX>([&](auto I) {
        constexpr int i = I.value;
        if (i >= N) return;
        const uint32_t tip = pos[i - 1];
        const uint32_t tref = tip & 0xFFFFFF00u;
        const uint32_t tq = tip - 5u;
        uint32_t occ = 0;
        if constexpr (i >= 2) occ = 1u << ((pos[i - 2] - tq) & 31u); // bonded predecessor
        static_for<0, (i >= 4 ? i / 2 - 1 : 0)>([&](auto Q) {
            constexpr int j = i - 4 - 2 * Q.value;
            const uint32_t L = __builtin_amdgcn_msad_u8(pos[j], tref, 0u);
            const uint32_t bit = __builtin_elementwise_sub_sat(2u, L);
            occ = (bit << ((pos[j] - tq) & 31u)) | occ;
        });
        const uint32_t freem = amask & ~occ;
        const uint32_t m = __builtin_popcount(freem);

        // 16-bit selection word: half i mod 8 of one Philox block per 8 steps
        if constexpr (i == 1 || (i & 7) == 0) blk = draw(a.seed, g, (uint32_t)(i >> 3), kSlotSelect, 0);
        constexpr int h = i & 7;
        const uint32_t wd = (h >> 1) == 0 ? blk.x0 : ((h >> 1) == 1 ? blk.x1 : ((h >> 1) == 2 ? blk.x2 : blk.x3));
        const uint32_t x = (h & 1) ? (wd >> 16) : (wd & 0xFFFFu);
        const uint32_t p = x * m; // < 2^19
        uint32_t r = p >> 16;
        if (__builtin_expect((p & 0xFFFFu) < m, 0)) // superset of Lemire's rejection
            r = lemire_redraw16(a.seed, g, (uint32_t)i, m, x, &rng_fail);

        // byte address of LUT[5 mask + r] is 5 freem + 4 r (freem = mask << 2)
        const uint32_t mv = *(const uint32_t *)((const char *)lut + (freem * kLutStride + (r << 2)));
        pos[i] = renorm(tip + mv);
        // field of m: bit 6 (m - 2) mod 32 (m = 1 lands at 26; m = 0 only
        // after a dead end, where log W is -inf anyway); step 1 has m = 6
        if constexpr (i >= 2) cntp += 1u << ((6u * m + 20u) & 31u);
        if constexpr (EXACT) wx = wx * (uint64_t)m;
        amask = m != 0 ? amask : 0u;
        cnt += amask;
    });

    const bool alive = amask != 0;
    // log W = sum over m = 1..6, ascending, of n_m log m, one rounding each
    double lw = 0.0;
    if (N >= 2) {
        lw = lw + (double)(cntp & 63u) * logm[2];
        lw = lw + (double)((cntp >> 6) & 63u) * logm[3];
        lw = lw + (double)((cntp >> 12) & 63u) * logm[4];
        lw = lw + (double)((cntp >> 18) & 63u) * logm[5];
        lw = lw + logm[6];
    }
    if (!alive) lw = -__builtin_huge_val();
    const int grown = N < 2 ? 1 : 1 + (int)(cnt / kCand);

    // observables over monomers 0..N-1; a dead chain's frozen tip repeats in
    // slots grown..N-1 and is subtracted again below
    uint32_t sx = 0, sy = 0, sz = 0, s2 = 0, last = kOrigin;
    static_for<0, NMAX>([&](auto J) {
        constexpr int j = J.value;
        if (j < N) {
            const uint32_t w = pos[j];
            const uint32_t wc = w & 0xFFFFFF00u;
            sx = __builtin_amdgcn_udot4(w, 0x00000100u, sx, false);
            sy = __builtin_amdgcn_udot4(w, 0x00010000u, sy, false);
            sz = __builtin_amdgcn_udot4(w, 0x01000000u, sz, false);
            s2 = __builtin_amdgcn_udot4(wc, wc, s2, false);
            last = w;
        }
    });
    const int64_t gg = grown;
    const int64_t extra = (int64_t)N - gg; // copies of the frozen tip
    const int64_t bx = (int64_t)((last >> 8) & 0xFFu), by = (int64_t)((last >> 16) & 0xFFu),
                  bz = (int64_t)(last >> 24);
    const int64_t ux = (int64_t)sx - extra * bx, uy = (int64_t)sy - extra * by, uz = (int64_t)sz - extra * bz;
    const int64_t u2 = (int64_t)s2 - extra * (bx * bx + by * by + bz * bz);
    const int64_t Sx = ux - 128 * gg, Sy = uy - 128 * gg, Sz = uz - 128 * gg;
    const int64_t S2 = u2 - 256 * (ux + uy + uz) + 3 * 16384 * gg;
    const int64_t nn = gg * S2 - (Sx * Sx + Sy * Sy + Sz * Sz);
    const int32_t ex = (int32_t)bx - 128, ey = (int32_t)by - 128, ez = (int32_t)bz - 128;

    if (valid) {
        if (a.log_w) a.log_w[c] = lw;
        if (EXACT && a.w_exact) a.w_exact[c] = alive ? wx : 0ull;
        if (a.r_end) {
            CT *re = (CT *)a.r_end;
            re[c] = (CT)ex;
            re[a.n_chains + c] = (CT)ey;
            re[2 * a.n_chains + c] = (CT)ez;
        }
        if (a.r2) a.r2[c] = (double)(ex * ex + ey * ey + ez * ez);
        if (a.n2rg2) a.n2rg2[c] = nn;
        if (a.rg2) a.rg2[c] = (double)nn / ((double)gg * (double)gg);
        if (a.n_grown) a.n_grown[c] = (uint16_t)grown;
    }
    if (rng_fail) atomicExch(a.status, 6);
    const uint64_t bits = alive ? (uint64_t)__double_as_longlong(lw) : 0ull;
    const uint64_t wmax = wave_max_u64(bits);
    if ((threadIdx.x & 63) == 0 && wmax != 0) atomicMax(a.log_w_max_bits, (unsigned long long)wmax);
}

template <int NMAX, bool EXACT, typename CT>
static hipError_t launch(const GrowArgs &a, hipStream_t s)
{
    const uint64_t blocks = (a.n_chains + 255) / 256;
    hipLaunchKernelGGL((grow_lattice_reg<NMAX, EXACT, CT>), dim3((uint32_t)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

// Dispatch on the N bucket, exact-weight flag and output coordinate type.
hipError_t launch_grow_lattice(const GrowArgs &a, bool exact, bool i16, hipStream_t s)
{
    const int N = a.n_monomers;
    if (exact) {
        // RSAW_EXACT_W is limited to N <= 28 by the caller
        if (N <= 16) return i16 ? launch<16, true, int16_t>(a, s) : launch<16, true, int32_t>(a, s);
        return i16 ? launch<32, true, int16_t>(a, s) : launch<32, true, int32_t>(a, s);
    }
    if (N <= 16) return i16 ? launch<16, false, int16_t>(a, s) : launch<16, false, int32_t>(a, s);
    if (N <= 32) return i16 ? launch<32, false, int16_t>(a, s) : launch<32, false, int32_t>(a, s);
    return i16 ? launch<64, false, int16_t>(a, s) : launch<64, false, int32_t>(a, s);
}

} // namespace rsaw
