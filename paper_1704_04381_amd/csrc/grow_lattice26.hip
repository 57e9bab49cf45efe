// 26-neighbour lattice variant (the "z = 26 possible lattice space" of Sec.
// 3.3.2): the candidates of a step are all 26 sites within Chebyshev
// distance 1 of the tip, numbered by the code (dx + 1) + 3 (dy + 1) +
// 9 (dz + 1) (13, the tip itself, excluded); the growth rule and weight are
// those of Algorithm 1 and Eq. 3 with m_i <= 26.
//
// Chains beyond N = 64: G lanes per chain (4 to 64, by N), the history in
// monomer order (no bipartite pruning on this lattice: a diagonal step
// keeps the parity).  Up to N = 640 one byte word per monomer and up to
// N = 4096 one packed word, each with a box and a regrowth of the chains
// that leave it (both described further down), held in the group's
// registers where its lanes' 64 slots hold the chain (N <= 64 G), else in
// LDS; beyond, and for the regrowth, two words per monomer ("wide") in LDS,
// A = (x + 2^15) | (y + 2^15) << 16 and B = z + 2^15, in two planes of H
// words.  Entries not yet placed hold A = 0 (x = y = -2^15, far from every
// tip) and B = 2^15.
// Wide pair test of monomer j against tip t:
//   (dx, dy) as packed 16-bit differences of the A words, dz = B_j - B_t
//   q  = dx^2 + dy^2 + dz^2          (dot2 onto a 24-bit product)
//   s  = |dx| + |dy| + |dz|          (two chained sad_u16 operations)
//   the site is a candidate iff max(|dx|, |dy|, |dz|) <= 1, i.e. iff q = s
//   (d^2 = |d| for |d| <= 1, d^2 >= |d| + 2 otherwise), so
//   bit = sat((s + 1) - q) and code = dx + 3 dy + 9 dz + 13 (dot2 onto a
//   24-bit multiply-add);  occ |= bit << code
// ten operations per pair.  The G partial masks are OR-reduced across the
// group; every lane then picks the same r-th free code (Lemire on the same
// 16-bit words as the six-neighbour lattice; the code by a binary search
// over the free mask in this LDS kernel, from the byte-rank table in the
// register kernel further down; the move computed from the code), and
// lane (m - 1) mod G counts the steps with m free candidates for log W.
// Short chains (N <= 64) use the one-lane-per-chain kernel further down.
#include "rsaw_device.hpp"

namespace rsaw {

__device__ __forceinline__ void z26_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int G>
__device__ __forceinline__ uint32_t z26_group_or(uint32_t v)
{
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);
    if constexpr (G >= 4) v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);
    if constexpr (G >= 8) v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);
    if constexpr (G >= 16) v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false);
    if constexpr (G >= 32) {
        const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        v = p[0] | p[1];
    }
    if constexpr (G >= 64) {
        const auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        v = p[0] | p[1];
    }
    return v;
}

typedef short short2_t __attribute__((ext_vector_type(2)));

constexpr uint32_t kZ26OriginA = 0x80008000u; // x = y = 0
constexpr uint32_t kZ26OriginB = 0x00008000u; // z = 0 (also the B sentinel)
constexpr uint32_t kZ26Codes = 0x7FFFFFFu & ~(1u << 13);

__device__ __forceinline__ uint32_t z26_bits(uint32_t wa, uint32_t wb, uint32_t ta, uint32_t tb)
{
    // (dx, dy) as 16-bit wrapping differences: exact for placed monomers
    // (|d| < 2^15), at least 2^14 + 1 in |dx| against the zero A sentinel;
    // dz exact (both B words are below 2^16, the sentinel's z is 0).  Hence
    // q < 2^32 without wrap, and q < s + 1 only for true neighbours.
    const short2_t dA = __builtin_bit_cast(short2_t, wa) - __builtin_bit_cast(short2_t, ta);
    const int dz = (int)(wb - tb);
    const short2_t w13 = {1, 3};
    const uint32_t q = (uint32_t)__builtin_amdgcn_sdot2(dA, dA, __mul24(dz, dz), false);
    const uint32_t s1 = __builtin_amdgcn_sad_u16(wa, ta, __builtin_amdgcn_sad_u16(wb, tb, 1u));
    const int code = __builtin_amdgcn_sdot2(dA, w13, __mul24(dz, 9) + 13, false);
    const uint32_t bit = __builtin_elementwise_sub_sat(s1, q);
    return bit << ((uint32_t)code & 31u);
}

// Index of the r-th (from 0) set bit of f, r < popcount(f) <= 27: the byte
// holding it from three prefix counts, then sel[byte][k], the index of the
// k-th set bit of a byte value (a 2 KB table in LDS).
__device__ __forceinline__ uint32_t z26_select(uint32_t f, uint32_t r, const uint8_t *sel)
{
    const uint32_t c0 = __builtin_popcount(f & 0xFFu);
    const uint32_t c1 = __builtin_popcount(f & 0xFFFFu);
    const uint32_t c2 = __builtin_popcount(f & 0xFFFFFFu);
    uint32_t k = 0, before = 0;
    if (r >= c0) { k = 8; before = c0; }
    if (r >= c1) { k = 16; before = c1; }
    if (r >= c2) { k = 24; before = c2; }
    const uint32_t byte = (f >> k) & 0xFFu;
    return k + sel[byte * 8 + (r - before)];
}

// Index of the r-th (from 0) set bit of f, r < popcount(f): a binary search
// over halves of the remaining word, in registers.
__device__ __forceinline__ uint32_t z26_select_bits(uint32_t f, uint32_t r)
{
    uint32_t pos = 0;
#pragma unroll
    for (int w = 16; w >= 1; w >>= 1) {
        const uint32_t c = __builtin_popcount(f & ((1u << w) - 1u));
        const bool up = r >= c;
        r = up ? r - c : r;
        f = up ? f >> w : f;
        pos = up ? pos + (uint32_t)w : pos;
    }
    return pos;
}

// A- and B-word moves of code c = (dx + 1) + 3 (dy + 1) + 9 (dz + 1), c < 27.
__device__ __forceinline__ void z26_move(uint32_t code, uint32_t &da, uint32_t &db)
{
    const uint32_t z = (code * 57u) >> 9;         // code / 9
    const uint32_t rem = code - 9u * z;
    const uint32_t y = (rem * 11u) >> 5;          // rem / 3
    const uint32_t x = rem - 3u * y;
    da = (x - 1u) + ((y - 1u) << 16);
    db = z - 1u;
}

__device__ __forceinline__ void z26_fill_select_table(uint8_t *sel)
{
    for (int q = threadIdx.x; q < 2048; q += blockDim.x) {
        const uint32_t byte = (uint32_t)q >> 3, k = (uint32_t)q & 7u;
        uint32_t b = byte;
        for (uint32_t j = 0; j < k && b; ++j) b &= b - 1u;
        sel[q] = (uint8_t)(b ? __builtin_ctz(b) : 0);
    }
}

// Byte words of the group kernel (N <= 640): one word per monomer, bytes
// (x + 64, y + 64, z + 64) plus 128 each, the pair test of the one-lane
// kernel (z26_bits8, six operations) against the tip's raw word.  The test
// needs every tip coordinate within [-62, 63] (at least 2 from the sentinel
// at -64) and every stored one within [-64, 63]; a chain whose new tip
// reaches |coordinate| = E (62, or the launch's byte_box if smaller) stops,
// writes nothing and is grown again, from its first draw, in wide words by
// the same block once its other chains are done (the same draws and tests
// give the same chain, Sec. 3.3.2).
constexpr int kZ26ByteMaxN = 640;
constexpr int kZ26ByteEdge = 62;
constexpr int kZ26ListWords = 65; // count + one slot per chain of a block (<= 64)
constexpr uint32_t kZ26Bias = 0x00808080u;
constexpr uint32_t kZ26LaneOrigin = 0x00404040u; // raw (64, 64, 64): the origin

// Pair test of a stored byte word w (raw bytes + 128) against
// tp = tip + 0x7F7F7F (raw tip bytes + 127), for tips at least 2 from the
// sentinel: v = w - tp has bytes d + 1 for d = raw_w - raw_tip when every
// |d| <= 1 (no byte borrows); a byte with d <= -2 borrows and is left at
// 0x80 or above, a byte with d >= 2 is left at 3 or above.  So the site is a
// candidate iff every byte of v and of v + 0x010101 stays below 4, and its
// code (dx + 1) + 3 (dy + 1) + 9 (dz + 1) is dot4(v, (1, 3, 9, 0)).
__device__ __forceinline__ uint32_t z26_bits8(uint32_t w, uint32_t tp)
{
    const uint32_t v = w - tp;
    const uint32_t bad = (v | (v + 0x010101u)) & 0x00FCFCFCu;
    const uint32_t code = __builtin_amdgcn_udot4(v, 0x00090301u, 0u, false);
    return __builtin_elementwise_sub_sat(1u, bad) << (code & 31u);
}

// Bytes (dx + 1, dy + 1, dz + 1) of code c = (dx + 1) + 3 (dy + 1) + 9 (dz + 1).
__device__ __forceinline__ uint32_t z26_move_bytes(uint32_t code)
{
    const uint32_t z = (code * 57u) >> 9; // code / 9
    const uint32_t rem = code - 9u * z;
    const uint32_t y = (rem * 11u) >> 5; // rem / 3
    return (rem - 3u * y) | (y << 8) | (z << 16);
}

// Packed words of the group kernel (640 < N <= 4096): one word per
// monomer, x + 1024 in bits 0-10, y + 1024 in bits 11-21, z + 512 in bits
// 22-31.  The byte test carries over field by field: with
// tp = tip - (1, 1, 1), v = w - tp has fields d + 1 when every |d| <= 1; a
// field with d <= -2 borrows and, for |d| <= 2^(width - 1) - 2, is left at
// 2^(width - 1) + 2 or above, one with d >= 2 at 3 or above.  Tips stay
// within |coordinate| <= 253 (a box like the byte words'), stored monomers
// within 254, the sentinel (-512, -512, -256) is at least 3 away, so every
// difference meets that bound.  The code (dx + 1) + 3 (dy + 1) + 9 (dz + 1)
// of a candidate is bits 22-26 of v * (2^22 + 3 * 2^11 + 9) (24-bit
// multiply; the lower products stay below 2^22).  Seven operations.
constexpr int kZ26PackedMaxN = 4096;
constexpr int kZ26PackedEdge = 254;
constexpr uint32_t kP32One = 1u | (1u << 11) | (1u << 22);
constexpr uint32_t kP32Origin = 1024u | (1024u << 11) | (512u << 22);
constexpr uint32_t kP32Sentinel = 512u | (512u << 11) | (256u << 22);
constexpr uint32_t kP32High = 0x7FCu | (0x7FCu << 11) | (0x3FCu << 22); // field bits above 1
constexpr uint32_t kP32Code = (1u << 22) + (3u << 11) + 9u;

__device__ __forceinline__ uint32_t z26_bits32(uint32_t w, uint32_t tp)
{
    const uint32_t v = w - tp;
    const uint32_t bad = (v | (v + kP32One)) & kP32High;
    const uint32_t code = __umul24(v, kP32Code) >> 22;
    return __builtin_elementwise_sub_sat(1u, bad) << (code & 31u);
}

// Fields (dx + 1, dy + 1, dz + 1) of code c in the packed layout.
__device__ __forceinline__ uint32_t z26_move_packed(uint32_t code)
{
    const uint32_t z = (code * 57u) >> 9; // code / 9
    const uint32_t rem = code - 9u * z;
    const uint32_t y = (rem * 11u) >> 5; // rem / 3
    return (rem - 3u * y) | (y << 11) | (z << 22);
}

// Lanes per chain and plane length of the wide regrowth.
__host__ __device__ __forceinline__ int z26_regrow_lanes(int N) { return N <= 512 ? 8 : 32; }
__host__ __device__ __forceinline__ int z26_regrow_plane(int N)
{
    const int q = 4 * z26_regrow_lanes(N);
    return (N + q - 1) / q * q;
}

// Word formats of the group kernel.
constexpr int kZ26Wide = 0, kZ26Byte = 1, kZ26Packed = 2;

// Grows chain c of this thread's group of G lanes, its history at PA (wide
// words: planes PA and PA + H; byte or packed words: one plane of H words),
// and writes its outputs.  With box > 0 (byte and packed words) a chain
// whose tip reaches |coordinate| = box stops, writes nothing and contributes
// nothing to the side channels; the function then returns true on the
// group's lanes.
template <int G, bool EXACT, typename CT, int FMT>
__device__ __forceinline__ bool z26_grow(const GrowArgs &a, const double *logm, uint32_t *PA, int H, uint64_t c,
                                         bool valid, int box)
{
    const int t = threadIdx.x & (G - 1);
    const int lane = threadIdx.x & 63;
    const int gbase = lane & ~(G - 1);
    const uint64_t g = a.chain_offset + c;
    const int N = a.n_monomers;
    uint32_t *PB = PA + H;
    constexpr bool BYTE = FMT == kZ26Byte, PACKED = FMT == kZ26Packed, ONE = FMT != kZ26Wide;

    // tip: A and B words (wide), the raw byte word (byte) or the packed word
    uint32_t ta = 0, tb = 0;
    bool alive = false;
    bool left_box = false;
    int grown = 1;
    // steps with m free candidates: lane t counts the m with (m - 1) mod G
    // = t, in FW-bit fields at (m - 1) / G (one field for G >= 32; 8-bit
    // fields for G = 4, whose seven fields need N <= 256)
    constexpr uint32_t FW = G >= 8 ? 16u : 8u;
    uint64_t n_mine = 0;
    uint64_t wx = 1;
    bool rng_fail = false;
    Philox4 blk{0, 0, 0, 0};
    double res_lw = -__builtin_huge_val();
    uint64_t res_wx = 0;
    int64_t res_nn = 0;
    int32_t res_ex = 0, res_ey = 0, res_ez = 0;
    int res_grown = 1;
    bool res_alive = false;
    bool res_set = false;
    bool pending = valid;

    for (uint32_t rd = 0; rd < a.max_rounds; ++rd) {
        if (pending) {
            if (rd > 0) {
                if constexpr (ONE) {
                    for (int w = t; w < H; w += G) PA[w] = BYTE ? kZ26Bias : kP32Sentinel;
                } else {
                    for (int w = t; w < 2 * H; w += G) PA[w] = w < H ? 0u : kZ26OriginB;
                }
            }
            ta = BYTE ? kZ26LaneOrigin : (PACKED ? kP32Origin : kZ26OriginA);
            tb = ONE ? 0u : kZ26OriginB;
            n_mine = 0;
            wx = 1;
        }
        z26_wave_sync();
        if (pending && t == 0) {
            if constexpr (ONE) {
                PA[0] = BYTE ? ta + kZ26Bias : ta;
            } else {
                PA[0] = ta;
                PB[0] = tb;
            }
        }
        z26_wave_sync();
        alive = pending;
        grown = 1;
        const uint32_t hi = rd << 16;

        for (int i = 1; i < N; ++i) {
            // monomers 0 .. i-2 can occupy a candidate site (i-1 is the tip)
            const int nrel = i - 1;
            const int passes = (nrel + 4 * G - 1) / (4 * G);
            uint32_t occ = 0, occ2 = 0;
            const uint32_t tp = PACKED ? ta - kP32One : ta + 0x7F7F7Fu;
            // two passes per iteration, so that the second pass's reads are in
            // flight while the first is tested; entries at nrel and beyond hold
            // the sentinel (never a candidate) or the tip (code 13, masked)
            auto test4 = [&](const uint4 &wa, const uint4 &wb) {
                if constexpr (BYTE) {
                    occ |= z26_bits8(wa.x, tp);
                    occ2 |= z26_bits8(wa.y, tp);
                    occ |= z26_bits8(wa.z, tp);
                    occ2 |= z26_bits8(wa.w, tp);
                } else if constexpr (PACKED) {
                    occ |= z26_bits32(wa.x, tp);
                    occ2 |= z26_bits32(wa.y, tp);
                    occ |= z26_bits32(wa.z, tp);
                    occ2 |= z26_bits32(wa.w, tp);
                } else {
                    occ |= z26_bits(wa.x, wb.x, ta, tb);
                    occ2 |= z26_bits(wa.y, wb.y, ta, tb);
                    occ |= z26_bits(wa.z, wb.z, ta, tb);
                    occ2 |= z26_bits(wa.w, wb.w, ta, tb);
                }
            };
            int q = 0;
            for (; q + 1 < passes; q += 2) {
                const int k1 = q * 4 * G + 4 * t, k2 = k1 + 4 * G;
                const uint4 a1 = *(const uint4 *)(PA + k1), a2 = *(const uint4 *)(PA + k2);
                uint4 b1 = make_uint4(0u, 0u, 0u, 0u), b2 = b1;
                if constexpr (!ONE) {
                    b1 = *(const uint4 *)(PB + k1);
                    b2 = *(const uint4 *)(PB + k2);
                }
                test4(a1, b1);
                test4(a2, b2);
            }
            if (q < passes) {
                const int k1 = q * 4 * G + 4 * t;
                uint4 b1 = make_uint4(0u, 0u, 0u, 0u);
                if constexpr (!ONE) b1 = *(const uint4 *)(PB + k1);
                test4(*(const uint4 *)(PA + k1), b1);
            }
            occ = z26_group_or<G>(occ | occ2);
            const uint32_t freem = ~occ & kZ26Codes;
            const uint32_t m = __builtin_popcount(freem);

            if (i == 1 || (i & 7) == 0) blk = draw(a.seed, g, (uint32_t)(i >> 3) | hi, kSlotSelect, 0);
            const uint32_t x = half_word(blk, (uint32_t)(i & 7));
            const uint32_t p = x * m;
            uint32_t r = p >> 16;
            if (__builtin_expect(alive && (p & 0xFFFFu) < m, 0)) {
                r = lemire_redraw16_inline(a.seed, g, (uint32_t)i | hi, m, x);
                if (r == kPickFailed) {
                    rng_fail = true;
                    r = 0;
                }
            }
            const uint32_t code = m ? z26_select_bits(freem, r) : 13u; // the r-th free code

            bool step_ok = alive && m != 0;
            if (alive && m == 0) {
                alive = false;
                grown = i;
            }
            uint32_t na = ta, nb = tb;
            if constexpr (BYTE) {
                // bytes dx + 1, dy + 1, dz + 1 added, then 1 taken from each:
                // no carry or borrow for a tip inside the box
                na = ta + z26_move_bytes(code) - 0x010101u;
            } else if constexpr (PACKED) {
                na = ta + z26_move_packed(code) - kP32One; // no carry or borrow in the box
            } else {
                uint32_t da, db;
                z26_move(code, da, db);
                na = ta + da;
                nb = tb + db;
            }
            if constexpr (BYTE) {
                // |coordinate| >= E: bytes b = x + 64 with b < 65 - E or
                // 127 - b < 64 - E (byte-wise "has a byte below n", exact
                // for n <= 128), possible from step E on
                if (box > 0 && i >= box) {
                    const uint32_t v = na, w = 0x7F7F7Fu - na;
                    const uint32_t lo = (uint32_t)(65 - box) * 0x010101u, hb = (uint32_t)(64 - box) * 0x010101u;
                    const uint32_t edge = (((v - lo) & ~v) | ((w - hb) & ~w)) & 0x808080u;
                    if (step_ok && edge != 0u) {
                        step_ok = false;
                        alive = false;
                        left_box = true;
                    }
                }
            } else if constexpr (PACKED) {
                // |coordinate| >= E, possible from step E on
                if (box > 0 && i >= box) {
                    const int ex = (int)(na & 0x7FFu) - 1024, ey = (int)((na >> 11) & 0x7FFu) - 1024,
                              ez = (int)(na >> 22) - 512;
                    const uint32_t span = 2u * (uint32_t)box - 2u; // |e| < E iff e + E - 1 <= 2 E - 2
                    const bool out = (uint32_t)(ex + box - 1) > span || (uint32_t)(ey + box - 1) > span ||
                                     (uint32_t)(ez + box - 1) > span;
                    if (step_ok && out) {
                        step_ok = false;
                        alive = false;
                        left_box = true;
                    }
                }
            }
            if (step_ok) {
                ta = na;
                tb = nb;
                const uint32_t mm1 = m - 1u;
                n_mine += (mm1 & (G - 1)) == (uint32_t)t ? 1ull << (FW * (mm1 / G)) : 0ull;
                if (EXACT) wx = wx * (uint64_t)m;
                if (t == 0) {
                    if constexpr (ONE) {
                        PA[i] = BYTE ? ta + kZ26Bias : ta;
                    } else {
                        PA[i] = ta;
                        PB[i] = tb;
                    }
                }
            }
            z26_wave_sync();
        }
        if (alive) grown = N;

        // log W = sum over m = 1..26, ascending, of n_m log m; n_m is field
        // (m - 1) / G of lane (m - 1) mod G of the group
        double lw = 0.0;
#pragma unroll 1
        for (int mm = 1; mm <= 26; ++mm) {
            const int f = (mm - 1) / G;                    // field index
            const int per = 32 / (int)FW;                     // fields per 32-bit half
            const uint32_t half = (uint32_t)(n_mine >> (32 * (f / per)));
            const uint32_t v = (uint32_t)__shfl((int)half, gbase + ((mm - 1) & (G - 1)), 64);
            const uint32_t nm = (v >> (FW * (uint32_t)(f % per))) & ((1u << FW) - 1u);
            lw = lw + (double)nm * logm[mm];
        }
        // observables over the placed monomers (integer sums: any order)
        int32_t sx = 0, sy = 0, sz = 0;
        int64_t s2 = 0;
        for (int j = t; j < grown; j += G) {
            int32_t xx, yy, zz;
            if constexpr (BYTE) {
                const uint32_t w = PA[j];
                xx = (int32_t)(w & 0xFFu) - 192;
                yy = (int32_t)((w >> 8) & 0xFFu) - 192;
                zz = (int32_t)((w >> 16) & 0xFFu) - 192;
            } else if constexpr (PACKED) {
                const uint32_t w = PA[j];
                xx = (int32_t)(w & 0x7FFu) - 1024;
                yy = (int32_t)((w >> 11) & 0x7FFu) - 1024;
                zz = (int32_t)(w >> 22) - 512;
            } else {
                xx = (int32_t)(PA[j] & 0xFFFFu) - 32768;
                yy = (int32_t)(PA[j] >> 16) - 32768;
                zz = (int32_t)(PB[j] & 0xFFFFu) - 32768;
            }
            sx += xx;
            sy += yy;
            sz += zz;
            s2 += (int64_t)(xx * xx + yy * yy + zz * zz);
        }
#pragma unroll
        for (int off = 1; off < G; off <<= 1) {
            sx += __shfl_xor(sx, off, 64);
            sy += __shfl_xor(sy, off, 64);
            sz += __shfl_xor(sz, off, 64);
            const int lo = __shfl_xor((int)(uint32_t)s2, off, 64);
            const int hh = __shfl_xor((int)(uint32_t)((uint64_t)s2 >> 32), off, 64);
            s2 += (int64_t)(((uint64_t)(uint32_t)hh << 32) | (uint32_t)lo);
        }
        if (pending && left_box) {
            pending = false; // grown again in wide words
        } else if (pending && (alive || rd + 1 >= a.max_rounds)) {
            const int64_t gg = grown;
            res_nn = gg * s2 - ((int64_t)sx * sx + (int64_t)sy * sy + (int64_t)sz * sz);
            if constexpr (BYTE) {
                res_ex = (int32_t)(ta & 0xFFu) - 64;
                res_ey = (int32_t)((ta >> 8) & 0xFFu) - 64;
                res_ez = (int32_t)((ta >> 16) & 0xFFu) - 64;
            } else if constexpr (PACKED) {
                res_ex = (int32_t)(ta & 0x7FFu) - 1024;
                res_ey = (int32_t)((ta >> 11) & 0x7FFu) - 1024;
                res_ez = (int32_t)(ta >> 22) - 512;
            } else {
                res_ex = (int32_t)(ta & 0xFFFFu) - 32768;
                res_ey = (int32_t)(ta >> 16) - 32768;
                res_ez = (int32_t)(tb & 0xFFFFu) - 32768;
            }
            res_lw = alive ? lw : -__builtin_huge_val();
            res_wx = alive ? wx : 0ull;
            res_grown = grown;
            res_alive = alive;
            res_set = true;
            pending = false;
        }
        if (__ballot(pending) == 0) break;
    }

    if (res_set && t == 0) {
        if (a.log_w) a.log_w[c] = res_lw;
        if (EXACT && a.w_exact) a.w_exact[c] = res_wx;
        if (a.r_end) {
            CT *re = (CT *)a.r_end;
            re[c] = (CT)res_ex;
            re[a.n_chains + c] = (CT)res_ey;
            re[2 * a.n_chains + c] = (CT)res_ez;
        }
        if (a.r2) a.r2[c] = (double)((int64_t)res_ex * res_ex + (int64_t)res_ey * res_ey + (int64_t)res_ez * res_ez);
        if (a.n2rg2) a.n2rg2[c] = res_nn;
        if (a.rg2) a.rg2[c] = (double)res_nn / ((double)res_grown * (double)res_grown);
        if (a.n_grown) a.n_grown[c] = (uint16_t)res_grown;
    }
    if (rng_fail && !left_box) atomicExch(a.status, 6);
    const uint64_t bits = (res_alive && t == 0) ? (uint64_t)__double_as_longlong(res_lw) : 0ull;
    const uint64_t wmax = wave_max_u64(bits);
    if ((threadIdx.x & 63) == 0 && wmax != 0) atomicMax(a.log_w_max_bits, (unsigned long long)wmax);
    return left_box;
}

// Register-resident one-word formats (byte or packed words, N <= 64 G):
// entry j (monomer j) of the chain sits in lane j mod G of its group, slot
// j / G of a 64-slot array.  A step tests the slots that can hold monomers
// 0 .. i - 2, four at a time behind one wave-uniform count test, two in a
// last group with one or two slots left (4-6 % faster than whole groups;
// slots past them hold the tip, code 13, masked, or the sentinel), and
// appends the new word with one indexed register read and write (uniform
// slot; the lane that holds entry i takes it).  The r-th free code comes
// from the one-lane kernel's byte-rank table in LDS (2 KB), about 20
// operations where the binary search takes about 45 (3-4 % faster at
// N = 256 and 2048, the same with 2 lanes).  Against the same mapping with
// the words in LDS (MI355X, kernel time, bit-identical, before the last
// two changes): N = 100, 2.57 -> 2.07 ms; N = 256, 15.2 -> 8.27 ms;
// N = 640, 35.8 -> 25.8 ms; N = 2048, 49.4 -> 35.9 ms; N = 4000, 81.0 ->
// 51.0 ms.  The step loses its scan loads and their
// round trips, and the kernel runs at 3 waves per SIMD (168 VGPRs; the
// compiler spills a few values outside the step loop) where the LDS kernel
// ran at 2; unbounded it takes 192 VGPRs and runs 10-40 % slower.
constexpr int kZ26Slots = 64;

template <int G, typename CT, int FMT>
__device__ __forceinline__ bool z26_grp_grow(const GrowArgs &a, const double *logm, const uint8_t *sel, uint64_t c,
                                             bool valid, int box)
{
    constexpr int SL = kZ26Slots;
    constexpr bool BYTE = FMT == kZ26Byte;
    constexpr uint32_t SENT = BYTE ? kZ26Bias : kP32Sentinel;
    const int t = threadIdx.x & (G - 1);
    const int lane = threadIdx.x & 63;
    const int gbase = lane & ~(G - 1);
    const uint64_t g = a.chain_offset + c;
    const int N = a.n_monomers;

    // slots 0-31 and 32-63 as two arrays (each indexed append stays in
    // registers)
    uint32_t pl[SL / 2], ph[SL / 2];
#pragma unroll
    for (int s = 0; s < SL / 2; ++s) pl[s] = ph[s] = SENT;
    uint32_t ta = 0;
    bool alive = false;
    bool left_box = false;
    int grown = 1;
    // n_m counters as in the LDS kernel; with G = 2 (N <= 128) a lane's 13
    // 8-bit fields take a second word for fields 8 and up
    constexpr uint32_t FW = G >= 8 ? 16u : 8u;
    uint64_t n_mine = 0, n_mine2 = 0;
    bool rng_fail = false;
    Philox4 blk{0, 0, 0, 0};
    double res_lw = -__builtin_huge_val();
    int64_t res_nn = 0;
    int32_t res_ex = 0, res_ey = 0, res_ez = 0;
    int res_grown = 1;
    bool res_alive = false;
    bool res_set = false;
    bool pending = valid;

    for (uint32_t rd = 0; rd < a.max_rounds; ++rd) {
        if (rd > 0) {
#pragma unroll
            for (int s = 0; s < SL / 2; ++s) {
                pl[s] = pending ? SENT : pl[s];
                ph[s] = pending ? SENT : ph[s];
            }
        }
        if (pending) {
            ta = BYTE ? kZ26LaneOrigin : kP32Origin;
            n_mine = 0;
            n_mine2 = 0;
        }
        pl[0] = (pending && t == 0) ? (BYTE ? kZ26LaneOrigin + kZ26Bias : kP32Origin) : pl[0];
        alive = pending;
        grown = 1;
        const uint32_t hi = rd << 16;

        for (int i = 1; i < N; ++i) {
            const int ns = (i - 1 + G - 1) / G; // slots that can hold monomers 0 .. i - 2
            uint32_t occ = 0, occ2 = 0;
            const uint32_t tp = BYTE ? ta + 0x7F7F7Fu : ta - kP32One;
            const auto test2 = [&](uint32_t w0, uint32_t w1) {
                if constexpr (BYTE) {
                    occ |= z26_bits8(w0, tp);
                    occ2 |= z26_bits8(w1, tp);
                } else {
                    occ |= z26_bits32(w0, tp);
                    occ2 |= z26_bits32(w1, tp);
                }
            };
            const auto word = [&](int sl) { return sl < SL / 2 ? pl[sl] : ph[sl - SL / 2]; };
#pragma unroll
            for (int q = 0; q < SL / 4; ++q) {
                if (4 * q >= ns) break;
                test2(word(4 * q), word(4 * q + 1));
                if (4 * q + 2 >= ns) break; // a tail of one or two slots
                test2(word(4 * q + 2), word(4 * q + 3));
            }
            occ = z26_group_or<G>(occ | occ2);
            const uint32_t freem = ~occ & kZ26Codes;
            const uint32_t m = __builtin_popcount(freem);

            if (i == 1 || (i & 7) == 0) blk = draw(a.seed, g, (uint32_t)(i >> 3) | hi, kSlotSelect, 0);
            const uint32_t x = half_word(blk, (uint32_t)(i & 7));
            const uint32_t p = x * m;
            uint32_t r = p >> 16;
            if (__builtin_expect(alive && (p & 0xFFFFu) < m, 0)) {
                r = lemire_redraw16_inline(a.seed, g, (uint32_t)i | hi, m, x);
                if (r == kPickFailed) {
                    rng_fail = true;
                    r = 0;
                }
            }
            const uint32_t code = m ? z26_select(freem, r, sel) : 13u;

            bool step_ok = alive && m != 0;
            grown = (alive && m == 0) ? i : grown;
            alive = alive && m != 0;
            const uint32_t na =
                BYTE ? ta + z26_move_bytes(code) - 0x010101u : ta + z26_move_packed(code) - kP32One;
            if (box > 0 && i >= box) {
                bool out;
                if constexpr (BYTE) {
                    const uint32_t v = na, w = 0x7F7F7Fu - na;
                    const uint32_t lo = (uint32_t)(65 - box) * 0x010101u, hb = (uint32_t)(64 - box) * 0x010101u;
                    out = ((((v - lo) & ~v) | ((w - hb) & ~w)) & 0x808080u) != 0u;
                } else {
                    const int ex = (int)(na & 0x7FFu) - 1024, ey = (int)((na >> 11) & 0x7FFu) - 1024,
                              ez = (int)(na >> 22) - 512;
                    const uint32_t span = 2u * (uint32_t)box - 2u;
                    out = (uint32_t)(ex + box - 1) > span || (uint32_t)(ey + box - 1) > span ||
                          (uint32_t)(ez + box - 1) > span;
                }
                left_box = left_box || (step_ok && out);
                alive = alive && !(step_ok && out);
                step_ok = step_ok && !out;
            }
            ta = step_ok ? na : ta;
            const uint32_t mm1 = m - 1u;
            const bool counts = step_ok && (mm1 & (G - 1)) == (uint32_t)t;
            if constexpr (G == 2) {
                const uint32_t f = mm1 / G;
                const bool upper = f >= 8u;
                const uint64_t inc = 1ull << (FW * (upper ? f - 8u : f));
                n_mine += (counts && !upper) ? inc : 0ull;
                n_mine2 += (counts && upper) ? inc : 0ull;
            } else {
                n_mine += counts ? 1ull << (FW * (mm1 / G)) : 0ull;
            }
            const bool mine = step_ok && t == (i & (G - 1));
            const uint32_t nw = BYTE ? na + kZ26Bias : na;
            const int slot = i / G;
            if (slot < SL / 2) {
                const uint32_t old = pl[slot];
                pl[slot] = mine ? nw : old;
            } else {
                const uint32_t old = ph[slot - SL / 2];
                ph[slot - SL / 2] = mine ? nw : old;
            }
        }
        if (alive) grown = N;

        double lw = 0.0;
#pragma unroll 1
        for (int mm = 1; mm <= 26; ++mm) {
            const int f0 = (mm - 1) / G;
            const bool upper = G == 2 && f0 >= 8;
            const int f = upper ? f0 - 8 : f0;
            const int per = 32 / (int)FW;
            const uint32_t half = (uint32_t)((upper ? n_mine2 : n_mine) >> (32 * (f / per)));
            const uint32_t v = (uint32_t)__shfl((int)half, gbase + ((mm - 1) & (G - 1)), 64);
            const uint32_t nm = (v >> (FW * (uint32_t)(f % per))) & ((1u << FW) - 1u);
            lw = lw + (double)nm * logm[mm];
        }
        // observables over the placed monomers (the slots off the sentinel;
        // integer sums: any order)
        int32_t sx = 0, sy = 0, sz = 0;
        int64_t s2 = 0;
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const uint32_t w = s < SL / 2 ? pl[s] : ph[s - SL / 2];
            const bool placed = w != SENT;
            int32_t xx, yy, zz;
            if constexpr (BYTE) {
                xx = (int32_t)(w & 0xFFu) - 192;
                yy = (int32_t)((w >> 8) & 0xFFu) - 192;
                zz = (int32_t)((w >> 16) & 0xFFu) - 192;
            } else {
                xx = (int32_t)(w & 0x7FFu) - 1024;
                yy = (int32_t)((w >> 11) & 0x7FFu) - 1024;
                zz = (int32_t)(w >> 22) - 512;
            }
            xx = placed ? xx : 0;
            yy = placed ? yy : 0;
            zz = placed ? zz : 0;
            sx += xx;
            sy += yy;
            sz += zz;
            s2 += (int64_t)(xx * xx + yy * yy + zz * zz);
        }
#pragma unroll
        for (int off = 1; off < G; off <<= 1) {
            sx += __shfl_xor(sx, off, 64);
            sy += __shfl_xor(sy, off, 64);
            sz += __shfl_xor(sz, off, 64);
            const int lo = __shfl_xor((int)(uint32_t)s2, off, 64);
            const int hh = __shfl_xor((int)(uint32_t)((uint64_t)s2 >> 32), off, 64);
            s2 += (int64_t)(((uint64_t)(uint32_t)hh << 32) | (uint32_t)lo);
        }
        if (pending && left_box) {
            pending = false; // grown again in wide words
        } else if (pending && (alive || rd + 1 >= a.max_rounds)) {
            const int64_t gg = grown;
            res_nn = gg * s2 - ((int64_t)sx * sx + (int64_t)sy * sy + (int64_t)sz * sz);
            if constexpr (BYTE) {
                res_ex = (int32_t)(ta & 0xFFu) - 64;
                res_ey = (int32_t)((ta >> 8) & 0xFFu) - 64;
                res_ez = (int32_t)((ta >> 16) & 0xFFu) - 64;
            } else {
                res_ex = (int32_t)(ta & 0x7FFu) - 1024;
                res_ey = (int32_t)((ta >> 11) & 0x7FFu) - 1024;
                res_ez = (int32_t)(ta >> 22) - 512;
            }
            res_lw = alive ? lw : -__builtin_huge_val();
            res_grown = grown;
            res_alive = alive;
            res_set = true;
            pending = false;
        }
        if (__ballot(pending) == 0) break;
    }

    if (res_set && t == 0) {
        if (a.log_w) a.log_w[c] = res_lw;
        if (a.r_end) {
            CT *re = (CT *)a.r_end;
            re[c] = (CT)res_ex;
            re[a.n_chains + c] = (CT)res_ey;
            re[2 * a.n_chains + c] = (CT)res_ez;
        }
        if (a.r2) a.r2[c] = (double)((int64_t)res_ex * res_ex + (int64_t)res_ey * res_ey + (int64_t)res_ez * res_ez);
        if (a.n2rg2) a.n2rg2[c] = res_nn;
        if (a.rg2) a.rg2[c] = (double)res_nn / ((double)res_grown * (double)res_grown);
        if (a.n_grown) a.n_grown[c] = (uint16_t)res_grown;
    }
    if (rng_fail && !left_box) atomicExch(a.status, 6);
    const uint64_t bits = (res_alive && t == 0) ? (uint64_t)__double_as_longlong(res_lw) : 0ull;
    const uint64_t wmax = wave_max_u64(bits);
    if ((threadIdx.x & 63) == 0 && wmax != 0) atomicMax(a.log_w_max_bits, (unsigned long long)wmax);
    return left_box;
}

// Passes of the wide regrowth with GW lanes per chain: `slots` chains at a
// time from the list at z26_lds[1..n].
template <int GW, typename CT>
__device__ void z26_regrow_passes(const GrowArgs &a, const double *logm, uint64_t first_chain, int n, int slots)
{
    extern __shared__ uint32_t z26_lds[];
    const int HW = z26_regrow_plane(a.n_monomers);
    uint32_t *planes = z26_lds + kZ26ListWords;
    const int gw = threadIdx.x / GW;
    for (int b0 = 0; b0 < n; b0 += slots) {
        __syncthreads();
        for (int w = threadIdx.x; w < slots * 2 * HW; w += blockDim.x)
            planes[w] = ((w / HW) & 1) ? kZ26OriginB : 0u;
        __syncthreads();
        const bool v = gw < slots && b0 + gw < n;
        const uint64_t c = first_chain + (v ? z26_lds[1 + b0 + gw] : 0u);
        if (__ballot(v) != 0) // waves without such a chain skip the growth
            z26_grow<GW, false, CT, kZ26Wide>(a, logm, planes + (v ? gw : 0) * 2 * HW, HW, c, v, 0);
    }
}

// Chains of the block that left the box of the byte or packed words (`mine`
// on the leader lane of each), grown again in wide words (8 lanes per chain
// up to N = 512, 32 beyond) in the block's own LDS of `words` words, as many
// at a time as fit.  Every thread of the block calls this.
template <typename CT>
__device__ void z26_regrow_wide(const GrowArgs &a, const double *logm, uint64_t first_chain, bool mine,
                                uint32_t chb, int words)
{
    extern __shared__ uint32_t z26_lds[];
    __syncthreads(); // every chain of the block is done with its plane
    if (threadIdx.x == 0) z26_lds[0] = 0u;
    const int n = __syncthreads_count(mine);
    if (n == 0) return;
    if (mine) z26_lds[1 + atomicAdd(&z26_lds[0], 1u)] = chb;
    const int N = a.n_monomers;
    const int room = (words - kZ26ListWords) / (2 * z26_regrow_plane(N));
    const int per_block = (int)blockDim.x / z26_regrow_lanes(N);
    const int slots = room < per_block ? room : per_block; // >= 1: checked by the launch shape
    if (z26_regrow_lanes(N) == 8)
        z26_regrow_passes<8, CT>(a, logm, first_chain, n, slots);
    else
        z26_regrow_passes<32, CT>(a, logm, first_chain, n, slots);
}

// Box edge of the byte (62) and packed (254) words; a launch's byte_box in
// 1..127 lowers it (tests), 0 keeps it.
__device__ __forceinline__ int z26_box(const GrowArgs &a, int natural)
{
    return (a.byte_box > 0 && a.byte_box < natural) ? a.byte_box : natural;
}

template <int G, bool EXACT, typename CT, int FMT>
__device__ __forceinline__ void grow_lattice26_body(const GrowArgs &a, uint64_t bid, int H)
{
    constexpr bool ONE = FMT != kZ26Wide;
    constexpr int WPM = ONE ? 1 : 2; // words per monomer
    const int cpb = blockDim.x / G;
    extern __shared__ uint32_t z26_lds[];
    uint32_t *chains = z26_lds; // cpb chains of WPM H words
    __shared__ double logm[27];
    for (int q = threadIdx.x; q < 27; q += blockDim.x) logm[q] = a.logm[q];
    for (int w = threadIdx.x; w < cpb * WPM * H; w += blockDim.x)
        chains[w] = FMT == kZ26Byte ? kZ26Bias
                                    : (FMT == kZ26Packed ? kP32Sentinel : (((w / H) & 1) ? kZ26OriginB : 0u));
    __syncthreads();

    const int t = threadIdx.x & (G - 1);
    const int chb = threadIdx.x / G;
    const uint64_t c = bid * cpb + chb;
    const int box = FMT == kZ26Byte ? z26_box(a, kZ26ByteEdge) : (FMT == kZ26Packed ? z26_box(a, kZ26PackedEdge) : 0);
    const bool left = z26_grow<G, EXACT, CT, FMT>(a, logm, chains + chb * WPM * H, H, c, c < a.n_chains, box);
    if constexpr (ONE) z26_regrow_wide<CT>(a, logm, bid * cpb, left && t == 0, (uint32_t)chb, cpb * H);
}

template <int G, bool EXACT, typename CT, int FMT>
__global__ __launch_bounds__(256) void grow_lattice26(GrowArgs a, int H, uint64_t base)
{
    grow_lattice26_body<G, EXACT, CT, FMT>(a, base + blockIdx.x, H);
}

template <int G, bool EXACT, typename CT, int FMT>
__global__ __launch_bounds__(256) void grow_lattice26_batch(const GrowEntry *tab, const uint64_t *block0, int n,
                                                            uint64_t base)
{
    const uint64_t bid = base + blockIdx.x;
    const int e = find_segment(block0, n, bid);
    grow_lattice26_body<G, EXACT, CT, FMT>(tab[e].a, bid - block0[e], tab[e].H);
}

// Register formats: one block grows its chains with their words in the
// groups' registers, then regrows the chains that left the box in wide
// words in its `words` of LDS.
template <int G, typename CT, int FMT>
__device__ __forceinline__ void grow_lattice26_grp_body(const GrowArgs &a, uint64_t bid, int words)
{
    const int cpb = blockDim.x / G;
    __shared__ double logm[27];
    __shared__ uint8_t sel[2048];
    for (int q = threadIdx.x; q < 27; q += blockDim.x) logm[q] = a.logm[q];
    z26_fill_select_table(sel);
    __syncthreads();
    const int t = threadIdx.x & (G - 1);
    const int chb = threadIdx.x / G;
    const uint64_t c = bid * cpb + chb;
    const int box = FMT == kZ26Byte ? z26_box(a, kZ26ByteEdge) : z26_box(a, kZ26PackedEdge);
    const bool left = z26_grp_grow<G, CT, FMT>(a, logm, sel, c, c < a.n_chains, box);
    z26_regrow_wide<CT>(a, logm, bid * cpb, left && t == 0, (uint32_t)chb, words);
}

// At least 3 waves per SIMD: the register budget of 168 VGPRs.
template <int G, typename CT, int FMT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void
grow_lattice26_grp(GrowArgs a, int words, uint64_t base)
{
    grow_lattice26_grp_body<G, CT, FMT>(a, base + blockIdx.x, words);
}

template <int G, typename CT, int FMT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void
grow_lattice26_grp_batch(const GrowEntry *tab, const uint64_t *block0, int n, uint64_t base)
{
    const uint64_t bid = base + blockIdx.x;
    const int e = find_segment(block0, n, bid);
    grow_lattice26_grp_body<G, CT, FMT>(tab[e].a, bid - block0[e], tab[e].S);
}

// Short chains (N <= 64): one lane per chain.  The lane's history sits in
// LDS as one word per monomer, bytes (x + 64, y + 64, z + 64) plus 128 each
// (coordinates stay within +-63), four monomers to a 16-byte group; group g
// of lane L is entry g * T + L of the block's group array, so a wave reads
// 1 KB of consecutive groups per ds_read_b128.  Unplaced entries hold the
// sentinel 0x00808080 (raw coordinates -64, at least 2 from every tip).
// Pair test of a stored word w against the tip word t (raw, unbiased), with
// tp = t + 0x7F7F7F (z26_bits8):
//   v    = w - tp                    bytes d + 1 when every |d| <= 1
//   bad  = (v | (v + 0x010101)) & 0xFCFCFC   0 iff every |d| <= 1
//   code = dot4(v, (1, 3, 9, 0));    occ |= sat(1 - bad) << code
// six operations.  The counts n_m of the
// steps with m free candidates are 8-bit fields in LDS (seven words per
// lane); the r-th free code comes from the byte holding it and a 2 KB table
// of the k-th set bit of every byte value.
constexpr int kZ26LaneMax = 64;
constexpr int kZ26LaneThreads = 256;

__host__ __device__ constexpr size_t z26_lane_shmem(int N, int T)
{
    return (size_t)((N + 3) / 4) * T * 16 + (size_t)7 * T * 4 + 32 * 4 + 2048;
}


template <bool EXACT, typename CT>
__device__ __forceinline__ void grow_lattice26_lane_body(const GrowArgs &a, uint64_t bid)
{
    constexpr int T = kZ26LaneThreads;
    const int N = a.n_monomers;
    const int NQ = (N + 3) >> 2;
    extern __shared__ uint4 z26l_lds[];
    uint4 *groups = z26l_lds;                                   // [NQ][T]
    uint32_t *hist = (uint32_t *)(groups + (size_t)NQ * T);     // [7][T]
    uint32_t *lut = hist + 7 * T;                               // [32]
    uint8_t *sel = (uint8_t *)(lut + 32);                       // [256][8]
    __shared__ double logm[27];
    for (int q = threadIdx.x; q < 27; q += T) {
        const int dx = q % 3, dy = (q / 3) % 3, dz = q / 9; // each + 1
        lut[q] = (uint32_t)(dx | dy << 8 | dz << 16);
        logm[q] = a.logm[q];
    }
    z26_fill_select_table(sel);
    const uint4 sent = {kZ26Bias, kZ26Bias, kZ26Bias, kZ26Bias};
    for (int q = threadIdx.x; q < NQ * T; q += T) groups[q] = sent;
    __syncthreads();

    const int L = threadIdx.x;
    const uint64_t c = bid * T + L;
    const bool valid = c < a.n_chains;
    const uint64_t g = a.chain_offset + c;
    uint32_t *words = (uint32_t *)groups;
    auto slot = [&](int j) -> uint32_t & { return words[(((size_t)(j >> 2) * T + L) << 2) + (j & 3)]; };

    uint32_t tip = kZ26LaneOrigin;
    bool alive = false;
    int grown = 1;
    uint64_t wx = 1;
    bool rng_fail = false;
    Philox4 blk{0, 0, 0, 0};
    double res_lw = -__builtin_huge_val();
    uint64_t res_wx = 0;
    int64_t res_nn = 0;
    int32_t res_ex = 0, res_ey = 0, res_ez = 0;
    int res_grown = 1;
    bool res_alive = false;
    bool pending = valid;

    for (uint32_t rd = 0; rd < a.max_rounds; ++rd) {
        if (pending) {
            if (rd > 0)
                for (int q = 0; q < NQ; ++q) groups[(size_t)q * T + L] = sent;
            for (int q = 0; q < 7; ++q) hist[q * T + L] = 0u;
            tip = kZ26LaneOrigin;
            slot(0) = tip + kZ26Bias;
            wx = 1;
        }
        alive = pending;
        grown = 1;
        const uint32_t hi = rd << 16;

        for (int i = 1; i < N; ++i) {
            // monomers 0 .. i-2 in groups of four; the last group may also hold
            // the tip (code 13, masked) and sentinels
            const int ng = (i + 2) >> 2;
            const uint32_t tp = tip + 0x7F7F7Fu;
            uint32_t occ = 0, occ2 = 0;
            auto test4 = [&](const uint4 &w) {
                occ |= z26_bits8(w.x, tp);
                occ2 |= z26_bits8(w.y, tp);
                occ |= z26_bits8(w.z, tp);
                occ2 |= z26_bits8(w.w, tp);
            };
            int q = 0;
            for (; q + 1 < ng; q += 2) { // two groups in flight, as in the group kernel
                const uint4 w1 = groups[(size_t)q * T + L];
                const uint4 w2 = groups[(size_t)(q + 1) * T + L];
                test4(w1);
                test4(w2);
            }
            if (q < ng) test4(groups[(size_t)q * T + L]);
            const uint32_t freem = ~(occ | occ2) & kZ26Codes;
            const uint32_t m = __builtin_popcount(freem);

            if (i == 1 || (i & 7) == 0) blk = draw(a.seed, g, (uint32_t)(i >> 3) | hi, kSlotSelect, 0);
            const uint32_t x = half_word(blk, (uint32_t)(i & 7));
            const uint32_t p = x * m;
            uint32_t r = p >> 16;
            if (__builtin_expect(alive && (p & 0xFFFFu) < m, 0)) {
                r = lemire_redraw16_inline(a.seed, g, (uint32_t)i | hi, m, x);
                if (r == kPickFailed) {
                    rng_fail = true;
                    r = 0;
                }
            }
            if (alive && m == 0) {
                alive = false;
                grown = i;
            }
            if (alive) {
                const uint32_t code = z26_select(freem, r, sel);
                tip = tip + lut[code] - 0x00010101u;
                slot(i) = tip + kZ26Bias;
                atomicAdd(&hist[(m >> 2) * T + L], 1u << ((m & 3u) * 8u));
                if (EXACT) wx = wx * (uint64_t)m;
            }
        }
        if (alive) grown = N;

        if (pending && (alive || rd + 1 >= a.max_rounds)) {
            // log W = sum over m = 1..26, ascending, of n_m log m
            double lw = 0.0;
#pragma unroll 1
            for (int mm = 1; mm <= 26; ++mm) {
                const uint32_t nm = (hist[(mm >> 2) * T + L] >> ((mm & 3) * 8)) & 0xFFu;
                lw = lw + (double)nm * logm[mm];
            }
            int32_t sx = 0, sy = 0, sz = 0, s2 = 0;
            for (int j = 0; j < grown; ++j) {
                const uint32_t w = slot(j) - kZ26Bias;
                const int32_t xx = (int32_t)(w & 0xFFu) - 64;
                const int32_t yy = (int32_t)((w >> 8) & 0xFFu) - 64;
                const int32_t zz = (int32_t)((w >> 16) & 0xFFu) - 64;
                sx += xx;
                sy += yy;
                sz += zz;
                s2 += xx * xx + yy * yy + zz * zz;
            }
            const int64_t gg = grown;
            res_nn = gg * (int64_t)s2 - ((int64_t)sx * sx + (int64_t)sy * sy + (int64_t)sz * sz);
            res_ex = (int32_t)(tip & 0xFFu) - 64;
            res_ey = (int32_t)((tip >> 8) & 0xFFu) - 64;
            res_ez = (int32_t)((tip >> 16) & 0xFFu) - 64;
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

template <bool EXACT, typename CT>
__global__ __launch_bounds__(kZ26LaneThreads) void grow_lattice26_lane(GrowArgs a, uint64_t base)
{
    grow_lattice26_lane_body<EXACT, CT>(a, base + blockIdx.x);
}

template <bool EXACT, typename CT>
__global__ __launch_bounds__(kZ26LaneThreads) void grow_lattice26_lane_batch(const GrowEntry *tab,
                                                                            const uint64_t *block0, int n,
                                                                            uint64_t base)
{
    const uint64_t bid = base + blockIdx.x;
    const int e = find_segment(block0, n, bid);
    grow_lattice26_lane_body<EXACT, CT>(tab[e].a, bid - block0[e]);
}

int lattice26_max_monomers() { return 16384; }

// Shape of the group kernel for N monomers, G lanes per chain and `threads`
// per block in one word format.  hipErrorInvalidValue when the block's LDS
// exceeds the CU's 160 KiB or, for byte and packed words, holds no chain of
// the wide regrowth.
static hipError_t z26_shape_fmt(int N, bool i16, int G, int threads, int fmt, GrowVariant *v)
{
    const int WPM = fmt == kZ26Wide ? 2 : 1;
    const int H = (N + 4 * G - 1) / (4 * G) * (4 * G);
    const int cpb = threads / G;
    const size_t words = (size_t)cpb * WPM * H;
    if (words * sizeof(uint32_t) > 163840) return hipErrorInvalidValue;
    if (fmt != kZ26Wide && (int)words - kZ26ListWords < 2 * z26_regrow_plane(N)) return hipErrorInvalidValue;
    v->family = 3;
    v->p0 = G;
    v->p1 = fmt;
    v->p2 = i16 ? 1 : 0;
    v->threads = threads;
    v->cpb = cpb;
    v->shmem = words * sizeof(uint32_t);
    v->H = H;
    v->S = 0;
    return hipSuccess;
}

// Shape of the group kernel for a mapping: G lanes per chain (4: 8-bit n_m
// fields, N <= 256; 8..64: 16-bit fields), `threads` per block (64 or 256);
// byte words up to N = 640 and packed words up to N = 4096, in the group's
// registers where N <= 64 G (formats 3 and 4; LDS for the regrowth only),
// else in LDS where the block can host the regrowth; else wide words.  Up to N = 4096 wide words always
// fit when the one-word formats lack that room (at most two chains per
// block), so a mapping legal at some N is legal at every smaller N of the
// group kernel.
static hipError_t z26_shape(int N, bool i16, int G, int threads, GrowVariant *v)
{
    if (G != 2 && G != 4 && G != 8 && G != 16 && G != 32 && G != 64) return hipErrorInvalidValue;
    if (threads != 64 && threads != 256) return hipErrorInvalidValue;
    if (G == 4 && N > 256) return hipErrorInvalidValue;
    if (G == 2 && N > kZ26Slots * 2) return hipErrorInvalidValue; // registers only
    const int fmt = N <= kZ26ByteMaxN ? kZ26Byte : (N <= kZ26PackedMaxN ? kZ26Packed : kZ26Wide);
    if (fmt != kZ26Wide && N <= kZ26Slots * G) {
        // registers: LDS for the regrowth of up to four chains at a time
        // (fewer where they would pass 40 KiB)
        int room = 4;
        while (room > 1 && (kZ26ListWords + room * 2 * z26_regrow_plane(N)) * 4 > 40960) --room;
        v->family = 3;
        v->p0 = G;
        v->p1 = fmt + 2; // 3: byte words, 4: packed words, in registers
        v->p2 = i16 ? 1 : 0;
        v->threads = threads;
        v->cpb = threads / G;
        v->S = kZ26ListWords + room * 2 * z26_regrow_plane(N);
        v->shmem = (size_t)v->S * sizeof(uint32_t);
        v->H = 0;
        return hipSuccess;
    }
    if (fmt != kZ26Wide && z26_shape_fmt(N, i16, G, threads, fmt, v) == hipSuccess) return hipSuccess;
    return z26_shape_fmt(N, i16, G, threads, kZ26Wide, v);
}

// One lane per chain up to N = 64 (and for exact weights, N <= 14); above,
// G lanes per chain, the fewest whose 64 register slots hold the chain:
// 2 up to N = 128, 4 up to 256, 8 up to 512, 16 up to 1024, 32 up to 2048
// and 64 beyond (wide words in LDS past N = 4096).  Against the widths
// measured best when the words sat in LDS (10^5 to 10^6 chains): N = 500,
// 18.5 -> 13.9 ms (8 lanes, not 16); N = 1000, 15.4 -> 11.9 ms (16, not
// 32); N = 2000, 31.2 -> 24.1 ms (32, not 64); with 2 lanes a wave's 32
// chains share each step's pick (N = 65, 1.30 -> 0.85 ms; N = 100, 2.10 ->
// 1.54 ms against 4 lanes).  256-thread blocks when the block's LDS fits in
// half a CU's, else one wave.  A legal mapping of the tuning table replaces
// the rule for the group kernel.
hipError_t lattice26_variant(const GrowArgs &a, bool exact, bool i16, GrowVariant *v)
{
    const int N = a.n_monomers;
    if (N <= kZ26LaneMax) {
        v->family = 3;
        v->p0 = 1;
        v->p1 = exact ? 1 : 0;
        v->p2 = i16 ? 1 : 0;
        v->threads = kZ26LaneThreads;
        v->cpb = kZ26LaneThreads;
        v->shmem = z26_lane_shmem(N, kZ26LaneThreads);
        v->H = 0;
        v->S = 0;
        return hipSuccess;
    }
    if (exact) return hipErrorInvalidValue;
    int tl = 0, tt = 0;
    if (tuned_mapping(2 /* 26-neighbour lattice */, N, a.k_trials, &tl, &tt) &&
        z26_shape(N, i16, tl, tt, v) == hipSuccess)
        return hipSuccess;
    const int G = N <= 128 ? 2 : (N <= 256 ? 4 : (N <= 512 ? 8 : (N <= 1024 ? 16 : (N <= 2048 ? 32 : 64))));
    GrowVariant half_cu;
    if (z26_shape(N, i16, G, 256, &half_cu) == hipSuccess && half_cu.shmem <= 81920) {
        *v = half_cu;
        return hipSuccess;
    }
    return z26_shape(N, i16, G, 64, v);
}

template <bool EXACT, typename CT>
static hipError_t launch26_lane(const GrowArgs &a, const GrowVariant &v, const GrowEntry *tab,
                                const uint64_t *block0, int n, uint64_t blocks, size_t shmem, hipStream_t s)
{
    const void *fn = tab ? (const void *)grow_lattice26_lane_batch<EXACT, CT>
                         : (const void *)grow_lattice26_lane<EXACT, CT>;
    if (shmem > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess) return e;
    }
    return launch_sliced(blocks, v.threads, [&](uint64_t b0, uint32_t nb) {
        if (tab)
            hipLaunchKernelGGL((grow_lattice26_lane_batch<EXACT, CT>), dim3(nb), dim3(v.threads), shmem, s, tab,
                               block0, n, b0);
        else
            hipLaunchKernelGGL((grow_lattice26_lane<EXACT, CT>), dim3(nb), dim3(v.threads), shmem, s, a, b0);
    });
}

template <int G, typename CT, int FMT>
static hipError_t launch26(const GrowArgs &a, const GrowVariant &v, const GrowEntry *tab, const uint64_t *block0,
                           int n, uint64_t blocks, size_t shmem, hipStream_t s)
{
    const void *fn = tab ? (const void *)grow_lattice26_batch<G, false, CT, FMT>
                         : (const void *)grow_lattice26<G, false, CT, FMT>;
    if (shmem > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess) return e;
    }
    return launch_sliced(blocks, v.threads, [&](uint64_t b0, uint32_t nb) {
        if (tab)
            hipLaunchKernelGGL((grow_lattice26_batch<G, false, CT, FMT>), dim3(nb), dim3(v.threads), shmem, s, tab,
                               block0, n, b0);
        else
            hipLaunchKernelGGL((grow_lattice26<G, false, CT, FMT>), dim3(nb), dim3(v.threads), shmem, s, a, v.H,
                               b0);
    });
}

template <int G, typename CT, int FMT>
static hipError_t launch26_grp(const GrowArgs &a, const GrowVariant &v, const GrowEntry *tab,
                               const uint64_t *block0, int n, uint64_t blocks, size_t shmem, hipStream_t s)
{
    const void *fn = tab ? (const void *)grow_lattice26_grp_batch<G, CT, FMT>
                         : (const void *)grow_lattice26_grp<G, CT, FMT>;
    if (shmem > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess) return e;
    }
    return launch_sliced(blocks, v.threads, [&](uint64_t b0, uint32_t nb) {
        if (tab)
            hipLaunchKernelGGL((grow_lattice26_grp_batch<G, CT, FMT>), dim3(nb), dim3(v.threads), shmem, s, tab,
                               block0, n, b0);
        else
            hipLaunchKernelGGL((grow_lattice26_grp<G, CT, FMT>), dim3(nb), dim3(v.threads), shmem, s, a, v.S, b0);
    });
}

template <int G, typename CT>
static hipError_t launch26_ct(const GrowArgs &a, const GrowVariant &v, const GrowEntry *tab,
                              const uint64_t *block0, int n, uint64_t blocks, size_t shmem, hipStream_t s)
{
    if constexpr (G == 2) { // byte words in registers only (N <= 128)
        return launch26_grp<2, CT, kZ26Byte>(a, v, tab, block0, n, blocks, shmem, s);
    } else {
        if (v.p1 == kZ26Byte + 2) return launch26_grp<G, CT, kZ26Byte>(a, v, tab, block0, n, blocks, shmem, s);
        if (v.p1 == kZ26Packed + 2) return launch26_grp<G, CT, kZ26Packed>(a, v, tab, block0, n, blocks, shmem, s);
        if (v.p1 == kZ26Byte) return launch26<G, CT, kZ26Byte>(a, v, tab, block0, n, blocks, shmem, s);
        if (v.p1 == kZ26Packed) return launch26<G, CT, kZ26Packed>(a, v, tab, block0, n, blocks, shmem, s);
        return launch26<G, CT, kZ26Wide>(a, v, tab, block0, n, blocks, shmem, s);
    }
}

template <int G>
static hipError_t launch26_g(const GrowArgs &a, const GrowVariant &v, const GrowEntry *tab, const uint64_t *block0,
                             int n, uint64_t blocks, size_t shmem, hipStream_t s)
{
    return v.p2 ? launch26_ct<G, int16_t>(a, v, tab, block0, n, blocks, shmem, s)
                : launch26_ct<G, int32_t>(a, v, tab, block0, n, blocks, shmem, s);
}

static hipError_t dispatch26(const GrowArgs &a, const GrowVariant &v, const GrowEntry *tab, const uint64_t *block0,
                             int n, uint64_t blocks, size_t shmem, hipStream_t s)
{
    const bool i16 = v.p2 != 0;
    if (v.p0 == 1) {
        if (v.p1)
            return i16 ? launch26_lane<true, int16_t>(a, v, tab, block0, n, blocks, shmem, s)
                       : launch26_lane<true, int32_t>(a, v, tab, block0, n, blocks, shmem, s);
        return i16 ? launch26_lane<false, int16_t>(a, v, tab, block0, n, blocks, shmem, s)
                   : launch26_lane<false, int32_t>(a, v, tab, block0, n, blocks, shmem, s);
    }
    switch (v.p0) {
    case 2: return launch26_g<2>(a, v, tab, block0, n, blocks, shmem, s);
    case 4: return launch26_g<4>(a, v, tab, block0, n, blocks, shmem, s);
    case 8: return launch26_g<8>(a, v, tab, block0, n, blocks, shmem, s);
    case 16: return launch26_g<16>(a, v, tab, block0, n, blocks, shmem, s);
    case 32: return launch26_g<32>(a, v, tab, block0, n, blocks, shmem, s);
    default: return launch26_g<64>(a, v, tab, block0, n, blocks, shmem, s);
    }
}

hipError_t launch_grow_lattice26(const GrowArgs &a, bool exact, bool i16, hipStream_t s)
{
    GrowVariant v;
    hipError_t e = lattice26_variant(a, exact, i16, &v);
    if (e != hipSuccess) return e;
    const uint64_t blocks = (a.n_chains + v.cpb - 1) / v.cpb;
    return dispatch26(a, v, nullptr, nullptr, 0, blocks, v.shmem, s);
}

hipError_t launch_lattice26_batch(const GrowVariant &v, const GrowEntry *tab, const uint64_t *block0, int n,
                                  uint64_t blocks, size_t shmem, hipStream_t s)
{
    return dispatch26(GrowArgs{}, v, tab, block0, n, blocks, shmem, s);
}

} // namespace rsaw
