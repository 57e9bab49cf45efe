// Lattice chain growth for chains too long to keep in one lane's registers
// (N > 64): the same growth rule as the register kernel (Sec. 3.3.2,
// Algorithm 1; weight of Eq. 3) with G lanes per chain.  Two kernels share
// the step: one keeps the chain history in the group's VGPRs (byte words,
// N <= 64 G, so N <= 4096), the other in LDS (any N to 16384).
//
// On the bipartite cubic lattice the monomers that can neighbour the tip at
// step i are those of index i - 2, i - 4, ..., i.e. the first floor(i / 2)
// entries of the plane of parity i (monomers of even, or odd, index), so
// both kernels keep two parity planes and scan one run of one of them.
// Entries not yet placed hold 0, a sentinel that is never adjacent to any
// tip, so a scan may run past the chain's last entry without a bounds test.
//
// Registers.  Entry k of a plane sits in lane k mod G of the group, slot
// k / G of that lane's 32-slot array (64 VGPRs for both planes).  A step
// tests the slots that hold entries, four at a time behind one wave-uniform
// count test (two in a last group with one or two slots left: 0.5-2 %
// faster, bit-identical), and appends the new monomer with one indexed
// register read and write (uniform slot; the lane holding it takes the
// new word).
//
// LDS.  Each chain owns S words: two planes of H words each, times one
// (byte format) or two (wide format) words per monomer.  Lane t of the
// chain's group reads 4 consecutive words (one b128 load) per pass, the
// group 4 G words, and H is the half length rounded up to 4 G.
//
// Monomer words.
//   byte format (N <= 2048 in LDS, N <= 4096 in registers; coordinates
//     within [-127, 127], exact by construction up to N = 128, kept by the
//     box and the regrowth below beyond): as in the register kernel, (Q mod 256, x + 128, y + 128,
//     z + 128); pair test L = msad(r_j, tip & ~0xFF), bit = sat(2 - L),
//     code = (r_j - tip + 3) mod 32 from the Q byte, 4 operations.
//   wide format (LDS beyond, and the regrowth): A = (x + 2^15) | (y + 2^15) << 16 and
//     B = (64 + Q mod 32) | (z + 2^15) << 16; pair test
//     L = sad_u16(A_j, A_t) + sad_u16(B_j & 0xFFFF0000, B_t & 0xFFFF0000),
//     bit = sat(2 - L), code = (B_j - B_t + 3) mod 32, 6 operations.  A move
//     adds per-field deltas that never carry across a field; one AND-OR
//     brings B's low field back to 64 + (Q mod 32).
//
// Per step the G partial occupancy masks are OR-reduced across the group
// (cross-lane DPP and permute operations, no LDS round trip);
// every lane of the group then performs the same pick (same Philox words),
// and the lane that holds the new entry appends it to its parity plane.
#include "lattice_common.hpp"

namespace rsaw {

// Orders the LDS accesses of the lanes of one wave.
__device__ __forceinline__ void lattice_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr uint32_t kByteOrigin = 0x80808000u;            // origin, Q = 0
constexpr uint32_t kWideOriginA = 0x80008000u;           // x = y = 0
constexpr uint32_t kWideOriginB = 0x80000000u | 64u;     // z = 0, Q = 0

// OR over the aligned group of G lanes, every lane receiving the result:
// DPP butterflies within quads, half rows and rows of 16, then the gfx950
// row-swap permutes for 32 and 64 lanes.  All lanes must be active.
template <int G>
__device__ __forceinline__ uint32_t group_or(uint32_t v)
{
    if constexpr (G >= 2) v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);
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

template <bool WIDE>
__device__ __forceinline__ uint32_t pair_bits(uint32_t wa, uint32_t wb, uint32_t ta, uint32_t tbh,
                                              uint32_t tq)
{
    if constexpr (WIDE) {
        uint32_t L = __builtin_amdgcn_sad_u16(wa, ta, 0u);
        L = __builtin_amdgcn_sad_u16(wb & 0xFFFF0000u, tbh, L);
        const uint32_t bit = __builtin_elementwise_sub_sat(2u, L);
        return bit << ((wb - tq) & 31u);
    } else {
        const uint32_t L = __builtin_amdgcn_msad_u8(wa, ta, 0u);
        const uint32_t bit = __builtin_elementwise_sub_sat(2u, L);
        return bit << ((wa - tq) & 31u);
    }
}

// Byte words hold each coordinate plus 128 in one byte.  Up to N = 128 no
// coordinate can leave [-127, 127].  Longer chains ("boxed" byte words)
// stop growing a chain whose new tip reaches |coordinate| = E (127, or the
// launch's byte_box when a caller lowers it), before the byte test and the
// carry-free move could stop being exact at -128 and +128; the block then
// grows that chain again from its first draw in wide words (the same draws
// and the same tests give the same chain, Sec. 3.3.2), so every chain's
// result is exact whichever word format produced it.
constexpr int kByteExactN = 128;
constexpr int kByteBoxedMaxN = 2048;
constexpr int kRegrowListWords = 65; // count + one slot per chain of a block (<= 64)

// A- and B-word deltas of a byte-format move (coordinate bytes | dQ).
__device__ __forceinline__ void wide_move(uint32_t mv, uint32_t &da, uint32_t &db)
{
    const int dq = (int)(int8_t)(mv & 0xFFu);
    const int axis = dq < 0 ? -dq : dq;
    const int sg = dq < 0 ? -1 : 1;
    da = axis == 1 ? (uint32_t)sg : (axis == 2 ? (uint32_t)(sg * 65536) : 0u);
    db = (uint32_t)((axis == 3 ? sg * 65536 : 0) + dq);
}

__device__ __forceinline__ void lattice_lds_luts(uint32_t *lut, uint32_t *lutb, bool wide)
{
    for (int idx = threadIdx.x; idx < kLutSize; idx += blockDim.x) {
        const uint32_t mv = lattice_move((uint32_t)idx);
        if (wide)
            wide_move(mv, lut[idx], lutb[idx]);
        else
            lut[idx] = mv;
    }
}

// Grows the chain c of this thread's group of G lanes, its history in the S
// words at `base`, and writes its outputs.  With `boxed` (byte words only) a
// chain whose tip reaches the edge of the byte range stops, writes nothing
// and contributes nothing to the side channels; the function then returns
// true on the group's lanes.
template <int G, bool WIDE, typename CT, bool TABLE = true>
__device__ __forceinline__ bool lattice_lds_grow(const GrowArgs &a, const uint32_t *lut, const uint32_t *lutb,
                                                 uint32_t *base, int H, int S, uint64_t c, bool valid, bool boxed)
{
    constexpr int WPM = WIDE ? 2 : 1; // words per monomer
    const int t = threadIdx.x & (G - 1);
    const uint64_t g = a.chain_offset + c;
    const int N = a.n_monomers;
    const int edge = a.byte_box > 0 ? a.byte_box : 127; // box of the byte words

    uint32_t ta = 0, tb = 0; // tip: A word (or the byte word) and B word (wide only)
    bool alive = false;
    bool left_box = false;
    int grown = 1;
    // steps with m free candidates: 16-bit fields for m = 2, 3, 4, 5 (wide
    // words; step 1 has m = 6), 12-bit fields at 12 (m - 1) for m = 1..6
    // (byte words, N <= 2048: no test of m or i needed)
    uint64_t cnt = 0;
    bool rng_fail = false;
    Philox4 blk{0, 0, 0, 0};
    // outputs of the attempt that ends the chain (see the register kernel)
    double res_lw = -__builtin_huge_val();
    int64_t res_nn = 0;
    int32_t res_ex = 0, res_ey = 0, res_ez = 0;
    int res_grown = 1;
    bool res_alive = false;
    bool res_set = false;
    bool pending = valid;

    for (uint32_t rd = 0; rd < a.max_rounds; ++rd) {
        // (re)start the chains still growing: clear their planes back to the
        // sentinel and place monomer 0 at the origin
        if (pending) {
            if (rd > 0)
                for (int w = t; w < S; w += G) base[w] = 0u;
            ta = WIDE ? kWideOriginA : kByteOrigin;
            tb = WIDE ? kWideOriginB : 0u;
            cnt = 0;
        }
        lattice_wave_sync();
        if (pending && t == 0) {
            base[0] = ta;
            if constexpr (WIDE) base[H] = tb;
        }
        lattice_wave_sync();
        alive = pending;
        grown = 1;
        const uint32_t hi = rd << 16; // attempt in the high half of the step word

        for (int i = 1; i < N; ++i) {
            // occupied-neighbour mask: the group scans the plane of parity i
            const uint32_t *pa = base + (i & 1) * WPM * H;
            const uint32_t *pb = pa + H;
            const int nrel = i >> 1;
            const int passes = (nrel + 4 * G - 1) / (4 * G);
            const uint32_t tref = WIDE ? ta : (ta & 0xFFFFFF00u);
            const uint32_t tbh = tb & 0xFFFF0000u;
            const uint32_t tq = (WIDE ? tb : ta) - 3u;
            uint32_t occ = 0, occ2 = 0;
            const auto test4 = [&](const uint4 &wa, const uint4 &wb) {
                occ |= pair_bits<WIDE>(wa.x, wb.x, tref, tbh, tq);
                occ2 |= pair_bits<WIDE>(wa.y, wb.y, tref, tbh, tq);
                occ |= pair_bits<WIDE>(wa.z, wb.z, tref, tbh, tq);
                occ2 |= pair_bits<WIDE>(wa.w, wb.w, tref, tbh, tq);
            };
            // two passes per iteration, so that the second pass's reads are
            // in flight while the first is tested
            int q = 0;
            for (; q + 1 < passes; q += 2) {
                const int k1 = q * 4 * G + 4 * t, k2 = k1 + 4 * G;
                const uint4 a1 = *(const uint4 *)(pa + k1), a2 = *(const uint4 *)(pa + k2);
                uint4 b1 = make_uint4(0u, 0u, 0u, 0u), b2 = b1;
                if constexpr (WIDE) {
                    b1 = *(const uint4 *)(pb + k1);
                    b2 = *(const uint4 *)(pb + k2);
                }
                test4(a1, b1);
                test4(a2, b2);
            }
            if (q < passes) {
                const int k1 = q * 4 * G + 4 * t;
                uint4 b1 = make_uint4(0u, 0u, 0u, 0u);
                if constexpr (WIDE) b1 = *(const uint4 *)(pb + k1);
                test4(*(const uint4 *)(pa + k1), b1);
            }
            occ |= occ2;
            occ = group_or<G>(occ);
            const uint32_t freem = ~occ & 0x77u;
            const uint32_t m = __builtin_popcount(freem);

            // 16-bit selection word: half i mod 8 of one Philox block per 8 steps
            if (i == 1 || (i & 7) == 0) blk = draw(a.seed, g, (uint32_t)(i >> 3) | hi, kSlotSelect, 0);
            const uint32_t x = half_word(blk, (uint32_t)(i & 7));
            const uint32_t p = x * m;
            uint32_t r = p >> 16;
            if (__builtin_expect(alive && (p & 0xFFFFu) < m, 0)) {
                r = lemire_redraw16(a.seed, g, (uint32_t)i | hi, m, x);
                if (r == kPickFailed) {
                    rng_fail = true;
                    r = 0;
                }
            }

            bool step_ok = alive && m != 0;
            const uint32_t li = (freem << 3) | r; // r < m <= 6, or 0
            uint32_t na, nb = 0u;
            if constexpr (WIDE) {
                uint32_t da, db;
                if constexpr (TABLE) {
                    da = lut[li];
                    db = lutb[li];
                } else {
                    wide_move(lattice_move(li), da, db);
                }
                na = ta + da;
                nb = ((tb + db) & 0xFFFF001Fu) | 0x40u;
            } else {
                const uint32_t mv = lut[li];
                na = ((ta & 0xFFFFFF00u) + (mv & 0xFFFFFF00u)) | ((ta + mv) & 0xFFu);
                // |coordinate| >= E (127, or the launch's byte_box if set;
                // possible from step E on):
                // the chain leaves the box here.  Coordinate bytes b = x + 128
                // with b < 129 - E or 255 - b < 128 - E, as two byte-wise
                // "has a byte below n" tests (exact for n <= 128) on the
                // three bytes and on their complements.
                if (boxed && i >= edge) {
                    const uint32_t v = na >> 8, w = v ^ 0xFFFFFFu;
                    const uint32_t lo = (uint32_t)(129 - edge) * 0x010101u;
                    const uint32_t hi = (uint32_t)(128 - edge) * 0x010101u;
                    const uint32_t edge = (((v - lo) & ~v) | ((w - hi) & ~w)) & 0x808080u;
                    if (step_ok && edge != 0u) {
                        step_ok = false;
                        alive = false;
                        left_box = true;
                    }
                }
            }
            if (alive && m == 0) {
                alive = false;
                grown = i;
            }
            if (step_ok) {
                ta = na;
                tb = nb;
                if constexpr (WIDE) {
                    if (i >= 2 && m >= 2) cnt += 1ull << (16u * (m - 2u));
                } else {
                    cnt += 1ull << (12u * (m - 1u));
                }
                if (t == 0) {
                    uint32_t *wp = base + (i & 1) * WPM * H + (i >> 1);
                    wp[0] = na;
                    if constexpr (WIDE) wp[H] = nb;
                }
            }
            lattice_wave_sync();
            // one chain per wave: once it has ended (a third of N = 3000 chains
            // meet a dead end, two thirds of N = 5000 ones), the wave leaves
            // the step loop instead of scanning on (N = 5000, 2 10^4 chains:
            // 94.2 -> 62.4 ms; N = 10000, 5 10^3 chains: 188.7 -> 79.0 ms)
            if constexpr (G == 64) {
                if (__ballot(alive) == 0) break;
            }
        }
        if (alive) grown = N;
        // log W = sum over m = 1..6, ascending, of n_m log m; n_1 log 1 = 0 and
        // m_1 = 6 always
        double lw = 0.0;
        if (N >= 2) {
            const int f0 = WIDE ? 0 : 12, fw = WIDE ? 16 : 12;
            const uint64_t fm = WIDE ? 0xFFFFu : 0xFFFu;
            lw = lw + (double)(uint32_t)((cnt >> f0) & fm) * a.logm[2];
            lw = lw + (double)(uint32_t)((cnt >> (f0 + fw)) & fm) * a.logm[3];
            lw = lw + (double)(uint32_t)((cnt >> (f0 + 2 * fw)) & fm) * a.logm[4];
            lw = lw + (double)(uint32_t)((cnt >> (f0 + 3 * fw)) & fm) * a.logm[5];
            lw = lw + a.logm[6];
        }

        // observables over the placed monomers (integer sums: any order)
        int32_t sx = 0, sy = 0, sz = 0;
        int64_t s2 = 0;
        for (int j = t; j < grown; j += G) {
            const uint32_t *wp = base + (j & 1) * WPM * H + (j >> 1);
            int32_t x, y, z;
            if constexpr (WIDE) {
                const uint32_t wa = wp[0], wb = wp[H];
                x = (int32_t)(wa & 0xFFFFu) - 32768;
                y = (int32_t)(wa >> 16) - 32768;
                z = (int32_t)(wb >> 16) - 32768;
            } else {
                const uint32_t w = wp[0];
                x = (int32_t)((w >> 8) & 0xFFu) - 128;
                y = (int32_t)((w >> 16) & 0xFFu) - 128;
                z = (int32_t)(w >> 24) - 128;
            }
            sx += x;
            sy += y;
            sz += z;
            s2 += (int64_t)(x * x + y * y + z * z);
        }
    #pragma unroll
        for (int off = 1; off < G; off <<= 1) {
            sx += __shfl_xor(sx, off, 64);
            sy += __shfl_xor(sy, off, 64);
            sz += __shfl_xor(sz, off, 64);
            const int lo = __shfl_xor((int)(uint32_t)s2, off, 64);
            const int hi = __shfl_xor((int)(uint32_t)((uint64_t)s2 >> 32), off, 64);
            s2 += (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
        }
        const int64_t gg = grown;
        const int64_t nn = gg * s2 - ((int64_t)sx * sx + (int64_t)sy * sy + (int64_t)sz * sz);
        int32_t ex, ey, ez;
        if constexpr (WIDE) {
            ex = (int32_t)(ta & 0xFFFFu) - 32768;
            ey = (int32_t)(ta >> 16) - 32768;
            ez = (int32_t)(tb >> 16) - 32768;
        } else {
            ex = (int32_t)((ta >> 8) & 0xFFu) - 128;
            ey = (int32_t)((ta >> 16) & 0xFFu) - 128;
            ez = (int32_t)(ta >> 24) - 128;
        }
        if (pending && left_box) {
            pending = false; // grown again in wide words
        } else if (pending && (alive || rd + 1 >= a.max_rounds)) {
            res_lw = alive ? lw : -__builtin_huge_val();
            res_nn = nn;
            res_ex = ex;
            res_ey = ey;
            res_ez = ez;
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

// Lanes per chain, plane length and chain stride (words) of the wide
// regrowth; the same formulas as the launch shapes.
__host__ __device__ __forceinline__ int regrow_lanes(int N) { return N <= 512 ? 8 : 32; }
__host__ __device__ __forceinline__ int regrow_plane(int N)
{
    const int half = (N + 1) / 2, q = 4 * regrow_lanes(N);
    return (half + q - 1) / q * q;
}
__host__ __device__ __forceinline__ int regrow_stride(int N)
{
    const int q = 4 * regrow_lanes(N);
    return 4 * regrow_plane(N) + (q < 64 ? q : 0);
}

// Passes of the regrowth: `slots` chains at a time from the list at
// lds_u[1..n]; moves computed per step (no tables: the regrowth is rare).
template <int GW, typename CT>
__device__ void regrow_passes(const GrowArgs &a, uint64_t first_chain, int n, int slots, uint32_t *planes)
{
    extern __shared__ uint32_t lds_u[];
    const int N = a.n_monomers;
    const int HW = regrow_plane(N), SW = regrow_stride(N);
    const int gw = threadIdx.x / GW;
    for (int b0 = 0; b0 < n; b0 += slots) {
        __syncthreads();
        for (int w = threadIdx.x; w < slots * SW; w += blockDim.x) planes[w] = 0u;
        __syncthreads();
        const bool v = gw < slots && b0 + gw < n;
        const uint64_t c = first_chain + (v ? lds_u[1 + b0 + gw] : 0u);
        if (__ballot(v) != 0) // waves without such a chain skip the growth
            lattice_lds_grow<GW, true, CT, false>(a, nullptr, nullptr, planes + (v ? gw : 0) * SW, HW, SW, c, v,
                                                  false);
    }
}

// Chains of the block that left the byte box (`mine` on the leader lane of
// each), grown again in wide words in the block's own LDS of `words` words,
// as many at a time as fit.  Every thread of the block calls this.
template <typename CT>
__device__ void regrow_wide(const GrowArgs &a, uint64_t first_chain, bool mine, uint32_t chb, int words)
{
    extern __shared__ uint32_t lds_u[];
    __syncthreads(); // every chain of the block is done with its planes
    if (threadIdx.x == 0) lds_u[0] = 0u;
    const int n = __syncthreads_count(mine);
    if (n == 0) return;
    if (mine) lds_u[1 + atomicAdd(&lds_u[0], 1u)] = chb;
    const int N = a.n_monomers;
    uint32_t *planes = lds_u + kRegrowListWords;
    const int room = (words - kRegrowListWords) / regrow_stride(N);
    const int per_block = (int)blockDim.x / regrow_lanes(N);
    const int slots = room < per_block ? room : per_block; // >= 1: checked by the launch shape
    if (regrow_lanes(N) == 8)
        regrow_passes<8, CT>(a, first_chain, n, slots, planes);
    else
        regrow_passes<32, CT>(a, first_chain, n, slots, planes);
}

// Register-resident byte words, the layout of the file header: N <= 64 G,
// with 2 lanes up to N = 128 and 4 to 64 lanes beyond.  Against the LDS
// kernel (same lanes, 10^5 to 10^6 chains, MI355X, bit-identical) the step
// loses its scan loads and their round trips, and the block's LDS shrinks
// to the move table and the regrowth, so the kernel runs at 3 waves per
// SIMD (168 VGPRs) where the LDS kernel ran at 2 to 3: N = 160, 2.09 ->
// 1.86 ms; N = 256, 4.95 -> 3.49 ms; N = 384, 13.5 -> 9.2 ms; N = 512,
// 19.9 -> 13.7 ms; N = 2048, 35.0 -> 26.1 ms.  With 64 lanes (one chain per
// wave, which leaves the step loop once its chain has ended) against wide
// words in LDS: N = 2049, 32.5 -> 20.4 ms; N = 3000, 43.1 -> 23.5 ms;
// N = 4096, 57.9 -> 45.5 ms (3 10^4 chains; 10^4 chains, 21.3 -> 22.9 ms:
// 3.5 % of N = 4096 chains leave the box and are regrown).  Up to N = 128
// the LDS kernel's chains are short enough for 4 waves per SIMD, and 4
// lanes in registers only tie (N = 80: 0.86 against 0.83 ms); but 2 lanes
// per chain, which only registers allow, let a wave's 32 chains share each
// step's pick and bookkeeping: N = 65, 0.84 -> 0.43 ms; N = 80, 0.82 ->
// 0.52 ms; N = 100, 1.03 -> 0.67 ms; N = 128, 1.36 -> 0.92 ms.  Unbounded,
// the compiler takes 186 VGPRs (2 waves per SIMD: 4.20 ms at N = 256); at
// 4 waves it spills in the step loop.
constexpr int kGrpSlots = 32; // slots per lane and plane

template <int G, typename CT>
__device__ __forceinline__ bool lattice_grp_grow(const GrowArgs &a, const uint32_t *lut, uint64_t c, bool valid)
{
    constexpr int SL = kGrpSlots;
    const int t = threadIdx.x & (G - 1);
    const uint64_t g = a.chain_offset + c;
    const int N = a.n_monomers;
    const bool boxed = N > kByteExactN;
    const int edge = a.byte_box > 0 ? a.byte_box : 127; // box of the byte words

    uint32_t pe[SL], po[SL]; // planes of even and odd monomers
#pragma unroll
    for (int s = 0; s < SL; ++s) pe[s] = po[s] = 0u;
    uint32_t ta = 0;
    bool alive = false;
    bool left_box = false;
    int grown = 1;
    uint64_t cnt = 0; // n_m in 12-bit fields at 12 (m - 1), m = 1..6
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
            for (int s = 0; s < SL; ++s) {
                pe[s] = pending ? 0u : pe[s];
                po[s] = pending ? 0u : po[s];
            }
        }
        if (pending) {
            ta = kByteOrigin;
            cnt = 0;
        }
        pe[0] = (pending && t == 0) ? kByteOrigin : pe[0];
        alive = pending;
        grown = 1;
        const uint32_t hi = rd << 16;

        const auto step = [&](int i, uint32_t(&pl)[SL]) {
            const int ns = ((i >> 1) + G - 1) / G; // slots holding entries of plane i mod 2
            const uint32_t tref = ta & 0xFFFFFF00u;
            const uint32_t tq = ta - 3u;
            uint32_t occ = 0, occ2 = 0;
#pragma unroll
            for (int q = 0; q < SL / 4; ++q) {
                if (4 * q >= ns) break;
                occ |= pair_bits<false>(pl[4 * q], 0u, tref, 0u, tq);
                occ2 |= pair_bits<false>(pl[4 * q + 1], 0u, tref, 0u, tq);
                if (4 * q + 2 >= ns) break; // a tail of one or two slots
                occ |= pair_bits<false>(pl[4 * q + 2], 0u, tref, 0u, tq);
                occ2 |= pair_bits<false>(pl[4 * q + 3], 0u, tref, 0u, tq);
            }
            occ |= occ2;
            occ = group_or<G>(occ);
            const uint32_t freem = ~occ & 0x77u;
            const uint32_t m = __builtin_popcount(freem);

            if (i == 1 || (i & 7) == 0) blk = draw(a.seed, g, (uint32_t)(i >> 3) | hi, kSlotSelect, 0);
            const uint32_t x = half_word(blk, (uint32_t)(i & 7));
            const uint32_t p = x * m;
            uint32_t r = p >> 16;
            if (__builtin_expect(alive && (p & 0xFFFFu) < m, 0)) {
                r = lemire_redraw16(a.seed, g, (uint32_t)i | hi, m, x);
                if (r == kPickFailed) {
                    rng_fail = true;
                    r = 0;
                }
            }

            bool step_ok = alive && m != 0;
            const uint32_t mv = lut[(freem << 3) | r];
            const uint32_t na = ((ta & 0xFFFFFF00u) + (mv & 0xFFFFFF00u)) | ((ta + mv) & 0xFFu);
            if (boxed && i >= edge) {
                const uint32_t v = na >> 8, w = v ^ 0xFFFFFFu;
                const uint32_t lo = (uint32_t)(129 - edge) * 0x010101u;
                const uint32_t hb = (uint32_t)(128 - edge) * 0x010101u;
                const bool out = ((((v - lo) & ~v) | ((w - hb) & ~w)) & 0x808080u) != 0u;
                left_box = left_box || (step_ok && out);
                alive = alive && !(step_ok && out);
                step_ok = step_ok && !out;
            }
            grown = (alive && m == 0) ? i : grown;
            alive = alive && m != 0;
            ta = step_ok ? na : ta;
            cnt += step_ok ? (1ull << (12u * (m - 1u))) : 0ull;
            const int k = i >> 1;
            const uint32_t old = pl[k / G];
            pl[k / G] = (step_ok && t == (k & (G - 1))) ? na : old;
        };
        for (int i = 1; i < N; i += 2) {
            step(i, po);
            if (i + 1 < N) step(i + 1, pe);
            // one chain per wave: the wave leaves once its chain has ended
            if constexpr (G == 64) {
                if (__ballot(alive) == 0) break;
            }
        }
        if (alive) grown = N;
        double lw = 0.0;
        if (N >= 2) {
            lw = lw + (double)(uint32_t)((cnt >> 12) & 0xFFFu) * a.logm[2];
            lw = lw + (double)(uint32_t)((cnt >> 24) & 0xFFFu) * a.logm[3];
            lw = lw + (double)(uint32_t)((cnt >> 36) & 0xFFFu) * a.logm[4];
            lw = lw + (double)(uint32_t)((cnt >> 48) & 0xFFFu) * a.logm[5];
            lw = lw + a.logm[6];
        }

        // observables over the placed monomers (the non-zero words; integer
        // sums: any order)
        int32_t sx = 0, sy = 0, sz = 0;
        int64_t s2 = 0;
        const auto add = [&](uint32_t w) {
            const int32_t x = w ? (int32_t)((w >> 8) & 0xFFu) - 128 : 0;
            const int32_t y = w ? (int32_t)((w >> 16) & 0xFFu) - 128 : 0;
            const int32_t z = w ? (int32_t)(w >> 24) - 128 : 0;
            sx += x;
            sy += y;
            sz += z;
            s2 += (int64_t)(x * x + y * y + z * z);
        };
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            add(pe[s]);
            add(po[s]);
        }
#pragma unroll
        for (int off = 1; off < G; off <<= 1) {
            sx += __shfl_xor(sx, off, 64);
            sy += __shfl_xor(sy, off, 64);
            sz += __shfl_xor(sz, off, 64);
            const int lo = __shfl_xor((int)(uint32_t)s2, off, 64);
            const int hi2 = __shfl_xor((int)(uint32_t)((uint64_t)s2 >> 32), off, 64);
            s2 += (int64_t)(((uint64_t)(uint32_t)hi2 << 32) | (uint32_t)lo);
        }
        const int64_t gg = grown;
        const int64_t nn = gg * s2 - ((int64_t)sx * sx + (int64_t)sy * sy + (int64_t)sz * sz);
        const int32_t ex = (int32_t)((ta >> 8) & 0xFFu) - 128;
        const int32_t ey = (int32_t)((ta >> 16) & 0xFFu) - 128;
        const int32_t ez = (int32_t)(ta >> 24) - 128;
        if (pending && left_box) {
            pending = false; // grown again in wide words
        } else if (pending && (alive || rd + 1 >= a.max_rounds)) {
            res_lw = alive ? lw : -__builtin_huge_val();
            res_nn = nn;
            res_ex = ex;
            res_ey = ey;
            res_ez = ez;
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

// One block: the move table, each group's chain, then the regrowth of the
// block's chains that left the byte box, in the block's `words` of LDS.
template <int G, typename CT>
__device__ __forceinline__ void grow_lattice_grp_body(const GrowArgs &a, uint64_t bid, int words)
{
    const int cpb = blockDim.x / G;
    extern __shared__ uint32_t lds_u[];
    lattice_lds_luts(lds_u, nullptr, false);
    __syncthreads();
    const int t = threadIdx.x & (G - 1);
    const int chb = threadIdx.x / G;
    const uint64_t c = bid * cpb + chb;
    const bool left = lattice_grp_grow<G, CT>(a, lds_u, c, c < a.n_chains);
    if (a.n_monomers > kByteExactN) regrow_wide<CT>(a, bid * cpb, left && t == 0, (uint32_t)chb, words);
}

// At least 3 waves per SIMD: the register budget of 168 VGPRs.
template <int G, typename CT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void
grow_lattice_grp(GrowArgs a, int words, uint64_t base)
{
    grow_lattice_grp_body<G, CT>(a, base + blockIdx.x, words);
}

// Batched launch: block b serves the ensemble whose block range holds b.
template <int G, typename CT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void
grow_lattice_grp_batch(const GrowEntry *tab, const uint64_t *block0, int n, uint64_t base)
{
    const uint64_t bid = base + blockIdx.x;
    const int e = find_segment(block0, n, bid);
    grow_lattice_grp_body<G, CT>(tab[e].a, bid - block0[e], tab[e].S);
}

template <int G, bool WIDE, typename CT>
__device__ __forceinline__ void grow_lattice_lds_body(const GrowArgs &a, uint64_t bid, int H, int S)
{
    constexpr int WPM = WIDE ? 2 : 1; // words per monomer
    const int cpb = blockDim.x / G;   // chains per block
    extern __shared__ uint32_t lds_u[];
    uint32_t *lut = lds_u;                     // byte-format move, or the A move
    uint32_t *lutb = lds_u + kLutSize;         // B move (wide only)
    uint32_t *chains = lds_u + WPM * kLutSize; // cpb chains of S words
    lattice_lds_luts(lut, lutb, WIDE);
    for (int w = threadIdx.x; w < cpb * S; w += blockDim.x) chains[w] = 0u;
    __syncthreads();

    const int t = threadIdx.x & (G - 1);
    const int chb = threadIdx.x / G;
    const uint64_t c = bid * cpb + chb;
    const bool boxed = !WIDE && a.n_monomers > kByteExactN;
    const bool left =
        lattice_lds_grow<G, WIDE, CT>(a, lut, lutb, chains + chb * S, H, S, c, c < a.n_chains, boxed);
    if constexpr (!WIDE) {
        if (boxed) regrow_wide<CT>(a, bid * cpb, left && t == 0, (uint32_t)chb, WPM * kLutSize + cpb * S);
    }
}

template <int G, bool WIDE, typename CT>
__global__ __launch_bounds__(256) void grow_lattice_lds(GrowArgs a, int H, int S, uint64_t base)
{
    grow_lattice_lds_body<G, WIDE, CT>(a, base + blockIdx.x, H, S);
}

// Batched launch: block b serves the ensemble whose block range holds b.
template <int G, bool WIDE, typename CT>
__global__ __launch_bounds__(256) void grow_lattice_lds_batch(const GrowEntry *tab, const uint64_t *block0,
                                                              int n, uint64_t base)
{
    const uint64_t bid = base + blockIdx.x;
    const int e = find_segment(block0, n, bid);
    grow_lattice_lds_body<G, WIDE, CT>(tab[e].a, bid - block0[e], tab[e].H, tab[e].S);
}

// Largest lattice chain of the LDS kernel (wide words: 128 KiB per chain).
int lattice_lds_max_monomers() { return 16384; }

// Shape of a lattice group kernel for N monomers, G lanes per chain and
// `threads` per block (64 or 256) in one word format: byte words (in the
// group's registers where 128 < N <= 64 G, or G = 2 and N <= 128, format
// 2, else in LDS up to N = 2048, format 0) or wide words (LDS, format 1).  hipErrorInvalidValue when the
// block's LDS exceeds the CU's 160 KiB or, for boxed byte words, holds no
// chain of the wide regrowth.
static hipError_t lds_shape_fmt(int N, bool i16, int G, int threads, bool wide, GrowVariant *v)
{
    if (!wide && (N > kByteExactN || G == 2) && N <= 2 * kGrpSlots * G) {
        // registers: LDS for the move table and the regrowth of up to four
        // chains at a time (fewer where they would pass 40 KiB)
        int room = N > kByteExactN ? 4 : 0;
        while (room > 1 && (kRegrowListWords + room * regrow_stride(N)) * 4 > 40960) --room;
        int words = kRegrowListWords + room * regrow_stride(N);
        if (words < kLutSize) words = kLutSize;
        v->family = 1;
        v->p0 = G;
        v->p1 = 2;
        v->p2 = i16 ? 1 : 0;
        v->threads = threads;
        v->cpb = threads / G;
        v->shmem = (size_t)words * sizeof(uint32_t);
        v->H = 0;
        v->S = words;
        return hipSuccess;
    }
    const int WPM = wide ? 2 : 1;
    const int half = (N + 1) / 2;
    const int H = (half + 4 * G - 1) / (4 * G) * (4 * G);
    // chain stride: pad so that the chains of a wave start on different banks
    const int S = 2 * WPM * H + (4 * G < 64 ? 4 * G : 0);
    const int cpb = threads / G;
    const int words = WPM * kLutSize + cpb * S;
    if ((size_t)words * sizeof(uint32_t) > 163840) return hipErrorInvalidValue;
    if (!wide && N > kByteExactN && words - kRegrowListWords < regrow_stride(N)) return hipErrorInvalidValue;
    v->family = 1;
    v->p0 = G;
    v->p1 = wide ? 1 : 0;
    v->p2 = i16 ? 1 : 0;
    v->threads = threads;
    v->cpb = cpb;
    v->shmem = (size_t)words * sizeof(uint32_t);
    v->H = H;
    v->S = S;
    return hipSuccess;
}

// Shape for a mapping: byte words (boxed beyond N = 128) in the group's
// registers for 128 < N <= 64 G and with G = 2 (N <= 128 only), else in
// LDS up to N = 2048 where the block can host the regrowth, else wide
// words (G >= 8).  Byte words need less
// LDS than wide ones, and their regrowth room does not grow back as N
// shrinks, so a mapping legal at some N is legal at every smaller N of the
// kernel.
static hipError_t lds_shape(int N, bool i16, int G, int threads, GrowVariant *v)
{
    if (G != 2 && G != 4 && G != 8 && G != 16 && G != 32 && G != 64) return hipErrorInvalidValue;
    if (G == 2 && N > 2 * kGrpSlots * 2) return hipErrorInvalidValue;
    if (threads != 64 && threads != 256) return hipErrorInvalidValue;
    if ((N <= kByteBoxedMaxN || (N > kByteExactN && N <= 2 * kGrpSlots * G)) &&
        lds_shape_fmt(N, i16, G, threads, false, v) == hipSuccess)
        return hipSuccess;
    if (G == 4) return hipErrorInvalidValue;
    return lds_shape_fmt(N, i16, G, threads, true, v);
}

// Variant for 64 < N <= 16384.  Built-in rule (measured on MI355X, 10^4 to
// 10^6 chains): byte words in the group's registers with 2 lanes per chain
// up to N = 128, 4 up to 256, 8 up to 512, 16 up to 1024, 32 up to 2048
// and 64 up to 4096 (the fewest lanes whose 32 slots hold a plane); wide words beyond, 32 lanes in 256-thread blocks
// while eight chains fit in a CU's LDS, else 64 lanes.
// Four or more waves per block share the move table when the block fits in
// half a CU's LDS.  A legal mapping of the tuning table replaces the rule.
hipError_t lattice_lds_variant(const GrowArgs &a, bool i16, GrowVariant *v)
{
    const int N = a.n_monomers;
    int tl = 0, tt = 0;
    if (tuned_mapping(0 /* simple cubic lattice */, N, a.k_trials, &tl, &tt) &&
        lds_shape(N, i16, tl, tt, v) == hipSuccess)
        return hipSuccess;
    const int G = N <= 128 ? 2 : N <= 256 ? 4 : (N <= 512 ? 8 : (N <= 1024 ? 16 : (N <= 2048 ? 32 : 64)));
    // wide words past N = 4096: eight chains of 32 lanes in one 256-thread
    // block per CU while they fit (N = 2200, before the registers took
    // N <= 4096: 37.8 against 49.2 ms for one-chain blocks of 64 lanes)
    if (N > 2 * kGrpSlots * 64 && lds_shape(N, i16, 32, 256, v) == hipSuccess) return hipSuccess;
    GrowVariant half_cu;
    if (lds_shape(N, i16, G, 256, &half_cu) == hipSuccess && half_cu.shmem <= 81920) {
        *v = half_cu;
        return hipSuccess;
    }
    return lds_shape(N, i16, G, 64, v);
}

template <int G, typename CT>
static hipError_t launch_grp(const GrowArgs &a, const GrowVariant &v, const GrowEntry *tab,
                             const uint64_t *block0, int n, uint64_t blocks, size_t shmem, hipStream_t s)
{
    const void *fn = tab ? (const void *)grow_lattice_grp_batch<G, CT> : (const void *)grow_lattice_grp<G, CT>;
    if (shmem > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess) return e;
    }
    return launch_sliced(blocks, v.threads, [&](uint64_t b0, uint32_t nb) {
        if (tab)
            hipLaunchKernelGGL((grow_lattice_grp_batch<G, CT>), dim3(nb), dim3(v.threads), shmem, s, tab, block0,
                               n, b0);
        else
            hipLaunchKernelGGL((grow_lattice_grp<G, CT>), dim3(nb), dim3(v.threads), shmem, s, a, v.S, b0);
    });
}

template <int G, bool WIDE, typename CT>
static hipError_t launch_lds(const GrowArgs &a, const GrowVariant &v, const GrowEntry *tab,
                             const uint64_t *block0, int n, uint64_t blocks, size_t shmem, hipStream_t s)
{
    const void *fn = tab ? (const void *)grow_lattice_lds_batch<G, WIDE, CT>
                         : (const void *)grow_lattice_lds<G, WIDE, CT>;
    if (shmem > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess) return e;
    }
    return launch_sliced(blocks, v.threads, [&](uint64_t b0, uint32_t nb) {
        if (tab)
            hipLaunchKernelGGL((grow_lattice_lds_batch<G, WIDE, CT>), dim3(nb), dim3(v.threads), shmem, s, tab,
                               block0, n, b0);
        else
            hipLaunchKernelGGL((grow_lattice_lds<G, WIDE, CT>), dim3(nb), dim3(v.threads), shmem, s, a, v.H, v.S,
                               b0);
    });
}

static hipError_t dispatch_lds(const GrowArgs &a, const GrowVariant &v, const GrowEntry *tab,
                               const uint64_t *block0, int n, uint64_t blocks, size_t shmem, hipStream_t s)
{
    const bool i16 = v.p2 != 0;
#define RSAW_LDS(G, W)                                                                                \
    return i16 ? launch_lds<G, W, int16_t>(a, v, tab, block0, n, blocks, shmem, s)                    \
               : launch_lds<G, W, int32_t>(a, v, tab, block0, n, blocks, shmem, s)
#define RSAW_GRP(G)                                                                                   \
    return i16 ? launch_grp<G, int16_t>(a, v, tab, block0, n, blocks, shmem, s)                       \
               : launch_grp<G, int32_t>(a, v, tab, block0, n, blocks, shmem, s)
    if (v.p1 == 2) {
        switch (v.p0) {
        case 2: RSAW_GRP(2);
        case 4: RSAW_GRP(4);
        case 8: RSAW_GRP(8);
        case 16: RSAW_GRP(16);
        case 32: RSAW_GRP(32);
        default: RSAW_GRP(64);
        }
    }
#undef RSAW_GRP
    switch (v.p0) {
    case 4: RSAW_LDS(4, false);
    case 8:
        if (!v.p1) RSAW_LDS(8, false);
        RSAW_LDS(8, true);
    case 16:
        if (!v.p1) RSAW_LDS(16, false);
        RSAW_LDS(16, true);
    case 32:
        if (!v.p1) RSAW_LDS(32, false);
        RSAW_LDS(32, true);
    default:
        if (!v.p1) RSAW_LDS(64, false);
        RSAW_LDS(64, true);
    }
#undef RSAW_LDS
}

hipError_t launch_grow_lattice_lds(const GrowArgs &a, bool i16, hipStream_t s)
{
    GrowVariant v;
    hipError_t e = lattice_lds_variant(a, i16, &v);
    if (e != hipSuccess) return e;
    const uint64_t blocks = (a.n_chains + v.cpb - 1) / v.cpb;
    return dispatch_lds(a, v, nullptr, nullptr, 0, blocks, v.shmem, s);
}

hipError_t launch_lattice_lds_batch(const GrowVariant &v, const GrowEntry *tab, const uint64_t *block0,
                                    int n, uint64_t blocks, size_t shmem, hipStream_t s)
{
    return dispatch_lds(GrowArgs{}, v, tab, block0, n, blocks, shmem, s);
}

} // namespace rsaw
