// Device-side building blocks of librsaw: the Philox4x32-10 block function,
// Lemire's uniform pick, wave-level helpers and the kernel argument blocks.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by
// the 64-bit seed; the counter is (lo32(g), hi32(g), c2, slot << 16 | attempt)
// with g the global chain index.  Word use per growth step i:
//   slot 0xFFFF, c2 = i >> 3      : primary 16-bit selection word, half i & 7
//   slot 0xFFFE, c2 = i, attempt a: redraw half-words of Lemire's rejection
//   slot t < 64, c2 = i, attempt a: real-space trial t, Marsaglia attempt a
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsaw {

constexpr uint32_t kSlotSelect = 0xFFFFu;
constexpr uint32_t kSlotRedraw = 0xFFFEu;
constexpr uint32_t kMaxAttempt = 65536u;

struct Philox4 {
    uint32_t x0, x1, x2, x3;
};

// Three-way XOR in one gfx950 bitop3 instruction (truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Ten Philox rounds; the key schedule adds the Weyl constants after each
// round.  Per round two 32 x 32 -> 64-bit multiplies and two three-way XORs.
__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Philox4{c0, c1, c2, c3};
}

// Square root of x in [2^-60, 1], correctly rounded (checked bit for bit
// against the host over the Marsaglia domain 1 - s by rsaw_fp64_check): the
// hardware estimate y of 1/sqrt(x), refined by Goldschmidt's iteration to
// g ~ sqrt(x) and h ~ 1/(2 g), then two Newton corrections of g on the
// remainder x - g^2, each a fused multiply-add.  Without the scaling and the
// special cases of the general square root, which this domain never needs.
__device__ __forceinline__ double sqrt_unit(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double e = __builtin_fma(-h, g, 0.5);
    g = __builtin_fma(g, e, g);
    h = __builtin_fma(h, e, h);
    double d = __builtin_fma(-g, g, x);
    g = __builtin_fma(d, h, g);
    d = __builtin_fma(-g, g, x);
    return __builtin_fma(d, h, g);
}

__device__ __forceinline__ Philox4 draw(uint64_t seed, uint64_t g, uint32_t c2, uint32_t slot,
                                        uint32_t attempt)
{
    return philox4x32_10((uint32_t)g, (uint32_t)(g >> 32), c2, (slot << 16) | attempt,
                         (uint32_t)seed, (uint32_t)(seed >> 32));
}

__device__ __forceinline__ uint32_t word(const Philox4 &b, uint32_t w)
{
    return w == 0 ? b.x0 : (w == 1 ? b.x1 : (w == 2 ? b.x2 : b.x3));
}

// 16-bit half h (0..7) of a block: word h / 2, low half for even h.
__device__ __forceinline__ uint32_t half_word(const Philox4 &b, uint32_t h)
{
    const uint32_t w = word(b, h >> 1);
    return (h & 1u) ? (w >> 16) : (w & 0xFFFFu);
}

// Lemire's method on 16-bit words, slow path: the primary word x of step
// `step` is accepted when (x m) mod 2^16 >= 2^16 mod m, else the eight
// halves of each redraw block (slot 0xFFFE, attempt 0, 1, ...) are tried in
// order.  Returns (x m) / 2^16 of the accepted word, or kPickFailed at the
// attempt cap.  m >= 1.  The failure travels in the return value so that no
// flag of the caller has its address taken (which would put it in scratch).
constexpr uint32_t kPickFailed = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t lemire_redraw16_inline(uint64_t seed, uint64_t g, uint32_t step,
                                                           uint32_t m, uint32_t x)
{
    const uint32_t threshold = 65536u % m;
    uint32_t p = x * m;
    if ((p & 0xFFFFu) >= threshold) return p >> 16;
    for (uint32_t a = 0; a < kMaxAttempt; ++a) {
        const Philox4 b = draw(seed, g, step, kSlotRedraw, a);
        for (uint32_t h = 0; h < 8; ++h) {
            p = half_word(b, h) * m;
            if ((p & 0xFFFFu) >= threshold) return p >> 16;
        }
    }
    return kPickFailed;
}

// The same as an out-of-line call: kernels whose live state across the rare
// slow path is small keep it out of their code; the others inline it and
// avoid the registers the call convention reserves.
__device__ __noinline__ uint32_t lemire_redraw16(uint64_t seed, uint64_t g, uint32_t step,
                                                 uint32_t m, uint32_t x)
{
    return lemire_redraw16_inline(seed, g, step, m, x);
}

// Wave-wide max of a 64-bit value (all 64 lanes must be active).
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// ---------------------------------------------------------------------------
// Kernel argument blocks (passed by value).
// ---------------------------------------------------------------------------
struct GrowArgs {
    uint64_t seed;
    uint64_t chain_offset;
    uint64_t n_chains;
    int32_t n_monomers;
    int32_t k_trials;
    double bond_length;
    double sigma2;
    double cull2; // (b + sigma)^2 (1 + 2^-30): beads at or beyond it cannot overlap
    uint32_t max_rounds; // growth attempts per chain: 1, or 65536 when a dead end restarts
    int32_t byte_box;    // boxed lattice words: |coordinate| (1..127) at which a chain is regrown in wide words; 0: each format's own edge
    double *bead_slots;  // hard spheres beyond the LDS limit: n_slots regions of 3 N doubles (HBM)
    uint32_t n_slots;
    // per-chain outputs (device, any may be null)
    double *log_w;
    uint64_t *w_exact;
    void *r_end;
    double *r2;
    double *rg2;
    int64_t *n2rg2;
    uint16_t *n_grown;
    // reduction side channels
    unsigned long long *log_w_max_bits; // atomicMax of the bit pattern (log W >= 0)
    int32_t *status;                    // RSAW_E_RNG on a rejection-cap hit
    double logm[65];                    // ln(m) correctly rounded, m = 0..64
};

// One ensemble of a batched launch: its arguments and, for the LDS lattice
// kernel, its plane length H and chain stride S (words).
struct GrowEntry {
    GrowArgs a;
    int32_t H, S;
};

// Segment of block `bid` in a batched launch: the last e with block0[e] <= bid
// (block0 ascending, block0[0] = 0, n >= 1).
__device__ __forceinline__ int find_segment(const uint64_t *block0, int n, uint64_t bid)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (block0[mid] <= bid) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Grids are issued in slices of at most 2^31 work-items (a dispatch packet
// counts work-items in 32 bits); each slice passes its first block index
// `base`, and block b of it serves block base + b of the whole grid.
template <typename F>
inline hipError_t launch_sliced(uint64_t blocks, int threads, F &&launch_one)
{
    const uint64_t step = ((uint64_t)1 << 31) / (uint64_t)threads;
    for (uint64_t b0 = 0; b0 < blocks; b0 += step) {
        const uint64_t nb = blocks - b0 < step ? blocks - b0 : step;
        launch_one(b0, (uint32_t)nb);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Launch shape of one growth kernel variant; ensembles with equal kernel,
// template parameters and block size share one batched launch.
struct GrowVariant {
    int family;         // 0 lattice (registers), 1 lattice (LDS), 2 hard spheres, 3 26-neighbour lattice
    int p0, p1, p2;     // template parameters of the family
    int threads;        // threads per block
    int cpb;            // chains per block
    size_t shmem;       // dynamic LDS bytes per block
    int32_t H, S;       // LDS lattice plane length and chain stride
};

// Lane mapping (lanes per chain, threads per block) that the tuning table
// holds for a group-kernel call of this geometry, N and k: the calling
// thread's forced mapping while the autotuner times a candidate, else the
// newest table entry covering N.  False when neither applies; the variant
// functions then use their built-in rule, and they also fall back to it
// when a mapping is not legal for the call.
bool tuned_mapping(int geometry, int n_monomers, int k_trials, int *lanes, int *threads);

} // namespace rsaw
