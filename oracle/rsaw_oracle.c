/*
 * Plain CPU oracle for Rosenbluth chain growth (Guo & Baulin, "GPU
 * implementation of the Rosenbluth generation method for static Monte Carlo
 * simulations", Comput. Phys. Commun. 2017).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the HIP library: both are written separately from the same rules.
 *
 * What it computes, in the paper's terms:
 *   - Sec. 3.3.2 / Algorithm 1: grow a self-avoiding chain on the simple cubic
 *     lattice, monomer 0 at the origin, one monomer per step next to the tip.
 *   - Sec. 3.3.3 / Algorithm 2: grow a hard-sphere chain in continuous space,
 *     each step trying k random bond directions of fixed length.
 *   - Eq. (3): the Rosenbluth weight W = product over steps of the number m_i
 *     of ways the chain can continue (free candidates); a step with m_i = 0 is
 *     a dead end and the chain keeps weight zero (attrition).
 *   - Eq. (2) with the Boltzmann factor of hard cores (0 or 1): the weighted
 *     average sum(W A) / sum(W); Eq. (6): the number of self-avoiding walks
 *     is estimated by the plain mean of W over all chains, dead ones included.
 *
 * Everything is written the slow, obvious way: every candidate is compared
 * with every earlier monomer, sums run sequentially in chain/step order with
 * Neumaier compensation, and no reordering or pruning is done.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), keyed by the 64-bit seed; the
 * 128-bit counter names (chain, step, slot, attempt) so that every chain can
 * be recomputed alone.  Uniform integers in [0, m) use Lemire's multiply-and-
 * reject method (ACM TOMACS 29(1), 2019) on 16-bit words.  Unit vectors use Marsaglia's
 * disc method (Ann. Math. Stat. 43 (1972) 645).
 *
 * Floating point: IEEE binary64, round to nearest, built without
 * contraction (-ffp-contract=off) and without fast-math, SSE2 arithmetic.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORO_OK 0
#define ORO_E_INVALID 1
#define ORO_E_RNG 6
#define ORO_E_NOMEM 4

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 block function (SC'11, Sec. 3 and Table 2 constants).       */
/* ------------------------------------------------------------------------ */
void oro_philox4x32_10(const uint32_t ctr_in[4], uint64_t seed, uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Counter layout: (lo32(chain), hi32(chain), c2, (slot << 16) | attempt). */
static void draw_block(uint64_t seed, uint64_t chain, uint32_t c2,
                       uint32_t slot, uint32_t attempt, uint32_t out[4])
{
    uint32_t ctr[4];
    ctr[0] = (uint32_t)chain;
    ctr[1] = (uint32_t)(chain >> 32);
    ctr[2] = c2;
    ctr[3] = (slot << 16) | attempt;
    oro_philox4x32_10(ctr, seed, out);
}

#define SLOT_SELECT 0xFFFFu   /* primary selection half-words, one block per 8 steps */
#define SLOT_REDRAW 0xFFFEu   /* Lemire redraw half-words for step i                */
#define MAX_ATTEMPT 65536u
#define ORO_RESTART 2        /* flag: a dead end restarts the chain (Sec. 3.3.2)  */
#define ORO_Z26 4            /* flag: the 26 neighbours of the tip are candidates */
#define MAX_ROUNDS 65536u    /* growth attempts of a chain with ORO_RESTART       */

/* 16-bit half h (0..7) of a Philox block: word h / 2, low half for even h. */
static uint32_t half_word(const uint32_t blk[4], uint32_t h)
{
    uint32_t w = blk[h >> 1];
    return (h & 1u) ? (w >> 16) : (w & 0xFFFFu);
}

/* ------------------------------------------------------------------------ */
/* Uniform index in [0, m): Lemire's method on 16-bit words.  The word       */
/* stream for step i is the primary half-word (half i mod 8 of block         */
/* (i / 8, SLOT_SELECT)), then the eight halves of block (i, SLOT_REDRAW,    */
/* attempt 0), then attempt 1, ...  Accept x when (x m) mod 2^16 >=          */
/* 2^16 mod m; the index is (x m) / 2^16.                                    */
/* ------------------------------------------------------------------------ */
int oro_lemire16(uint32_t x, uint32_t m, uint32_t *index)
{
    uint32_t threshold = 65536u % m;
    uint32_t p = x * m;
    if ((p & 0xFFFFu) < threshold) return 0;
    *index = p >> 16;
    return 1;
}

/* The pick of step i; *redraws counts the rejected half-words.  `step` is
 * the step word i | (r << 16) of growth attempt r (restarts): the primary
 * block has c2 = (i >> 3) | (r << 16), the redraw blocks c2 = step. */
int oro_pick(uint64_t seed, uint64_t chain, uint32_t step, uint32_t m,
             uint32_t *index, uint32_t *redraws)
{
    uint32_t blk[4];
    uint32_t rejected = 0;
    draw_block(seed, chain, ((step & 0xFFFFu) >> 3) | (step & 0xFFFF0000u), SLOT_SELECT, 0, blk);
    if (oro_lemire16(half_word(blk, step & 7u), m, index)) {
        if (redraws) *redraws = 0;
        return ORO_OK;
    }
    ++rejected;
    for (uint32_t a = 0; a < MAX_ATTEMPT; ++a) {
        draw_block(seed, chain, step, SLOT_REDRAW, a, blk);
        for (uint32_t h = 0; h < 8; ++h) {
            if (oro_lemire16(half_word(blk, h), m, index)) {
                if (redraws) *redraws = rejected;
                return ORO_OK;
            }
            ++rejected;
        }
    }
    return ORO_E_RNG;
}

static int pick_uniform(uint64_t seed, uint64_t chain, uint32_t step,
                        uint32_t m, uint32_t *index)
{
    return oro_pick(seed, chain, step, m, index, NULL);
}

/* ------------------------------------------------------------------------ */
/* log W (Eq. 3): W = prod_i m_i = prod_m m^(n_m), with n_m the number of     */
/* steps that had m free candidates.  log W = sum over m = 1 .. K, ascending, */
/* of n_m * log(m), each product and sum rounded once in binary64.  This is   */
/* the same quantity as the step-by-step sum of log m_i, with K - 1 products  */
/* and additions instead of one addition per step.                          */
/* ------------------------------------------------------------------------ */
static double log_weight(const int64_t *n_of_m, int K)
{
    double lw = 0.0;
    for (int m = 1; m <= K; ++m) lw = lw + (double)n_of_m[m] * log((double)m);
    return lw;
}

/* ------------------------------------------------------------------------ */
/* Simple cubic lattice (Sec. 3.3.2, Algorithm 1).                          */
/* Candidates of a step: the six neighbours of the tip, in the fixed order   */
/* -z, -y, -x, +x, +y, +z.                                                   */
/* ------------------------------------------------------------------------ */
static const int32_t LATTICE_DIR[6][3] = {
    {0, 0, -1}, {0, -1, 0}, {-1, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}
};

/* The 26-neighbour variant (the "z = 26 possible lattice space" of Sec.
 * 3.3.2): every displacement in {-1, 0, 1}^3 but zero, in the order of the
 * code (dx + 1) + 3 (dy + 1) + 9 (dz + 1).  Its six face neighbours come in
 * the same relative order as LATTICE_DIR. */
static int32_t DIR26[26][3];

static void init_dir26(void)
{
    int q = 0;
    for (int c = 0; c < 27; ++c) {
        if (c == 13) continue;
        DIR26[q][0] = c % 3 - 1;
        DIR26[q][1] = (c / 3) % 3 - 1;
        DIR26[q][2] = c / 9 - 1;
        ++q;
    }
}

/*
 * Grow one lattice chain of N monomers for RNG chain index `chain`.
 * Outputs (each pointer may be NULL):
 *   xyz[3*N]   coordinates of the placed monomers (rest untouched)
 *   m_seq[N]   m_i for step i (m_seq[0] = 0; steps past a dead end untouched)
 *   log_w      log W = sum over m of n_m log(m) (see log_weight); -inf if dead
 *   w_exact    product of m_i as an integer; 0 for a dead chain;
 *              UINT64_MAX-saturated with *w_exact_ok = 0 when it overflows
 *   n_grown    number of monomers placed (N for a complete chain)
 *   end[3]     coordinates of the last placed monomer (monomer 0 is origin)
 *   r2         squared end-to-end distance of the placed part
 *   n2rg2      g^2 Rg^2 = g * sum |r|^2 - |sum r|^2 over the g placed monomers
 *   rg2        n2rg2 / g^2 (one IEEE division)
 */
int oro_lattice_chain(uint64_t seed, uint64_t chain, int32_t N,
                      int32_t *xyz, int32_t *m_seq, double *log_w,
                      uint64_t *w_exact, int32_t *w_exact_ok, int32_t *n_grown,
                      int32_t end[3], int64_t *r2, int64_t *n2rg2, double *rg2,
                      int32_t flags, int32_t *rounds)
{
    if (N < 1) return ORO_E_INVALID;
    int32_t *pos = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)N);
    if (!pos) return ORO_E_NOMEM;
    int64_t n_of_m[27];
    const int nd = (flags & ORO_Z26) ? 26 : 6;
    if (nd == 26) init_dir26();
    const int32_t (*dir)[3] = (nd == 26) ? (const int32_t (*)[3])DIR26 : LATTICE_DIR;
    uint64_t w;
    int w_ok;
    int32_t g;
    int dead;
    int status = ORO_OK;
    const uint32_t max_rounds = (flags & ORO_RESTART) ? MAX_ROUNDS : 1u;
    uint32_t round = 0;
    /* A dead end discards the attempt and, with ORO_RESTART, the chain grows
     * again from the origin with the next round of random numbers. */
    for (;;) {
    pos[0] = 0; pos[1] = 0; pos[2] = 0;
    for (int q = 0; q < 27; ++q) n_of_m[q] = 0; /* steps with m_i = m */
    w = 1;
    w_ok = 1;
    g = 1;
    dead = 0;
    if (m_seq) m_seq[0] = 0;

    for (int32_t i = 1; i < N; ++i) {
        const int32_t *tip = &pos[3 * (i - 1)];
        int free_[26];
        uint32_t m = 0;
        for (int d = 0; d < nd; ++d) {
            int32_t cx = tip[0] + dir[d][0];
            int32_t cy = tip[1] + dir[d][1];
            int32_t cz = tip[2] + dir[d][2];
            free_[d] = 1;
            for (int32_t j = 0; j < i; ++j) {
                if (pos[3 * j] == cx && pos[3 * j + 1] == cy && pos[3 * j + 2] == cz)
                    free_[d] = 0;
            }
            m += (uint32_t)free_[d];
        }
        if (m_seq) m_seq[i] = (int32_t)m;
        if (m == 0) {
            dead = 1;
            break;
        }
        uint32_t pick;
        status = pick_uniform(seed, chain, (uint32_t)i | (round << 16), m, &pick);
        if (status != ORO_OK) break;
        int chosen = -1;
        uint32_t seen = 0;
        for (int d = 0; d < nd; ++d) {
            if (free_[d]) {
                if (seen == pick) { chosen = d; break; }
                ++seen;
            }
        }
        pos[3 * i] = tip[0] + dir[chosen][0];
        pos[3 * i + 1] = tip[1] + dir[chosen][1];
        pos[3 * i + 2] = tip[2] + dir[chosen][2];
        g = i + 1;
        n_of_m[m] += 1;
        if (w_ok && w > UINT64_MAX / m) w_ok = 0;
        if (w_ok) w = w * m;
    }
    if (status != ORO_OK || !dead || round + 1 >= max_rounds) break;
    ++round;
    }
    if (status != ORO_OK) {
        free(pos);
        return status;
    }
    if (rounds) *rounds = (int32_t)round + 1;

    double lw = log_weight(n_of_m, nd);

    /* Observables of the placed monomers 0 .. g-1. */
    int64_t sx = 0, sy = 0, sz = 0, s2 = 0;
    for (int32_t i = 0; i < g; ++i) {
        int64_t x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
        sx += x; sy += y; sz += z;
        s2 += x * x + y * y + z * z;
    }
    int64_t ex = pos[3 * (g - 1)], ey = pos[3 * (g - 1) + 1], ez = pos[3 * (g - 1) + 2];
    int64_t nn = (int64_t)g * s2 - (sx * sx + sy * sy + sz * sz);
    if (xyz) memcpy(xyz, pos, sizeof(int32_t) * 3 * (size_t)g);
    if (log_w) *log_w = dead ? -INFINITY : lw;
    if (w_exact) *w_exact = dead ? 0 : (w_ok ? w : UINT64_MAX);
    if (w_exact_ok) *w_exact_ok = dead ? 1 : w_ok;
    if (n_grown) *n_grown = g;
    if (end) { end[0] = (int32_t)ex; end[1] = (int32_t)ey; end[2] = (int32_t)ez; }
    if (r2) *r2 = ex * ex + ey * ey + ez * ez;
    if (n2rg2) *n2rg2 = nn;
    if (rg2) *rg2 = (double)nn / ((double)g * (double)g);
    free(pos);
    return ORO_OK;
}

/* ------------------------------------------------------------------------ */
/* Continuous space, hard spheres (Sec. 3.3.3, Algorithm 2).                */
/* ------------------------------------------------------------------------ */

/* Marsaglia (1972) unit vector for trial t of step i: the first attempt a
 * whose pair (v1, v2), each a 53-bit uniform on [-1, 1), falls strictly
 * inside the unit disc and off its centre. */
int oro_unit_vector(uint64_t seed, uint64_t chain, uint32_t step, uint32_t t,
                    double e[3], uint32_t *attempts)
{
    const double two_m52 = 2.220446049250313080847263336181640625e-16; /* 2^-52 */
    uint32_t blk[4];
    for (uint32_t a = 0; a < MAX_ATTEMPT; ++a) {
        draw_block(seed, chain, step, t, a, blk);
        int64_t j1 = ((int64_t)(blk[0] >> 5) << 26) + (int64_t)(blk[1] >> 6);
        int64_t j2 = ((int64_t)(blk[2] >> 5) << 26) + (int64_t)(blk[3] >> 6);
        double v1 = (double)(j1 - ((int64_t)1 << 52)) * two_m52;
        double v2 = (double)(j2 - ((int64_t)1 << 52)) * two_m52;
        double s = v1 * v1 + v2 * v2;
        if (s < 1.0 && s != 0.0) {
            double q = 2.0 * sqrt(1.0 - s);
            e[0] = v1 * q;
            e[1] = v2 * q;
            e[2] = 1.0 - 2.0 * s;
            if (attempts) *attempts = a + 1;
            return ORO_OK;
        }
    }
    return ORO_E_RNG;
}

/* Overlap rule: the candidate c overlaps bead j when the squared distance,
 * evaluated as ((dx dx + dy dy) + dz dz), is below sigma^2. */
int oro_overlaps(const double c[3], const double r[3], double sigma2)
{
    double dx = c[0] - r[0];
    double dy = c[1] - r[1];
    double dz = c[2] - r[2];
    double d2 = dx * dx + dy * dy;
    d2 = d2 + dz * dz;
    return d2 < sigma2;
}

/*
 * Grow one hard-sphere chain: N beads, k trial directions per step, bond
 * length b, bead diameter sigma.  A candidate is tested against every bead
 * except the tip it is bonded to (beads 0 .. i-2 at step i).
 * Outputs as for the lattice; coordinates are doubles, r2 is a double and
 * rg2 = (1/g) sum_i |r_i - cm|^2 with cm = (sum_i r_i) / g.
 */
int oro_real_chain(uint64_t seed, uint64_t chain, int32_t N, int32_t k,
                   double b, double sigma, double *xyz, int32_t *m_seq,
                   double *log_w, int32_t *n_grown, double end[3], double *r2,
                   double *rg2, int32_t flags, int32_t *rounds)
{
    if (N < 1 || k < 1 || k > 64 || !(b > 0.0) || !(sigma >= 0.0)) return ORO_E_INVALID;
    double *pos = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    if (!pos) return ORO_E_NOMEM;
    double cand[64][3];
    int free_[64];
    double sigma2 = sigma * sigma;
    int64_t n_of_m[65];
    int32_t g;
    int dead;
    int status = ORO_OK;
    const uint32_t max_rounds = (flags & ORO_RESTART) ? MAX_ROUNDS : 1u;
    uint32_t round = 0;
    /* Restart rule as for the lattice. */
    for (;;) {
    pos[0] = 0.0; pos[1] = 0.0; pos[2] = 0.0;
    for (int q = 0; q <= 64; ++q) n_of_m[q] = 0;
    g = 1;
    dead = 0;
    if (m_seq) m_seq[0] = 0;

    for (int32_t i = 1; i < N && status == ORO_OK; ++i) {
        const double *tip = &pos[3 * (i - 1)];
        const uint32_t sw = (uint32_t)i | (round << 16); /* step word */
        uint32_t m = 0;
        for (int32_t t = 0; t < k; ++t) {
            double e[3];
            status = oro_unit_vector(seed, chain, sw, (uint32_t)t, e, NULL);
            if (status != ORO_OK) break;
            cand[t][0] = tip[0] + b * e[0];
            cand[t][1] = tip[1] + b * e[1];
            cand[t][2] = tip[2] + b * e[2];
            free_[t] = 1;
            for (int32_t j = 0; j <= i - 2; ++j) {
                if (oro_overlaps(cand[t], &pos[3 * j], sigma2)) free_[t] = 0;
            }
            m += (uint32_t)free_[t];
        }
        if (status != ORO_OK) break;
        if (m_seq) m_seq[i] = (int32_t)m;
        if (m == 0) {
            dead = 1;
            break;
        }
        uint32_t pick;
        status = pick_uniform(seed, chain, sw, m, &pick);
        if (status != ORO_OK) break;
        int chosen = -1;
        uint32_t seen = 0;
        for (int32_t t = 0; t < k; ++t) {
            if (free_[t]) {
                if (seen == pick) { chosen = t; break; }
                ++seen;
            }
        }
        pos[3 * i] = cand[chosen][0];
        pos[3 * i + 1] = cand[chosen][1];
        pos[3 * i + 2] = cand[chosen][2];
        g = i + 1;
        n_of_m[m] += 1;
    }
    if (status != ORO_OK || !dead || round + 1 >= max_rounds) break;
    ++round;
    }
    if (status != ORO_OK) {
        free(pos);
        return status;
    }
    if (rounds) *rounds = (int32_t)round + 1;
    double lw = log_weight(n_of_m, k);

    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int32_t i = 0; i < g; ++i) {
        sx = sx + pos[3 * i];
        sy = sy + pos[3 * i + 1];
        sz = sz + pos[3 * i + 2];
    }
    double cx = sx / (double)g, cy = sy / (double)g, cz = sz / (double)g;
    double acc = 0.0;
    for (int32_t i = 0; i < g; ++i) {
        double dx = pos[3 * i] - cx;
        double dy = pos[3 * i + 1] - cy;
        double dz = pos[3 * i + 2] - cz;
        double q = dx * dx + dy * dy;
        q = q + dz * dz;
        acc = acc + q;
    }
    double ex = pos[3 * (g - 1)], ey = pos[3 * (g - 1) + 1], ez = pos[3 * (g - 1) + 2];
    if (xyz) memcpy(xyz, pos, sizeof(double) * 3 * (size_t)g);
    if (log_w) *log_w = dead ? -INFINITY : lw;
    if (n_grown) *n_grown = g;
    if (end) { end[0] = ex; end[1] = ey; end[2] = ez; }
    if (r2) {
        double q = ex * ex + ey * ey;
        *r2 = q + ez * ez;
    }
    if (rg2) *rg2 = acc / (double)g;
    free(pos);
    return ORO_OK;
}

/* ------------------------------------------------------------------------ */
/* Batch drivers: chains chain_offset .. chain_offset + n - 1, written to     */
/* per-chain arrays (structure of arrays; r_end has 3 planes of n).  Every   */
/* output pointer may be NULL.                                               */
/* ------------------------------------------------------------------------ */
int oro_gen_lattice(uint64_t seed, uint64_t chain_offset, uint64_t n, int32_t N,
                    double *log_w, uint64_t *w_exact, int32_t *w_exact_ok,
                    int32_t *r_end, int64_t *r2, int64_t *n2rg2, double *rg2,
                    int32_t *n_grown, int32_t flags)
{
    for (uint64_t c = 0; c < n; ++c) {
        double lw, rg;
        uint64_t we;
        int32_t ok, g, e[3];
        int64_t rr, nn;
        int s = oro_lattice_chain(seed, chain_offset + c, N, NULL, NULL, &lw, &we, &ok,
                                  &g, e, &rr, &nn, &rg, flags, NULL);
        if (s != ORO_OK) return s;
        if (log_w) log_w[c] = lw;
        if (w_exact) w_exact[c] = we;
        if (w_exact_ok) w_exact_ok[c] = ok;
        if (r_end) { r_end[c] = e[0]; r_end[n + c] = e[1]; r_end[2 * n + c] = e[2]; }
        if (r2) r2[c] = rr;
        if (n2rg2) n2rg2[c] = nn;
        if (rg2) rg2[c] = rg;
        if (n_grown) n_grown[c] = g;
    }
    return ORO_OK;
}

int oro_gen_real(uint64_t seed, uint64_t chain_offset, uint64_t n, int32_t N, int32_t k,
                 double b, double sigma, double *log_w, double *r_end, double *r2,
                 double *rg2, int32_t *n_grown, int32_t flags)
{
    for (uint64_t c = 0; c < n; ++c) {
        double lw, e[3], rr, rg;
        int32_t g;
        int s = oro_real_chain(seed, chain_offset + c, N, k, b, sigma, NULL, NULL, &lw, &g,
                               e, &rr, &rg, flags, NULL);
        if (s != ORO_OK) return s;
        if (log_w) log_w[c] = lw;
        if (r_end) { r_end[c] = e[0]; r_end[n + c] = e[1]; r_end[2 * n + c] = e[2]; }
        if (r2) r2[c] = rr;
        if (rg2) rg2[c] = rg;
        if (n_grown) n_grown[c] = g;
    }
    return ORO_OK;
}

/* ------------------------------------------------------------------------ */
/* Reductions: Eq. (2) weighted averages and Eq. (6) mean weight.            */
/* ------------------------------------------------------------------------ */
typedef struct {
    double sum, comp;
} neumaier;

static void nm_add(neumaier *a, double x)
{
    double t = a->sum + x;
    if (fabs(a->sum) >= fabs(x))
        a->comp += (a->sum - t) + x;
    else
        a->comp += (x - t) + a->sum;
    a->sum = t;
}

static double nm_val(const neumaier *a) { return a->sum + a->comp; }

/* Output layout of oro_reduce (all doubles):
 *  [0]  M (chains)            [1]  alive chains        [2]  L = max log W
 *  [3]  S0 = sum w            [4]  S2 = sum w^2         w = exp(log W - L)
 *  [5]  sum w R2              [6]  sum w^2 R2           [7]  sum w^2 R2^2
 *  [8]  sum w Rg2             [9]  sum w^2 Rg2          [10] sum w^2 Rg2^2
 *  [11] log c estimate = L + log(S0 / M)
 *  [12] relative std. error of the c estimate
 *  [13] <R2>   [14] its std. error   [15] <Rg2>   [16] its std. error
 *  [17] effective sample size S0^2 / S2
 *  [18] steps executed = sum (n_grown - 1)
 * hist_w[bins] and hist_n[bins] (optional): W-weighted (w) and plain counts
 * of live chains by R2 bin floor(R2 * bins / (n^2 + 1)), n = N - 1.
 */
void oro_reduce(uint64_t M, int32_t N, const double *log_w, const double *r2,
                const double *rg2, const int32_t *n_grown, int32_t bins,
                double *out, double *hist_w, uint64_t *hist_n)
{
    double L = -INFINITY;
    uint64_t alive = 0;
    double steps = 0.0;
    for (uint64_t c = 0; c < M; ++c) {
        if (log_w[c] > -INFINITY) {
            ++alive;
            if (log_w[c] > L) L = log_w[c];
        }
        steps += (double)(n_grown[c] - 1);
    }
    neumaier s0 = {0, 0}, s2 = {0, 0}, a1 = {0, 0}, a2 = {0, 0}, a3 = {0, 0},
             g1 = {0, 0}, g2 = {0, 0}, g3 = {0, 0};
    neumaier *hb = NULL;
    if (bins > 0 && hist_w) {
        hb = (neumaier *)calloc((size_t)bins, sizeof(neumaier));
    }
    if (bins > 0 && hist_n) {
        for (int32_t b = 0; b < bins; ++b) hist_n[b] = 0;
    }
    double nsq1 = (double)(N - 1) * (double)(N - 1) + 1.0;
    for (uint64_t c = 0; c < M; ++c) {
        if (!(log_w[c] > -INFINITY)) continue;
        double w = exp(log_w[c] - L);
        double ww = w * w;
        nm_add(&s0, w);
        nm_add(&s2, ww);
        nm_add(&a1, w * r2[c]);
        nm_add(&a2, ww * r2[c]);
        nm_add(&a3, ww * r2[c] * r2[c]);
        nm_add(&g1, w * rg2[c]);
        nm_add(&g2, ww * rg2[c]);
        nm_add(&g3, ww * rg2[c] * rg2[c]);
        if (bins > 0) {
            double q = floor((r2[c] * (double)bins) / nsq1);
            int32_t bin = q < 0.0 ? 0 : (q >= (double)bins ? bins - 1 : (int32_t)q);
            if (hb) nm_add(&hb[bin], w);
            if (hist_n) hist_n[bin] += 1;
        }
    }
    double S0 = nm_val(&s0), S2 = nm_val(&s2);
    double A1 = nm_val(&a1), A2 = nm_val(&a2), A3 = nm_val(&a3);
    double G1 = nm_val(&g1), G2 = nm_val(&g2), G3 = nm_val(&g3);
    out[0] = (double)M;
    out[1] = (double)alive;
    out[2] = L;
    out[3] = S0; out[4] = S2;
    out[5] = A1; out[6] = A2; out[7] = A3;
    out[8] = G1; out[9] = G2; out[10] = G3;
    out[11] = (alive > 0) ? L + log(S0 / (double)M) : -INFINITY;
    out[12] = (alive > 0 && M > 1)
                  ? sqrt(((double)M * S2 / (S0 * S0) - 1.0) / ((double)M - 1.0))
                  : NAN;
    double mr = A1 / S0, mg = G1 / S0;
    out[13] = (alive > 0) ? mr : NAN;
    out[14] = (alive > 0) ? sqrt(fabs(A3 - 2.0 * mr * A2 + mr * mr * S2)) / S0 : NAN;
    out[15] = (alive > 0) ? mg : NAN;
    out[16] = (alive > 0) ? sqrt(fabs(G3 - 2.0 * mg * G2 + mg * mg * S2)) / S0 : NAN;
    out[17] = (alive > 0) ? S0 * S0 / S2 : 0.0;
    out[18] = steps;
    if (hb) {
        for (int32_t b = 0; b < bins; ++b) hist_w[b] = nm_val(&hb[b]);
        free(hb);
    }
}

/* Exact integer sums for lattice chains whose W fits in 64 bits:
 * out128[0..1] = sum W, [2..3] = sum W R2, [4..5] = sum W n2rg2 as (lo, hi). */
void oro_reduce_exact(uint64_t M, const uint64_t *w_exact, const int64_t *r2,
                      const int64_t *n2rg2, uint64_t out128[6])
{
    unsigned __int128 sw = 0, swr = 0, swg = 0;
    for (uint64_t c = 0; c < M; ++c) {
        unsigned __int128 w = w_exact[c];
        sw += w;
        swr += w * (unsigned __int128)(uint64_t)r2[c];
        swg += w * (unsigned __int128)(uint64_t)n2rg2[c];
    }
    out128[0] = (uint64_t)sw; out128[1] = (uint64_t)(sw >> 64);
    out128[2] = (uint64_t)swr; out128[3] = (uint64_t)(swr >> 64);
    out128[4] = (uint64_t)swg; out128[5] = (uint64_t)(swg >> 64);
}
