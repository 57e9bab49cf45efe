/*
 * Brute-force enumeration of self-avoiding walks on the simple cubic lattice,
 * used to pin the oracle (test infrastructure; independent of the oracle's
 * code).  For n steps it walks every SAW by depth-first search on an
 * occupancy grid and reports
 *   c_n                    number of n-step SAWs
 *   sum R^2                over all SAWs (end-to-end distance squared)
 *   sum N^2 Rg^2           over all SAWs, N = n + 1 monomers, computed as the
 *                          pair sum  sum_{i<j} |r_i - r_j|^2
 *   for every SAW its Rosenbluth weight W = prod m_i, where m_i is the number
 *   of unoccupied neighbours of the tip before step i (Eq. 3): a histogram
 *   {W: number of SAWs with that W}
 *   for every trapped prefix (a walk whose tip has no free neighbour before
 *   step i <= n) the product of m over its steps: a histogram
 *   {(i, product): count}
 *
 * Rosenbluth growth reaches a complete SAW with probability 1/W and a trapped
 * prefix with probability 1/product, so these histograms give the exact law
 * of the weight and the exact attrition probability.
 *
 * Output: one "key value..." line per quantity, parsed by the tests.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#define MAXN 14
#define G (2 * MAXN + 3)
static unsigned char occ[G][G][G];
static int px[MAXN + 1], py[MAXN + 1], pz[MAXN + 1];
static int nsteps;
static int origin;
static uint64_t count;
static uint64_t sum_r2, sum_n2rg2;

#define HCAP 200000
static uint64_t hw_key[HCAP], hw_cnt[HCAP];
static int hw_len;
static uint64_t ht_key[HCAP], ht_cnt[HCAP];
static int ht_step[HCAP];
static int ht_len;

static const int D[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};

static void add_w(uint64_t w)
{
    for (int i = 0; i < hw_len; ++i)
        if (hw_key[i] == w) { hw_cnt[i]++; return; }
    if (hw_len >= HCAP) { fprintf(stderr, "histogram full\n"); exit(2); }
    hw_key[hw_len] = w; hw_cnt[hw_len] = 1; hw_len++;
}

static void add_trap(int step, uint64_t w)
{
    for (int i = 0; i < ht_len; ++i)
        if (ht_key[i] == w && ht_step[i] == step) { ht_cnt[i]++; return; }
    if (ht_len >= HCAP) { fprintf(stderr, "trap histogram full\n"); exit(2); }
    ht_key[ht_len] = w; ht_step[ht_len] = step; ht_cnt[ht_len] = 1; ht_len++;
}

static void dfs(int i, uint64_t w)
{
    /* monomers 0..i-1 are placed; place monomer i */
    if (i > nsteps) {
        count++;
        int64_t x = px[nsteps] - origin, y = py[nsteps] - origin, z = pz[nsteps] - origin;
        sum_r2 += (uint64_t)(x * x + y * y + z * z);
        int64_t pair = 0;
        for (int a = 0; a <= nsteps; ++a)
            for (int b = a + 1; b <= nsteps; ++b) {
                int64_t dx = px[a] - px[b], dy = py[a] - py[b], dz = pz[a] - pz[b];
                pair += dx * dx + dy * dy + dz * dz;
            }
        sum_n2rg2 += (uint64_t)pair;
        add_w(w);
        return;
    }
    int tx = px[i - 1], ty = py[i - 1], tz = pz[i - 1];
    int m = 0;
    for (int d = 0; d < 6; ++d)
        if (!occ[tx + D[d][0]][ty + D[d][1]][tz + D[d][2]]) m++;
    if (m == 0) {
        add_trap(i, w);
        return;
    }
    for (int d = 0; d < 6; ++d) {
        int x = tx + D[d][0], y = ty + D[d][1], z = tz + D[d][2];
        if (occ[x][y][z]) continue;
        occ[x][y][z] = 1;
        px[i] = x; py[i] = y; pz[i] = z;
        dfs(i + 1, w * (uint64_t)m);
        occ[x][y][z] = 0;
    }
}

int main(int argc, char **argv)
{
    if (argc < 2) { fprintf(stderr, "usage: saw_enum n_steps\n"); return 1; }
    nsteps = atoi(argv[1]);
    if (nsteps < 0 || nsteps > MAXN) { fprintf(stderr, "n out of range\n"); return 1; }
    int o = MAXN + 1;
    origin = o;
    px[0] = o; py[0] = o; pz[0] = o;
    occ[o][o][o] = 1;
    dfs(1, 1);
    printf("n %d\n", nsteps);
    printf("c %llu\n", (unsigned long long)count);
    printf("sum_r2 %llu\n", (unsigned long long)sum_r2);
    printf("sum_n2rg2 %llu\n", (unsigned long long)sum_n2rg2);
    for (int i = 0; i < hw_len; ++i)
        printf("w %llu %llu\n", (unsigned long long)hw_key[i], (unsigned long long)hw_cnt[i]);
    for (int i = 0; i < ht_len; ++i)
        printf("trap %d %llu %llu\n", ht_step[i], (unsigned long long)ht_key[i],
               (unsigned long long)ht_cnt[i]);
    return 0;
}
