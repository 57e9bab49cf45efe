/*
 * Driver for a sanitizer build of the oracle (AddressSanitizer and
 * UndefinedBehaviorSanitizer, host only): runs every oracle entry point over
 * the edge cases of its arguments (one monomer, empty ensembles, dead ends,
 * restarts, the 26-neighbour lattice, k = 1 and 64, sigma = 0, all-dead and
 * single-live reductions, histograms) and checks a few invariants.  Any
 * out-of-bounds access, leak, overflow or other undefined behaviour aborts
 * the run with a report.  Prints "ok" on success.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oro_philox4x32_10(const uint32_t ctr_in[4], uint64_t seed, uint32_t out[4]);
int oro_lemire16(uint32_t x, uint32_t m, uint32_t *index);
int oro_pick(uint64_t seed, uint64_t chain, uint32_t step, uint32_t m, uint32_t *index, uint32_t *redraws);
int oro_lattice_chain(uint64_t seed, uint64_t chain, int32_t N, int32_t *xyz, int32_t *m_seq, double *log_w,
                      uint64_t *w_exact, int32_t *w_exact_ok, int32_t *n_grown, int32_t end[3], int64_t *r2,
                      int64_t *n2rg2, double *rg2, int32_t flags, int32_t *rounds);
int oro_unit_vector(uint64_t seed, uint64_t chain, uint32_t step, uint32_t t, double e[3], uint32_t *attempts);
int oro_overlaps(const double c[3], const double r[3], double sigma2);
int oro_real_chain(uint64_t seed, uint64_t chain, int32_t N, int32_t k, double b, double sigma, double *xyz,
                   int32_t *m_seq, double *log_w, int32_t *n_grown, double end[3], double *r2, double *rg2,
                   int32_t flags, int32_t *rounds);
int oro_gen_lattice(uint64_t seed, uint64_t chain_offset, uint64_t n, int32_t N, double *log_w, uint64_t *w_exact,
                    int32_t *w_exact_ok, int32_t *r_end, int64_t *r2, int64_t *n2rg2, double *rg2,
                    int32_t *n_grown, int32_t flags);
int oro_gen_real(uint64_t seed, uint64_t chain_offset, uint64_t n, int32_t N, int32_t k, double b, double sigma,
                 double *log_w, double *r_end, double *r2, double *rg2, int32_t *n_grown, int32_t flags);
void oro_reduce(uint64_t M, int32_t N, const double *log_w, const double *r2, const double *rg2,
                const int32_t *n_grown, int32_t bins, double *out, double *hist_w, uint64_t *hist_n);
void oro_reduce_exact(uint64_t M, const uint64_t *w_exact, const int64_t *r2, const int64_t *n2rg2,
                      uint64_t out128[6]);

#define RESTART 2
#define Z26 4

static int failures = 0;
#define CHECK(cond)                                                                  \
    do {                                                                             \
        if (!(cond)) {                                                               \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                              \
        }                                                                            \
    } while (0)

static void lattice_ensemble(uint64_t seed, uint64_t off, uint64_t n, int32_t N, int32_t flags, int32_t bins)
{
    double *lw = malloc(sizeof(double) * (n + 1)), *rg = malloc(sizeof(double) * (n + 1));
    uint64_t *we = malloc(sizeof(uint64_t) * (n + 1));
    int32_t *ok = malloc(sizeof(int32_t) * (n + 1)), *ng = malloc(sizeof(int32_t) * (n + 1));
    int32_t *end = malloc(sizeof(int32_t) * 3 * (n + 1));
    int64_t *r2 = malloc(sizeof(int64_t) * (n + 1)), *nn = malloc(sizeof(int64_t) * (n + 1));
    double *r2d = malloc(sizeof(double) * (n + 1));
    double out[19];
    double *hw = bins ? malloc(sizeof(double) * bins) : NULL;
    uint64_t *hn = bins ? malloc(sizeof(uint64_t) * bins) : NULL;
    CHECK(oro_gen_lattice(seed, off, n, N, lw, we, ok, end, r2, nn, rg, ng, flags) == 0);
    for (uint64_t c = 0; c < n; ++c) {
        r2d[c] = (double)r2[c];
        CHECK(ng[c] >= 1 && ng[c] <= N);
        CHECK((ng[c] == N) == (lw[c] > -INFINITY));
        CHECK(r2[c] >= 0 && nn[c] >= 0);
    }
    oro_reduce(n, N, lw, r2d, rg, ng, bins, out, hw, hn);
    uint64_t ex[6];
    oro_reduce_exact(n, we, r2, nn, ex);
    /* also the NULL-output form of the batch driver */
    CHECK(oro_gen_lattice(seed, off, n, N, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, flags) == 0);
    free(lw); free(rg); free(we); free(ok); free(ng); free(end); free(r2); free(nn); free(r2d);
    free(hw); free(hn);
}

static void real_ensemble(uint64_t seed, uint64_t off, uint64_t n, int32_t N, int32_t k, double b, double sigma,
                          int32_t flags, int32_t bins)
{
    double *lw = malloc(sizeof(double) * (n + 1)), *rg = malloc(sizeof(double) * (n + 1));
    double *end = malloc(sizeof(double) * 3 * (n + 1)), *r2 = malloc(sizeof(double) * (n + 1));
    int32_t *ng = malloc(sizeof(int32_t) * (n + 1));
    double out[19];
    double *hw = bins ? malloc(sizeof(double) * bins) : NULL;
    uint64_t *hn = bins ? malloc(sizeof(uint64_t) * bins) : NULL;
    CHECK(oro_gen_real(seed, off, n, N, k, b, sigma, lw, end, r2, rg, ng, flags) == 0);
    for (uint64_t c = 0; c < n; ++c) {
        CHECK(ng[c] >= 1 && ng[c] <= N);
        CHECK(r2[c] >= 0.0 && rg[c] >= 0.0);
    }
    oro_reduce(n, N, lw, r2, rg, ng, bins, out, hw, hn);
    free(lw); free(rg); free(end); free(r2); free(ng); free(hw); free(hn);
}

int main(void)
{
    /* Philox, Lemire, pick, unit vector, overlap rule */
    uint32_t ctr[4] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, out[4];
    oro_philox4x32_10(ctr, UINT64_MAX, out);
    uint32_t idx = 0, rej = 0;
    for (uint32_t m = 1; m <= 64; ++m)
        for (uint32_t x = 0; x < 65536; x += 97) (void)oro_lemire16(x, m, &idx);
    for (uint32_t m = 1; m <= 26; ++m) {
        CHECK(oro_pick(3, UINT64_MAX - 1, 0xFFFFu | (7u << 16), m, &idx, &rej) == 0);
        CHECK(idx < m);
    }
    double e[3];
    uint32_t att = 0;
    for (uint32_t t = 0; t < 64; ++t) CHECK(oro_unit_vector(9, (1ull << 40) + t, 5, t, e, &att) == 0);
    const double c0[3] = {0.0, 0.0, 0.0}, c1[3] = {1.0, 0.0, 0.0};
    CHECK(!oro_overlaps(c0, c1, 1.0));
    CHECK(oro_overlaps(c0, c1, 1.0000001));

    /* single chains with every output, N = 1 upwards */
    int32_t xyz[3 * 300], mseq[300], g, ok, rounds, iend[3];
    double dxyz[3 * 300], lw, rg, dend[3], r2d;
    uint64_t we;
    int64_t r2, nn;
    for (int32_t N = 1; N <= 300; N += (N < 8 ? 1 : 37)) {
        for (int32_t fl = 0; fl < 8; fl += 2) {
            if ((fl & Z26) && N > 14 && (fl & RESTART)) continue;
            CHECK(oro_lattice_chain(1, (uint64_t)N, N, xyz, mseq, &lw, &we, &ok, &g, iend, &r2, &nn, &rg, fl,
                                    &rounds) == 0);
        }
        for (int32_t k = 1; k <= 64; k += 21) {
            CHECK(oro_real_chain(2, (uint64_t)N, N, k, 1.0, 1.0, dxyz, mseq, &lw, &g, dend, &r2d, &rg, 0,
                                 &rounds) == 0);
            CHECK(oro_real_chain(2, (uint64_t)N, N, k, 1.5, 0.0, dxyz, mseq, &lw, &g, dend, &r2d, &rg, 0,
                                 &rounds) == 0);
        }
    }
    /* argument errors are reported, not crashed on */
    CHECK(oro_lattice_chain(1, 0, 0, NULL, NULL, &lw, &we, &ok, &g, iend, &r2, &nn, &rg, 0, NULL) != 0);
    CHECK(oro_real_chain(1, 0, 4, 65, 1.0, 1.0, NULL, NULL, &lw, &g, dend, &r2d, &rg, 0, NULL) != 0);
    CHECK(oro_real_chain(1, 0, 4, 8, 0.0, 1.0, NULL, NULL, &lw, &g, dend, &r2d, &rg, 0, NULL) != 0);

    /* ensembles: empty, ragged, dead ends, restarts, z = 26, exact weights */
    lattice_ensemble(1, 0, 0, 16, 0, 16);
    lattice_ensemble(1, 0, 2000, 16, 0, 0);
    lattice_ensemble(11, 5, 3000, 64, 0, 256);        /* some trapped chains */
    lattice_ensemble(12, 1ull << 33, 300, 64, RESTART, 32);
    lattice_ensemble(13, 0, 500, 14, Z26, 8);
    lattice_ensemble(14, 0, 100, 130, Z26 | RESTART, 8);
    lattice_ensemble(15, 0, 10, 1, 0, 4);
    real_ensemble(1, 0, 0, 16, 8, 1.0, 1.0, 0, 16);
    real_ensemble(2, 7, 500, 40, 4, 1.0, 1.4, 0, 64);  /* frequent dead ends */
    real_ensemble(3, 0, 300, 20, 4, 1.0, 1.4, RESTART, 8);
    real_ensemble(4, 0, 100, 3, 1, 1.0, 1.0, 0, 4);
    real_ensemble(5, 0, 50, 30, 64, 1.0, 0.0, 0, 0);
    real_ensemble(6, 0, 40, 2, 8, 1.0, 1.0, 0, 256);
    /* reductions: all dead, one live chain, single chain */
    {
        double l[3] = {-INFINITY, -INFINITY, -INFINITY}, a[3] = {1, 2, 3}, b2[3] = {0.5, 0.5, 0.5}, o[19];
        int32_t gg[3] = {2, 3, 1};
        double hw[8];
        uint64_t hn[8];
        oro_reduce(3, 5, l, a, b2, gg, 8, o, hw, hn);
        CHECK(o[1] == 0.0);
        l[1] = 4.0;
        gg[1] = 5;
        oro_reduce(3, 5, l, a, b2, gg, 8, o, hw, hn);
        CHECK(o[1] == 1.0);
        oro_reduce(1, 5, l + 1, a, b2, gg + 1, 0, o, NULL, NULL);
    }
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}
