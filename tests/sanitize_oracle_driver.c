/*
 * Drives every entry point of the FP64 oracle (oracle/stdecomp_oracle.c) on
 * small seeded problems, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_oracle_sanitized.py).  Inputs come
 * from a plain linear congruential generator; the checks here are only that
 * every call succeeds or rejects bad arguments, that sample orders are
 * permutations and that results are finite -- the values themselves are
 * pinned by the Python tests.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_perm(int64_t T, uint64_t seed, int64_t epoch, int64_t *out);
int orc_segments(int64_t m, const int32_t *rows, int32_t *sigma, int32_t *seg_off, int32_t *seg_row,
                 int32_t *nseg);
int orc_predict(int N, const int64_t *dims, const int32_t *ranks, const double *A, const double *G, int64_t q,
                const int32_t *idx, double *out);
int orc_loss(int N, const int64_t *dims, const int32_t *ranks, const double *A, const double *G, int64_t q,
             const int32_t *idx, const float *vals, double lam_A, double lam_G, double *out);
int orc_run(int N, const int64_t *dims, const int32_t *ranks, double *A, double *G, int64_t T, const int32_t *idx,
            const float *vals, int64_t M, double gam_A, double lam_A, double gam_G, double lam_G,
            const int64_t *perm, uint64_t seed, int64_t epoch0, int64_t n_epochs, int64_t max_batches,
            int64_t *batches_run);
int orc_run_momentum(int N, const int64_t *dims, const int32_t *ranks, double *A, double *G, double *VA,
                     double *VG, int64_t T, const int32_t *idx, const float *vals, int64_t M, double gam_A,
                     double lam_A, double gam_G, double lam_G, double mu, const int64_t *perm, uint64_t seed,
                     int64_t epoch0, int64_t n_epochs, int64_t max_batches, int64_t *batches_run);
int orc_kruskal_core(int N, const int32_t *ranks, int R, const double *B, double *G);
int orc_run_kruskal(int N, const int64_t *dims, const int32_t *ranks, double *A, int R, double *B, double *G,
                    int64_t T, const int32_t *idx, const float *vals, int64_t M, double gam_A, double lam_A,
                    double gam_B, double lam_B, const int64_t *perm, uint64_t seed, int64_t epoch0,
                    int64_t n_epochs, int64_t max_batches, int64_t *batches_run);

static uint64_t lcg = 12345;
static double unif(void)
{
    lcg = lcg * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

static int fails = 0;
#define CHECK(c)                                                           \
    do {                                                                   \
        if (!(c)) {                                                        \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            fails++;                                                       \
        }                                                                  \
    } while (0)

static int all_finite(const double *x, int64_t n)
{
    for (int64_t i = 0; i < n; i++)
        if (!isfinite(x[i])) return 0;
    return 1;
}

int main(void)
{
    /* sample orders */
    const int64_t Ts[] = {1, 2, 3, 17, 1000, 4099};
    for (int c = 0; c < 6; c++) {
        int64_t T = Ts[c];
        int64_t *p = malloc(sizeof(int64_t) * T);
        char *seen = calloc(T, 1);
        CHECK(orc_perm(T, 77 + c, c, p) == 0);
        for (int64_t i = 0; i < T; i++) {
            CHECK(p[i] >= 0 && p[i] < T);
            if (p[i] >= 0 && p[i] < T) seen[p[i]]++;
        }
        for (int64_t i = 0; i < T; i++) CHECK(seen[i] == 1);
        free(p);
        free(seen);
    }
    CHECK(orc_perm(0, 1, 0, NULL) != 0);

    /* segments, including the empty minibatch */
    {
        int32_t rows[9] = {4, 1, 4, 4, 0, 1, 7, 0, 4}, sigma[9], off[10], srow[9], nseg = -1;
        CHECK(orc_segments(9, rows, sigma, off, srow, &nseg) == 0);
        CHECK(nseg == 4 && off[0] == 0 && off[nseg] == 9);
        CHECK(orc_segments(0, NULL, NULL, NULL, NULL, &nseg) == 0 && nseg == 0);
    }

    /* dense-core epochs, orders 2..5, ragged last minibatch */
    for (int N = 2; N <= 5; N++) {
        int64_t dims[8];
        int32_t ranks[8];
        int64_t nA = 0, P = 1;
        for (int n = 0; n < N; n++) {
            dims[n] = 5 + 3 * n;
            ranks[n] = 1 + (n % 3);
            nA += dims[n] * ranks[n];
            P *= ranks[n];
        }
        const int64_t T = 211;
        int32_t *idx = malloc(sizeof(int32_t) * N * T);
        float *vals = malloc(sizeof(float) * T);
        double *A = malloc(sizeof(double) * nA), *G = malloc(sizeof(double) * P);
        for (int n = 0; n < N; n++)
            for (int64_t t = 0; t < T; t++) idx[n * T + t] = (int32_t)(unif() * dims[n]);
        for (int64_t t = 0; t < T; t++) vals[t] = (float)(unif() - 0.5);
        for (int64_t i = 0; i < nA; i++) A[i] = unif() - 0.5;
        for (int64_t i = 0; i < P; i++) G[i] = unif() - 0.5;
        int64_t done = -1;
        CHECK(orc_run(N, dims, ranks, A, G, T, idx, vals, 16, 0.05, 0.01, 0.05, 0.01, NULL, 3, 0, 2, -1, &done) == 0);
        CHECK(done == 2 * ((T + 15) / 16));
        CHECK(all_finite(A, nA) && all_finite(G, P));
        double *pred = malloc(sizeof(double) * T), loss[4];
        CHECK(orc_predict(N, dims, ranks, A, G, T, idx, pred) == 0 && all_finite(pred, T));
        CHECK(orc_loss(N, dims, ranks, A, G, T, idx, vals, 0.01, 0.01, loss) == 0 && all_finite(loss, 4));
        /* heavy-ball momentum; mu outside [0, 1) rejected */
        double *VA = calloc((size_t)nA, sizeof(double)), *VG = calloc((size_t)P, sizeof(double));
        CHECK(orc_run_momentum(N, dims, ranks, A, G, VA, VG, T, idx, vals, 16, 0.05, 0.01, 0.05, 0.01, 0.9, NULL,
                               3, 2, 1, -1, &done) == 0);
        CHECK(done == (T + 15) / 16);
        CHECK(all_finite(A, nA) && all_finite(G, P) && all_finite(VA, nA) && all_finite(VG, P));
        CHECK(orc_run_momentum(N, dims, ranks, A, G, VA, VG, T, idx, vals, 16, 0.05, 0.01, 0.05, 0.01, 1.0, NULL,
                               3, 2, 1, -1, &done) != 0);
        free(VA);
        free(VG);
        idx[0] = (int32_t)dims[0]; /* out of range: rejected */
        CHECK(orc_predict(N, dims, ranks, A, G, T, idx, pred) != 0);
        free(pred);
        /* Kruskal core, R = 1..3 */
        for (int R = 1; R <= 3; R++) {
            idx[0] = 0;
            int64_t nB = 0;
            for (int n = 0; n < N; n++) nB += (int64_t)ranks[n] * R;
            double *B = malloc(sizeof(double) * nB);
            for (int64_t i = 0; i < nB; i++) B[i] = unif() - 0.5;
            CHECK(orc_kruskal_core(N, ranks, R, B, G) == 0 && all_finite(G, P));
            CHECK(orc_run_kruskal(N, dims, ranks, A, R, B, G, T, idx, vals, 32, 0.05, 0.01, 0.05, 0.01, NULL, 5,
                                  0, 1, -1, &done) == 0);
            CHECK(all_finite(A, nA) && all_finite(B, nB) && all_finite(G, P));
            free(B);
        }
        free(idx);
        free(vals);
        free(A);
        free(G);
    }
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("SANITIZED_ORACLE_OK\n");
    return 0;
}
