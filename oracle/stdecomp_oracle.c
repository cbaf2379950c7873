/*
 * stdecomp_oracle.c -- plain, slow, single-threaded FP64 CPU oracle for the
 * SGD_Tucker minibatch update (sparse Tucker decomposition fitted by SGD).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code with the GPU library.
 *
 * Every function states the passage of the paper (arXiv 2012.03550,
 * "SGD_Tucker: A Novel Stochastic Optimization Strategy for Parallel Sparse
 * Tucker Decomposition") it follows.  Readings of silent or ambiguous passages
 * are marked READING and listed in the design notes of the repository.
 *
 * Conventions (0-based):
 *   - N modes, mode sizes I[n], core ranks J[n], P = prod_n J[n].
 *   - Factor matrices A(n) are I[n] x J[n], row-major, stored back to back in
 *     one array: A(n) starts at offset sum_{k<n} I[k]*J[k].
 *   - The core G is stored flat with j_0 fastest: lin(j) = sum_n j_n prod_{k<n} J[k]
 *     (Definition "Tensor Unfolding" applied to G, then "Vectorization").
 *   - The mode-n unfolding G_(n)[j_n, col] with
 *     col = sum_{k != n} j_k prod_{k' < k, k' != n} J[k'] (lowest mode fastest),
 *     which is the column order of S(n) = A(N) (x) ... (x) A(n+1) (x) A(n-1) (x) ... (x) A(1)
 *     (Section "Optimization Process for Factor Matrices", Eq. optimization_for_factor).
 *   - COO indices are SoA: idx[n*T + t] is i_n of entry t.
 *
 * Parity status of each function is documented in its comment; all are pinned
 * by tests (finite differences, brute-force reconstruction, planted models,
 * closed forms, the paper's worked examples) except where it says otherwise.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_MAXN 8

/* ------------------------------------------------------------------------ */
/* Sampler.                                                                  */
/* The paper draws the minibatch Psi "randomly" from Omega (Eq. SGD and the   */
/* SGD solutions of Section "Stochastic Optimization") without fixing how.   */
/* READING: an epoch is one pass over Omega without replacement in the order */
/* of a keyed pseudo-random permutation pi_e of [0, T).  pi_e is a 4-round    */
/* balanced Feistel network on 2h-bit words (Luby-Rackoff construction) made */
/* a permutation of [0, T) by cycle walking (Black and Rogaway, "Ciphers     */
/* with Arbitrary Finite Domains", 2002).  The round function and the key    */
/* schedule use the SplitMix64 output function (Steele, Lea and Flood,       */
/* "Fast Splittable Pseudorandom Number Generators", OOPSLA 2014).           */
/* ------------------------------------------------------------------------ */

/* SplitMix64: advance the state by the golden-ratio increment, then mix. */
uint64_t orc_sm64(uint64_t state)
{
    uint64_t z = state + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Half width h (>= 1) of the Feistel words: the smallest h with 4^h >= T. */
int orc_feistel_half_bits(int64_t T)
{
    int h = 1;
    while (h < 31 && ((uint64_t)1 << (2 * h)) < (uint64_t)T) h++;
    return h;
}

/* Round key r of epoch e. */
uint64_t orc_round_key(uint64_t seed, int64_t epoch, int r)
{
    return orc_sm64(seed ^ orc_sm64((uint64_t)(4 * epoch + r)));
}

static uint64_t feistel_encrypt(uint64_t x, int h, const uint64_t key[4])
{
    uint64_t mask = ((uint64_t)1 << h) - 1;
    uint64_t L = x >> h, R = x & mask;
    for (int r = 0; r < 4; r++) {
        uint64_t F = orc_sm64(R ^ key[r]) & mask;
        uint64_t newR = L ^ F;
        L = R;
        R = newR;
    }
    return (L << h) | R;
}

/* pi_e(q) for every q in [0, T): the first Feistel iterate of q that is < T. */
int orc_perm(int64_t T, uint64_t seed, int64_t epoch, int64_t *out)
{
    if (T < 1 || !out) return ORC_EINVAL;
    int h = orc_feistel_half_bits(T);
    uint64_t key[4];
    for (int r = 0; r < 4; r++) key[r] = orc_round_key(seed, epoch, r);
    for (int64_t q = 0; q < T; q++) {
        uint64_t y = feistel_encrypt((uint64_t)q, h, key);
        while (y >= (uint64_t)T) y = feistel_encrypt(y, h, key);
        out[q] = (int64_t)y;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Per-row segments of a minibatch (the sets (Psi_M^(n))_{i_n} of Eq.        */
/* SGD_factor_matrix; Algorithm 1 loops over them row by row).               */
/* READING: the order inside a row is the position in the minibatch, so the  */
/* key (i_n, position) is unique and the sorted order is unique.             */
/* ------------------------------------------------------------------------ */
static const int32_t *g_sort_rows; /* qsort has no context argument */

static int cmp_row_pos(const void *a, const void *b)
{
    int32_t pa = *(const int32_t *)a, pb = *(const int32_t *)b;
    int32_t ra = g_sort_rows[pa], rb = g_sort_rows[pb];
    if (ra != rb) return ra < rb ? -1 : 1;
    return pa < pb ? -1 : (pa > pb ? 1 : 0);
}

/* rows[p] = i_n of sample p.  Writes sigma (positions sorted by (row, p)),
 * the segment offsets seg_off[0..nseg], the row of each segment and nseg. */
int orc_segments(int64_t m, const int32_t *rows, int32_t *sigma,
                 int32_t *seg_off, int32_t *seg_row, int32_t *nseg)
{
    if (m < 0 || (m > 0 && (!rows || !sigma || !seg_off || !seg_row)) || !nseg)
        return ORC_EINVAL;
    for (int64_t p = 0; p < m; p++) sigma[p] = (int32_t)p;
    g_sort_rows = rows;
    if (m > 0) qsort(sigma, (size_t)m, sizeof(int32_t), cmp_row_pos);
    int32_t d = 0;
    for (int64_t q = 0; q < m; q++) {
        if (q == 0 || rows[sigma[q]] != rows[sigma[q - 1]]) {
            seg_off[d] = (int32_t)q;
            seg_row[d] = rows[sigma[q]];
            d++;
        }
    }
    if (m > 0) seg_off[d] = (int32_t)m;
    else if (seg_off) seg_off[0] = 0;
    *nseg = d;
    return ORC_OK;
}

/* Column of X^(n) that holds tensor entry (i_0..i_{N-1}) (Definition "Tensor
 * Unfolding", written 0-based: col = sum_{k != n} i_k prod_{k' < k, k' != n} I[k']). */
int64_t orc_unfold_col(int N, const int64_t *dims, const int64_t *index, int n)
{
    int64_t col = 0, stride = 1;
    for (int k = 0; k < N; k++) {
        if (k == n) continue;
        col += index[k] * stride;
        stride *= dims[k];
    }
    return col;
}

/* ------------------------------------------------------------------------ */
/* Model helpers.                                                            */
/* ------------------------------------------------------------------------ */
static int check_model(int N, const int64_t *dims, const int32_t *ranks, int64_t *P)
{
    if (N < 2 || N > ORC_MAXN || !dims || !ranks) return ORC_EINVAL;
    int64_t p = 1;
    for (int n = 0; n < N; n++) {
        if (dims[n] < 1 || ranks[n] < 1) return ORC_EINVAL;
        p *= ranks[n];
    }
    *P = p;
    return ORC_OK;
}

static void factor_offsets(int N, const int64_t *dims, const int32_t *ranks, int64_t *off)
{
    int64_t o = 0;
    for (int n = 0; n < N; n++) {
        off[n] = o;
        o += dims[n] * ranks[n];
    }
}

/* Row pointer of a(n)_{i,:}. */
static const double *row_of(const double *A, const int64_t *off, const int32_t *ranks,
                            int n, int64_t i)
{
    return A + off[n] + i * ranks[n];
}

/* Advance the multi-index j (j_0 fastest) by one step over the core. */
static void odometer_next(int N, const int32_t *ranks, int *j)
{
    for (int k = 0; k < N; k++) {
        if (++j[k] < ranks[k]) return;
        j[k] = 0;
    }
}

/* x_hat of one entry by the definition of the Sparse Tucker Decomposition:
 * x_hat = sum over all core positions j of G[j] * prod_k A(k)[i_k, j_k]. */
static double predict_one(int N, const int32_t *ranks, const int64_t *off, const double *A,
                          const double *G, int64_t P, const int64_t *i)
{
    int j[ORC_MAXN] = {0};
    double acc = 0.0;
    for (int64_t lin = 0; lin < P; lin++) {
        double h = G[lin];
        for (int k = 0; k < N; k++) h *= row_of(A, off, ranks, k, i[k])[j[k]];
        acc += h;
        odometer_next(N, ranks, j);
    }
    return acc;
}

static int check_indices(int N, const int64_t *dims, int64_t q, const int32_t *idx)
{
    for (int n = 0; n < N; n++)
        for (int64_t t = 0; t < q; t++)
            if (idx[n * q + t] < 0 || idx[n * q + t] >= dims[n]) return ORC_EINVAL;
    return ORC_OK;
}

/* Prediction for q entries (Definition "Sparse Tucker Decomposition"). */
int orc_predict(int N, const int64_t *dims, const int32_t *ranks, const double *A,
                const double *G, int64_t q, const int32_t *idx, double *out)
{
    int64_t P, off[ORC_MAXN], i[ORC_MAXN];
    if (check_model(N, dims, ranks, &P) || q < 0) return ORC_EINVAL;
    if (check_indices(N, dims, q, idx)) return ORC_EINVAL;
    factor_offsets(N, dims, ranks, off);
    for (int64_t t = 0; t < q; t++) {
        for (int k = 0; k < N; k++) i[k] = idx[k * q + t];
        out[t] = predict_one(N, ranks, off, A, G, P, i);
    }
    return ORC_OK;
}

/* RMSE and MAE over a set (Section "Experimental Settings"); also the sum of
 * squared residuals and the regularised objective
 *   0.5*SSE/n + 0.5*lambda_A*sum_n ||A(n)||^2 + 0.5*lambda_G*||G||^2.
 * out = {rmse, mae, sse, objective}. */
int orc_loss(int N, const int64_t *dims, const int32_t *ranks, const double *A,
             const double *G, int64_t q, const int32_t *idx, const float *vals,
             double lam_A, double lam_G, double *out)
{
    int64_t P, off[ORC_MAXN], i[ORC_MAXN];
    if (check_model(N, dims, ranks, &P) || q < 1 || !out) return ORC_EINVAL;
    if (check_indices(N, dims, q, idx)) return ORC_EINVAL;
    factor_offsets(N, dims, ranks, off);
    double sse = 0.0, sae = 0.0;
    for (int64_t t = 0; t < q; t++) {
        for (int k = 0; k < N; k++) i[k] = idx[k * q + t];
        double r = (double)vals[t] - predict_one(N, ranks, off, A, G, P, i);
        sse += r * r;
        sae += fabs(r);
    }
    double reg_A = 0.0, reg_G = 0.0;
    int64_t nA = 0;
    for (int n = 0; n < N; n++) nA += dims[n] * ranks[n];
    for (int64_t e = 0; e < nA; e++) reg_A += A[e] * A[e];
    for (int64_t e = 0; e < P; e++) reg_G += G[e] * G[e];
    out[0] = sqrt(sse / (double)q);
    out[1] = sae / (double)q;
    out[2] = sse;
    out[3] = 0.5 * sse / (double)q + 0.5 * lam_A * reg_A + 0.5 * lam_G * reg_G;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Core sub-step.                                                            */
/* READING (dense core): the core objective of Eq.                           */
/* approximated_core_tensor_optimization, ||x - H g||^2 + lambda ||g||^2, is */
/* minimised by the averaged SGD rule of Eq. SGD directly in the dense core  */
/* vector g = Vec(G) (the Kruskal substitution of Eq. CP-Decomposition is    */
/* not applied), once per minibatch.  Row p of H_Psi is                       */
/* h_p[lin(j)] = prod_k A(k)[i_k(p), j_k].  With the 1/2 convention the step  */
/* is the exact gradient of f_C(G) = (1/2m) sum_p r_p^2 + (lambda_G/2)||G||^2: */
/*   G <- G - gamma_G * ( -(1/m) sum_p r_p h_p + lambda_G G ),                */
/* with r_p = x_p - x_hat_p from the current A and G.                        */
/* idx is SoA [N][m] for the m samples of the minibatch.                      */
/* ------------------------------------------------------------------------ */
static int core_step_impl(int N, const int64_t *dims, const int32_t *ranks, const double *A,
                          double *G, int64_t m, const int32_t *idx, const float *x,
                          double gam_G, double lam_G, double *VG, double mu);

int orc_core_step(int N, const int64_t *dims, const int32_t *ranks, const double *A,
                  double *G, int64_t m, const int32_t *idx, const float *x,
                  double gam_G, double lam_G)
{
    return core_step_impl(N, dims, ranks, A, G, m, idx, x, gam_G, lam_G, NULL, 0.0);
}

/* The same step with heavy-ball momentum when VG is given (see
 * orc_step_momentum): VG <- mu VG + grad, G <- G - gamma_G VG. */
static int core_step_impl(int N, const int64_t *dims, const int32_t *ranks, const double *A,
                          double *G, int64_t m, const int32_t *idx, const float *x,
                          double gam_G, double lam_G, double *VG, double mu)
{
    int64_t P, off[ORC_MAXN], i[ORC_MAXN];
    if (check_model(N, dims, ranks, &P) || m < 1) return ORC_EINVAL;
    if (check_indices(N, dims, m, idx)) return ORC_EINVAL;
    factor_offsets(N, dims, ranks, off);
    double *sum_rh = (double *)calloc((size_t)P, sizeof(double));
    if (!sum_rh) return ORC_ENOMEM;
    for (int64_t p = 0; p < m; p++) {
        for (int k = 0; k < N; k++) i[k] = idx[k * m + p];
        double r = (double)x[p] - predict_one(N, ranks, off, A, G, P, i);
        int j[ORC_MAXN] = {0};
        for (int64_t lin = 0; lin < P; lin++) {
            double h = 1.0;
            for (int k = 0; k < N; k++) h *= row_of(A, off, ranks, k, i[k])[j[k]];
            sum_rh[lin] += r * h;
            odometer_next(N, ranks, j);
        }
    }
    for (int64_t lin = 0; lin < P; lin++) {
        double grad = -sum_rh[lin] / (double)m + lam_G * G[lin];
        if (VG) {
            VG[lin] = mu * VG[lin] + grad;
            G[lin] -= gam_G * VG[lin];
        } else {
            G[lin] -= gam_G * grad;
        }
    }
    free(sum_rh);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Mode-n sub-step (Algorithm 1, factor loop; Eq. SGD_factor_matrix and     */
/* Eq. Gradient_factor_matrix).                                              */
/* For every sample p: E_p = G_(n) s_p, where s_p is the row of S(n) built    */
/* from the current rows of the other modes, and r_p = x_p - a(n)_{i_n} E_p.  */
/* All residuals are formed before any row of mode n changes.  Each sampled  */
/* row i then takes one step on                                              */
/*   f_{n,i}(a) = (1/2c_i) sum_{p in seg(i)} (x_p - a E_p)^2 + (lambda_A/2)||a||^2: */
/*   a <- a - gamma_A * ( F/c_i + lambda_A a ),  F = sum_{p in seg(i)} (-r_p E_p), */
/* summed in (row, position) order.                                          */
/* READING: the normaliser is the row count c_i = |(Psi_M^(n))_{i_n}| (the    */
/* SGD call of Algorithm 1), not the minibatch size of Eq.                    */
/* Gradient_factor_matrix; rows absent from the minibatch are not touched.   */
/* ------------------------------------------------------------------------ */
static int mode_step_impl(int N, const int64_t *dims, const int32_t *ranks, double *A,
                          const double *G, int64_t m, const int32_t *idx, const float *x,
                          int n, double gam_A, double lam_A, double *VA, double mu);

int orc_mode_step(int N, const int64_t *dims, const int32_t *ranks, double *A,
                  const double *G, int64_t m, const int32_t *idx, const float *x,
                  int n, double gam_A, double lam_A)
{
    return mode_step_impl(N, dims, ranks, A, G, m, idx, x, n, gam_A, lam_A, NULL, 0.0);
}

/* The same step with heavy-ball momentum when VA (velocities laid out as A)
 * is given (see orc_step_momentum): for each sampled row,
 * v <- mu v + (F/c_i + lambda_A a), a <- a - gamma_A v. */
static int mode_step_impl(int N, const int64_t *dims, const int32_t *ranks, double *A,
                          const double *G, int64_t m, const int32_t *idx, const float *x,
                          int n, double gam_A, double lam_A, double *VA, double mu)
{
    int64_t P, off[ORC_MAXN], i[ORC_MAXN];
    if (check_model(N, dims, ranks, &P) || m < 1 || n < 0 || n >= N) return ORC_EINVAL;
    if (ranks[n] > 256) return ORC_EINVAL;
    if (check_indices(N, dims, m, idx)) return ORC_EINVAL;
    factor_offsets(N, dims, ranks, off);
    int Jn = ranks[n];
    double *E = (double *)calloc((size_t)(m * Jn), sizeof(double));
    double *r = (double *)calloc((size_t)m, sizeof(double));
    int32_t *rows = (int32_t *)malloc((size_t)m * sizeof(int32_t));
    int32_t *sigma = (int32_t *)malloc((size_t)m * sizeof(int32_t));
    int32_t *seg_off = (int32_t *)malloc((size_t)(m + 1) * sizeof(int32_t));
    int32_t *seg_row = (int32_t *)malloc((size_t)m * sizeof(int32_t));
    if (!E || !r || !rows || !sigma || !seg_off || !seg_row) {
        free(E); free(r); free(rows); free(sigma); free(seg_off); free(seg_row);
        return ORC_ENOMEM;
    }
    for (int64_t p = 0; p < m; p++) {
        for (int k = 0; k < N; k++) i[k] = idx[k * m + p];
        /* E_p[j_n] = sum over the core of G[j] * prod_{k != n} A(k)[i_k, j_k] */
        int j[ORC_MAXN] = {0};
        for (int64_t lin = 0; lin < P; lin++) {
            double s = G[lin];
            for (int k = 0; k < N; k++)
                if (k != n) s *= row_of(A, off, ranks, k, i[k])[j[k]];
            E[p * Jn + j[n]] += s;
            odometer_next(N, ranks, j);
        }
        const double *a = row_of(A, off, ranks, n, i[n]);
        double xh = 0.0;
        for (int jn = 0; jn < Jn; jn++) xh += a[jn] * E[p * Jn + jn];
        r[p] = (double)x[p] - xh;
        rows[p] = i[n];
    }
    int32_t nseg = 0;
    orc_segments(m, rows, sigma, seg_off, seg_row, &nseg);
    double F[256];
    for (int32_t s = 0; s < nseg; s++) {
        double *a = A + off[n] + (int64_t)seg_row[s] * Jn;
        int32_t c = seg_off[s + 1] - seg_off[s];
        for (int jn = 0; jn < Jn; jn++) F[jn] = 0.0;
        for (int32_t q = seg_off[s]; q < seg_off[s + 1]; q++) {
            int32_t p = sigma[q];
            for (int jn = 0; jn < Jn; jn++) F[jn] += -r[p] * E[(int64_t)p * Jn + jn];
        }
        if (VA) {
            double *v = VA + off[n] + (int64_t)seg_row[s] * Jn;
            for (int jn = 0; jn < Jn; jn++) {
                v[jn] = mu * v[jn] + (F[jn] / (double)c + lam_A * a[jn]);
                a[jn] -= gam_A * v[jn];
            }
        } else {
            for (int jn = 0; jn < Jn; jn++)
                a[jn] -= gam_A * (F[jn] / (double)c + lam_A * a[jn]);
        }
    }
    free(E); free(r); free(rows); free(sigma); free(seg_off); free(seg_row);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* One minibatch: the core sub-step, then modes 0..N-1 in order, each using  */
/* the rows and core left by the sub-steps before it (Algorithm 1 order;     */
/* alternating minimisation of Section "SGD_Tucker").                        */
/* ------------------------------------------------------------------------ */
int orc_step(int N, const int64_t *dims, const int32_t *ranks, double *A, double *G,
             int64_t m, const int32_t *idx, const float *x, double gam_A, double lam_A,
             double gam_G, double lam_G)
{
    int rc = orc_core_step(N, dims, ranks, A, G, m, idx, x, gam_G, lam_G);
    for (int n = 0; rc == ORC_OK && n < N; n++)
        rc = orc_mode_step(N, dims, ranks, A, G, m, idx, x, n, gam_A, lam_A);
    return rc;
}

/* Epochs of minibatch SGD over all T entries.  Epoch e visits the entries in
 * the order perm[e*T + q] if perm is given, else in the order pi_{epoch0+e}
 * of the sampler above with the given seed.  Minibatch b of an epoch holds
 * positions [bM, min((b+1)M, T)); the last one may be shorter.  At most
 * max_batches minibatches are run in total (negative: no limit), which lets
 * a caller time or compare a prefix of an epoch.  Returns the number of
 * minibatches run in *batches_run. */
int orc_run(int N, const int64_t *dims, const int32_t *ranks, double *A, double *G,
            int64_t T, const int32_t *idx, const float *vals, int64_t M, double gam_A,
            double lam_A, double gam_G, double lam_G, const int64_t *perm, uint64_t seed,
            int64_t epoch0, int64_t n_epochs, int64_t max_batches, int64_t *batches_run)
{
    int64_t P;
    if (check_model(N, dims, ranks, &P) || T < 1 || M < 1 || n_epochs < 0) return ORC_EINVAL;
    if (check_indices(N, dims, T, idx)) return ORC_EINVAL;
    int64_t *order = (int64_t *)malloc((size_t)T * sizeof(int64_t));
    int32_t *bidx = (int32_t *)malloc((size_t)(N * M) * sizeof(int32_t));
    float *bx = (float *)malloc((size_t)M * sizeof(float));
    if (!order || !bidx || !bx) {
        free(order); free(bidx); free(bx);
        return ORC_ENOMEM;
    }
    int64_t done = 0;
    int rc = ORC_OK;
    for (int64_t e = 0; e < n_epochs && rc == ORC_OK; e++) {
        if (perm) memcpy(order, perm + e * T, (size_t)T * sizeof(int64_t));
        else orc_perm(T, seed, epoch0 + e, order);
        for (int64_t b0 = 0; b0 < T && rc == ORC_OK; b0 += M) {
            if (max_batches >= 0 && done >= max_batches) break;
            int64_t m = (T - b0 < M) ? (T - b0) : M;
            for (int64_t p = 0; p < m; p++) {
                int64_t t = order[b0 + p];
                for (int k = 0; k < N; k++) bidx[k * m + p] = idx[k * T + t];
                bx[p] = vals[t];
            }
            rc = orc_step(N, dims, ranks, A, G, m, bidx, bx, gam_A, lam_A, gam_G, lam_G);
            done++;
        }
    }
    if (batches_run) *batches_run = done;
    free(order); free(bidx); free(bx);
    return rc;
}

/* ======================================================================== */
/* Heavy-ball momentum (Section "Conclusion and Future Works" names momentum  */
/* as an extension of SGD_Tucker without fixing it).                         */
/* READING: Polyak's heavy ball on each sub-step's stochastic gradient:      */
/* v <- mu v + g, theta <- theta - gamma v, with the core's velocity VG       */
/* updated once per minibatch and one velocity per factor row (VA, laid out  */
/* as A) updated when its row is sampled; like the rows themselves (lazy     */
/* rows), the velocity of a row absent from a minibatch neither changes nor  */
/* decays.  mu = 0 is the plain method.                                      */
/* ======================================================================== */
int orc_step_momentum(int N, const int64_t *dims, const int32_t *ranks, double *A, double *G,
                      double *VA, double *VG, int64_t m, const int32_t *idx, const float *x,
                      double gam_A, double lam_A, double gam_G, double lam_G, double mu)
{
    int64_t P;
    if (check_model(N, dims, ranks, &P) || !VA || !VG || !(mu >= 0.0 && mu < 1.0)) return ORC_EINVAL;
    int rc = core_step_impl(N, dims, ranks, A, G, m, idx, x, gam_G, lam_G, VG, mu);
    for (int n = 0; rc == ORC_OK && n < N; n++)
        rc = mode_step_impl(N, dims, ranks, A, G, m, idx, x, n, gam_A, lam_A, VA, mu);
    return rc;
}

/* Epochs as orc_run, each minibatch by orc_step_momentum. */
int orc_run_momentum(int N, const int64_t *dims, const int32_t *ranks, double *A, double *G,
                     double *VA, double *VG, int64_t T, const int32_t *idx, const float *vals,
                     int64_t M, double gam_A, double lam_A, double gam_G, double lam_G, double mu,
                     const int64_t *perm, uint64_t seed, int64_t epoch0, int64_t n_epochs,
                     int64_t max_batches, int64_t *batches_run)
{
    int64_t P;
    if (check_model(N, dims, ranks, &P) || T < 1 || M < 1 || n_epochs < 0) return ORC_EINVAL;
    if (check_indices(N, dims, T, idx)) return ORC_EINVAL;
    int64_t *order = (int64_t *)malloc((size_t)T * sizeof(int64_t));
    int32_t *bidx = (int32_t *)malloc((size_t)(N * M) * sizeof(int32_t));
    float *bx = (float *)malloc((size_t)M * sizeof(float));
    if (!order || !bidx || !bx) {
        free(order); free(bidx); free(bx);
        return ORC_ENOMEM;
    }
    int64_t done = 0;
    int rc = ORC_OK;
    for (int64_t e = 0; e < n_epochs && rc == ORC_OK; e++) {
        if (perm) memcpy(order, perm + e * T, (size_t)T * sizeof(int64_t));
        else orc_perm(T, seed, epoch0 + e, order);
        for (int64_t b0 = 0; b0 < T && rc == ORC_OK; b0 += M) {
            if (max_batches >= 0 && done >= max_batches) break;
            int64_t m = (T - b0 < M) ? (T - b0) : M;
            for (int64_t p = 0; p < m; p++) {
                int64_t t = order[b0 + p];
                for (int k = 0; k < N; k++) bidx[k * m + p] = idx[k * T + t];
                bx[p] = vals[t];
            }
            rc = orc_step_momentum(N, dims, ranks, A, G, VA, VG, m, bidx, bx, gam_A, lam_A, gam_G, lam_G, mu);
            done++;
        }
    }
    if (batches_run) *batches_run = done;
    free(order); free(bidx); free(bx);
    return rc;
}

/* ======================================================================== */
/* Kruskal core (Section "Optimization Process for the Core Tensor").        */
/* The core is approximated by the R_core Kruskal product of the matrices    */
/* B(n) in R^{J_n x R} (Eq. CP-Decomposition).  B is stored with each B(n)   */
/* row-major J_n x R, the modes back to back (B(n) starts at                 */
/* sum_{k<n} J_k * R).                                                       */
/* READING: the paper requires R_core <= J_n but its rank study uses         */
/* R_core up to 25 at J_n = 5, so any R >= 1 is accepted here.               */
/* ======================================================================== */

static void b_offsets(int N, const int32_t *ranks, int R, int64_t *off)
{
    int64_t o = 0;
    for (int n = 0; n < N; n++) {
        off[n] = o;
        o += (int64_t)ranks[n] * R;
    }
}

/* G[lin(j)] = sum_r prod_k B(k)[j_k, r] (Eq. CP-Decomposition; G flat with
 * j_0 fastest, as everywhere in this file). */
int orc_kruskal_core(int N, const int32_t *ranks, int R, const double *B, double *G)
{
    int64_t P, boff[ORC_MAXN];
    int64_t dims1[ORC_MAXN];
    for (int n = 0; n < N && n < ORC_MAXN; n++) dims1[n] = 1;
    if (check_model(N, dims1, ranks, &P) || R < 1 || !B || !G) return ORC_EINVAL;
    b_offsets(N, ranks, R, boff);
    int j[ORC_MAXN] = {0};
    for (int64_t lin = 0; lin < P; lin++) {
        double acc = 0.0;
        for (int r = 0; r < R; r++) {
            double t = 1.0;
            for (int k = 0; k < N; k++) t *= B[boff[k] + (int64_t)j[k] * R + r];
            acc += t;
        }
        G[lin] = acc;
        odometer_next(N, ranks, j);
    }
    return ORC_OK;
}

/* W_r of mode n for the m samples of a minibatch, built as Algorithm 1's
 * core loop builds it: the rows of H_Psi in the mode-n vectorisation of Eq.
 * approximated_core_tensor_optimization (entry j_n + J_n*col holds
 * prod_k A(k)[i_k, j_k], col the mode-n unfolding column of Definition
 * "Tensor Unfolding"), the column q_r of the Khatri-Rao product
 * Q(n) = B(N) (.) ... (.) B(n+1) (.) B(n-1) (.) ... (.) B(1) of Eq. eventual0
 * (entry col holds prod_{k != n} B(k)[j_k, r]), the block matrix O_r of Eq. Q_r
 * (the J_n x J_n identity scaled by q_{col,r} in block row col), and
 * W_r = H_Psi O_r (m x J_n, row-major), all formed explicitly. */
int orc_kruskal_W(int N, const int64_t *dims, const int32_t *ranks, const double *A, int R,
                  const double *B, int64_t m, const int32_t *idx, int n, int r, double *W)
{
    int64_t P, off[ORC_MAXN], boff[ORC_MAXN], i[ORC_MAXN];
    if (check_model(N, dims, ranks, &P) || R < 1 || m < 1 || n < 0 || n >= N || r < 0 || r >= R || !W)
        return ORC_EINVAL;
    if (check_indices(N, dims, m, idx)) return ORC_EINVAL;
    factor_offsets(N, dims, ranks, off);
    b_offsets(N, ranks, R, boff);
    const int Jn = ranks[n];
    const int64_t K = P / Jn;
    double *H = (double *)malloc((size_t)(m * P) * sizeof(double));
    double *q = (double *)malloc((size_t)K * sizeof(double));
    double *O = (double *)calloc((size_t)(P * Jn), sizeof(double));
    if (!H || !q || !O) {
        free(H); free(q); free(O);
        return ORC_ENOMEM;
    }
    /* H_Psi and q_r, walking the core positions j (j_0 fastest) */
    int j[ORC_MAXN] = {0};
    for (int64_t lin = 0; lin < P; lin++) {
        int64_t col = 0, stride = 1;
        for (int k = 0; k < N; k++) {
            if (k == n) continue;
            col += j[k] * stride;
            stride *= ranks[k];
        }
        const int64_t v = j[n] + (int64_t)Jn * col;
        for (int64_t s = 0; s < m; s++) {
            double h = 1.0;
            for (int k = 0; k < N; k++) {
                i[k] = idx[k * m + s];
                h *= row_of(A, off, ranks, k, i[k])[j[k]];
            }
            H[s * P + v] = h;
        }
        double qv = 1.0;
        for (int k = 0; k < N; k++)
            if (k != n) qv *= B[boff[k] + (int64_t)j[k] * R + r];
        q[col] = qv;
        odometer_next(N, ranks, j);
    }
    /* O_r: block row col is q_{col,r} times the identity */
    for (int64_t col = 0; col < K; col++)
        for (int jj = 0; jj < Jn; jj++) O[(jj + Jn * col) * Jn + jj] = q[col];
    /* W_r = H_Psi O_r */
    for (int64_t s = 0; s < m; s++)
        for (int jj = 0; jj < Jn; jj++) {
            double acc = 0.0;
            for (int64_t v = 0; v < P; v++) acc += H[s * P + v] * O[v * Jn + jj];
            W[s * Jn + jj] = acc;
        }
    free(H); free(q); free(O);
    return ORC_OK;
}

/* The cyclic block steps on the columns rc0..rc1-1 of B(n) (Eq.
 * eventual_approximated, solved by the averaged SGD of Eq. SGD_core_tensor
 * with the gradient of Eq. Gradient_core_tensor; Algorithm 1, core loop):
 * with the W_r of every r computed once for mode n, each column in turn forms
 *   x_hat = x - sum_{r != rc} W_r b_r          (current columns),
 *   C = W_rc^T W_rc,  V = -W_rc^T x_hat + C b_rc,
 *   b_rc <- b_rc - gamma_B * ( V / m + lambda_B b_rc ),
 * the exact gradient step of (1/2m) ||x - sum_r W_r b_r||^2 + (lambda_B/2)||b_rc||^2
 * (the 1/M of Eq. Gradient_core_tensor with M = m, the minibatch's size). */
static int kruskal_columns(int N, const int64_t *dims, const int32_t *ranks, const double *A, int R,
                           double *B, int64_t m, const int32_t *idx, const float *x, int n, int rc0,
                           int rc1, double gam_B, double lam_B)
{
    int64_t boff[ORC_MAXN];
    b_offsets(N, ranks, R, boff);
    const int Jn = ranks[n];
    double *W = (double *)malloc((size_t)(R * m * Jn) * sizeof(double));
    double *xh = (double *)malloc((size_t)m * sizeof(double));
    double *C = (double *)malloc((size_t)(Jn * Jn) * sizeof(double));
    double *V = (double *)malloc((size_t)Jn * sizeof(double));
    if (!W || !xh || !C || !V) {
        free(W); free(xh); free(C); free(V);
        return ORC_ENOMEM;
    }
    int rc = ORC_OK;
    for (int r = 0; r < R && rc == ORC_OK; r++)
        rc = orc_kruskal_W(N, dims, ranks, A, R, B, m, idx, n, r, W + (int64_t)r * m * Jn);
    double *Bn = B + boff[n];
    for (int c = rc0; c < rc1 && rc == ORC_OK; c++) {
        const double *Wc = W + (int64_t)c * m * Jn;
        for (int64_t s = 0; s < m; s++) {
            double v = (double)x[s];
            for (int r = 0; r < R; r++) {
                if (r == c) continue;
                for (int jj = 0; jj < Jn; jj++) v -= W[((int64_t)r * m + s) * Jn + jj] * Bn[jj * R + r];
            }
            xh[s] = v;
        }
        for (int a = 0; a < Jn; a++)
            for (int b = 0; b < Jn; b++) {
                double acc = 0.0;
                for (int64_t s = 0; s < m; s++) acc += Wc[s * Jn + a] * Wc[s * Jn + b];
                C[a * Jn + b] = acc;
            }
        for (int a = 0; a < Jn; a++) {
            double v = 0.0;
            for (int64_t s = 0; s < m; s++) v -= Wc[s * Jn + a] * xh[s];
            for (int b = 0; b < Jn; b++) v += C[a * Jn + b] * Bn[b * R + c];
            V[a] = v;
        }
        for (int a = 0; a < Jn; a++)
            Bn[a * R + c] -= gam_B * (V[a] / (double)m + lam_B * Bn[a * R + c]);
    }
    free(W); free(xh); free(C); free(V);
    return rc;
}

/* One block step on column rc of B(n) alone (for the gradient pins). */
int orc_kruskal_column_step(int N, const int64_t *dims, const int32_t *ranks, const double *A, int R,
                            double *B, int64_t m, const int32_t *idx, const float *x, int n, int rc,
                            double gam_B, double lam_B)
{
    int64_t P;
    if (check_model(N, dims, ranks, &P) || R < 1 || m < 1 || n < 0 || n >= N || rc < 0 || rc >= R || !B)
        return ORC_EINVAL;
    if (check_indices(N, dims, m, idx)) return ORC_EINVAL;
    return kruskal_columns(N, dims, ranks, A, R, B, m, idx, x, n, rc, rc + 1, gam_B, lam_B);
}

/* The Kruskal core sub-step of one minibatch (Algorithm 1, core loop and the
 * forming of the core): for n = 1..N in order, every column of B(n) in
 * order, each mode's W_r built from the B(k) left by the modes before it;
 * then G = the Kruskal product of the updated B (Eq. CP-Decomposition). */
int orc_kruskal_core_step(int N, const int64_t *dims, const int32_t *ranks, const double *A, int R,
                          double *B, double *G, int64_t m, const int32_t *idx, const float *x,
                          double gam_B, double lam_B)
{
    int64_t P;
    if (check_model(N, dims, ranks, &P) || R < 1 || m < 1 || !B || !G) return ORC_EINVAL;
    if (check_indices(N, dims, m, idx)) return ORC_EINVAL;
    int rc = ORC_OK;
    for (int n = 0; n < N && rc == ORC_OK; n++)
        rc = kruskal_columns(N, dims, ranks, A, R, B, m, idx, x, n, 0, R, gam_B, lam_B);
    if (rc == ORC_OK) rc = orc_kruskal_core(N, ranks, R, B, G);
    return rc;
}

/* One minibatch with the Kruskal core: the core sub-step above, then the
 * factor sub-steps of modes 0..N-1 with the core it formed (Algorithm 1). */
int orc_step_kruskal(int N, const int64_t *dims, const int32_t *ranks, double *A, int R, double *B,
                     double *G, int64_t m, const int32_t *idx, const float *x, double gam_A, double lam_A,
                     double gam_B, double lam_B)
{
    int rc = orc_kruskal_core_step(N, dims, ranks, A, R, B, G, m, idx, x, gam_B, lam_B);
    for (int n = 0; rc == ORC_OK && n < N; n++)
        rc = orc_mode_step(N, dims, ranks, A, G, m, idx, x, n, gam_A, lam_A);
    return rc;
}

/* Epochs as orc_run, each minibatch by orc_step_kruskal. */
int orc_run_kruskal(int N, const int64_t *dims, const int32_t *ranks, double *A, int R, double *B, double *G,
                    int64_t T, const int32_t *idx, const float *vals, int64_t M, double gam_A,
                    double lam_A, double gam_B, double lam_B, const int64_t *perm, uint64_t seed,
                    int64_t epoch0, int64_t n_epochs, int64_t max_batches, int64_t *batches_run)
{
    int64_t P;
    if (check_model(N, dims, ranks, &P) || R < 1 || T < 1 || M < 1 || n_epochs < 0) return ORC_EINVAL;
    if (check_indices(N, dims, T, idx)) return ORC_EINVAL;
    int64_t *order = (int64_t *)malloc((size_t)T * sizeof(int64_t));
    int32_t *bidx = (int32_t *)malloc((size_t)(N * M) * sizeof(int32_t));
    float *bx = (float *)malloc((size_t)M * sizeof(float));
    if (!order || !bidx || !bx) {
        free(order); free(bidx); free(bx);
        return ORC_ENOMEM;
    }
    int64_t done = 0;
    int rc = orc_kruskal_core(N, ranks, R, B, G);
    for (int64_t e = 0; e < n_epochs && rc == ORC_OK; e++) {
        if (perm) memcpy(order, perm + e * T, (size_t)T * sizeof(int64_t));
        else orc_perm(T, seed, epoch0 + e, order);
        for (int64_t b0 = 0; b0 < T && rc == ORC_OK; b0 += M) {
            if (max_batches >= 0 && done >= max_batches) break;
            int64_t m = (T - b0 < M) ? (T - b0) : M;
            for (int64_t p = 0; p < m; p++) {
                int64_t t = order[b0 + p];
                for (int k = 0; k < N; k++) bidx[k * m + p] = idx[k * T + t];
                bx[p] = vals[t];
            }
            rc = orc_step_kruskal(N, dims, ranks, A, R, B, G, m, bidx, bx, gam_A, lam_A, gam_B, lam_B);
            done++;
        }
    }
    if (batches_run) *batches_run = done;
    free(order); free(bidx); free(bx);
    return rc;
}
