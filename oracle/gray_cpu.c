/*
 * The paper's own method on host cores -- a TIMING BASELINE, test
 * infrastructure like the oracle beside it.  Only the tests and the
 * benchmark's CPU-baseline leg load this file's library; the product path
 * (the HIP library) never calls it and shares no code with it.
 *
 * What it runs is the improved brute force of Sec. 2.2 / Algorithm 1 with the
 * prefix split of Sec. 3.1, in float64 as the paper's code is:
 *
 *   - the 2^s states of a suffix of s bits are visited in reflected Gray-code
 *     order, g(t) = t ^ (t >> 1); step t flips the single bit l = ctz(t);
 *   - the objective changes by (1 - 2 x_l) h_l (Eq. 2, 3), where the local
 *     field of bit j is h_j = Q_jj + sum_{i != j} S_ij x_i and S = Q + Q^T off
 *     the diagonal;
 *   - after the flip every field moves by +S_jl (x_l became 1) or -S_jl
 *     (x_l became 0): O(n) work per state;
 *   - the top m = n - s bits are a prefix fixed per task; OpenMP threads take
 *     prefixes dynamically (Sec. 3.1 gives each thread one prefix; more
 *     prefixes than threads only balance the load).
 *
 * The incumbent starts at each prefix's first state and is replaced when a
 * state is lower, ties going to the lower mask, so the result compares with
 * the oracle's k = 1 answer (same order: energy, then mask).  Bit i of a mask
 * is x_i; the prefix holds the top m bits in natural order.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define QG_OK 0
#define QG_ERR_ARG -1
#define QG_MAXN 63

/* Walks the 2^s suffix states under prefix p: S is the symmetric n x n
 * off-diagonal coupling (zero diagonal, row-major), d the diagonal. */
__attribute__((target_clones("avx2", "default")))
static void walk_prefix(const double *S, const double *d, int n, int s, uint64_t p,
                        double *best_e, uint64_t *best_m)
{
    double h[QG_MAXN + 1];
    uint64_t x = p << s;
    /* value of the prefix part alone (the suffix starts at zero) */
    double v = 0.0;
    for (int i = s; i < n; ++i) {
        if (!((x >> i) & 1u))
            continue;
        v += d[i];
        for (int j = i + 1; j < n; ++j)
            if ((x >> j) & 1u)
                v += S[(size_t)i * n + j];
    }
    /* fields of the suffix bits */
    for (int j = 0; j < s; ++j) {
        double f = d[j];
        for (int i = s; i < n; ++i)
            if ((x >> i) & 1u)
                f += S[(size_t)j * n + i];
        h[j] = f;
    }
    double be = v;
    uint64_t bm = x;
    const uint64_t steps = (uint64_t)1 << s;
    for (uint64_t t = 1; t < steps; ++t) {
        const int l = __builtin_ctzll(t);
        const double *col = S + (size_t)l * n;
        x ^= (uint64_t)1 << l;
        if ((x >> l) & 1u) {
            v += h[l];
            for (int j = 0; j < s; ++j)
                h[j] += col[j];
        } else {
            v -= h[l];
            for (int j = 0; j < s; ++j)
                h[j] -= col[j];
        }
        if (v < be || (v == be && x < bm)) {
            be = v;
            bm = x;
        }
    }
    *best_e = be;
    *best_m = bm;
}

/* Minimum of f_Q over the states whose top m bits are one of the listed
 * prefixes (all 2^m prefixes when `prefixes` is NULL).  Q: float32, row
 * stride ldq, entries with i > j ignored.  threads <= 0: all OpenMP threads.
 * Returns QG_OK, or QG_ERR_ARG for n outside [1, 63], m outside [0, min(n, 62)], or
 * more than 2^m listed prefixes / a prefix >= 2^m. */
int qg_min_f32(const float *Q, int n, int64_t ldq, int m, const uint64_t *prefixes, int64_t count,
               int threads, double *out_e, uint64_t *out_m)
{
    if (!Q || !out_e || !out_m || n < 1 || n > QG_MAXN || m < 0 || m > n || m > 62 || ldq < n)
        return QG_ERR_ARG;
    const int s = n - m;
    const int64_t np = prefixes ? count : ((int64_t)1 << m);
    if (np < 1)
        return QG_ERR_ARG;
    if (prefixes)
        for (int64_t i = 0; i < np; ++i)
            if (prefixes[i] >= ((uint64_t)1 << m))
                return QG_ERR_ARG;
    double *S = calloc((size_t)n * n, sizeof(double));
    double *d = calloc((size_t)n, sizeof(double));
    if (!S || !d) {
        free(S);
        free(d);
        return QG_ERR_ARG;
    }
    for (int i = 0; i < n; ++i) {
        d[i] = (double)Q[(size_t)i * ldq + i];
        for (int j = i + 1; j < n; ++j) {
            S[(size_t)i * n + j] = (double)Q[(size_t)i * ldq + j];
            S[(size_t)j * n + i] = (double)Q[(size_t)i * ldq + j];
        }
    }
    const int T = threads > 0 ? threads : omp_get_max_threads();
    double be = 0.0;
    uint64_t bm = ~(uint64_t)0;
    int have = 0;
#pragma omp parallel num_threads(T)
    {
        double le = 0.0;
        uint64_t lm = ~(uint64_t)0;
        int lh = 0;
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < np; ++i) {
            const uint64_t p = prefixes ? prefixes[i] : (uint64_t)i;
            double e;
            uint64_t mk;
            walk_prefix(S, d, n, s, p, &e, &mk);
            if (!lh || e < le || (e == le && mk < lm)) {
                le = e;
                lm = mk;
                lh = 1;
            }
        }
#pragma omp critical
        {
            if (lh && (!have || le < be || (le == be && lm < bm))) {
                be = le;
                bm = lm;
                have = 1;
            }
        }
    }
    free(S);
    free(d);
    *out_e = be;
    *out_m = bm;
    return QG_OK;
}

int qg_max_threads(void) { return omp_get_max_threads(); }
