/*
 * CPU oracle for exhaustive QUBO solving -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this file's library.  The product path (the HIP library)
 * never calls it and shares no code, header, table or constant with it.
 *
 * What it computes is the plain definition, written out slowly:
 *
 *   f_Q(x) = sum_{i <= j} Q_ij x_i x_j            (Eq. 1, Q upper triangular)
 *
 * evaluated from scratch, O(n^2), for every mask in natural binary order
 * (Sec. 3, the naive solver: bit i of the counter is x_i, counting from 1 but
 * with the zero vector, value 0, as the starting incumbent).  No Gray code, no
 * incremental update, no table: a reader can check it against Eq. 1 by eye.
 *
 * Readings of the paper taken here (the paper is silent or inconsistent):
 *   - entries with i > j are ignored (Eq. 1, right-hand side);
 *   - bit i of a mask is x_i, 0-based (the decoding of Sec. 3);
 *   - the zero vector is a candidate with value 0 (Sec. 2.1, Sec. 3 code);
 *   - ties are broken by the lower natural mask, i.e. candidates are ordered
 *     lexicographically by (energy, mask);
 *   - float Q is widened exactly to double; integer Q to int64 (float64 and
 *     int64 Q are used as stored).
 *
 * Summation order of one energy (the canonical order, used for bitwise
 * comparison of rescored values): i ascending; for each i with x_i = 1 the row
 * term starts at Q_ii and adds Q_ij for j = i+1 .. n-1 with x_j = 1, in
 * ascending j; the row terms are added to the total in ascending i.  Build with
 * -ffp-contract=off (there are no products anyway).
 *
 * Log-partition and gradient (extensions beyond the paper, defined plainly):
 *   logZ(beta) = log sum_x exp(-beta f(x))
 *     pass A: M = max_x (-beta f(x)); pass B: S = sum_x exp(-beta f(x) - M)
 *     with Neumaier-compensated summation; logZ = M + log S.
 *   G_ij = d logZ / d Q_ij = -beta sum_x p(x) x_i x_j  (i <= j; x_i x_i = x_i),
 *     p(x) = exp(-beta f(x) - logZ), Neumaier-compensated; G_ij = 0 for i > j.
 *
 * Threading: the mask range is cut into T contiguous chunks (the top bits of
 * the mask, as in the prefix split of Sec. 3.1); each thread keeps its own
 * top-k list / partial sums, merged afterwards in thread order.  Top-k results
 * do not depend on T.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define QO_OK 0
#define QO_ERR_ARG -1

/* ---------------------------------------------------------------- energy */

static double energy_f(const float *Q, int n, int64_t ldq, uint64_t mask)
{
    double total = 0.0;
    for (int i = 0; i < n; ++i) {
        if (!((mask >> i) & 1u))
            continue;
        double row = (double)Q[(int64_t)i * ldq + i];
        for (int j = i + 1; j < n; ++j)
            if ((mask >> j) & 1u)
                row += (double)Q[(int64_t)i * ldq + j];
        total += row;
    }
    return total;
}

static int64_t energy_i(const int32_t *Q, int n, int64_t ldq, uint64_t mask)
{
    int64_t total = 0;
    for (int i = 0; i < n; ++i) {
        if (!((mask >> i) & 1u))
            continue;
        int64_t row = (int64_t)Q[(int64_t)i * ldq + i];
        for (int j = i + 1; j < n; ++j)
            if ((mask >> j) & 1u)
                row += (int64_t)Q[(int64_t)i * ldq + j];
        total += row;
    }
    return total;
}

double qo_energy_f32(const float *Q, int n, int64_t ldq, uint64_t mask)
{
    return energy_f(Q, n, ldq, mask);
}

int64_t qo_energy_i32(const int32_t *Q, int n, int64_t ldq, uint64_t mask)
{
    return energy_i(Q, n, ldq, mask);
}

/* Energies of many masks (for rescoring checks). */
void qo_energies_f32(const float *Q, int n, int64_t ldq, const uint64_t *masks,
                     int64_t count, double *out)
{
    for (int64_t c = 0; c < count; ++c)
        out[c] = energy_f(Q, n, ldq, masks[c]);
}

void qo_energies_i32(const int32_t *Q, int n, int64_t ldq, const uint64_t *masks,
                     int64_t count, int64_t *out)
{
    for (int64_t c = 0; c < count; ++c)
        out[c] = energy_i(Q, n, ldq, masks[c]);
}

/*
 * float64 and int64 Q: the same definition and summation order.  float64 Q is
 * used as stored; int64 sums are exact while sum |Q_ij| < 2^63.
 */
static double energy_d(const double *Q, int n, int64_t ldq, uint64_t mask)
{
    double total = 0.0;
    for (int i = 0; i < n; ++i) {
        if (!((mask >> i) & 1u))
            continue;
        double row = Q[(int64_t)i * ldq + i];
        for (int j = i + 1; j < n; ++j)
            if ((mask >> j) & 1u)
                row += Q[(int64_t)i * ldq + j];
        total += row;
    }
    return total;
}

static int64_t energy_l(const int64_t *Q, int n, int64_t ldq, uint64_t mask)
{
    int64_t total = 0;
    for (int i = 0; i < n; ++i) {
        if (!((mask >> i) & 1u))
            continue;
        int64_t row = Q[(int64_t)i * ldq + i];
        for (int j = i + 1; j < n; ++j)
            if ((mask >> j) & 1u)
                row += Q[(int64_t)i * ldq + j];
        total += row;
    }
    return total;
}

double qo_energy_f64(const double *Q, int n, int64_t ldq, uint64_t mask)
{
    return energy_d(Q, n, ldq, mask);
}

int64_t qo_energy_i64(const int64_t *Q, int n, int64_t ldq, uint64_t mask)
{
    return energy_l(Q, n, ldq, mask);
}

void qo_energies_f64(const double *Q, int n, int64_t ldq, const uint64_t *masks,
                     int64_t count, double *out)
{
    for (int64_t c = 0; c < count; ++c)
        out[c] = energy_d(Q, n, ldq, masks[c]);
}

void qo_energies_i64(const int64_t *Q, int n, int64_t ldq, const uint64_t *masks,
                     int64_t count, int64_t *out)
{
    for (int64_t c = 0; c < count; ++c)
        out[c] = energy_l(Q, n, ldq, masks[c]);
}

/* ----------------------------------------------------------- top-k lists */

/* (ea, ma) strictly before (eb, mb) in (energy, mask) order */
static int before_d(double ea, uint64_t ma, double eb, uint64_t mb)
{
    return ea < eb || (ea == eb && ma < mb);
}

static int before_i(int64_t ea, uint64_t ma, int64_t eb, uint64_t mb)
{
    return ea < eb || (ea == eb && ma < mb);
}

/* Insert into an ascending list of length k (slots beyond `*len` unused). */
static void insert_d(double *E, uint64_t *M, int k, int *len, double e, uint64_t m)
{
    if (*len == k && !before_d(e, m, E[k - 1], M[k - 1]))
        return;
    int pos = (*len < k) ? *len : k - 1;
    while (pos > 0 && before_d(e, m, E[pos - 1], M[pos - 1])) {
        E[pos] = E[pos - 1];
        M[pos] = M[pos - 1];
        --pos;
    }
    E[pos] = e;
    M[pos] = m;
    if (*len < k)
        ++*len;
}

static void insert_i(int64_t *E, uint64_t *M, int k, int *len, int64_t e, uint64_t m)
{
    if (*len == k && !before_i(e, m, E[k - 1], M[k - 1]))
        return;
    int pos = (*len < k) ? *len : k - 1;
    while (pos > 0 && before_i(e, m, E[pos - 1], M[pos - 1])) {
        E[pos] = E[pos - 1];
        M[pos] = M[pos - 1];
        --pos;
    }
    E[pos] = e;
    M[pos] = m;
    if (*len < k)
        ++*len;
}

/* Thread t of nt takes the t-th of nt contiguous, near-equal chunks. */
static void chunk(uint64_t lo, uint64_t span, int t, int nt, uint64_t *a, uint64_t *b)
{
    uint64_t base = span / (uint64_t)nt, rem = span % (uint64_t)nt, tt = (uint64_t)t;
    *a = lo + base * tt + (tt < rem ? tt : rem);
    *b = *a + base + (tt < rem ? 1 : 0);
}

static int threads_for(int requested)
{
    return requested > 0 ? requested : omp_get_max_threads();
}

/*
 * The k lowest (energy, mask) pairs among masks in [lo, hi), natural order.
 * Unused trailing slots get energy +inf and mask ~0.
 */
int qo_topk_f32(const float *Q, int n, int64_t ldq, uint64_t lo, uint64_t hi, int k,
                double *E_out, uint64_t *M_out, int nthreads)
{
    if (n < 1 || n > 63 || k < 1 || lo > hi || hi > (1ull << n))
        return QO_ERR_ARG;
    int T = threads_for(nthreads);
    double *E = (double *)malloc(sizeof(double) * (size_t)T * k);
    uint64_t *M = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)T * k);
    int *len = (int *)calloc((size_t)T, sizeof(int));
    uint64_t span = hi - lo;
#pragma omp parallel num_threads(T)
    {
        int t = omp_get_thread_num();
        int nt = omp_get_num_threads();
        uint64_t a, b;
        chunk(lo, span, t, nt, &a, &b);
        for (uint64_t x = a; x < b; ++x)
            insert_d(E + (size_t)t * k, M + (size_t)t * k, k, &len[t], energy_f(Q, n, ldq, x), x);
    }
    int outlen = 0;
    for (int i = 0; i < k; ++i) {
        E_out[i] = INFINITY;
        M_out[i] = ~0ull;
    }
    for (int t = 0; t < T; ++t)
        for (int i = 0; i < len[t]; ++i)
            insert_d(E_out, M_out, k, &outlen, E[(size_t)t * k + i], M[(size_t)t * k + i]);
    free(E);
    free(M);
    free(len);
    return QO_OK;
}

int qo_topk_i32(const int32_t *Q, int n, int64_t ldq, uint64_t lo, uint64_t hi, int k,
                int64_t *E_out, uint64_t *M_out, int nthreads)
{
    if (n < 1 || n > 63 || k < 1 || lo > hi || hi > (1ull << n))
        return QO_ERR_ARG;
    int T = threads_for(nthreads);
    int64_t *E = (int64_t *)malloc(sizeof(int64_t) * (size_t)T * k);
    uint64_t *M = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)T * k);
    int *len = (int *)calloc((size_t)T, sizeof(int));
    uint64_t span = hi - lo;
#pragma omp parallel num_threads(T)
    {
        int t = omp_get_thread_num();
        int nt = omp_get_num_threads();
        uint64_t a, b;
        chunk(lo, span, t, nt, &a, &b);
        for (uint64_t x = a; x < b; ++x)
            insert_i(E + (size_t)t * k, M + (size_t)t * k, k, &len[t], energy_i(Q, n, ldq, x), x);
    }
    int outlen = 0;
    for (int i = 0; i < k; ++i) {
        E_out[i] = INT64_MAX;
        M_out[i] = ~0ull;
    }
    for (int t = 0; t < T; ++t)
        for (int i = 0; i < len[t]; ++i)
            insert_i(E_out, M_out, k, &outlen, E[(size_t)t * k + i], M[(size_t)t * k + i]);
    free(E);
    free(M);
    free(len);
    return QO_OK;
}

/* The same selection for float64 and int64 Q. */
int qo_topk_f64(const double *Q, int n, int64_t ldq, uint64_t lo, uint64_t hi, int k,
                double *E_out, uint64_t *M_out, int nthreads)
{
    if (n < 1 || n > 63 || k < 1 || lo > hi || hi > (1ull << n))
        return QO_ERR_ARG;
    int T = threads_for(nthreads);
    double *E = (double *)malloc(sizeof(double) * (size_t)T * k);
    uint64_t *M = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)T * k);
    int *len = (int *)calloc((size_t)T, sizeof(int));
    uint64_t span = hi - lo;
#pragma omp parallel num_threads(T)
    {
        int t = omp_get_thread_num();
        int nt = omp_get_num_threads();
        uint64_t a, b;
        chunk(lo, span, t, nt, &a, &b);
        for (uint64_t x = a; x < b; ++x)
            insert_d(E + (size_t)t * k, M + (size_t)t * k, k, &len[t], energy_d(Q, n, ldq, x), x);
    }
    int outlen = 0;
    for (int i = 0; i < k; ++i) {
        E_out[i] = INFINITY;
        M_out[i] = ~0ull;
    }
    for (int t = 0; t < T; ++t)
        for (int i = 0; i < len[t]; ++i)
            insert_d(E_out, M_out, k, &outlen, E[(size_t)t * k + i], M[(size_t)t * k + i]);
    free(E);
    free(M);
    free(len);
    return QO_OK;
}

int qo_topk_i64(const int64_t *Q, int n, int64_t ldq, uint64_t lo, uint64_t hi, int k,
                int64_t *E_out, uint64_t *M_out, int nthreads)
{
    if (n < 1 || n > 63 || k < 1 || lo > hi || hi > (1ull << n))
        return QO_ERR_ARG;
    int T = threads_for(nthreads);
    int64_t *E = (int64_t *)malloc(sizeof(int64_t) * (size_t)T * k);
    uint64_t *M = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)T * k);
    int *len = (int *)calloc((size_t)T, sizeof(int));
    uint64_t span = hi - lo;
#pragma omp parallel num_threads(T)
    {
        int t = omp_get_thread_num();
        int nt = omp_get_num_threads();
        uint64_t a, b;
        chunk(lo, span, t, nt, &a, &b);
        for (uint64_t x = a; x < b; ++x)
            insert_i(E + (size_t)t * k, M + (size_t)t * k, k, &len[t], energy_l(Q, n, ldq, x), x);
    }
    int outlen = 0;
    for (int i = 0; i < k; ++i) {
        E_out[i] = INT64_MAX;
        M_out[i] = ~0ull;
    }
    for (int t = 0; t < T; ++t)
        for (int i = 0; i < len[t]; ++i)
            insert_i(E_out, M_out, k, &outlen, E[(size_t)t * k + i], M[(size_t)t * k + i]);
    free(E);
    free(M);
    free(len);
    return QO_OK;
}

/* ------------------------------------------------------- compensated sums */

typedef struct {
    double s, c;
} nsum_t;

static void nsum_add(nsum_t *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

static double nsum_val(const nsum_t *a)
{
    return a->s + a->c;
}

/* --------------------------------------------------------- log-partition */

/*
 * logZ(beta) = log sum_x exp(-beta f(x)), two passes (max, then compensated
 * sum of shifted exponentials).  Also returns E_p[f] through *mean_energy when
 * non-NULL (d logZ / d beta = -E_p[f]).
 */
double qo_logz_f32(const float *Q, int n, int64_t ldq, double beta, double *mean_energy,
                   int nthreads)
{
    if (n < 1 || n > 40)
        return NAN;
    int T = threads_for(nthreads);
    uint64_t total = 1ull << n;
    double M = -INFINITY;
#pragma omp parallel for num_threads(T) schedule(static) reduction(max : M)
    for (int64_t x = 0; x < (int64_t)total; ++x) {
        double a = -beta * energy_f(Q, n, ldq, (uint64_t)x);
        if (a > M)
            M = a;
    }
    nsum_t *S = (nsum_t *)calloc((size_t)T, sizeof(nsum_t));
    nsum_t *W = (nsum_t *)calloc((size_t)T, sizeof(nsum_t));
#pragma omp parallel num_threads(T)
    {
        int t = omp_get_thread_num();
        int nt = omp_get_num_threads();
        uint64_t a = total / nt * t, b = (t == nt - 1) ? total : total / nt * (t + 1);
        for (uint64_t x = a; x < b; ++x) {
            double e = energy_f(Q, n, ldq, x);
            double w = exp(-beta * e - M);
            nsum_add(&S[t], w);
            nsum_add(&W[t], w * e);
        }
    }
    nsum_t s = {0.0, 0.0}, we = {0.0, 0.0};
    for (int t = 0; t < T; ++t) {
        nsum_add(&s, nsum_val(&S[t]));
        nsum_add(&we, nsum_val(&W[t]));
    }
    free(S);
    free(W);
    double sum = nsum_val(&s);
    if (mean_energy)
        *mean_energy = nsum_val(&we) / sum;
    return M + log(sum);
}

/*
 * G (n x n, row-major, f64): G_ij = -beta sum_x p(x) x_i x_j for i <= j, 0 below
 * the diagonal; p(x) = exp(-beta f(x) - logz).
 */
int qo_grad_f32(const float *Q, int n, int64_t ldq, double beta, double logz, double *G,
                int nthreads)
{
    if (n < 1 || n > 40)
        return QO_ERR_ARG;
    int T = threads_for(nthreads);
    uint64_t total = 1ull << n;
    size_t nn = (size_t)n * n;
    nsum_t *acc = (nsum_t *)calloc((size_t)T * nn, sizeof(nsum_t));
#pragma omp parallel num_threads(T)
    {
        int t = omp_get_thread_num();
        int nt = omp_get_num_threads();
        nsum_t *A = acc + (size_t)t * nn;
        uint64_t a = total / nt * t, b = (t == nt - 1) ? total : total / nt * (t + 1);
        for (uint64_t x = a; x < b; ++x) {
            double p = exp(-beta * energy_f(Q, n, ldq, x) - logz);
            for (int i = 0; i < n; ++i) {
                if (!((x >> i) & 1u))
                    continue;
                for (int j = i; j < n; ++j)
                    if ((x >> j) & 1u)
                        nsum_add(&A[(size_t)i * n + j], p);
            }
        }
    }
    for (size_t e = 0; e < nn; ++e) {
        nsum_t s = {0.0, 0.0};
        for (int t = 0; t < T; ++t)
            nsum_add(&s, nsum_val(&acc[(size_t)t * nn + e]));
        size_t i = e / (size_t)n, j = e % (size_t)n;
        G[e] = (i <= j) ? -beta * nsum_val(&s) : 0.0;
    }
    free(acc);
    return QO_OK;
}

int qo_max_threads(void)
{
    return omp_get_max_threads();
}
