/*
 * Oracle: sparse L-QSW superoperator and truncated-Taylor expmv on the CPU.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled by gcc into a host
 * library that the tests, the smoke check and the CPU-baseline leg of the
 * benchmark load.  It shares no code with the GPU path and no product file
 * includes, links or calls it.
 *
 * Everything is plain float64 / complex128, one obvious loop per formula.
 *
 * Superoperator (Section 2.5.1 eq. qsw with the vectorisation of eq.
 * vec_mappings, written for the ROW-MAJOR vec index r(a,b) = a*N + b of
 * rho_ab).  With L_k = sqrt(R_ij)|i><j| (eq. lindblad, R_ij = |M_ij|) one has
 * L_k rho L_k^dag = R_ij rho_jj |i><i| and sum_k L_k^dag L_k = diag(K),
 * K_j = sum_i R_ij, so entry (a,b) of d(rho)/dt is
 *
 *   -i(1-w) ( sum_c H_ac rho_cb - sum_c rho_ac H_cb )
 *   + w ( [a==b] sum_j R_aj rho_jj - 1/2 (K_a + K_b) rho_ab ).
 *
 * oracle_superop_csr writes exactly these terms for every row, then sorts
 * the row by column and adds coinciding columns.  Entries whose value
 * happens to be zero are kept, so the pattern does not depend on w.
 *
 * Taylor expmv: one application of the Al-Mohy--Higham single-time
 * algorithm (the paper's `step`, Section 3.1) with given degree m and
 * scaling s:
 *   F = b; for s steps { c1 = |b|inf; for j = 1..m { b = (t/(s j)) A b;
 *   c2 = |b|inf; F += b; stop if c1 + c2 <= tol |F|inf; c1 = c2 } b = F }.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex zdouble;

typedef struct {
    int64_t col;
    zdouble val;
} entry_t;

static int cmp_entry(const void *x, const void *y)
{
    const entry_t *p = (const entry_t *)x, *q = (const entry_t *)y;
    return (p->col > q->col) - (p->col < q->col);
}

/* Collect, sort and merge the entries of row (a,b).  Returns the count. */
static int64_t build_row(int64_t N, int64_t a, int64_t b,
                         const int64_t *hp, const int32_t *hi, const zdouble *hv,
                         const int64_t *rp, const int32_t *ri, const double *rv,
                         const double *K, double w, entry_t *buf)
{
    int64_t cnt = 0;
    const zdouble mi = -I * (1.0 - w); /* -i(1-w) */
    /* -i(1-w) sum_c H_ac rho_cb : column r(c,b) = c*N + b */
    for (int64_t e = hp[a]; e < hp[a + 1]; ++e) {
        buf[cnt].col = (int64_t)hi[e] * N + b;
        buf[cnt].val = mi * hv[e];
        ++cnt;
    }
    /* +i(1-w) sum_c rho_ac H_cb : column r(a,c); H_cb = conj(H_bc) */
    for (int64_t e = hp[b]; e < hp[b + 1]; ++e) {
        buf[cnt].col = a * N + (int64_t)hi[e];
        buf[cnt].val = -mi * conj(hv[e]);
        ++cnt;
    }
    /* -w/2 (K_a + K_b) rho_ab */
    buf[cnt].col = a * N + b;
    buf[cnt].val = -0.5 * w * (K[a] + K[b]);
    ++cnt;
    /* w [a==b] sum_j R_aj rho_jj : column r(j,j) */
    if (a == b) {
        for (int64_t e = rp[a]; e < rp[a + 1]; ++e) {
            int64_t j = ri[e];
            buf[cnt].col = j * N + j;
            buf[cnt].val = w * rv[e];
            ++cnt;
        }
    }
    qsort(buf, (size_t)cnt, sizeof(entry_t), cmp_entry);
    int64_t out = 0;
    for (int64_t e = 0; e < cnt; ++e) {
        if (out > 0 && buf[out - 1].col == buf[e].col)
            buf[out - 1].val += buf[e].val;
        else
            buf[out++] = buf[e];
    }
    return out;
}

/*
 * H: N x N Hermitian CSR (complex, interleaved re/im), may hold a diagonal.
 * R: N x N CSR of rates R_ij = |ML_ij|^2 >= 0, may hold a diagonal.
 * Pass 1 (val == NULL): fills row_ptr (length N*N+1) only.
 * Pass 2: fills col and val as well (row_ptr must come from pass 1).
 * Returns nnz, or -1 on allocation failure.
 */
int64_t oracle_superop_csr(int64_t N,
                           const int64_t *hp, const int32_t *hi, const double *hv_ri,
                           const int64_t *rp, const int32_t *ri, const double *rv,
                           double w, int64_t *row_ptr, int32_t *col, double *val_ri)
{
    const zdouble *hv = (const zdouble *)hv_ri;
    zdouble *val = (zdouble *)val_ri;
    double *K = (double *)calloc((size_t)N, sizeof(double));
    if (!K) return -1;
    /* K_j = sum_i R_ij (column sums of R) */
    for (int64_t i = 0; i < N; ++i)
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) K[ri[e]] += rv[e];
    int64_t maxdeg = 0;
    for (int64_t i = 0; i < N; ++i) {
        int64_t d = hp[i + 1] - hp[i];
        if (d > maxdeg) maxdeg = d;
        d = rp[i + 1] - rp[i];
        if (d > maxdeg) maxdeg = d;
    }
    const int64_t cap = 3 * maxdeg + 2;
    const int64_t n = N * N;
    int failed = 0;
    if (val == NULL) {
        int64_t *len = (int64_t *)malloc((size_t)n * sizeof(int64_t));
        if (!len) { free(K); return -1; }
#pragma omp parallel
        {
            entry_t *buf = (entry_t *)malloc((size_t)cap * sizeof(entry_t));
            if (!buf) {
#pragma omp atomic write
                failed = 1;
            } else {
#pragma omp for schedule(static)
                for (int64_t r = 0; r < n; ++r)
                    len[r] = build_row(N, r / N, r % N, hp, hi, hv, rp, ri, rv, K, w, buf);
            }
            free(buf);
        }
        row_ptr[0] = 0;
        for (int64_t r = 0; r < n; ++r) row_ptr[r + 1] = row_ptr[r] + len[r];
        free(len);
    } else {
#pragma omp parallel
        {
            entry_t *buf = (entry_t *)malloc((size_t)cap * sizeof(entry_t));
            if (!buf) {
#pragma omp atomic write
                failed = 1;
            } else {
#pragma omp for schedule(static)
                for (int64_t r = 0; r < n; ++r) {
                    int64_t c = build_row(N, r / N, r % N, hp, hi, hv, rp, ri, rv, K, w, buf);
                    int64_t o = row_ptr[r];
                    for (int64_t e = 0; e < c; ++e) {
                        col[o + e] = (int32_t)buf[e].col;
                        val[o + e] = buf[e].val;
                    }
                }
            }
            free(buf);
        }
    }
    free(K);
    return failed ? -1 : row_ptr[n];
}

/* ||A||_1 = max_j sum_i |A_ij| (column sums, accumulated in storage order). */
double oracle_norm1(int64_t n, const int64_t *rp, const int32_t *ci, const double *val_ri)
{
    const zdouble *val = (const zdouble *)val_ri;
    double *cs = (double *)calloc((size_t)n, sizeof(double));
    if (!cs) return -1.0;
    for (int64_t r = 0; r < n; ++r)
        for (int64_t e = rp[r]; e < rp[r + 1]; ++e) cs[ci[e]] += cabs(val[e]);
    double m = 0.0;
    for (int64_t j = 0; j < n; ++j)
        if (cs[j] > m) m = cs[j];
    free(cs);
    return m;
}

/* y = A x */
void oracle_spmv(int64_t n, const int64_t *rp, const int32_t *ci, const double *val_ri,
                 const double *x_ri, double *y_ri)
{
    const zdouble *val = (const zdouble *)val_ri;
    const zdouble *x = (const zdouble *)x_ri;
    zdouble *y = (zdouble *)y_ri;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
        zdouble acc = 0.0;
        for (int64_t e = rp[r]; e < rp[r + 1]; ++e) acc += val[e] * x[ci[e]];
        y[r] = acc;
    }
}

static double inf_norm(int64_t n, const zdouble *v)
{
    double m = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double a = cabs(v[i]);
        if (a > m || isnan(a)) m = a;
    }
    return m;
}

/*
 * F = T_m(t A / s)^s b  with the early-termination test of the single-time
 * algorithm.  b_ri is read only.  Returns the number of matrix-vector
 * products performed, or -1 on allocation failure.
 */
int64_t oracle_taylor_expmv(int64_t n, const int64_t *rp, const int32_t *ci,
                            const double *val_ri, const double *b_ri, double t,
                            int32_t m, int32_t s, double tol, double *F_ri)
{
    const zdouble *b0 = (const zdouble *)b_ri;
    zdouble *F = (zdouble *)F_ri;
    zdouble *b = (zdouble *)malloc((size_t)n * sizeof(zdouble));
    zdouble *y = (zdouble *)malloc((size_t)n * sizeof(zdouble));
    if (!b || !y) { free(b); free(y); return -1; }
    memcpy(F, b0, (size_t)n * sizeof(zdouble));
    memcpy(b, b0, (size_t)n * sizeof(zdouble));
    int64_t products = 0;
    for (int32_t i = 1; i <= s; ++i) {
        double c1 = inf_norm(n, b);
        for (int32_t j = 1; j <= m; ++j) {
            oracle_spmv(n, rp, ci, (const double *)val_ri, (const double *)b, (double *)y);
            ++products;
            const double coef = t / ((double)s * (double)j);
            for (int64_t r = 0; r < n; ++r) b[r] = coef * y[r];
            double c2 = inf_norm(n, b);
            for (int64_t r = 0; r < n; ++r) F[r] += b[r];
            if (c1 + c2 <= tol * inf_norm(n, F)) break;
            c1 = c2;
        }
        memcpy(b, F, (size_t)n * sizeof(zdouble));
    }
    free(b);
    free(y);
    return products;
}
