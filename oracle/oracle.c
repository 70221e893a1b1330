/*
 * oracle.c -- plain, slow, obviously correct CPU reference for the SpMV / CG
 * path of "Morpheus unleashed: Fast cross-platform SpMV on emerging
 * architectures" (arXiv 2304.09511).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library and includes none of its files.
 *
 * Precision: FP64 throughout, except the FP32 inner solve of the mixed
 * refinement, whose vectors are float by definition.  Built with
 * -ffp-contract=off and without -ffast-math: every product and every sum is
 * rounded separately, in the order written.
 *
 * Storage conventions (Section III-B):
 *   COO  ai[k], aj[k], av[k], k in [0, nnz)
 *   CSR  irp[nrows+1] (irp[0]=0, irp[nrows]=nnz), aj[nnz], av[nnz]
 *   DIA  doff[ndiag] ascending, av[d*nrows + i] = A(i, i+doff[d])
 *        (the value of diagonal d that multiplies x[i+doff[d]] in row i;
 *        the paper's av(i,j) with the two indices swapped in memory)
 *
 * Status codes returned by the checking routines:
 *    0 ok, 1 not converged, -2 index out of range, -3 unsorted,
 *   -4 duplicate, -8 breakdown, -9 non-finite input.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_INDEX_RANGE (-2)
#define ORC_UNSORTED (-3)
#define ORC_DUPLICATE (-4)
#define ORC_BREAKDOWN (-8)
#define ORC_NONFINITE (-9)

/* ======================================================================
 * SpMV: the three algorithms of Section III-B
 * ==================================================================== */

/* Algorithm 1 (COO SpMV): y(ai(i)) += av(i)*x(aj(i)) over all stored entries.
 * The algorithm accumulates into y; here y is cleared first so the routine
 * computes y = A*x, the statement of the problem. */
void orc_coo_spmv(int64_t nrows, int64_t nnz, const int32_t *ai, const int32_t *aj,
                  const double *av, const double *x, double *y)
{
    for (int64_t i = 0; i < nrows; ++i)
        y[i] = 0.0;
    for (int64_t k = 0; k < nnz; ++k)
        y[ai[k]] += av[k] * x[aj[k]];
}

/* Algorithm 1 with float matrix, vectors and accumulation. */
void orc_coo_spmv_f32(int64_t nrows, int64_t nnz, const int32_t *ai, const int32_t *aj,
                      const float *av, const float *x, float *y)
{
    for (int64_t i = 0; i < nrows; ++i)
        y[i] = 0.0f;
    for (int64_t k = 0; k < nnz; ++k)
        y[ai[k]] += av[k] * x[aj[k]];
}

/* Algorithm 2 (CSR SpMV): per row, sum av(j)*x(aj(j)) over j in
 * [irp(i), irp(i+1)) and assign the sum to y(i). */
void orc_csr_spmv(int64_t nrows, const int32_t *irp, const int32_t *aj, const double *av,
                  const double *x, double *y)
{
    for (int64_t i = 0; i < nrows; ++i) {
        double sum = 0.0;
        for (int64_t j = irp[i]; j < irp[i + 1]; ++j)
            sum += av[j] * x[aj[j]];
        y[i] = sum;
    }
}

/* Algorithm 3 (DIA SpMV): per row, for each diagonal j, k = i + doff(j); if
 * 0 <= k < N add av(i,j)*x(k).  N is the number of columns. */
void orc_dia_spmv(int64_t nrows, int64_t ncols, int64_t ndiag, const int32_t *doff,
                  const double *av, const double *x, double *y)
{
    for (int64_t i = 0; i < nrows; ++i) {
        double sum = 0.0;
        for (int64_t j = 0; j < ndiag; ++j) {
            int64_t k = i + (int64_t)doff[j];
            if (k >= 0 && k < ncols)
                sum += av[j * nrows + i] * x[k];
        }
        y[i] = sum;
    }
}

/* ======================================================================
 * Canonical containers and conversions (Section III-B)
 * ==================================================================== */

/* Checks COO indices: range first, then (row, col) order.  Strictly
 * ascending keys are canonical; an equal neighbour is a duplicate; a
 * descending neighbour means unsorted (duplicates in unsorted input are
 * found after sorting). */
int orc_coo_check(int64_t nrows, int64_t ncols, int64_t nnz, const int32_t *ai,
                  const int32_t *aj)
{
    for (int64_t k = 0; k < nnz; ++k)
        if (ai[k] < 0 || ai[k] >= nrows || aj[k] < 0 || aj[k] >= ncols)
            return ORC_INDEX_RANGE;
    int unsorted = 0, dup = 0;
    for (int64_t k = 1; k < nnz; ++k) {
        if (ai[k] < ai[k - 1] || (ai[k] == ai[k - 1] && aj[k] < aj[k - 1]))
            unsorted = 1;
        else if (ai[k] == ai[k - 1] && aj[k] == aj[k - 1])
            dup = 1;
    }
    if (unsorted)
        return ORC_UNSORTED;
    if (dup)
        return ORC_DUPLICATE;
    return ORC_OK;
}

/* Stable counting sort of one key array; permutes perm accordingly. */
static void counting_pass(int64_t nnz, int64_t nkeys, const int32_t *key, int64_t *perm,
                          int64_t *tmp)
{
    int64_t *cnt = (int64_t *)calloc((size_t)nkeys + 1, sizeof(int64_t));
    for (int64_t k = 0; k < nnz; ++k)
        cnt[key[perm[k]] + 1]++;
    for (int64_t c = 0; c < nkeys; ++c)
        cnt[c + 1] += cnt[c];
    for (int64_t k = 0; k < nnz; ++k)
        tmp[cnt[key[perm[k]]]++] = perm[k];
    memcpy(perm, tmp, (size_t)nnz * sizeof(int64_t));
    free(cnt);
}

/* Sorts COO triples by (row, col): a stable pass by column, then a stable
 * pass by row.  Indices must be in range. */
void orc_coo_sort(int64_t nrows, int64_t ncols, int64_t nnz, int32_t *ai, int32_t *aj,
                  double *av)
{
    if (nnz == 0)
        return;
    int64_t *perm = (int64_t *)malloc((size_t)nnz * sizeof(int64_t));
    int64_t *tmp = (int64_t *)malloc((size_t)nnz * sizeof(int64_t));
    for (int64_t k = 0; k < nnz; ++k)
        perm[k] = k;
    counting_pass(nnz, ncols, aj, perm, tmp);
    counting_pass(nnz, nrows, ai, perm, tmp);
    int32_t *bi = (int32_t *)malloc((size_t)nnz * sizeof(int32_t));
    int32_t *bj = (int32_t *)malloc((size_t)nnz * sizeof(int32_t));
    double *bv = (double *)malloc((size_t)nnz * sizeof(double));
    for (int64_t k = 0; k < nnz; ++k) {
        bi[k] = ai[perm[k]];
        bj[k] = aj[perm[k]];
        bv[k] = av[perm[k]];
    }
    memcpy(ai, bi, (size_t)nnz * sizeof(int32_t));
    memcpy(aj, bj, (size_t)nnz * sizeof(int32_t));
    memcpy(av, bv, (size_t)nnz * sizeof(double));
    free(bi); free(bj); free(bv); free(perm); free(tmp);
}

/* CSR row pointers from sorted COO: irp[r] = number of entries whose row is
 * below r (so irp[0] = 0 and irp[nrows] = nnz).  aj and av carry over. */
void orc_coo_to_csr(int64_t nrows, int64_t nnz, const int32_t *ai, int32_t *irp)
{
    for (int64_t r = 0; r <= nrows; ++r)
        irp[r] = 0;
    for (int64_t k = 0; k < nnz; ++k)
        irp[ai[k] + 1]++;
    for (int64_t r = 0; r < nrows; ++r)
        irp[r + 1] += irp[r];
}

/* COO row indices from CSR: entries irp[r] .. irp[r+1]-1 belong to row r. */
void orc_csr_to_coo(int64_t nrows, const int32_t *irp, int32_t *ai)
{
    for (int64_t r = 0; r < nrows; ++r)
        for (int64_t k = irp[r]; k < irp[r + 1]; ++k)
            ai[k] = (int32_t)r;
}

/* Checks CSR structure: irp[0] = 0, monotone, irp[nrows] = nnz, columns in
 * range, columns strictly ascending within a row. */
int orc_csr_check(int64_t nrows, int64_t ncols, int64_t nnz, const int32_t *irp,
                  const int32_t *aj)
{
    if (irp[0] != 0 || irp[nrows] != nnz)
        return ORC_INDEX_RANGE;
    for (int64_t r = 0; r < nrows; ++r)
        if (irp[r + 1] < irp[r])
            return ORC_INDEX_RANGE;
    for (int64_t k = 0; k < nnz; ++k)
        if (aj[k] < 0 || aj[k] >= ncols)
            return ORC_INDEX_RANGE;
    int unsorted = 0, dup = 0;
    for (int64_t r = 0; r < nrows; ++r)
        for (int64_t k = irp[r] + 1; k < irp[r + 1]; ++k) {
            if (aj[k] < aj[k - 1])
                unsorted = 1;
            else if (aj[k] == aj[k - 1])
                dup = 1;
        }
    if (unsorted)
        return ORC_UNSORTED;
    if (dup)
        return ORC_DUPLICATE;
    return ORC_OK;
}

/* The distinct diagonal offsets j - i of the stored entries, ascending.
 * doff must hold nrows + ncols - 1 entries; returns ndiag. */
int64_t orc_dia_offsets(int64_t nrows, int64_t ncols, int64_t nnz, const int32_t *ai,
                        const int32_t *aj, int32_t *doff)
{
    int64_t span = nrows + ncols - 1;
    if (span <= 0)
        return 0;
    unsigned char *seen = (unsigned char *)calloc((size_t)span, 1);
    for (int64_t k = 0; k < nnz; ++k)
        seen[(int64_t)aj[k] - (int64_t)ai[k] + (nrows - 1)] = 1;
    int64_t nd = 0;
    for (int64_t s = 0; s < span; ++s)
        if (seen[s])
            doff[nd++] = (int32_t)(s - (nrows - 1));
    free(seen);
    return nd;
}

/* Band of a split matrix (a DIA band plus a remainder: the hybrid DIA/CSR
 * format among the further formats of Section IX, and the local/remote split
 * of the distributed HPCG runs, Section VII-D and Table III).  The band is
 * the diagonals, in ascending offset order, that hold at least one stored
 * entry and at least min_fill times as many stored entries as the diagonal
 * has slots inside the matrix (compared in FP64); entries on them form the
 * band and all others the remainder.  Returns the number of band offsets
 * written to doff. */
int64_t orc_split_offsets(int64_t nrows, int64_t ncols, int64_t nnz, const int32_t *ai,
                          const int32_t *aj, double min_fill, int32_t *doff)
{
    int64_t span = nrows + ncols - 1;
    if (span <= 0)
        return 0;
    int64_t *count = (int64_t *)calloc((size_t)span, sizeof(int64_t));
    for (int64_t k = 0; k < nnz; ++k)
        count[(int64_t)aj[k] - (int64_t)ai[k] + (nrows - 1)]++;
    int64_t nd = 0;
    for (int64_t s = 0; s < span; ++s) {
        int64_t d = s - (nrows - 1);
        /* rows i with 0 <= i < nrows and 0 <= i + d < ncols */
        int64_t lo = d < 0 ? -d : 0;
        int64_t hi = ncols - d < nrows ? ncols - d : nrows;
        int64_t slots = hi - lo;
        if (count[s] > 0 && (double)count[s] >= min_fill * (double)slots)
            doff[nd++] = (int32_t)d;
    }
    free(count);
    return nd;
}

/* DIA values from sorted COO: av_dia[d*nrows + i] = A(i, i + doff[d]), and
 * +0.0 in every slot that holds no stored entry. */
void orc_coo_to_dia(int64_t nrows, int64_t nnz, const int32_t *ai, const int32_t *aj,
                    const double *av, int64_t ndiag, const int32_t *doff, double *av_dia)
{
    for (int64_t s = 0; s < ndiag * nrows; ++s)
        av_dia[s] = 0.0;
    for (int64_t k = 0; k < nnz; ++k) {
        int64_t off = (int64_t)aj[k] - (int64_t)ai[k];
        int64_t d = -1;
        for (int64_t q = 0; q < ndiag; ++q)
            if (doff[q] == off) {
                d = q;
                break;
            }
        av_dia[d * nrows + ai[k]] = av[k];
    }
}

/* Number of in-range DIA slots whose value is not zero (+0.0 and -0.0 are
 * both dropped when converting back). */
int64_t orc_dia_nnz(int64_t nrows, int64_t ncols, int64_t ndiag, const int32_t *doff,
                    const double *av_dia)
{
    int64_t c = 0;
    for (int64_t i = 0; i < nrows; ++i)
        for (int64_t d = 0; d < ndiag; ++d) {
            int64_t k = i + (int64_t)doff[d];
            if (k >= 0 && k < ncols && av_dia[d * nrows + i] != 0.0)
                c++;
        }
    return c;
}

/* Number of in-range DIA slots (stored zeros included). */
int64_t orc_dia_slots(int64_t nrows, int64_t ncols, int64_t ndiag, const int32_t *doff)
{
    int64_t c = 0;
    for (int64_t i = 0; i < nrows; ++i)
        for (int64_t d = 0; d < ndiag; ++d) {
            int64_t k = i + (int64_t)doff[d];
            if (k >= 0 && k < ncols)
                c++;
        }
    return c;
}

/* Sorted COO from DIA: rows ascending; within a row the diagonals in
 * ascending offset order, which is ascending column order. */
void orc_dia_to_coo(int64_t nrows, int64_t ncols, int64_t ndiag, const int32_t *doff,
                    const double *av_dia, int32_t *ai, int32_t *aj, double *av)
{
    int64_t c = 0;
    for (int64_t i = 0; i < nrows; ++i)
        for (int64_t d = 0; d < ndiag; ++d) {
            int64_t k = i + (int64_t)doff[d];
            double v = av_dia[d * nrows + i];
            if (k >= 0 && k < ncols && v != 0.0) {
                ai[c] = (int32_t)i;
                aj[c] = (int32_t)k;
                av[c] = v;
                c++;
            }
        }
}

/* ======================================================================
 * Conjugate gradients (HPCG's solver with the preconditioner disabled,
 * Section VII-D).  Textbook Hestenes-Stiefel recurrence.
 * ==================================================================== */

static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s += a[i] * b[i];
    return s;
}

double orc_dot(int64_t n, const double *a, const double *b) { return dot(n, a, b); }

static int all_finite(int64_t n, const double *v)
{
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(v[i]))
            return 0;
    return 1;
}

/* Unpreconditioned CG on the COO matrix A (square, n rows).
 *   r = b - A x0; rho0 = r.r; p = r
 *   repeat: q = A p; sigma = p.q; alpha = rho/sigma; x += alpha p;
 *           r -= alpha q; rho' = r.r; stop when sqrt(rho') <= tol*sqrt(rho0);
 *           beta = rho'/rho; p = r + beta p
 * The iteration count is the number of loop SpMVs.  sigma <= 0 or non-finite
 * is a breakdown.  out[0] = ||r_k||/||r_0|| (recursive residual),
 * out[1] = ||b - A x||/||b|| (true residual). */
int orc_cg(int64_t n, int64_t nnz, const int32_t *ai, const int32_t *aj, const double *av,
           const double *b, double *x, double tol, int64_t maxit, int64_t *iters,
           double *out)
{
    *iters = 0;
    out[0] = out[1] = 0.0;
    if (!all_finite(n, b) || !all_finite(n, x))
        return ORC_NONFINITE;
    double *r = (double *)malloc((size_t)(n ? n : 1) * sizeof(double));
    double *p = (double *)malloc((size_t)(n ? n : 1) * sizeof(double));
    double *q = (double *)malloc((size_t)(n ? n : 1) * sizeof(double));
    int status = ORC_NOT_CONVERGED;
    orc_coo_spmv(n, nnz, ai, aj, av, x, q);
    for (int64_t i = 0; i < n; ++i)
        r[i] = b[i] - q[i];
    double rho0 = dot(n, r, r);
    double rho = rho0, rho_new = rho0;
    if (rho0 == 0.0) {
        status = ORC_OK;
    } else {
        for (int64_t i = 0; i < n; ++i)
            p[i] = r[i];
        for (int64_t k = 1; k <= maxit; ++k) {
            orc_coo_spmv(n, nnz, ai, aj, av, p, q);
            double sigma = dot(n, p, q);
            if (!(sigma > 0.0) || !isfinite(sigma)) {
                *iters = k;
                status = ORC_BREAKDOWN;
                break;
            }
            double alpha = rho / sigma;
            for (int64_t i = 0; i < n; ++i)
                x[i] += alpha * p[i];
            for (int64_t i = 0; i < n; ++i)
                r[i] -= alpha * q[i];
            rho_new = dot(n, r, r);
            *iters = k;
            if (sqrt(rho_new) <= tol * sqrt(rho0)) {
                status = ORC_OK;
                break;
            }
            double beta = rho_new / rho;
            for (int64_t i = 0; i < n; ++i)
                p[i] = r[i] + beta * p[i];
            rho = rho_new;
        }
    }
    out[0] = rho0 > 0.0 ? sqrt(rho_new) / sqrt(rho0) : 0.0;
    orc_coo_spmv(n, nnz, ai, aj, av, x, q);
    for (int64_t i = 0; i < n; ++i)
        q[i] = b[i] - q[i];
    double bn = sqrt(dot(n, b, b));
    out[1] = bn > 0.0 ? sqrt(dot(n, q, q)) / bn : sqrt(dot(n, q, q));
    free(r); free(p); free(q);
    return status;
}

/* ======================================================================
 * Mixed-precision iterative refinement (an addition to the paper's method):
 * FP64 outer residual and update, FP32 inner CG.
 * ==================================================================== */

/* Dot of two float vectors accumulated in double. */
static double dot_f32(int64_t n, const float *a, const float *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s += (double)a[i] * (double)b[i];
    return s;
}

/* Inner solve: CG on A32 d = r32 from d = 0, float vectors, float SpMV,
 * dots accumulated in double, alpha and beta in double and rounded to float
 * where they scale a float vector.  Stops when ||r_k|| <= rtol*||r_0||, after
 * maxit iterations, or at sigma <= 0 (the outer loop then continues from the
 * current correction).  Returns the iteration count. */
static int64_t inner_cg_f32(int64_t n, int64_t nnz, const int32_t *ai, const int32_t *aj,
                            const float *av32, const float *r0, float *d, double rtol,
                            int64_t maxit, float *r, float *p, float *q)
{
    for (int64_t i = 0; i < n; ++i) {
        d[i] = 0.0f;
        r[i] = r0[i];
        p[i] = r0[i];
    }
    double rho0 = dot_f32(n, r, r), rho = rho0;
    if (rho0 == 0.0)
        return 0;
    int64_t k;
    for (k = 1; k <= maxit; ++k) {
        orc_coo_spmv_f32(n, nnz, ai, aj, av32, p, q);
        double sigma = dot_f32(n, p, q);
        if (!(sigma > 0.0) || !isfinite(sigma))
            return k;
        float alpha = (float)(rho / sigma);
        for (int64_t i = 0; i < n; ++i)
            d[i] += alpha * p[i];
        for (int64_t i = 0; i < n; ++i)
            r[i] -= alpha * q[i];
        double rho_new = dot_f32(n, r, r);
        if (sqrt(rho_new) <= rtol * sqrt(rho0))
            return k;
        float beta = (float)(rho_new / rho);
        for (int64_t i = 0; i < n; ++i)
            p[i] = r[i] + beta * p[i];
        rho = rho_new;
    }
    return maxit;
}

/* Outer loop:
 *   r = b - A x (FP64); stop when ||r|| <= tol*||b||;
 *   s = ||r||; r32 = fp32(r/s); inner CG on fp32(A) d = r32; x += s*fp64(d);
 * at most max_outer corrections.  counts[0] = corrections applied,
 * counts[1] = total inner iterations; out[0] = final ||b - A x||/||b||. */
int orc_mixed_ir(int64_t n, int64_t nnz, const int32_t *ai, const int32_t *aj,
                 const double *av, const double *b, double *x, double tol, double inner_rtol,
                 int64_t inner_maxit, int64_t max_outer, int64_t *counts, double *out)
{
    counts[0] = counts[1] = 0;
    out[0] = 0.0;
    if (!all_finite(n, b) || !all_finite(n, x))
        return ORC_NONFINITE;
    size_t nb = (size_t)(n ? n : 1);
    float *av32 = (float *)malloc((size_t)(nnz ? nnz : 1) * sizeof(float));
    for (int64_t k = 0; k < nnz; ++k)
        av32[k] = (float)av[k];
    double *r = (double *)malloc(nb * sizeof(double));
    float *r32 = (float *)malloc(nb * sizeof(float));
    float *d = (float *)malloc(nb * sizeof(float));
    float *ri = (float *)malloc(nb * sizeof(float));
    float *pi = (float *)malloc(nb * sizeof(float));
    float *qi = (float *)malloc(nb * sizeof(float));
    double bn = sqrt(dot(n, b, b));
    int status = ORC_NOT_CONVERGED;
    for (int64_t outer = 0;; ++outer) {
        orc_coo_spmv(n, nnz, ai, aj, av, x, r);
        for (int64_t i = 0; i < n; ++i)
            r[i] = b[i] - r[i];
        double rn = sqrt(dot(n, r, r));
        out[0] = bn > 0.0 ? rn / bn : rn;
        if (rn <= tol * bn) {
            status = ORC_OK;
            break;
        }
        if (outer == max_outer)
            break;
        for (int64_t i = 0; i < n; ++i)
            r32[i] = (float)(r[i] / rn);
        counts[1] += inner_cg_f32(n, nnz, ai, aj, av32, r32, d, inner_rtol, inner_maxit, ri,
                                  pi, qi);
        for (int64_t i = 0; i < n; ++i)
            x[i] += rn * (double)d[i];
        counts[0]++;
    }
    free(av32); free(r); free(r32); free(d); free(ri); free(pi); free(qi);
    return status;
}

/* Mixed-precision CG with reliable updates (van der Vorst and Ye's residual
 * replacement, used for mixed precision by Clark et al.): one CG recurrence
 * runs in FP32 (SpMV with fp32(A), FP32 vectors, dot products accumulated
 * in FP64) and accumulates its correction in an FP32 vector d.  After each
 * iteration, when the recursive residual norm has dropped to delta times the
 * largest residual norm since the last update, or to the stopping threshold
 * tol*||b||, the update is made: x += fp64(d), d = 0, the residual is
 * recomputed as b - A x in FP64 and replaces the FP32 one, and the largest
 * norm restarts from it.  The search direction is kept.  The solve stops when
 * the recomputed residual meets ||b - A x|| <= tol*||b||.
 * counts[0] = updates, counts[1] = iterations; out[0] = ||b - A x||/||b||
 * of the returned x. */
int orc_mixed_ru(int64_t n, int64_t nnz, const int32_t *ai, const int32_t *aj,
                 const double *av, const double *b, double *x, double tol, double delta,
                 int64_t maxit, int64_t *counts, double *out)
{
    counts[0] = counts[1] = 0;
    out[0] = 0.0;
    if (!all_finite(n, b) || !all_finite(n, x))
        return ORC_NONFINITE;
    size_t nb = (size_t)(n ? n : 1);
    float *av32 = (float *)malloc((size_t)(nnz ? nnz : 1) * sizeof(float));
    for (int64_t k = 0; k < nnz; ++k)
        av32[k] = (float)av[k];
    double *r = (double *)malloc(nb * sizeof(double));
    float *r32 = (float *)malloc(nb * sizeof(float));
    float *d = (float *)malloc(nb * sizeof(float));
    float *p = (float *)malloc(nb * sizeof(float));
    float *q = (float *)malloc(nb * sizeof(float));
    double bn = sqrt(dot(n, b, b));
    double thresh = tol * bn;
    int status = ORC_NOT_CONVERGED;

    /* true residual, and the FP32 recurrence started from it */
    orc_coo_spmv(n, nnz, ai, aj, av, x, r);
    for (int64_t i = 0; i < n; ++i)
        r[i] = b[i] - r[i];
    double rn = sqrt(dot(n, r, r));
    out[0] = bn > 0.0 ? rn / bn : rn;
    if (rn <= thresh) {
        status = ORC_OK;
        goto done;
    }
    for (int64_t i = 0; i < n; ++i) {
        r32[i] = (float)r[i];
        p[i] = r32[i];
        d[i] = 0.0f;
    }
    double rho = dot_f32(n, r32, r32);
    double rmax = sqrt(rho);
    for (int64_t k = 1; k <= maxit; ++k) {
        orc_coo_spmv_f32(n, nnz, ai, aj, av32, p, q);
        double sigma = dot_f32(n, p, q);
        counts[1] = k;
        if (!(sigma > 0.0) || !isfinite(sigma)) {
            status = ORC_BREAKDOWN;
            break;
        }
        float alpha = (float)(rho / sigma);
        for (int64_t i = 0; i < n; ++i)
            d[i] += alpha * p[i];
        for (int64_t i = 0; i < n; ++i)
            r32[i] -= alpha * q[i];
        double rho_new = dot_f32(n, r32, r32);
        double rn32 = sqrt(rho_new);
        if (rn32 <= delta * rmax || rn32 <= thresh) {
            /* reliable update */
            for (int64_t i = 0; i < n; ++i) {
                x[i] += (double)d[i];
                d[i] = 0.0f;
            }
            counts[0]++;
            orc_coo_spmv(n, nnz, ai, aj, av, x, r);
            for (int64_t i = 0; i < n; ++i)
                r[i] = b[i] - r[i];
            rn = sqrt(dot(n, r, r));
            out[0] = bn > 0.0 ? rn / bn : rn;
            if (rn <= thresh) {
                status = ORC_OK;
                break;
            }
            for (int64_t i = 0; i < n; ++i)
                r32[i] = (float)r[i];
            rho_new = dot_f32(n, r32, r32);
            rmax = sqrt(rho_new);
        } else if (rn32 > rmax) {
            rmax = rn32;
        }
        float beta = (float)(rho_new / rho);
        for (int64_t i = 0; i < n; ++i)
            p[i] = r32[i] + beta * p[i];
        rho = rho_new;
    }
    if (status != ORC_OK) {
        /* fold in the correction not yet applied and report its residual */
        for (int64_t i = 0; i < n; ++i)
            x[i] += (double)d[i];
        orc_coo_spmv(n, nnz, ai, aj, av, x, r);
        for (int64_t i = 0; i < n; ++i)
            r[i] = b[i] - r[i];
        rn = sqrt(dot(n, r, r));
        out[0] = bn > 0.0 ? rn / bn : rn;
    }
done:
    free(av32); free(r); free(r32); free(d); free(p); free(q);
    return status;
}

/* ======================================================================
 * Format-selector features (an addition to the paper: its auto-tuners pick
 * a format per matrix, Sections VII-D and IX)
 * ==================================================================== */

/* Eight features of a sorted COO matrix:
 *   0 rows, 1 nnz, 2 mean row length, 3 population variance of row lengths,
 *   4 max row length, 5 number of distinct diagonals, 6 DIA fill ratio
 *   nnz/(ndiag*rows), 7 max |j - i| / ncols. */
void orc_features(int64_t nrows, int64_t ncols, int64_t nnz, const int32_t *ai,
                  const int32_t *aj, double *f)
{
    int64_t *len = (int64_t *)calloc((size_t)(nrows ? nrows : 1), sizeof(int64_t));
    for (int64_t k = 0; k < nnz; ++k)
        len[ai[k]]++;
    double mean = nrows ? (double)nnz / (double)nrows : 0.0;
    double var = 0.0;
    int64_t mx = 0;
    for (int64_t i = 0; i < nrows; ++i) {
        double dlt = (double)len[i] - mean;
        var += dlt * dlt;
        if (len[i] > mx)
            mx = len[i];
    }
    var = nrows ? var / (double)nrows : 0.0;
    int32_t *doff = (int32_t *)malloc((size_t)((nrows + ncols) > 1 ? nrows + ncols : 1) *
                                      sizeof(int32_t));
    int64_t nd = orc_dia_offsets(nrows, ncols, nnz, ai, aj, doff);
    int64_t bw = 0;
    for (int64_t k = 0; k < nnz; ++k) {
        int64_t o = (int64_t)aj[k] - (int64_t)ai[k];
        if (o < 0)
            o = -o;
        if (o > bw)
            bw = o;
    }
    f[0] = (double)nrows;
    f[1] = (double)nnz;
    f[2] = mean;
    f[3] = var;
    f[4] = (double)mx;
    f[5] = (double)nd;
    f[6] = (nd > 0 && nrows > 0) ? (double)nnz / ((double)nd * (double)nrows) : 0.0;
    f[7] = ncols > 0 ? (double)bw / (double)ncols : 0.0;
    free(len);
    free(doff);
}

/* ======================================================================
 * Selector network: MLP 8-64-64-7 with ReLU, softmax cross-entropy, Adam;
 * one output per format of the label set (COO, CSR, DIA, ELL, SELL, HYB,
 * HDC).
 * Parameter layout (row-major, input index first):
 *   W1[8][64], b1[64], W2[64][64], b2[64], W3[64][7], b3[7]  (5191 values)
 * ==================================================================== */
#define NI 8
#define NH 64
#define NO 7
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + NI * NH)
#define OFF_W2 (OFF_B1 + NH)
#define OFF_B2 (OFF_W2 + NH * NH)
#define OFF_W3 (OFF_B2 + NH)
#define OFF_B3 (OFF_W3 + NH * NO)
#define NPARAM (OFF_B3 + NO)

int64_t orc_mlp_nparam(void) { return NPARAM; }

/* Forward pass of one sample: pre-activations a1, a2, hidden h1, h2, logits z. */
static void mlp_sample(const double *w, const double *xin, double *a1, double *h1, double *a2,
                       double *h2, double *z)
{
    for (int j = 0; j < NH; ++j) {
        double s = w[OFF_B1 + j];
        for (int i = 0; i < NI; ++i)
            s += xin[i] * w[OFF_W1 + i * NH + j];
        a1[j] = s;
        h1[j] = s > 0.0 ? s : 0.0;
    }
    for (int k = 0; k < NH; ++k) {
        double s = w[OFF_B2 + k];
        for (int j = 0; j < NH; ++j)
            s += h1[j] * w[OFF_W2 + j * NH + k];
        a2[k] = s;
        h2[k] = s > 0.0 ? s : 0.0;
    }
    for (int c = 0; c < NO; ++c) {
        double s = w[OFF_B3 + c];
        for (int k = 0; k < NH; ++k)
            s += h2[k] * w[OFF_W3 + k * NO + c];
        z[c] = s;
    }
}

/* Logits of n samples (row-major X[n][8]) into z[n][3]. */
void orc_mlp_forward(const double *w, const double *X, int64_t n, double *z)
{
    double a1[NH], h1[NH], a2[NH], h2[NH];
    for (int64_t s = 0; s < n; ++s)
        mlp_sample(w, X + s * NI, a1, h1, a2, h2, z + s * NO);
}

/* Mean softmax cross-entropy over n samples and its gradient with respect to
 * every parameter (grad has the parameter layout).  ReLU'(0) is taken as 0. */
double orc_mlp_loss_grad(const double *w, const double *X, const int32_t *labels, int64_t n,
                         double *grad)
{
    double a1[NH], h1[NH], a2[NH], h2[NH], z[NO], dz[NO], dh2[NH], dh1[NH];
    for (int i = 0; i < NPARAM; ++i)
        grad[i] = 0.0;
    double loss = 0.0;
    for (int64_t s = 0; s < n; ++s) {
        const double *xin = X + s * NI;
        mlp_sample(w, xin, a1, h1, a2, h2, z);
        double m = z[0];
        for (int c = 1; c < NO; ++c)
            if (z[c] > m)
                m = z[c];
        double den = 0.0;
        for (int c = 0; c < NO; ++c)
            den += exp(z[c] - m);
        int y = labels[s];
        loss += -((z[y] - m) - log(den));
        for (int c = 0; c < NO; ++c)
            dz[c] = (exp(z[c] - m) / den - (c == y ? 1.0 : 0.0)) / (double)n;
        for (int c = 0; c < NO; ++c) {
            grad[OFF_B3 + c] += dz[c];
            for (int k = 0; k < NH; ++k)
                grad[OFF_W3 + k * NO + c] += h2[k] * dz[c];
        }
        for (int k = 0; k < NH; ++k) {
            double g = 0.0;
            for (int c = 0; c < NO; ++c)
                g += w[OFF_W3 + k * NO + c] * dz[c];
            dh2[k] = a2[k] > 0.0 ? g : 0.0;
        }
        for (int k = 0; k < NH; ++k) {
            grad[OFF_B2 + k] += dh2[k];
            for (int j = 0; j < NH; ++j)
                grad[OFF_W2 + j * NH + k] += h1[j] * dh2[k];
        }
        for (int j = 0; j < NH; ++j) {
            double g = 0.0;
            for (int k = 0; k < NH; ++k)
                g += w[OFF_W2 + j * NH + k] * dh2[k];
            dh1[j] = a1[j] > 0.0 ? g : 0.0;
        }
        for (int j = 0; j < NH; ++j) {
            grad[OFF_B1 + j] += dh1[j];
            for (int i = 0; i < NI; ++i)
                grad[OFF_W1 + i * NH + j] += xin[i] * dh1[j];
        }
    }
    return n ? loss / (double)n : 0.0;
}

/* One Adam step (Kingma and Ba, 2015, Algorithm 1) at step t >= 1. */
void orc_adam_step(int64_t np, double *w, double *m, double *v, const double *g, double lr,
                   int64_t t, double b1, double b2, double eps)
{
    double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int64_t i = 0; i < np; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        w[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* ------------------------------------------------------------------------
 * Symmetric Gauss-Seidel: the smoother of HPCG's preconditioner (Section
 * VII-D describes HPCG as PCG preconditioned by symmetric Gauss-Seidel
 * inside a multigrid cycle; the textbook sweep is Saad, Section 4.1).
 * One forward sweep visits the rows in `order`, one backward sweep visits
 * them in reverse; row i becomes x_i = (r_i - sum_{j != i} a_ij x_j) / a_ii
 * with the newest x_j.  The sum runs over row i's entries in storage
 * order, starting from r_i.  Returns ORC_BREAKDOWN when a visited row holds
 * no nonzero diagonal entry (x untouched from that row on), else ORC_OK.
 * ---------------------------------------------------------------------- */
static int gs_row(const int32_t *irp, const int32_t *aj, const double *av, int32_t i,
                  const double *r, double *x)
{
    double s = r[i], d = 0.0;
    for (int32_t k = irp[i]; k < irp[i + 1]; ++k) {
        if (aj[k] == i)
            d = av[k];
        else
            s -= av[k] * x[aj[k]];
    }
    if (d == 0.0)
        return ORC_BREAKDOWN;
    x[i] = s / d;
    return ORC_OK;
}

int orc_symgs(int64_t n, const int32_t *irp, const int32_t *aj, const double *av,
              const int32_t *order, const double *r, double *x)
{
    for (int64_t t = 0; t < n; ++t)
        if (gs_row(irp, aj, av, order[t], r, x) != ORC_OK)
            return ORC_BREAKDOWN;
    for (int64_t t = n - 1; t >= 0; --t)
        if (gs_row(irp, aj, av, order[t], r, x) != ORC_OK)
            return ORC_BREAKDOWN;
    return ORC_OK;
}

/* One forward (dir = 1) or backward (dir = -1) sweep alone. */
int orc_gs_sweep(int64_t n, const int32_t *irp, const int32_t *aj, const double *av,
                 const int32_t *order, int dir, const double *r, double *x)
{
    for (int64_t u = 0; u < n; ++u) {
        const int64_t t = dir > 0 ? u : n - 1 - u;
        if (gs_row(irp, aj, av, order[t], r, x) != ORC_OK)
            return ORC_BREAKDOWN;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Padded formats named as further work in Section IX.
 *
 * ELL (ELLPACK): every row gets K = (longest row) slots, stored column-major:
 * slot k of row i at k*nrows + i holds the row's k-th entry (columns
 * ascending); slots past the row's length hold column -1 and value +0.0.
 *
 * SELL-C-sigma (Kreutzer et al., SIAM J. Sci. Comput. 36(5), 2014): rows are
 * sorted by descending length, stably, inside windows of sigma consecutive
 * rows; perm[p] is the row at sorted position p.  Positions are cut into
 * slices of C; slice s is as wide as its longest row and starts at cs[s]
 * (cs[s+1] = cs[s] + C * width_s); slot k of position p in slice s is at
 * cs[s] + k*C + (p - s*C), padded as ELL (positions past the last row too).
 * ---------------------------------------------------------------------- */
int64_t orc_ell_width(int64_t nrows, const int32_t *irp)
{
    int64_t k = 0;
    for (int64_t i = 0; i < nrows; ++i)
        if (irp[i + 1] - irp[i] > k)
            k = irp[i + 1] - irp[i];
    return k;
}

void orc_csr_to_ell(int64_t nrows, const int32_t *irp, const int32_t *aj, const double *av,
                    int64_t K, int32_t *ecol, double *eval)
{
    for (int64_t i = 0; i < nrows; ++i)
        for (int64_t k = 0; k < K; ++k) {
            const int64_t len = irp[i + 1] - irp[i];
            ecol[k * nrows + i] = k < len ? aj[irp[i] + k] : -1;
            eval[k * nrows + i] = k < len ? av[irp[i] + k] : 0.0;
        }
}

/* y_i = sum over the row's slots, k ascending, of value * x[column]; padding
 * slots (column -1) are skipped. */
void orc_ell_spmv(int64_t nrows, int64_t K, const int32_t *ecol, const double *eval,
                  const double *x, double *y)
{
    for (int64_t i = 0; i < nrows; ++i) {
        double sum = 0.0;
        for (int64_t k = 0; k < K; ++k)
            if (ecol[k * nrows + i] >= 0)
                sum += eval[k * nrows + i] * x[ecol[k * nrows + i]];
        y[i] = sum;
    }
}

/* perm: stable descending-length order inside each window of sigma rows,
 * by counting: longer rows first, equal lengths in row order. */
void orc_sell_perm(int64_t nrows, const int32_t *irp, int64_t sigma, int32_t *perm)
{
    for (int64_t w0 = 0; w0 < nrows; w0 += sigma) {
        const int64_t w1 = w0 + sigma < nrows ? w0 + sigma : nrows;
        int64_t maxlen = 0;
        for (int64_t i = w0; i < w1; ++i)
            if (irp[i + 1] - irp[i] > maxlen)
                maxlen = irp[i + 1] - irp[i];
        int64_t p = w0;
        for (int64_t len = maxlen; len >= 0; --len)
            for (int64_t i = w0; i < w1; ++i)
                if (irp[i + 1] - irp[i] == len)
                    perm[p++] = (int32_t)i;
    }
}

/* cs[0..nslices] for slices of C positions; returns nslices. */
int64_t orc_sell_offsets(int64_t nrows, const int32_t *irp, const int32_t *perm, int64_t C,
                         int64_t *cs)
{
    const int64_t ns = (nrows + C - 1) / C;
    cs[0] = 0;
    for (int64_t s = 0; s < ns; ++s) {
        int64_t w = 0;
        for (int64_t p = s * C; p < (s + 1) * C && p < nrows; ++p) {
            const int64_t len = irp[perm[p] + 1] - irp[perm[p]];
            if (len > w)
                w = len;
        }
        cs[s + 1] = cs[s] + C * w;
    }
    return ns;
}

void orc_csr_to_sell(int64_t nrows, const int32_t *irp, const int32_t *aj, const double *av,
                     int64_t C, const int32_t *perm, const int64_t *cs, int32_t *scol, double *sval)
{
    const int64_t ns = (nrows + C - 1) / C;
    for (int64_t s = 0; s < ns; ++s) {
        const int64_t w = (cs[s + 1] - cs[s]) / C;
        for (int64_t r = 0; r < C; ++r) {
            const int64_t p = s * C + r;
            const int64_t i = p < nrows ? perm[p] : -1;
            const int64_t len = i >= 0 ? irp[i + 1] - irp[i] : 0;
            for (int64_t k = 0; k < w; ++k) {
                scol[cs[s] + k * C + r] = k < len ? aj[irp[i] + k] : -1;
                sval[cs[s] + k * C + r] = k < len ? av[irp[i] + k] : 0.0;
            }
        }
    }
}

/* y[perm[p]] = sum over position p's slots, k ascending (padding skipped). */
void orc_sell_spmv(int64_t nrows, int64_t C, const int32_t *perm, const int64_t *cs,
                   const int32_t *scol, const double *sval, const double *x, double *y)
{
    for (int64_t p = 0; p < nrows; ++p) {
        const int64_t s = p / C, r = p % C;
        const int64_t w = (cs[s + 1] - cs[s]) / C;
        double sum = 0.0;
        for (int64_t k = 0; k < w; ++k) {
            const int64_t q = cs[s] + k * C + r;
            if (scol[q] >= 0)
                sum += sval[q] * x[scol[q]];
        }
        y[perm[p]] = sum;
    }
}

/* ------------------------------------------------------------------------
 * HYB (Bell and Garland, SC'09): the first K entries of each row in ELL,
 * the rest in COO (canonical order).  The width rule keeps ELL dense: K is
 * the largest k such that at least max(4096, nrows/3) rows (all rows when
 * fewer) hold k or more entries (0 for an empty matrix).
 * ---------------------------------------------------------------------- */
int64_t orc_hyb_width(int64_t nrows, const int32_t *irp)
{
    int64_t need = nrows / 3 > 4096 ? nrows / 3 : 4096;
    if (need > nrows)
        need = nrows;
    int64_t best = 0;
    for (int64_t k = 1;; ++k) {
        int64_t rows = 0;
        for (int64_t i = 0; i < nrows; ++i)
            if (irp[i + 1] - irp[i] >= k)
                ++rows;
        if (rows < need || rows == 0)
            break;
        best = k;
    }
    return best;
}

/* Number of entries past the K-th of their row. */
int64_t orc_hyb_rest(int64_t nrows, const int32_t *irp, int64_t K)
{
    int64_t r = 0;
    for (int64_t i = 0; i < nrows; ++i)
        if (irp[i + 1] - irp[i] > K)
            r += irp[i + 1] - irp[i] - K;
    return r;
}

void orc_csr_to_hyb(int64_t nrows, const int32_t *irp, const int32_t *aj, const double *av,
                    int64_t K, int32_t *ecol, double *eval, int32_t *ri, int32_t *rj, double *rv)
{
    int64_t q = 0;
    for (int64_t i = 0; i < nrows; ++i) {
        const int64_t len = irp[i + 1] - irp[i];
        for (int64_t k = 0; k < K; ++k) {
            ecol[k * nrows + i] = k < len ? aj[irp[i] + k] : -1;
            eval[k * nrows + i] = k < len ? av[irp[i] + k] : 0.0;
        }
        for (int64_t k = K; k < len; ++k) {
            ri[q] = (int32_t)i;
            rj[q] = aj[irp[i] + k];
            rv[q] = av[irp[i] + k];
            ++q;
        }
    }
}
