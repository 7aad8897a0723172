/*
 * mi_oracle.c -- plain CPU oracle for all-pairs binary mutual information,
 * and for its extension to categorical variables (at the end of the file).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU path is checked against.  It shares no code with the
 * GPU library and the product path never loads it.
 *
 * What it computes (Section 1, Eq. 1 of the paper, unrolled over the four
 * cells in Eq. 2): for binary columns X_i, X_j of an m-row matrix,
 *
 *   MI(X_i; X_j) = sum over x, y in {0,1} of p(x,y) * log2( p(x,y) / (p(x) p(y)) )
 *
 * with p(x,y) = n_xy / m (joint counts over the rows, Section 2 step 2),
 * p(x) and p(y) the marginals (Section 2 step 3).  Reading adopted where the
 * paper is silent: a cell with n_xy = 0 contributes exactly 0 (0 log 0 = 0)
 * instead of the unspecified small epsilon of Section 2 step 5; when n_xy > 0
 * both marginals are positive, so no division by zero can occur.
 *
 * Counting is a direct loop over the rows for each pair, the definition of a
 * joint count.  For each cell the ratio p(x,y)/(p(x)p(y)) equals
 * (n_xy * m) / (n_x * n_y); both products are formed exactly in int64 before
 * the conversion to double, so the only rounding is the division, the log2
 * and the final sum.  Units are bits.
 *
 * Rows are samples and columns are variables (the paper's D is rows x cols,
 * Section 2 step 1); X is row-major with a row pitch ldx >= n.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>

/* One cell's contribution, in bits, multiplied by m: n_xy * log2(n_xy m / (n_x n_y)). */
static double cell_term(int64_t nxy, int64_t nx, int64_t ny, int64_t m)
{
    if (nxy == 0) return 0.0;                    /* 0 log 0 = 0 */
    double num = (double)(nxy * m);              /* exact below 2^53 */
    double den = (double)(nx * ny);
    return (double)nxy * log2(num / den);
}

/* Count the four cells of a pair of columns by looping over the rows.  Row k
 * of column i is xi[k * stride] (stride = ldx for the row-major X, 1 for a
 * column of the transposed layout), likewise for column j. */
static void count_pair(const uint8_t* xcol_i, const uint8_t* xcol_j, int64_t m, int64_t stride,
                       int64_t* n11, int64_t* n10, int64_t* n01, int64_t* n00)
{
    int64_t a = 0, b = 0, c = 0, d = 0;
    for (int64_t k = 0; k < m; ++k) {
        int xi = xcol_i[k * stride] != 0;
        int xj = xcol_j[k * stride] != 0;
        if (xi && xj) ++a;
        else if (xi && !xj) ++b;
        else if (!xi && xj) ++c;
        else ++d;
    }
    *n11 = a; *n10 = b; *n01 = c; *n00 = d;
}

/* MI of one pair from its four cell counts (Eq. 2), in bits. */
double mi_oracle_from_counts(int64_t n11, int64_t n10, int64_t n01, int64_t n00)
{
    int64_t m = n11 + n10 + n01 + n00;
    int64_t xi1 = n11 + n10, xi0 = n01 + n00;    /* marginal counts of X_i */
    int64_t xj1 = n11 + n01, xj0 = n10 + n00;    /* marginal counts of X_j */
    if (m <= 0) return NAN;
    double s = cell_term(n11, xi1, xj1, m)
             + cell_term(n10, xi1, xj0, m)
             + cell_term(n01, xi0, xj1, m)
             + cell_term(n00, xi0, xj0, m);
    return s / (double)m;
}

/* Column sums c_j = number of ones in column j (the marginal counts of Section 2 step 3). */
int mi_oracle_colsums(const uint8_t* X, int64_t m, int64_t n, int64_t ldx, int64_t* c)
{
    if (!X || !c || m <= 0 || n < 0 || ldx < n) return 1;
    for (int64_t j = 0; j < n; ++j) {
        int64_t s = 0;
        for (int64_t k = 0; k < m; ++k) s += X[k * ldx + j] != 0;
        c[j] = s;
    }
    return 0;
}

/*
 * A list of pairs.  For p in [0, npairs): counts and MI of (pi[p], pj[p]).
 * Any of the output arrays may be NULL.
 */
int mi_oracle_pairs(const uint8_t* X, int64_t m, int64_t n, int64_t ldx,
                    int64_t npairs, const int64_t* pi, const int64_t* pj,
                    int64_t* n11, int64_t* n10, int64_t* n01, int64_t* n00, double* mi)
{
    if (!X || m <= 0 || n < 0 || ldx < n || npairs < 0 || (npairs > 0 && (!pi || !pj))) return 1;
    for (int64_t p = 0; p < npairs; ++p)
        if (pi[p] < 0 || pi[p] >= n || pj[p] < 0 || pj[p] >= n) return 2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < npairs; ++p) {
        int64_t a, b, c, d;
        count_pair(X + pi[p], X + pj[p], m, ldx, &a, &b, &c, &d);
        if (n11) n11[p] = a;
        if (n10) n10[p] = b;
        if (n01) n01[p] = c;
        if (n00) n00[p] = d;
        if (mi) mi[p] = mi_oracle_from_counts(a, b, c, d);
    }
    return 0;
}

/*
 * The same two functions on the transposed layout: Xt is n x ldt bytes, row j
 * holding the m entries of column j (ldt >= m).  Only the addressing differs
 * (a column is contiguous), which makes a long column sample cheap to check.
 */
int mi_oracle_colsums_t(const uint8_t* Xt, int64_t m, int64_t n, int64_t ldt, int64_t* c)
{
    if (!Xt || !c || m <= 0 || n < 0 || ldt < m) return 1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j) {
        int64_t s = 0;
        for (int64_t k = 0; k < m; ++k) s += Xt[j * ldt + k] != 0;
        c[j] = s;
    }
    return 0;
}

int mi_oracle_pairs_t(const uint8_t* Xt, int64_t m, int64_t n, int64_t ldt,
                      int64_t npairs, const int64_t* pi, const int64_t* pj,
                      int64_t* n11, int64_t* n10, int64_t* n01, int64_t* n00, double* mi)
{
    if (!Xt || m <= 0 || n < 0 || ldt < m || npairs < 0 || (npairs > 0 && (!pi || !pj))) return 1;
    for (int64_t p = 0; p < npairs; ++p)
        if (pi[p] < 0 || pi[p] >= n || pj[p] < 0 || pj[p] >= n) return 2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < npairs; ++p) {
        int64_t a, b, c, d;
        count_pair(Xt + pi[p] * ldt, Xt + pj[p] * ldt, m, 1, &a, &b, &c, &d);
        if (n11) n11[p] = a;
        if (n10) n10[p] = b;
        if (n01) n01[p] = c;
        if (n00) n00[p] = d;
        if (mi) mi[p] = mi_oracle_from_counts(a, b, c, d);
    }
    return 0;
}

/*
 * The whole matrix: for every pair i <= j count the four cells and evaluate
 * MI; the lower triangle is the mirror (MI and the 1-1 count are symmetric).
 * n11 and mi are n x n row-major; either may be NULL.
 */
int mi_oracle_all(const uint8_t* X, int64_t m, int64_t n, int64_t ldx, int64_t* n11, double* mi)
{
    if (!X || m <= 0 || n < 0 || ldx < n) return 1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i; j < n; ++j) {
            int64_t a, b, c, d;
            count_pair(X + i, X + j, m, ldx, &a, &b, &c, &d);
            double v = mi_oracle_from_counts(a, b, c, d);
            if (n11) { n11[i * n + j] = a; n11[j * n + i] = a; }
            if (mi)  { mi[i * n + j] = v;  mi[j * n + i] = v; }
        }
    }
    return 0;
}

/* Threads the OpenMP loops above will use (1 when built without OpenMP). */
int mi_oracle_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------
 * Categorical variables (the extension to non-binary data named as future
 * work in the Conclusions).  Eq. 1 is a sum over the joint value set of two
 * discrete variables; the binary case restricts it to {0,1} x {0,1}.  Here
 * variable j takes the codes 0 .. L_j - 1, the joint counts of a pair form an
 * L_i x L_j contingency table, and
 *
 *   MI(X_i; X_j) = (1/m) sum_{x,y} n_xy log2( n_xy m / (r_x s_y) )
 *
 * with r_x and s_y the row and column sums of the table (the marginal
 * counts) and 0 log 0 = 0 as above.  The table is counted by a direct loop
 * over the rows, and the marginals are the table's own sums.
 * ---------------------------------------------------------------------- */

/* Contingency table of variables i and j: table[x * Lj + y] = number of rows
 * with X_i = x and X_j = y.  Returns 2 if a code is not below its level count. */
int mi_oracle_cat_table(const uint8_t* X, int64_t m, int64_t ldx, int64_t i, int64_t j,
                        int32_t Li, int32_t Lj, int64_t* table)
{
    if (!X || !table || m <= 0 || Li < 1 || Lj < 1) return 1;
    for (int64_t c = 0; c < (int64_t)Li * Lj; ++c) table[c] = 0;
    for (int64_t k = 0; k < m; ++k) {
        int x = X[k * ldx + i], y = X[k * ldx + j];
        if (x >= Li || y >= Lj) return 2;
        table[(int64_t)x * Lj + y] += 1;
    }
    return 0;
}

/* MI in bits of one pair from its contingency table. */
double mi_oracle_cat_from_table(const int64_t* table, int32_t Li, int32_t Lj)
{
    int64_t m = 0, col[256];
    if (Li < 1 || Lj < 1 || Lj > 256) return NAN;
    for (int32_t y = 0; y < Lj; ++y) col[y] = 0;
    for (int32_t x = 0; x < Li; ++x)
        for (int32_t y = 0; y < Lj; ++y) {
            col[y] += table[(int64_t)x * Lj + y];
            m += table[(int64_t)x * Lj + y];
        }
    if (m <= 0) return NAN;
    double s = 0.0;
    for (int32_t x = 0; x < Li; ++x) {
        int64_t r = 0;                                   /* row sum: marginal count of X_i = x */
        for (int32_t y = 0; y < Lj; ++y) r += table[(int64_t)x * Lj + y];
        for (int32_t y = 0; y < Lj; ++y) s += cell_term(table[(int64_t)x * Lj + y], r, col[y], m);
    }
    return s / (double)m;
}

/* The whole v x v matrix for variables with levels[j] codes each (1 <= levels[j]
 * <= 256).  mi is v x v row-major, both triangles.  Returns 2 on a code out
 * of range, 3 if a table cannot be allocated. */
int mi_oracle_cat_all(const uint8_t* X, int64_t m, int64_t v, int64_t ldx, const int32_t* levels, double* mi)
{
    if (!X || !levels || !mi || m <= 0 || v < 0 || ldx < v) return 1;
    for (int64_t j = 0; j < v; ++j)
        if (levels[j] < 1 || levels[j] > 256) return 1;
    int rc = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < v; ++i) {
        int64_t* table = (int64_t*)malloc(sizeof(int64_t) * 256 * 256);
        if (!table) {
#pragma omp atomic write
            rc = 3;
            continue;
        }
        for (int64_t j = i; j < v; ++j) {
            int r = mi_oracle_cat_table(X, m, ldx, i, j, levels[i], levels[j], table);
            if (r != 0) {
#pragma omp atomic write
                rc = r;
                break;
            }
            double val = mi_oracle_cat_from_table(table, levels[i], levels[j]);
            mi[i * v + j] = val;
            mi[j * v + i] = val;
        }
        free(table);
    }
    return rc;
}
