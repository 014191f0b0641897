/*
 * Plain, slow, sequential FP64 reference for the row-splitting ILU method.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the CPU oracle that the GPU library
 * is checked against. Only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark may load it; the library never links, calls or includes it
 * and shares no code with it.
 *
 * Everything here is written for readability, not speed: dense work vectors,
 * an explicit depth-first search, full sorts, sequential sums in index order.
 * Built with -ffp-contract=off so every a - (l*u) is two IEEE roundings.
 *
 * Contents
 *   orc_prescale       Section 5.1: scale each column of A to unit 2-norm.
 *   orc_ilup           Algorithms 4, 5 and 6: rectangular ILUP(p, tau) with
 *                      threshold partial pivoting by rows, minimum-row-count
 *                      pivot choice and small-pivot modification.
 *   orc_csr_matvec     y = A x, row by row, sequential sums.
 *   orc_lower_solve    forward substitution with a lower-triangular CSR.
 *   orc_upper_solve    back substitution with an upper-triangular CSR.
 *   orc_levels         depth of every row in the dependency DAG of a
 *                      triangular factor (longest path from a source).
 *   orc_explicit_y     Section 3.2: the rows of Y~ = L2 L1^{-1} as a sparse
 *                      matrix, by back substitution with L1^T on each sparse
 *                      row of L2, small entries dropped.
 *   orc_dot            sum_i a_i b_i, sequential in index order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Section 5.1: A is prescaled so that every column has unit 2-norm.
 * nrm_j = sqrt(sum_i a_ij^2) summed in ascending row order; a_ij / nrm_j.
 * A column with no entries keeps nrm_j = 1. */
int orc_prescale(int64_t n, const int64_t *colptr, const int32_t *rowind, const double *val,
                 double *sval, double *colnorm)
{
    (void)rowind;
    for (int64_t j = 0; j < n; ++j) {
        double s = 0.0;
        for (int64_t e = colptr[j]; e < colptr[j + 1]; ++e) {
            double sq = val[e] * val[e];
            s = s + sq;
        }
        double nrm = (colptr[j + 1] > colptr[j]) ? sqrt(s) : 1.0;
        if (nrm == 0.0) nrm = 1.0;
        colnorm[j] = nrm;
        for (int64_t e = colptr[j]; e < colptr[j + 1]; ++e) sval[e] = val[e] / nrm;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Helpers for the sorts used by the dropping rule and the reach. */

typedef struct {
    double absval;
    double val;
    int64_t key; /* original row index (L) or elimination step (U) */
} orc_entry;

/* larger |v| first; equal |v| -> smaller key first */
static int orc_cmp_drop(const void *pa, const void *pb)
{
    const orc_entry *a = (const orc_entry *)pa, *b = (const orc_entry *)pb;
    if (a->absval > b->absval) return -1;
    if (a->absval < b->absval) return 1;
    if (a->key < b->key) return -1;
    if (a->key > b->key) return 1;
    return 0;
}

static int orc_cmp_i64(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    return (a > b) - (a < b);
}

/* Keep the entries with v != 0 and |v| >= tau, then at most p of the largest
 * |v| (ties: smaller key). Entries are compacted to the front; returns count. */
static int64_t orc_drop(orc_entry *e, int64_t cnt, int64_t p, double tau)
{
    int64_t k = 0;
    for (int64_t i = 0; i < cnt; ++i) {
        if (e[i].val != 0.0 && e[i].absval >= tau) e[k++] = e[i];
    }
    if (k > p) {
        qsort(e, (size_t)k, sizeof(orc_entry), orc_cmp_drop);
        k = p;
    }
    return k;
}

/* Algorithm 6: the replacement value for a zero or too-small pivot,
 * max(beta * ||A(:,j)||_inf, small) with beta = 10^(-2(1 - j/n)), j 1-based. */
static double orc_modified_pivot(int64_t j1, int64_t n, double colmax, double small)
{
    double beta = pow(10.0, -2.0 * (1.0 - (double)j1 / (double)n));
    double v = beta * colmax;
    return v > small ? v : small;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 4: column-wise ILUP(p, tau) of the m x n matrix A (m >= n), given
 * in CSC with ascending row indices (already prescaled by the caller).
 *
 * Outputs
 *   perm[k]            original row placed at position k (k < n: rows of A1)
 *   lptr/lrow/lval     columns of L~ below the unit diagonal; entries are
 *                      (original row index, value); lptr has n+1 entries
 *   uptr/ustep/uval    columns of U~; entries are (elimination step, value),
 *                      the diagonal U(j,j) stored last in column j
 *   nmod               number of modified pivots (Algorithm 6 applications)
 * Capacities lcap / ucap are the lengths of the row/value arrays; the call
 * returns -2 if they are too small, -1 on bad arguments, 0 on success.
 *
 * Per column j (0-based here, j+1 in the paper):
 *   1. x <- A(:,j) scattered into a dense work vector indexed by original row.
 *   2. The steps k < j whose U(k,j) can be nonzero are found by a depth-first
 *      search from the already pivoted rows of A(:,j) through the columns of
 *      L~ (a pivoted row i leads to column pos[i]); they are then taken in
 *      ascending order k: u_k = x[perm[k]] and, if u_k != 0, every row i of
 *      L~(:,k) gets x[i] = x[i] - l_ik * u_k. This is the sparse triangular
 *      solve for U~(1:j-1, j) and the update of L~(j:m, j) (Alg. 4 steps 6, 7).
 *   3. Pivot choice on the unpivoted rows with x[i] != 0 (Algorithm 5):
 *      R = {i : |x_i| >= mu * max|x|}; the row of R with the smallest row count
 *      rc, ties to the larger |x_i|, then to the smaller original row index.
 *      If no unpivoted row is nonzero the row at position j becomes the pivot
 *      row with no interchange. A pivot that is absent or has |x| < small is
 *      replaced by the Algorithm 6 value and counted in nmod.
 *   4. Rows j and pivot are interchanged; U(j,j) = pivot; l_i = x_i / U(j,j).
 *   5. L~(:,j) and U~(1:j-1,j) keep the entries with |v| >= tau, then at most
 *      p of the largest (ties: smaller original row for L, smaller step for U).
 *      The diagonal is never dropped.
 *   6. rc(i) -= 1 for every row i with an entry in column j of A, so rc holds
 *      the number of entries of row i in the columns still to be eliminated.
 */
int orc_ilup(int64_t m, int64_t n, const int64_t *colptr, const int32_t *rowind, const double *val,
             int64_t p, double tau, double mu, double small, int32_t *perm, int64_t *lptr,
             int32_t *lrow, double *lval, int64_t lcap, int64_t *uptr, int32_t *ustep,
             double *uval, int64_t ucap, int64_t *nmod)
{
    if (m < n || n < 1 || p < 0 || !(mu > 0.0) || !(mu <= 1.0) || !(small > 0.0) || tau < 0.0)
        return -1;

    int64_t *pos = malloc(sizeof(int64_t) * (size_t)m);
    int64_t *rc = calloc((size_t)m, sizeof(int64_t));
    double *x = calloc((size_t)m, sizeof(double));
    char *touched = calloc((size_t)m, 1);
    int64_t *tlist = malloc(sizeof(int64_t) * (size_t)m);
    int64_t *visited = malloc(sizeof(int64_t) * (size_t)n);
    int64_t *stack = malloc(sizeof(int64_t) * (size_t)n);
    int64_t *reach = malloc(sizeof(int64_t) * (size_t)n);
    orc_entry *cand = malloc(sizeof(orc_entry) * (size_t)m);
    orc_entry *ucand = malloc(sizeof(orc_entry) * (size_t)n);
    int rcode = 0;
    if (!pos || !rc || !x || !touched || !tlist || !visited || !stack || !reach || !cand || !ucand) {
        rcode = -3;
        goto done;
    }

    for (int64_t i = 0; i < m; ++i) {
        perm[i] = (int32_t)i;
        pos[i] = i;
    }
    for (int64_t k = 0; k < n; ++k) visited[k] = -1;
    /* Algorithm 4 step 1: row counts of A */
    for (int64_t e = 0; e < colptr[n]; ++e) rc[rowind[e]] += 1;

    *nmod = 0;
    lptr[0] = 0;
    uptr[0] = 0;
    int64_t lnz = 0, unz = 0;

    for (int64_t j = 0; j < n; ++j) {
        int64_t nt = 0;
        double colmax = 0.0;
        /* 1. scatter A(:,j) */
        for (int64_t e = colptr[j]; e < colptr[j + 1]; ++e) {
            int64_t i = rowind[e];
            x[i] = val[e];
            if (!touched[i]) {
                touched[i] = 1;
                tlist[nt++] = i;
            }
            double a = fabs(val[e]);
            if (a > colmax) colmax = a;
        }

        /* 2a. reach of the pivoted rows of A(:,j) through the columns of L~ */
        int64_t nreach = 0;
        for (int64_t e = colptr[j]; e < colptr[j + 1]; ++e) {
            int64_t i = rowind[e];
            if (pos[i] >= j) continue;
            int64_t s0 = pos[i];
            if (visited[s0] == j) continue;
            int64_t top = 0;
            stack[top++] = s0;
            visited[s0] = j;
            while (top > 0) {
                int64_t k = stack[--top];
                reach[nreach++] = k;
                for (int64_t f = lptr[k]; f < lptr[k + 1]; ++f) {
                    int64_t r = lrow[f];
                    if (pos[r] < j && visited[pos[r]] != j) {
                        visited[pos[r]] = j;
                        stack[top++] = pos[r];
                    }
                }
            }
        }
        qsort(reach, (size_t)nreach, sizeof(int64_t), orc_cmp_i64);

        /* 2b. eliminate in ascending step order */
        for (int64_t t = 0; t < nreach; ++t) {
            int64_t k = reach[t];
            double uk = x[perm[k]];
            if (uk == 0.0) continue;
            for (int64_t f = lptr[k]; f < lptr[k + 1]; ++f) {
                int64_t r = lrow[f];
                double prod = lval[f] * uk;
                x[r] = x[r] - prod;
                if (!touched[r]) {
                    touched[r] = 1;
                    tlist[nt++] = r;
                }
            }
        }

        /* U candidates: the nonzero u_k of the reached steps */
        int64_t nu = 0;
        for (int64_t t = 0; t < nreach; ++t) {
            int64_t k = reach[t];
            double uk = x[perm[k]];
            if (uk != 0.0) {
                ucand[nu].val = uk;
                ucand[nu].absval = fabs(uk);
                ucand[nu].key = k;
                ++nu;
            }
        }

        /* L candidates: unpivoted rows with a nonzero value */
        int64_t nc = 0;
        for (int64_t t = 0; t < nt; ++t) {
            int64_t i = tlist[t];
            if (pos[i] >= j && x[i] != 0.0) {
                cand[nc].val = x[i];
                cand[nc].absval = fabs(x[i]);
                cand[nc].key = i;
                ++nc;
            }
        }

        /* 3. pivot choice (Algorithm 5) and modification (Algorithm 6) */
        int64_t piv;
        double pivval;
        if (nc == 0) {
            piv = perm[j];
            pivval = orc_modified_pivot(j + 1, n, colmax, small);
            *nmod += 1;
        } else {
            double amax = 0.0;
            for (int64_t c = 0; c < nc; ++c)
                if (cand[c].absval > amax) amax = cand[c].absval;
            double thr = mu * amax;
            int64_t best = -1;
            for (int64_t c = 0; c < nc; ++c) {
                if (!(cand[c].absval >= thr)) continue;
                if (best < 0) {
                    best = c;
                    continue;
                }
                int64_t ri = rc[cand[c].key], rb = rc[cand[best].key];
                if (ri < rb || (ri == rb && (cand[c].absval > cand[best].absval ||
                                             (cand[c].absval == cand[best].absval &&
                                              cand[c].key < cand[best].key))))
                    best = c;
            }
            piv = cand[best].key;
            pivval = cand[best].val;
            if (fabs(pivval) < small) {
                pivval = orc_modified_pivot(j + 1, n, colmax, small);
                *nmod += 1;
            }
        }

        /* 4. interchange rows at positions j and pos[piv] */
        {
            int64_t pp = pos[piv];
            int64_t rj = perm[j];
            perm[pp] = (int32_t)rj;
            pos[rj] = pp;
            perm[j] = (int32_t)piv;
            pos[piv] = j;
        }

        /* scale the L column by the pivot */
        int64_t nl = 0;
        for (int64_t c = 0; c < nc; ++c) {
            if (cand[c].key == piv) continue;
            double l = cand[c].val / pivval;
            cand[nl].val = l;
            cand[nl].absval = fabs(l);
            cand[nl].key = cand[c].key;
            ++nl;
        }

        /* 5. dropping */
        nl = orc_drop(cand, nl, p, tau);
        nu = orc_drop(ucand, nu, p, tau);
        if (lnz + nl > lcap || unz + nu + 1 > ucap) {
            rcode = -2;
            goto done;
        }
        for (int64_t c = 0; c < nl; ++c) {
            lrow[lnz] = (int32_t)cand[c].key;
            lval[lnz] = cand[c].val;
            ++lnz;
        }
        lptr[j + 1] = lnz;
        for (int64_t c = 0; c < nu; ++c) {
            ustep[unz] = (int32_t)ucand[c].key;
            uval[unz] = ucand[c].val;
            ++unz;
        }
        ustep[unz] = (int32_t)j;
        uval[unz] = pivval;
        ++unz;
        uptr[j + 1] = unz;

        /* 6. row counts of the columns still to come */
        for (int64_t e = colptr[j]; e < colptr[j + 1]; ++e) rc[rowind[e]] -= 1;

        /* clear the work vector */
        for (int64_t t = 0; t < nt; ++t) {
            x[tlist[t]] = 0.0;
            touched[tlist[t]] = 0;
        }
    }

done:
    free(pos);
    free(rc);
    free(x);
    free(touched);
    free(tlist);
    free(visited);
    free(stack);
    free(reach);
    free(cand);
    free(ucand);
    return rcode;
}

/* ------------------------------------------------------------------------ */
/* y = A x for CSR A (nrows rows), sums in stored order. */
void orc_csr_matvec(int64_t nrows, const int64_t *rowptr, const int32_t *col, const double *val,
                    const double *xin, double *y)
{
    for (int64_t i = 0; i < nrows; ++i) {
        double s = 0.0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            double prod = val[e] * xin[col[e]];
            s = s + prod;
        }
        y[i] = s;
    }
}

/* Forward substitution, rows ascending: x_i = (b_i - sum_{c<i} L_ic x_c) / d_i
 * with d_i = diag[i], or 1 when diag is NULL. Entries with c >= i are an
 * error (returns the offending row + 1). */
int64_t orc_lower_solve(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                        const double *diag, const double *b, double *xout)
{
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            if (col[e] >= i) return i + 1;
            double prod = val[e] * xout[col[e]];
            s = s + prod;
        }
        double r = b[i] - s;
        xout[i] = diag ? r / diag[i] : r;
    }
    return 0;
}

/* Back substitution, rows descending: x_i = (b_i - sum_{c>i} U_ic x_c) / d_i. */
int64_t orc_upper_solve(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                        const double *diag, const double *b, double *xout)
{
    for (int64_t i = n - 1; i >= 0; --i) {
        double s = 0.0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            if (col[e] <= i) return i + 1;
            double prod = val[e] * xout[col[e]];
            s = s + prod;
        }
        double r = b[i] - s;
        xout[i] = diag ? r / diag[i] : r;
    }
    return 0;
}

/* Level of each row of a triangular CSR: 0 if the row has no off-diagonal
 * entry, else 1 + the largest level among the rows it depends on.
 * forward != 0: dependencies are columns < i (lower); else columns > i. */
void orc_levels(int64_t n, const int64_t *rowptr, const int32_t *col, int forward, int32_t *level)
{
    for (int64_t t = 0; t < n; ++t) {
        int64_t i = forward ? t : n - 1 - t;
        int32_t lv = 0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            int32_t d = level[col[e]] + 1;
            if (d > lv) lv = d;
        }
        level[i] = lv;
    }
}

/* ------------------------------------------------------------------------ */
/* Section 3.2 offers to compute Y~ = L2 L1^{-1} and store it as a sparse
 * matrix by solving L1^T Y~^T = L2^T with a back substitution that handles a
 * sparse right-hand side. Row i of Y~ is the y with y L1 = l (l = row i of
 * L2; L1 unit lower triangular, strictly lower part given by rows). Taking the
 * positions k in descending order, y_k is final once every row k' > k has been
 * processed; a final y_k is then pushed into the lower positions of row k of
 * L1: y_j = y_j - (y_k * l_kj). Positions are reached only from l's pattern
 * and from kept entries, so a max-heap of reached positions gives the order.
 * A final value is dropped (and not pushed further) when it is zero or
 * |y_k| < tauY, the rule the ILUP applies to the entries of L.
 *
 * Rows row_begin.. are written into yptr/ycol/yval (yptr[row_begin] must hold
 * the running count) until the capacity `cap` would be exceeded. Returns the
 * number of rows completed; the caller grows the arrays and calls again from
 * there. Within a row the kept entries are stored in ascending column order. */
static void orc_heap_push(int64_t *h, int64_t *cnt, int64_t v)
{
    int64_t i = (*cnt)++;
    h[i] = v;
    while (i > 0) {
        int64_t parent = (i - 1) / 2;
        if (h[parent] >= h[i]) break;
        int64_t t = h[parent];
        h[parent] = h[i];
        h[i] = t;
        i = parent;
    }
}

static int64_t orc_heap_pop(int64_t *h, int64_t *cnt)
{
    int64_t top = h[0];
    int64_t last = h[--(*cnt)];
    int64_t i = 0;
    if (*cnt == 0) return top;
    h[0] = last;
    for (;;) {
        int64_t a = 2 * i + 1, b = 2 * i + 2, big = i;
        if (a < *cnt && h[a] > h[big]) big = a;
        if (b < *cnt && h[b] > h[big]) big = b;
        if (big == i) break;
        int64_t t = h[big];
        h[big] = h[i];
        h[i] = t;
        i = big;
    }
    return top;
}

int64_t orc_explicit_y(int64_t row_begin, int64_t nrows, int64_t n, const int64_t *l2ptr, const int32_t *l2col,
                       const double *l2val, const int64_t *l1ptr, const int32_t *l1col, const double *l1val,
                       double tauY, int64_t cap, int64_t *yptr, int32_t *ycol, double *yval)
{
    size_t nn = (size_t)(n > 0 ? n : 1);
    double *x = (double *)calloc(nn, sizeof(double));
    char *reached = (char *)calloc(nn, 1);
    int64_t *heap = (int64_t *)malloc(nn * sizeof(int64_t));
    int64_t *kcol = (int64_t *)malloc(nn * sizeof(int64_t));
    double *kval = (double *)malloc(nn * sizeof(double));
    if (!x || !reached || !heap || !kcol || !kval) {
        free(x); free(reached); free(heap); free(kcol); free(kval);
        return -1;
    }
    int64_t row = row_begin;
    for (; row < nrows; ++row) {
        int64_t hc = 0, nk = 0;
        for (int64_t e = l2ptr[row]; e < l2ptr[row + 1]; ++e) {
            int32_t j = l2col[e];
            x[j] = l2val[e];
            reached[j] = 1;
            orc_heap_push(heap, &hc, j);
        }
        while (hc > 0) {
            int64_t k = orc_heap_pop(heap, &hc);
            double yk = x[k];
            reached[k] = 0;
            x[k] = 0.0;
            if (yk == 0.0 || fabs(yk) < tauY) continue;
            kcol[nk] = k;
            kval[nk] = yk;
            nk++;
            for (int64_t e = l1ptr[k]; e < l1ptr[k + 1]; ++e) {
                int32_t j = l1col[e];
                double prod = yk * l1val[e];
                if (!reached[j]) {
                    reached[j] = 1;
                    x[j] = 0.0;
                    orc_heap_push(heap, &hc, j);
                }
                x[j] = x[j] - prod;
            }
        }
        if (yptr[row] + nk > cap) break;
        /* found in descending position order: store ascending */
        for (int64_t t = 0; t < nk; ++t) {
            ycol[yptr[row] + t] = (int32_t)kcol[nk - 1 - t];
            yval[yptr[row] + t] = kval[nk - 1 - t];
        }
        yptr[row + 1] = yptr[row] + nk;
    }
    free(x);
    free(reached);
    free(heap);
    free(kcol);
    free(kval);
    return row;
}

/* sum_i a_i b_i, accumulated sequentially in index order. */
double orc_dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double prod = a[i] * b[i];
        s = s + prod;
    }
    return s;
}
