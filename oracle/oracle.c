/*
 * CPU oracle for the supernodal sparse Cholesky path -- TEST INFRASTRUCTURE.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline legs
 * (one matrix on one core; the batched matrices on a process pool) may load
 * this file's library.  It shares no code with the HIP library: its
 * symbolic analysis follows the plain definitions, its numeric factorization
 * is a scalar left-looking column Cholesky, and everything runs on one core in
 * IEEE binary64 (build with -O2 -ffp-contract=off).
 *
 * What it computes, and where the paper defines it (arXiv:1608.00044):
 *   - A = L L^T with L lower triangular (Section II-A, equation (1));
 *     here for the permuted matrix C = P A P^T, the fill-reducing ordering of
 *     Section V applied first;
 *   - the column algorithm of Algorithm 1 (Section II-A), reorganised
 *     left-looking as described in Section II-C: every update to column j is
 *     applied before column j is factored;
 *   - fill and supernodes (Section II-B), the elimination tree (Section II-B,
 *     parent(j) = first off-diagonal nonzero row of column j of L);
 *   - the 150-column supernode cap (Section III-B);
 *   - the two triangular solves that follow the factorization (Section II-A).
 * Readings where the paper is silent (input triangle, non-fundamental
 * supernodes, cap split, amalgamation rule) are listed with each function.
 *
 * Status convention: 0 = success, >0 = 1-based column whose pivot was not
 * positive, <0 = argument or pattern error.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_ERR_ARG (-1)
#define ORC_ERR_PATTERN (-2)
#define ORC_ERR_OOM (-3)

/* ------------------------------------------------------------------------ */
/* input checks and permutation                                              */
/* ------------------------------------------------------------------------ */

/* The input is the lower triangle of a symmetric matrix in CSC form, 0-based,
 * with row indices strictly increasing inside each column and every row index
 * >= its column (reading: the paper states only that A is symmetric). */
int orc_validate(int64_t n, const int64_t *Ap, const int32_t *Ai, const int32_t *perm) {
    if (n < 0 || (n > 0 && (!Ap || (Ap[n] > 0 && !Ai)))) return ORC_ERR_ARG;
    if (n == 0) return 0;
    if (Ap[0] != 0) return ORC_ERR_PATTERN;
    for (int64_t j = 0; j < n; j++) {
        if (Ap[j + 1] < Ap[j]) return ORC_ERR_PATTERN;
        for (int64_t p = Ap[j]; p < Ap[j + 1]; p++) {
            int64_t i = Ai[p];
            if (i < j || i >= n) return ORC_ERR_PATTERN;
            if (p > Ap[j] && Ai[p - 1] >= i) return ORC_ERR_PATTERN;
        }
    }
    if (perm) {
        char *seen = (char *)calloc((size_t)n, 1);
        if (!seen) return ORC_ERR_OOM;
        int bad = 0;
        for (int64_t k = 0; k < n && !bad; k++) {
            if (perm[k] < 0 || perm[k] >= n || seen[perm[k]]) bad = 1;
            else seen[perm[k]] = 1;
        }
        free(seen);
        if (bad) return ORC_ERR_ARG;
    }
    return 0;
}

/* C = lower(P A P^T) with C_ij = A_{perm[i], perm[j]} (perm[new] = old, NULL =
 * identity).  Every stored A entry (i, j) moves to (max(i', j'), min(i', j'))
 * with i' = pinv[i].  Cp has n+1 entries, Ci/Cx nnz(A) entries; map (may be
 * NULL) receives, for each input entry, its position in C.  Rows of C come out
 * sorted because columns are filled by a counting sort over target rows in
 * increasing order. */
int orc_permute(int64_t n, const int64_t *Ap, const int32_t *Ai, const double *Ax,
                const int32_t *perm, int64_t *Cp, int32_t *Ci, double *Cx, int64_t *map) {
    int st = orc_validate(n, Ap, Ai, perm);
    if (st) return st;
    if (n == 0) { Cp[0] = 0; return 0; }
    int64_t nnz = Ap[n];
    int32_t *pinv = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *ti = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz ? nnz : 1));
    int32_t *tj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz ? nnz : 1));
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *byrow = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz ? nnz : 1));
    int64_t *rowptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!pinv || !ti || !tj || !cnt || !byrow || !rowptr) {
        free(pinv); free(ti); free(tj); free(cnt); free(byrow); free(rowptr);
        return ORC_ERR_OOM;
    }
    for (int64_t k = 0; k < n; k++) pinv[perm ? perm[k] : k] = (int32_t)k;
    for (int64_t j = 0; j < n; j++)
        for (int64_t p = Ap[j]; p < Ap[j + 1]; p++) {
            int32_t a = pinv[Ai[p]], b = pinv[j];
            ti[p] = a > b ? a : b;
            tj[p] = a > b ? b : a;
        }
    /* bucket entries by target row, then deal them to columns in row order */
    for (int64_t p = 0; p < nnz; p++) rowptr[ti[p] + 1]++;
    for (int64_t i = 0; i < n; i++) rowptr[i + 1] += rowptr[i];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    memcpy(fill, rowptr, sizeof(int64_t) * (size_t)n);
    for (int64_t p = 0; p < nnz; p++) byrow[fill[ti[p]]++] = p;
    for (int64_t p = 0; p < nnz; p++) cnt[tj[p] + 1]++;
    for (int64_t j = 0; j < n; j++) cnt[j + 1] += cnt[j];
    memcpy(Cp, cnt, sizeof(int64_t) * (size_t)(n + 1));
    memcpy(fill, cnt, sizeof(int64_t) * (size_t)n);
    for (int64_t q = 0; q < nnz; q++) {
        int64_t p = byrow[q];
        int64_t dst = fill[tj[p]]++;
        Ci[dst] = ti[p];
        if (Cx) Cx[dst] = Ax ? Ax[p] : 0.0;
        if (map) map[p] = dst;
    }
    free(fill); free(pinv); free(ti); free(tj); free(cnt); free(byrow); free(rowptr);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* symbolic analysis by definition                                           */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t n, nnz;
    int64_t *Lp;     /* n+1 */
    int32_t *Li;     /* nnz(L), rows sorted, diagonal first */
    int32_t *parent; /* n, -1 for roots */
    int32_t *cc;     /* n, column counts including the diagonal */
} orc_sym;

/* Structure of L from the elimination process (Section II-B):
 *   S_j = { i >= j : C_ij stored }  U  union over children c of j of (S_c \ {c}),
 *   parent(j) = min(S_j \ {j})  (-1 if empty),   colcount(j) = |S_j|.
 * Children have smaller indices than their parent, so one increasing sweep
 * over j builds every S_j.  No numerical cancellation is considered: stored
 * zeros and fill are structural.  The unsorted lists are sorted by two
 * transpositions (column lists -> row lists -> column lists). */
void *orc_sym_new(int64_t n, const int64_t *Cp, const int32_t *Ci) {
    if (n < 0) return NULL;
    orc_sym *S = (orc_sym *)calloc(1, sizeof(orc_sym));
    if (!S) return NULL;
    S->n = n;
    S->Lp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    S->parent = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    S->cc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int32_t *child_head = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int32_t *child_next = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int64_t cap = (n ? Cp[n] : 0) + n + 16;
    int32_t *U = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap); /* unsorted lists */
    if (!S->Lp || !S->parent || !S->cc || !mark || !child_head || !child_next || !U) goto fail;
    for (int64_t j = 0; j < n; j++) { mark[j] = -1; child_head[j] = -1; }
    int64_t top = 0;
    for (int64_t j = 0; j < n; j++) {
        int64_t start = top;
        /* room for the worst case: every row >= j */
        if (top + (n - j) > cap) {
            int64_t ncap = cap * 2;
            while (ncap < top + (n - j)) ncap *= 2;
            int32_t *nu = (int32_t *)realloc(U, sizeof(int32_t) * (size_t)ncap);
            if (!nu) goto fail;
            U = nu;
            cap = ncap;
        }
        mark[j] = (int32_t)j;
        U[top++] = (int32_t)j;
        for (int64_t p = Cp[j]; p < Cp[j + 1]; p++) {
            int32_t i = Ci[p];
            if (mark[i] != j) { mark[i] = (int32_t)j; U[top++] = i; }
        }
        for (int32_t c = child_head[j]; c != -1; c = child_next[c]) {
            for (int64_t p = S->Lp[c]; p < S->Lp[c + 1]; p++) {
                int32_t i = U[p];
                if (i == c) continue;
                if (mark[i] != j) { mark[i] = (int32_t)j; U[top++] = i; }
            }
        }
        S->Lp[j + 1] = top;
        S->cc[j] = (int32_t)(top - start);
        int32_t par = -1;
        for (int64_t p = start; p < top; p++)
            if (U[p] != j && (par == -1 || U[p] < par)) par = U[p];
        S->parent[j] = par;
        if (par != -1) { child_next[j] = child_head[par]; child_head[par] = (int32_t)j; }
    }
    S->nnz = top;
    {
        /* sort each column's rows: transpose to row lists (columns come out in
         * increasing order), then transpose back (rows come out increasing) */
        int64_t nnz = top;
        int64_t *Rp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
        int32_t *Rj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz ? nnz : 1));
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
        S->Li = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz ? nnz : 1));
        if (!Rp || !Rj || !fill || !S->Li) { free(Rp); free(Rj); free(fill); goto fail; }
        for (int64_t p = 0; p < nnz; p++) Rp[U[p] + 1]++;
        for (int64_t i = 0; i < n; i++) Rp[i + 1] += Rp[i];
        memcpy(fill, Rp, sizeof(int64_t) * (size_t)n);
        for (int64_t j = 0; j < n; j++)
            for (int64_t p = S->Lp[j]; p < S->Lp[j + 1]; p++) Rj[fill[U[p]]++] = (int32_t)j;
        memcpy(fill, S->Lp, sizeof(int64_t) * (size_t)n);
        for (int64_t i = 0; i < n; i++)
            for (int64_t p = Rp[i]; p < Rp[i + 1]; p++) S->Li[fill[Rj[p]]++] = (int32_t)i;
        free(Rp); free(Rj); free(fill);
    }
    free(U); free(mark); free(child_head); free(child_next);
    return S;
fail:
    free(U); free(mark); free(child_head); free(child_next);
    if (S) { free(S->Lp); free(S->parent); free(S->cc); free(S->Li); free(S); }
    return NULL;
}

int64_t orc_sym_nnz(const void *h) { return h ? ((const orc_sym *)h)->nnz : -1; }

void orc_sym_get(const void *h, int32_t *parent, int32_t *cc, int64_t *Lp, int32_t *Li) {
    const orc_sym *S = (const orc_sym *)h;
    if (!S) return;
    if (parent) memcpy(parent, S->parent, sizeof(int32_t) * (size_t)S->n);
    if (cc) memcpy(cc, S->cc, sizeof(int32_t) * (size_t)S->n);
    if (Lp) memcpy(Lp, S->Lp, sizeof(int64_t) * (size_t)(S->n + 1));
    if (Li) memcpy(Li, S->Li, sizeof(int32_t) * (size_t)S->nnz);
}

void orc_sym_free(void *h) {
    orc_sym *S = (orc_sym *)h;
    if (!S) return;
    free(S->Lp); free(S->Li); free(S->parent); free(S->cc); free(S);
}

/* ------------------------------------------------------------------------ */
/* supernode partition                                                       */
/* ------------------------------------------------------------------------ */

/* Supernodes (Section II-B): a maximal run of consecutive columns whose
 * diagonal block is dense and whose rows below it are shared.  Reading: the
 * non-fundamental form -- column j+1 continues column j's supernode iff
 * parent(j) = j+1 and colcount(j) = colcount(j+1) + 1 (this reproduces the ten
 * supernodes of Fig. 1).  Runs wider than cap (Section III-B, 150 columns) are
 * split into ceil(w/cap) pieces as equal as possible, the earlier pieces taking
 * the extra columns.  sn_ptr receives first columns plus the end sentinel n;
 * returns the number of supernodes. */
int64_t orc_supernodes(int64_t n, const int32_t *parent, const int32_t *cc, int32_t cap,
                       int32_t *sn_ptr) {
    if (cap < 1) return ORC_ERR_ARG;
    int64_t ns = 0;
    int64_t j = 0;
    while (j < n) {
        int64_t e = j + 1; /* run is [j, e) */
        while (e < n && parent[e - 1] == e && cc[e - 1] == cc[e] + 1) e++;
        int64_t w = e - j;
        int64_t k = (w + cap - 1) / cap;
        int64_t base = w / k, extra = w % k, c = j;
        for (int64_t q = 0; q < k; q++) {
            sn_ptr[ns++] = (int32_t)c;
            c += base + (q < extra ? 1 : 0);
        }
        j = e;
    }
    sn_ptr[ns] = (int32_t)n;
    return ns;
}

/* Relaxed amalgamation (the paper is silent; the workload asks for ratio 0.1).
 * Reading:
 *   - a supernode s may merge into its supernodal parent p only when p starts
 *     right after s ends (last(s) + 1 = first(p));
 *   - the merged supernode keeps p's rows below last(p) (r_p of them) and stores
 *     every column j of s densely: stored(j) = (last(p) - j + 1) + r_p;
 *   - z = sum over the merged columns of stored(j) - colcount(j) (explicit zeros
 *     relative to the exact structure), T = sum of stored(j); the merge is taken
 *     iff width(s) + width(p) <= cap and (double)z <= ratio * (double)T;
 *   - one pass visits the current supernodes in increasing column order and
 *     tries each against its parent; passes repeat until one merges nothing.
 * sn_ptr (length nsup+1) is rewritten in place; returns the new count. */
int64_t orc_amalgamate(int64_t n, const int32_t *parent, const int32_t *cc, int64_t nsup,
                       int32_t *sn_ptr, int32_t cap, double ratio) {
    if (nsup <= 1 || ratio <= 0.0) return nsup;
    int32_t *first = (int32_t *)malloc(sizeof(int32_t) * (size_t)nsup);
    int32_t *last = (int32_t *)malloc(sizeof(int32_t) * (size_t)nsup);
    int64_t *z = (int64_t *)malloc(sizeof(int64_t) * (size_t)nsup);
    int64_t *T = (int64_t *)malloc(sizeof(int64_t) * (size_t)nsup);
    int32_t *owner = (int32_t *)malloc(sizeof(int32_t) * (size_t)n); /* column -> supernode */
    char *alive = (char *)malloc((size_t)nsup);
    if (!first || !last || !z || !T || !owner || !alive) {
        free(first); free(last); free(z); free(T); free(owner); free(alive);
        return ORC_ERR_OOM;
    }
    for (int64_t s = 0; s < nsup; s++) {
        first[s] = sn_ptr[s];
        last[s] = sn_ptr[s + 1] - 1;
        alive[s] = 1;
        int64_t r = cc[last[s]] - 1;
        z[s] = 0;
        T[s] = 0;
        for (int32_t j = first[s]; j <= last[s]; j++) {
            int64_t stored = (int64_t)(last[s] - j + 1) + r;
            z[s] += stored - cc[j];
            T[s] += stored;
            owner[j] = (int32_t)s;
        }
    }
    int merged_any = 1;
    while (merged_any) {
        merged_any = 0;
        for (int64_t s = 0; s < nsup; s++) {
            if (!alive[s]) continue;
            int32_t pc = parent[last[s]];
            if (pc < 0) continue;
            int32_t p = owner[pc];
            if (first[p] != last[s] + 1) continue;
            if ((int64_t)(last[s] - first[s] + 1) + (last[p] - first[p] + 1) > cap) continue;
            int64_t rp = cc[last[p]] - 1;
            int64_t zn = z[p], Tn = T[p];
            for (int32_t j = first[s]; j <= last[s]; j++) {
                int64_t stored = (int64_t)(last[p] - j + 1) + rp;
                zn += stored - cc[j];
                Tn += stored;
            }
            if (!((double)zn <= ratio * (double)Tn)) continue;
            for (int32_t j = first[s]; j <= last[s]; j++) owner[j] = p;
            first[p] = first[s];
            z[p] = zn;
            T[p] = Tn;
            alive[s] = 0;
            merged_any = 1;
        }
    }
    int64_t ns = 0;
    for (int64_t s = 0; s < nsup; s++)
        if (alive[s]) sn_ptr[ns++] = first[s];
    sn_ptr[ns] = (int32_t)n;
    free(first); free(last); free(z); free(T); free(owner); free(alive);
    return ns;
}

/* ------------------------------------------------------------------------ */
/* numeric factorization                                                     */
/* ------------------------------------------------------------------------ */

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Left-looking column Cholesky of C (lower CSC, rows sorted) into the exact
 * structure (Lp, Li) of orc_sym_new.  For each column j: scatter C(:, j) into a
 * dense accumulator x; subtract, for every earlier column k with L(j, k) != 0
 * taken in increasing k, L(i, k) * L(j, k) from x[i] for the rows i >= j of
 * column k; take the pivot d = x[j]; stop with status j+1 unless d > 0;
 * L(j, j) = sqrt(d) and L(i, j) = x[i] / L(j, j).  This is Algorithm 1 with its
 * updates pulled before each column instead of pushed after it (Section II-C).
 * The columns k that update column j are found with per-row linked lists: after
 * column k is final it waits in the list of its next row below the current one.
 * Returns 0 or the 1-based failing column. */
int orc_factor(int64_t n, const int64_t *Cp, const int32_t *Ci, const double *Cx,
               const int64_t *Lp, const int32_t *Li, double *Lx) {
    if (n == 0) return 0;
    double *x = (double *)calloc((size_t)n, sizeof(double));
    int32_t *head = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *next = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int32_t *ks = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!x || !head || !next || !pos || !ks) {
        free(x); free(head); free(next); free(pos); free(ks);
        return ORC_ERR_OOM;
    }
    for (int64_t j = 0; j < n; j++) head[j] = -1;
    int status = 0;
    for (int64_t j = 0; j < n && !status; j++) {
        for (int64_t p = Cp[j]; p < Cp[j + 1]; p++) x[Ci[p]] = Cx[p];
        int64_t nk = 0;
        for (int32_t k = head[j]; k != -1; k = next[k]) ks[nk++] = k;
        head[j] = -1;
        qsort(ks, (size_t)nk, sizeof(int32_t), cmp_i32);
        for (int64_t q = 0; q < nk; q++) {
            int32_t k = ks[q];
            int64_t at = pos[k]; /* Li[at] == j */
            double ljk = Lx[at];
            for (int64_t t = at; t < Lp[k + 1]; t++) x[Li[t]] -= Lx[t] * ljk;
            pos[k] = at + 1;
            if (at + 1 < Lp[k + 1]) {
                int32_t r = Li[at + 1];
                next[k] = head[r];
                head[r] = k;
            }
        }
        double d = x[j];
        if (!(d > 0.0)) {
            status = (int)(j + 1);
            break;
        }
        double ljj = sqrt(d);
        Lx[Lp[j]] = ljj;
        for (int64_t t = Lp[j] + 1; t < Lp[j + 1]; t++) Lx[t] = x[Li[t]] / ljj;
        for (int64_t t = Lp[j]; t < Lp[j + 1]; t++) x[Li[t]] = 0.0;
        pos[j] = Lp[j] + 1;
        if (Lp[j] + 1 < Lp[j + 1]) {
            int32_t r = Li[Lp[j] + 1];
            next[j] = head[r];
            head[r] = (int32_t)j;
        }
    }
    free(x); free(head); free(next); free(pos); free(ks);
    return status;
}

/* ------------------------------------------------------------------------ */
/* triangular solves                                                         */
/* ------------------------------------------------------------------------ */

/* x = P^T L^{-T} L^{-1} P b for nrhs column-major right-hand sides (Section
 * II-A, the two triangular solves).  (P b)[i] = b[perm[i]]; the forward sweep is
 * column oriented, the backward sweep uses dot products with column j of L. */
int orc_solve(int64_t n, const int64_t *Lp, const int32_t *Li, const double *Lx,
              const int32_t *perm, int64_t nrhs, const double *b, int64_t ldb, double *xo,
              int64_t ldx) {
    if (n == 0) return 0;
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    if (!y) return ORC_ERR_OOM;
    for (int64_t c = 0; c < nrhs; c++) {
        const double *bc = b + c * ldb;
        double *xc = xo + c * ldx;
        for (int64_t i = 0; i < n; i++) y[i] = bc[perm ? perm[i] : i];
        for (int64_t j = 0; j < n; j++) {
            y[j] /= Lx[Lp[j]];
            double yj = y[j];
            for (int64_t t = Lp[j] + 1; t < Lp[j + 1]; t++) y[Li[t]] -= Lx[t] * yj;
        }
        for (int64_t j = n - 1; j >= 0; j--) {
            double s = y[j];
            for (int64_t t = Lp[j] + 1; t < Lp[j + 1]; t++) s -= Lx[t] * y[Li[t]];
            y[j] = s / Lx[Lp[j]];
        }
        for (int64_t i = 0; i < n; i++) xc[perm ? perm[i] : i] = y[i];
    }
    free(y);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* checks: products, residuals, backward error                              */
/* ------------------------------------------------------------------------ */

/* y = A z for a symmetric A given by its lower CSC (nrhs column-major). */
void orc_symv(int64_t n, const int64_t *Ap, const int32_t *Ai, const double *Ax, int64_t nrhs,
              const double *z, int64_t ldz, double *y, int64_t ldy) {
    for (int64_t c = 0; c < nrhs; c++) {
        const double *zc = z + c * ldz;
        double *yc = y + c * ldy;
        for (int64_t i = 0; i < n; i++) yc[i] = 0.0;
        for (int64_t j = 0; j < n; j++)
            for (int64_t p = Ap[j]; p < Ap[j + 1]; p++) {
                int64_t i = Ai[p];
                yc[i] += Ax[p] * zc[j];
                if (i != j) yc[j] += Ax[p] * zc[i];
            }
    }
}

/* Exact ||L L^T - C||_F / ||C||_F over the lower triangle (off-diagonal
 * entries counted twice).  Column j of L L^T below the diagonal is
 * sum over k <= j with L(j, k) != 0 of L(:, k) L(j, k); the columns k are found
 * from the row lists built as in orc_factor.  L has the exact structure of C's
 * factor (Lp, Li). */
double orc_residual_exact(int64_t n, const int64_t *Cp, const int32_t *Ci, const double *Cx,
                          const int64_t *Lp, const int32_t *Li, const double *Lx) {
    if (n == 0) return 0.0;
    double *x = (double *)calloc((size_t)n, sizeof(double));
    int32_t *head = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *next = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!x || !head || !next || !pos) {
        free(x); free(head); free(next); free(pos);
        return -1.0;
    }
    for (int64_t j = 0; j < n; j++) head[j] = -1;
    double num = 0.0, den = 0.0;
    for (int64_t j = 0; j < n; j++) {
        /* L(:, j) L(j, j) */
        double ljj = Lx[Lp[j]];
        for (int64_t t = Lp[j]; t < Lp[j + 1]; t++) x[Li[t]] += Lx[t] * ljj;
        int32_t k = head[j];
        head[j] = -1;
        while (k != -1) {
            int32_t nk = next[k];
            int64_t at = pos[k];
            double ljk = Lx[at];
            for (int64_t t = at; t < Lp[k + 1]; t++) x[Li[t]] += Lx[t] * ljk;
            pos[k] = at + 1;
            if (at + 1 < Lp[k + 1]) {
                int32_t r = Li[at + 1];
                next[k] = head[r];
                head[r] = k;
            }
            k = nk;
        }
        pos[j] = Lp[j] + 1;
        if (Lp[j] + 1 < Lp[j + 1]) {
            int32_t r = Li[Lp[j] + 1];
            next[j] = head[r];
            head[r] = (int32_t)j;
        }
        for (int64_t p = Cp[j]; p < Cp[j + 1]; p++) {
            x[Ci[p]] -= Cx[p];
            den += (Ci[p] == j ? 1.0 : 2.0) * Cx[p] * Cx[p];
        }
        for (int64_t t = Lp[j]; t < Lp[j + 1]; t++) {
            double v = x[Li[t]];
            num += (Li[t] == j ? 1.0 : 2.0) * v * v;
            x[Li[t]] = 0.0;
        }
    }
    free(x); free(head); free(next); free(pos);
    return den > 0.0 ? sqrt(num / den) : sqrt(num);
}

/* Probe estimate ||(L L^T - C) Z||_F / ||C Z||_F for m column-major probe
 * vectors Z (drawn by the caller). */
double orc_residual_probe(int64_t n, const int64_t *Cp, const int32_t *Ci, const double *Cx,
                          const int64_t *Lp, const int32_t *Li, const double *Lx, int64_t m,
                          const double *Z) {
    if (n == 0) return 0.0;
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    double *cz = (double *)malloc(sizeof(double) * (size_t)n);
    if (!w || !v || !cz) { free(w); free(v); free(cz); return -1.0; }
    double num = 0.0, den = 0.0;
    for (int64_t c = 0; c < m; c++) {
        const double *zc = Z + c * n;
        /* w = L^T z */
        for (int64_t j = 0; j < n; j++) {
            double s = 0.0;
            for (int64_t t = Lp[j]; t < Lp[j + 1]; t++) s += Lx[t] * zc[Li[t]];
            w[j] = s;
        }
        /* v = L w */
        for (int64_t i = 0; i < n; i++) v[i] = 0.0;
        for (int64_t j = 0; j < n; j++)
            for (int64_t t = Lp[j]; t < Lp[j + 1]; t++) v[Li[t]] += Lx[t] * w[j];
        orc_symv(n, Cp, Ci, Cx, 1, zc, n, cz, n);
        for (int64_t i = 0; i < n; i++) {
            double d = v[i] - cz[i];
            num += d * d;
            den += cz[i] * cz[i];
        }
    }
    free(w); free(v); free(cz);
    return den > 0.0 ? sqrt(num / den) : sqrt(num);
}

/* Normwise backward error of each solution column (Rigal-Gaches):
 * eta = ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf), A symmetric given
 * by its lower CSC.  eta receives nrhs values. */
void orc_backward_error(int64_t n, const int64_t *Ap, const int32_t *Ai, const double *Ax,
                        int64_t nrhs, const double *b, int64_t ldb, const double *x,
                        int64_t ldx, double *eta) {
    double *r = (double *)malloc(sizeof(double) * (size_t)(n ? n : 1));
    double *rs = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
    if (!r || !rs) { free(r); free(rs); return; }
    for (int64_t j = 0; j < n; j++)
        for (int64_t p = Ap[j]; p < Ap[j + 1]; p++) {
            rs[Ai[p]] += fabs(Ax[p]);
            if (Ai[p] != j) rs[j] += fabs(Ax[p]);
        }
    double anorm = 0.0;
    for (int64_t i = 0; i < n; i++) anorm = rs[i] > anorm ? rs[i] : anorm;
    for (int64_t c = 0; c < nrhs; c++) {
        const double *bc = b + c * ldb;
        const double *xc = x + c * ldx;
        orc_symv(n, Ap, Ai, Ax, 1, xc, n, r, n);
        double rn = 0.0, xn = 0.0, bn = 0.0;
        for (int64_t i = 0; i < n; i++) {
            double d = fabs(bc[i] - r[i]);
            rn = d > rn ? d : rn;
            xn = fabs(xc[i]) > xn ? fabs(xc[i]) : xn;
            bn = fabs(bc[i]) > bn ? fabs(bc[i]) : bn;
        }
        double den = anorm * xn + bn;
        eta[c] = den > 0.0 ? rn / den : rn;
    }
    free(r); free(rs);
}
